"""GPU parity of the LNS operators (paper, Sec. "Built-in Operator Hierarchy":
segment shuffle, scatter shuffle, guided rebuild; Tab. weight_preset: LNS
weights and caps), through the C interface, bit for bit against the oracle:
every state field and the run totals after each split of a run and the best
a solve reports, on TSP (every staging), QAP, the VRPTW giant tour (weighted
and lexicographic), with the LNS operators alone and beside the others, with
their initial weights raised so that many candidates hold LNS steps (the
epoch is long, so the cap applies late), per-solution weights, tiny sizes,
the 442-city instance (the largest destroyed part), and a batch."""
import dataclasses
import os
import time

import numpy as np
import pytest

import oracle
import synth
from paper_2603_19163_amd import gx

pytestmark = pytest.mark.gpu

KEYS = ["g", "stag", "T_q16", "epoch_ref", "accepted", "w_op", "w_k", "u_op", "v_op", "u_k", "v_k",
        "cur", "cur_f", "best", "best_f"]
TOT = [("u_op", "tot_u_op"), ("v_op", "tot_v_op"), ("u_k", "tot_u_k"), ("v_k", "tot_v_k")]
LNS, ALL = synth.LNS_OPS, synth.PERM_LNS_OPS
RAISED = [0, 0, 0, 0, 0, 30000, 30000, 30000]      # LNS weights raised for the first epoch
THREADS = max(1, min(16, os.cpu_count() or 1))


@pytest.fixture(scope="module")
def ctx():
    c = gx.gx_create(0)
    yield c
    gx.gx_destroy(c)


def P(G, **kw):
    kw.setdefault("alpha_q32", synth.alpha_q32_for(G))
    return synth.Params(generations=G, **kw)


def compare(ctx, job, p, inst, st, what, lex=False):
    g = gx.gx_snapshot(ctx, job, p.population, synth.solution_len(inst))
    for k in KEYS:
        a, b = np.asarray(g[k]), np.asarray(st[k])
        assert np.array_equal(a, b), f"{what}: {k} gpu {a.ravel()[:10]} oracle {b.ravel()[:10]}"
    if lex:
        v = gx.gx_snapshot_lex(ctx, job, p.population)
        for k in ("cur_v", "best_v", "ref_v"):
            assert np.array_equal(v[k], st[k]), f"{what}: {k}"
    s = gx.gx_job_stats(ctx, job)
    for gk, ok in TOT:
        assert np.array_equal(s[gk], st[ok]), f"{what}: run total {gk} gpu {s[gk]} oracle {st[ok]}"
    assert s["accepted"] == st["accepted"]


def run_parity(ctx, inst, p, splits, what, lex=False, threads=1):
    print(f"[lns] {what} kind={inst.kind} n={inst.n} P={p.population} C={p.candidates} mask={p.op_mask:#x}",
          flush=True)
    h = gx.gx_instance_upload(ctx, inst)
    job = gx.gx_job_create(ctx, h, p)
    o = oracle.OracleInstance(inst)
    st = o.init(p)
    compare(ctx, job, p, inst, st, f"{what} init", lex)
    for i, s in enumerate(splits):
        gx.gx_job_advance(ctx, job, s)
        o.run(p, st, s, threads=threads)
        compare(ctx, job, p, inst, st, f"{what} split {i}", lex)
    gx.gx_job_free(ctx, job)
    job = gx.gx_solve(ctx, h, p)
    gx.gx_wait(ctx, job)
    sol, f = gx.gx_fetch_best(ctx, job, synth.solution_len(inst))
    fo, io = o.best_of(st)
    assert f == fo and np.array_equal(sol, st["best"][io]), (what, f, fo)
    gx.gx_job_free(ctx, job)
    gx.gx_instance_free(ctx, h)
    return st


@pytest.mark.parametrize("staging", [1, 2, 3, 4])
def test_tsp_lns(ctx, staging):
    inst = synth.tsp_clustered(70, 2, key=21)
    p = P(36, seed=5, population=5, candidates=128, op_mask=ALL, epoch=30, staging=staging, init_weight_q16=RAISED)
    st = run_parity(ctx, inst, p, [7, 29], f"tsp staging {staging}")
    assert int(st["tot_u_op"][5:8].min()) > 0


@pytest.mark.parametrize("case", ["lns-only", "credit1", "sol-scope"])
def test_tsp_lns_modes(ctx, case):
    inst = synth.tsp_uniform(45, 3, key=22)
    kw = {"lns-only": dict(op_mask=LNS), "credit1": dict(op_mask=ALL, credit=1, init_weight_q16=RAISED),
          "sol-scope": dict(op_mask=ALL, aos_scope=1, epoch=4, init_weight_q16=RAISED)}[case]
    kw.setdefault("epoch", 25)
    p = P(30, seed=9, population=4, candidates=100, **kw)
    run_parity(ctx, inst, p, [11, 19], f"tsp {case}")


def test_qap_lns(ctx):
    inst = synth.qap_random(26, 3, key=23)
    p = P(30, seed=4, population=4, candidates=128, op_mask=ALL, epoch=25, init_weight_q16=RAISED)
    st = run_parity(ctx, inst, p, [9, 21], "qap")
    assert int(st["tot_u_op"][5:8].min()) > 0


def test_qap_lns_only_wide_sums(ctx):
    base = synth.qap_random(20, 4, key=24)
    inst = dataclasses.replace(base, a=base.a * 1000, b=base.b * 160)   # the 64-bit row sums
    run_parity(ctx, inst, P(20, seed=2, population=3, candidates=96, op_mask=LNS), [20], "qap wide")


@pytest.mark.parametrize("mode", ["weighted", "lex"])
def test_vrptw_lns(ctx, mode):
    base = synth.vrptw_random(30, 5, key=25)
    inst = dataclasses.replace(base, vehicles=4, obj_weights=(6, 2, 2)) if mode == "weighted" else \
        dataclasses.replace(base, vehicles=4, lex_order=(2, 1, 0), lex_tol=(0, 25, 0))
    p = P(30, seed=6, population=4, candidates=128, op_mask=ALL, epoch=25, init_weight_q16=RAISED)
    run_parity(ctx, inst, p, [13, 17], f"vrptw {mode}", lex=mode == "lex")


@pytest.mark.parametrize("n", [1, 2, 3, 17])
def test_lns_tiny(ctx, n):
    for inst in (synth.tsp_uniform(n, 1, key=30 + n), synth.qap_random(n, 1, key=40 + n)):
        run_parity(ctx, inst, P(12, seed=7, population=3, candidates=65, op_mask=ALL, init_weight_q16=RAISED),
                   [12], f"tiny {n}")


def test_tsp442_lns(ctx):
    """The 442-city instance: 29 entries destroyed per LNS step."""
    inst, _ = synth.c2_tsp442(population=64, generations=24)
    p = P(24, seed=42, population=64, candidates=128, op_mask=ALL, epoch=20, init_weight_q16=RAISED)
    run_parity(ctx, inst, p, [10, 14], "tsp442", threads=16)


def test_lns_batch(ctx):
    insts = [synth.tsp_uniform(40, 6, key=50), synth.qap_random(18, 6, key=51), synth.vrptw_random(20, 6, key=52),
             synth.tsp_uniform(33, 7, key=53)]
    masks = [ALL, ALL, ALL, synth.PERM_OPS]
    params = [P(25, seed=1 + i, population=3 + i, candidates=128, op_mask=m, epoch=20, init_weight_q16=RAISED)
              for i, m in enumerate(masks)]
    hs = [gx.gx_instance_upload(ctx, i) for i in insts]
    jobs = gx.gx_solve_batch(ctx, hs, params)
    gx.gx_wait(ctx)
    for inst, p, job in zip(insts, params, jobs):
        o = oracle.OracleInstance(inst)
        st = o.solve(p)
        fo, io = o.best_of(st)
        sol, f = gx.gx_fetch_best(ctx, job, inst.n)
        assert f == fo and np.array_equal(sol, st["best"][io]), (inst.kind, f, fo)
    for j in jobs:
        gx.gx_job_free(ctx, j)
    for h in hs:
        gx.gx_instance_free(ctx, h)


def test_lns_masks(ctx):
    """LNS bits are taken only where they are LNS operators."""
    h = gx.gx_instance_upload(ctx, synth.knapsack_random(20, 1, key=60))
    with pytest.raises(gx.GxError):
        gx.gx_job_create(ctx, h, P(5, seed=1, population=2, op_mask=LNS))
    gx.gx_instance_free(ctx, h)
    h = gx.gx_instance_upload(ctx, synth.tsp_uniform(20, 1, key=61))
    job = gx.gx_job_create(ctx, h, P(5, seed=1, population=2, op_mask=LNS))
    st = gx.gx_snapshot(ctx, job, 2, 20)
    assert (st["w_op"][5:8] > 0).all() and not st["w_op"][:5].any()
    gx.gx_job_free(ctx, job)
    job = gx.gx_job_create(ctx, h, P(5, seed=1, population=2))
    st = gx.gx_snapshot(ctx, job, 2, 20)
    assert not st["w_op"][5:8].any()                 # op_mask 0: no LNS
    gx.gx_job_free(ctx, job)
    gx.gx_instance_free(ctx, h)


def test_served_lanes_keep_variants_apart(ctx):
    """Requests of one kind that need different kernels (LNS or not, giant
    tour or rows) are served together, each equal to the oracle."""
    reqs = [(synth.tsp_uniform(40, 8, key=70), P(30, seed=1, population=4, op_mask=ALL, epoch=20,
                                                  init_weight_q16=RAISED)),
            (synth.tsp_uniform(40, 9, key=71), P(30, seed=2, population=4, op_mask=synth.PERM_OPS)),
            (synth.vrptw_random(20, 3, key=72), P(30, seed=3, population=4)),
            (synth.vrptw_rows(20, 3, key=73, vehicles=4), P(30, seed=4, population=4)),
            (synth.vrptw_random(20, 4, key=74), P(30, seed=5, population=4, op_mask=ALL, init_weight_q16=RAISED)),
            (synth.qap_random(16, 5, key=75), P(30, seed=6, population=4, op_mask=ALL, init_weight_q16=RAISED))]
    srv = gx.gx_server_create(ctx, quantum_epochs=1)
    tickets = [gx.gx_server_submit(srv, i, p) for i, p in reqs]
    got = {}
    t_end = time.time() + 60
    while len(got) < len(reqs) and time.time() < t_end:
        for k, t in enumerate(tickets):
            if k not in got:
                r = gx.gx_server_poll(srv, t, synth.solution_len(reqs[k][0]))
                if r is not None:
                    got[k] = r
        time.sleep(0.002)
    gx.gx_server_destroy(srv)
    assert len(got) == len(reqs), f"served {sorted(got)} of {len(reqs)}"
    for k, (inst, p) in enumerate(reqs):
        o = oracle.OracleInstance(inst)
        st = o.solve(p)
        fo, io = o.best_of(st)
        assert got[k][1] == fo and np.array_equal(got[k][0], st["best"][io]), (k, got[k][1], fo)


@pytest.mark.parametrize("scope", [0, 1])
def test_per_sequence_caps(ctx, scope):
    """Caller weight caps (one above the floor, one below it, defaults for the
    rest), under both AOS scopes, and on the multi-row VRPTW's row operators."""
    caps = [20000, 500, 0, 0, 0, 0, 900, 0]
    inst = synth.tsp_uniform(50, 4, key=80)
    p = P(40, seed=3, population=4, candidates=128, op_mask=ALL, epoch=4, aos_scope=scope, weight_cap_q16=caps)
    run_parity(ctx, inst, p, [13, 27], f"caps scope {scope}")
    rows = dataclasses.replace(synth.vrptw_rows(18, 5, key=81, vehicles=4), capacity=70)
    pr = P(30, seed=4, population=4, candidates=128, epoch=3, aos_scope=scope,
           weight_cap_q16=[0, 0, 3000, 0, 0, 600, 0, 40000])
    run_parity(ctx, rows, pr, [30], f"rows caps scope {scope}")


@pytest.mark.parametrize("mode", [dict(islands=2, migrate_epochs=2, migrate_mode=0, elite_epochs=3),
                                  dict(islands=4, migrate_epochs=1, migrate_mode=2, migrate_n=1)])
def test_lns_with_islands(ctx, mode):
    """The LNS kernels with island migration and elite injection at the epoch ends."""
    inst = synth.tsp_clustered(60, 5, key=90)
    p = P(36, seed=8, population=8, candidates=128, op_mask=ALL, epoch=3, init_weight_q16=RAISED, **mode)
    run_parity(ctx, inst, p, [7, 29], f"lns islands {mode['migrate_mode']}")
    vr = dataclasses.replace(synth.vrptw_random(24, 6, key=91), vehicles=4)
    run_parity(ctx, vr, P(24, seed=9, population=8, candidates=128, op_mask=ALL, epoch=3,
                          init_weight_q16=RAISED, **mode), [24], f"vrptw lns islands {mode['migrate_mode']}")



def test_c3_lns_whole_run(ctx):
    """The 100-customer giant-tour configuration with the LNS operators as the
    per-kind bench row runs it (P = 64, 5000 generations, presets): state and
    run totals compared with the oracle every 1000 generations."""
    base, p0 = synth.c3_vrptw(seed=42)
    p = p0.with_(op_mask=ALL)
    h = gx.gx_instance_upload(ctx, base)
    job = gx.gx_job_create(ctx, h, p)
    o = oracle.OracleInstance(base)
    st = o.init(p)
    compare(ctx, job, p, base, st, "C3 LNS init")
    for k in range(5):
        gx.gx_job_advance(ctx, job, 1000)
        t = time.perf_counter()
        o.run(p, st, 1000, threads=THREADS)
        print(f"[lns] C3 LNS generations {1000 * k}..{1000 * (k + 1)}: oracle {time.perf_counter() - t:.1f} s",
              flush=True)
        compare(ctx, job, p, base, st, f"C3 LNS generation {1000 * (k + 1)}")
    assert st["tot_v_op"][5:8].sum() > 0   # LNS steps were drawn
    sol, f = gx.gx_fetch_best(ctx, job, base.n)
    fo, io = o.best_of(st)
    assert f == fo and np.array_equal(sol, st["best"][io])
    gx.gx_job_free(ctx, job)
    gx.gx_instance_free(ctx, h)


def test_c2_lns_windows(ctx):
    """The 442-city LNS row of the per-kind bench (autosized population, the
    default staging, 20 000 generations): 20-generation windows at generations
    1000, 5000, 10 000 and 19 980 of one job, each resumed by the oracle from the GPU's state."""
    inst, p = synth.c2_tsp442(population=0, generations=20_000)
    p = p.with_(op_mask=synth.PERM4_OPS | LNS)
    h = gx.gx_instance_upload(ctx, inst)
    p = p.with_(population=gx.gx_autosize_population(ctx, h, p))
    job = gx.gx_job_create(ctx, h, p)
    o = oracle.OracleInstance(inst)
    g = 0
    for start in (1000, 5000, 10_000, 19_980):
        gx.gx_job_advance(ctx, job, start - g)
        a = gx.gx_snapshot(ctx, job, p.population, inst.n)
        gx.gx_job_advance(ctx, job, 20)
        b = gx.gx_snapshot(ctx, job, p.population, inst.n)
        g = start + 20
        assert a["g"] == start and b["g"] == g
        t = time.perf_counter()
        o.run(p, a, 20, threads=THREADS)
        print(f"[lns] C2 LNS P={p.population} window {start}..{g}: best {int(b['best_f'].min())}, "
              f"oracle {time.perf_counter() - t:.1f} s", flush=True)
        for k in KEYS:
            x, y = np.asarray(b[k]), np.asarray(a[k])
            assert np.array_equal(x, y), f"C2 LNS window {start}: {k} gpu {x.ravel()[:6]} oracle {y.ravel()[:6]}"
    gx.gx_job_free(ctx, job)
    gx.gx_instance_free(ctx, h)
