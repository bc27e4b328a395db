"""GPU parity of the multi-row VRPTW form (paper, Sec. "Solution Structure";
Tab. operators, row level; Tab. generality; Sec. "Partition Encoding Heuristic
Initialization"), through the C interface, bit for bit against the oracle:
every state field and the run totals after each split of a run, the best a
solve reports, with every operator set of the form (row operators alone,
with and without 3-opt, both credit rules), the weighted and lexicographic
objectives, per-solution weights, islands and elite injection, tiny and
degenerate row counts (one row: no split is possible; as many rows as
customers), a batch mixing forms and kinds, a served request, resume from a
snapshot, the refused inputs, and the 100-customer configuration over a
whole 5000-generation run.

Instances are the VRPTW stand-ins of synth.vrptw_random with the capacity set
so that loads above it occur (the row form's penalty takes part)."""
import dataclasses
import os
import time

import numpy as np
import pytest

import oracle
import synth
from paper_2603_19163_amd import gx

pytestmark = pytest.mark.gpu

DIST, VEH, LONG = 1, 2, 3
KEYS = ["g", "stag", "T_q16", "epoch_ref", "accepted", "w_op", "w_k", "u_op", "v_op", "u_k", "v_k",
        "cur", "cur_f", "best", "best_f"]
TOT = [("u_op", "tot_u_op"), ("v_op", "tot_v_op"), ("u_k", "tot_u_k"), ("v_k", "tot_v_k")]
THREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def ctx():
    c = gx.gx_create(0)
    yield c
    gx.gx_destroy(c)


def rows_inst(n, R, key, cap=80, **kw):
    return dataclasses.replace(synth.vrptw_rows(n, 13, key=key, vehicles=R), capacity=cap, **kw)


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
    assert s["accepted"] == st["accepted"] and s["generations_done"] == st["g"]


def run_parity(ctx, inst, p, splits, what, lex=False):
    print(f"[rows] {what} n={inst.n} rows={inst.vehicles} P={p.population} C={p.candidates} "
          f"mask={p.op_mask:#x}", flush=True)
    h = gx.gx_instance_upload(ctx, inst)
    job = gx.gx_job_create(ctx, h, p)
    o = oracle.OracleInstance(inst)
    st = o.init(p)
    compare(ctx, job, p, inst, st, f"{what} init", lex)
    for i, s in enumerate(splits):
        gx.gx_job_advance(ctx, job, s)
        o.run(p, st, s)
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


R_OPS, ALL = synth.ROW_OPS, synth.ROWS_ALL_OPS
CASES = {
    # name: (n, rows, capacity, params)
    "all-ops": (20, 5, 70, dict(candidates=128, op_mask=ALL)),
    "row-ops-only": (18, 6, 60, dict(candidates=100, op_mask=R_OPS)),
    "no-3opt-credit1": (22, 5, 90, dict(candidates=150, credit=1, op_mask=synth.PERM4_OPS | R_OPS)),
    "one-row": (15, 1, 10**4, dict(candidates=128, op_mask=ALL)),
    "row-per-customer": (12, 12, 50, dict(candidates=200, op_mask=ALL)),
    "3opt-and-merge": (16, 4, 70, dict(candidates=64, op_mask=(1 << synth.OP_3OPT) | (1 << synth.OP_ROWMERGE))),
    "split-merge": (20, 7, 50, dict(candidates=96, op_mask=(1 << synth.OP_ROWSPLIT) | (1 << synth.OP_ROWMERGE)
                                    | (1 << synth.OP_INSERT))),
}


@pytest.mark.parametrize("case", list(CASES))
def test_rows_parity(ctx, case):
    n, R, cap, kw = CASES[case]
    inst = rows_inst(n, R, 40 + len(case), cap)
    p = P(45, seed=17, population=6, epoch=4, stagnation_epochs=2, **kw)
    st = run_parity(ctx, inst, p, [9, 3, 25], case)
    if p.op_mask & R_OPS:   # the row operators were drawn and credited
        assert int(st["tot_u_op"][5:8].sum()) > 0


def test_rows_weighted_objectives(ctx):
    inst = rows_inst(24, 6, 35, 80, obj_weights=(6, 2, 2))
    run_parity(ctx, inst, P(40, seed=5, population=5, candidates=128, epoch=5), [13, 27], "weighted")


@pytest.mark.parametrize("order,tol", [((VEH, DIST, 0), (0, 30, 0)), ((DIST, LONG, VEH), (25, 5, 0))])
def test_rows_lexicographic(ctx, order, tol):
    inst = rows_inst(22, 6, 36 + order[0], 70, lex_order=order, lex_tol=tol)
    run_parity(ctx, inst, P(40, seed=9, population=6, candidates=128, epoch=4, stagnation_epochs=2),
               [11, 29], f"lex {order}", lex=True)


def test_rows_per_solution_weights(ctx):
    inst = rows_inst(20, 5, 37, 70)
    p = P(40, seed=3, population=5, candidates=128, epoch=4, aos_scope=1)
    h = gx.gx_instance_upload(ctx, inst)
    job = gx.gx_job_create(ctx, h, p)
    o = oracle.OracleInstance(inst)
    st = o.init(p)
    for s in (12, 28):
        gx.gx_job_advance(ctx, job, s)
        o.run(p, st, s)
        compare(ctx, job, p, inst, st, f"aos_scope 1 after {s}")
        assert gx.gx_snapshot_aos(ctx, job, p.population).tobytes() == st["saos"].tobytes()
    gx.gx_job_free(ctx, job)
    gx.gx_instance_free(ctx, h)


@pytest.mark.parametrize("mode", [dict(islands=2, migrate_epochs=2, migrate_mode=0, elite_epochs=3),
                                  dict(islands=4, migrate_epochs=1, migrate_mode=2, migrate_n=1)])
def test_rows_islands(ctx, mode):
    inst = rows_inst(20, 5, 38, 70)
    run_parity(ctx, inst, P(36, seed=11, population=8, candidates=128, epoch=3, **mode), [7, 29],
               f"islands {mode['migrate_mode']}")


@pytest.mark.parametrize("n,R", [(1, 1), (1, 3), (2, 1), (3, 2), (5, 5)])
def test_rows_tiny(ctx, n, R):
    inst = rows_inst(n, R, 50 + 10 * n + R, 60)
    run_parity(ctx, inst, P(12, seed=2, population=3, candidates=65, op_mask=ALL), [12], f"tiny {n}x{R}")


def test_rows_resume_and_restore_checks(ctx):
    inst = rows_inst(18, 5, 39, 70)
    p = P(40, seed=6, population=4, candidates=128, epoch=5)
    N = synth.solution_len(inst)
    h = gx.gx_instance_upload(ctx, inst)
    a = gx.gx_job_create(ctx, h, p)
    gx.gx_job_advance(ctx, a, 15)
    snap = gx.gx_snapshot(ctx, a, p.population, N)
    b = gx.gx_job_create(ctx, h, p)
    gx.gx_job_restore(ctx, b, snap)
    gx.gx_job_advance(ctx, a, 25)
    gx.gx_job_advance(ctx, b, 25)
    sa, sb = gx.gx_snapshot(ctx, a, p.population, N), gx.gx_snapshot(ctx, b, p.population, N)
    for k in KEYS:
        assert np.array_equal(np.asarray(sa[k]), np.asarray(sb[k])), k
    # a solution must end with a row marker
    bad = dict(snap)
    cur = snap["cur"].copy()
    cur[0, [-1, 0]] = cur[0, [0, -1]]
    if cur[0, -1] >= inst.n:          # the swap moved a marker to the end: take a customer instead
        j = int(np.argmax(cur[0] < inst.n))
        cur[0, [-1, j]] = cur[0, [j, -1]]
    bad["cur"] = cur
    with pytest.raises(gx.GxError):
        gx.gx_job_restore(ctx, b, bad)
    for j in (a, b):
        gx.gx_job_free(ctx, j)
    gx.gx_instance_free(ctx, h)


def test_rows_batch_and_served(ctx):
    insts = [rows_inst(25, 6, 60, 80), synth.vrptw_random(25, 12, key=61), rows_inst(14, 3, 62, 90),
             synth.tsp_uniform(30, 3, key=63)]
    params = [P(30, seed=1 + i, population=4 + i, candidates=128, epoch=5) for i in range(len(insts))]
    hs = [gx.gx_instance_upload(ctx, i) for i in insts]
    jobs = gx.gx_solve_batch(ctx, hs, params)
    gx.gx_wait(ctx)
    for inst, p, job in zip(insts, params, jobs):
        o = oracle.OracleInstance(inst)
        st = o.solve(p)
        fo, io = o.best_of(st)
        sol, f = gx.gx_fetch_best(ctx, job, synth.solution_len(inst))
        assert f == fo and np.array_equal(sol, st["best"][io]), (inst.kind, f, fo)
    for j in jobs:
        gx.gx_job_free(ctx, j)
    for h in hs:
        gx.gx_instance_free(ctx, h)
    reqs = [(rows_inst(22, 5, 64, 70), P(40, seed=3, population=4)),
            (rows_inst(16, 4, 65, 60, lex_order=(VEH, DIST, 0), lex_tol=(0, 10, 0)), P(40, seed=4, population=4))]
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
    assert len(got) == len(reqs)
    for k, (inst, p) in enumerate(reqs):
        o = oracle.OracleInstance(inst)
        st = o.solve(p)
        fo, io = o.best_of(st)
        assert got[k][1] == fo and np.array_equal(got[k][0], st["best"][io]), (k, got[k][1], fo)


def test_rows_refusals(ctx):
    base = rows_inst(12, 4, 66, 70)
    for kw in (dict(vehicles=0), dict(capacity=(1 << 22) + 1), dict(vehicles=251)):
        with pytest.raises(gx.GxError):
            gx.gx_instance_upload(ctx, dataclasses.replace(base, **kw))
    h = gx.gx_instance_upload(ctx, base)
    # operators of other encodings enable nothing here
    with pytest.raises(gx.GxError):
        gx.gx_job_create(ctx, h, P(5, seed=1, population=2, op_mask=1 << synth.OP_FLIP))
    # on the giant tour the same bits name the LNS operators, not the row ones
    gi = synth.vrptw_random(12, 2, key=67)
    g = gx.gx_instance_upload(ctx, gi)
    job = gx.gx_job_create(ctx, g, P(5, seed=1, population=2, op_mask=R_OPS))
    w = gx.gx_snapshot(ctx, job, 2, gi.n)["w_op"]
    o = oracle.OracleInstance(gi)
    assert list(w) == list(o.initial_weights(R_OPS)) and o.lns_cap() > 0
    gx.gx_job_free(ctx, job)
    gx.gx_instance_free(ctx, g)
    gx.gx_instance_free(ctx, h)


def test_c3_rows_whole_run(ctx):
    """The 100-customer configuration in the multi-row form (25 rows, every
    operator of the form, P = 64, 5000 generations) as the per-kind bench row
    runs it: state compared with the oracle every 1000 generations."""
    inst, p = synth.c3_vrptw_rows(seed=42)
    N = synth.solution_len(inst)
    h = gx.gx_instance_upload(ctx, inst)
    job = gx.gx_job_create(ctx, h, p)
    o = oracle.OracleInstance(inst)
    st = o.init(p)
    compare(ctx, job, p, inst, st, "C3 rows init")
    for k in range(5):
        gx.gx_job_advance(ctx, job, 1000)
        t = time.perf_counter()
        o.run(p, st, 1000, threads=THREADS)
        print(f"[rows] C3 rows generations {1000 * k}..{1000 * (k + 1)}: oracle {time.perf_counter() - t:.1f} s",
              flush=True)
        compare(ctx, job, p, inst, st, f"C3 rows generation {1000 * (k + 1)}")
    sol, f = gx.gx_fetch_best(ctx, job, N)
    fo, io = o.best_of(st)
    assert f == fo and np.array_equal(sol, st["best"][io])
    gx.gx_job_free(ctx, job)
    gx.gx_instance_free(ctx, h)
