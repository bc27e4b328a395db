"""GPU parity of the VRPTW lexicographic mode (paper, Sec. "Multi-Objective
Optimization Modes"; Tab. lexicographic_mode), through the C interface,
bit for bit against the oracle: every state field, the objective vectors of
every solution, the stagnation reference and the run totals after each split
of the run; the best solution a solve reports; a batch that mixes modes; a
served request; island migration and elite injection; the portfolio pick;
and the combinations the interface refuses.

The instances are VRPTW stand-ins (synth.vrptw_random) with a small fleet, so
that the penalty level (lateness and fleet excess) takes part in the
comparisons; the level orders and tolerances cover one, two and three levels,
tolerances of zero and wider than typical differences, and candidate counts
that end a chunk and a round of 64 early."""
import dataclasses
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


@pytest.fixture(scope="module")
def ctx():
    c = gx.gx_create(0)
    yield c
    gx.gx_destroy(c)


def lex_inst(n, key, order, tol, vehicles=3):
    base = synth.vrptw_random(n, 11, key=key)
    return dataclasses.replace(base, vehicles=vehicles, lex_order=order, lex_tol=tol)


def P(G, **kw):
    kw.setdefault("alpha_q32", synth.alpha_q32_for(G))
    return synth.Params(generations=G, **kw)


def compare(ctx, job, p, n, st, what):
    g = gx.gx_snapshot(ctx, job, p.population, n)
    for k in KEYS:
        a, b = np.asarray(g[k]), np.asarray(st[k])
        assert np.array_equal(a, b), f"{what}: {k} gpu {a.ravel()[:8]} oracle {b.ravel()[:8]}"
    v = gx.gx_snapshot_lex(ctx, job, p.population)
    for k in ("cur_v", "best_v", "ref_v"):
        assert np.array_equal(v[k], st[k]), f"{what}: {k} gpu {v[k].ravel()[:8]} oracle {st[k].ravel()[:8]}"
    s = gx.gx_job_stats(ctx, job)
    for gk, ok in TOT:
        assert np.array_equal(s[gk], st[ok]), f"{what}: run total {gk}"
    assert s["accepted"] == st["accepted"] and s["generations_done"] == st["g"]


CASES = {
    # name: (n, order, tol, params)
    "dist-veh-long": (24, (DIST, VEH, LONG), (30, 0, 5), dict(candidates=128)),
    "veh-dist": (30, (VEH, DIST, 0), (0, 100, 0), dict(candidates=100)),
    "long-only": (20, (LONG, 0, 0), (0, 0, 0), dict(candidates=200)),
    "dist-wide": (26, (DIST, LONG, 0), (10**6, 0, 0), dict(candidates=64)),
    "credit1-3opt": (28, (DIST, VEH, 0), (40, 0, 0), dict(candidates=150, credit=1, op_mask=synth.PERM_OPS)),
    "three-opt-only": (22, (VEH, LONG, DIST), (0, 20, 0), dict(candidates=96, op_mask=1 << synth.OP_3OPT)),
}


@pytest.mark.parametrize("case", list(CASES))
def test_lex_parity(ctx, case):
    n, order, tol, kw = CASES[case]
    inst = lex_inst(n, 60 + len(case), order, tol)
    p = P(57, seed=21, population=6, epoch=4, stagnation_epochs=2, **kw)
    print(f"[lex] {case} n={n} order={order} tol={tol} C={p.candidates}", flush=True)
    h = gx.gx_instance_upload(ctx, inst)
    job = gx.gx_job_create(ctx, h, p)
    o = oracle.OracleInstance(inst)
    assert o.lex
    st = o.init(p)
    compare(ctx, job, p, n, st, f"{case} init")
    for i, s in enumerate([9, 3, 25, 20]):
        gx.gx_job_advance(ctx, job, s)
        o.run(p, st, s)
        compare(ctx, job, p, n, st, f"{case} split {i}")
    gx.gx_job_free(ctx, job)
    # a whole solve reports the oracle's best (ordered scan over the best vectors)
    job = gx.gx_solve(ctx, h, p)
    gx.gx_wait(ctx, job)
    sol, f = gx.gx_fetch_best(ctx, job, n)
    fo, io = o.best_of(st)
    assert f == fo and np.array_equal(sol, st["best"][io]), (f, fo)
    gx.gx_job_free(ctx, job)
    gx.gx_instance_free(ctx, h)


ISLANDS = {
    "ring": dict(islands=2, migrate_epochs=2, migrate_mode=0),
    "top-n": dict(islands=4, migrate_epochs=1, migrate_mode=1, migrate_n=1),
    "top-2": dict(islands=2, migrate_epochs=1, migrate_mode=1, migrate_n=2),
    "hybrid-elite": dict(islands=2, migrate_epochs=2, migrate_mode=2, migrate_n=2, elite_epochs=3),
    "elite-only": dict(elite_epochs=2),
}


@pytest.mark.parametrize("case", list(ISLANDS))
def test_lex_islands_parity(ctx, case):
    """Island migration and elite injection in the lexicographic mode: the
    picks and the improvement test by the mode's relation, vectors copied
    with the solutions, the stagnation reference taken before the exchange."""
    inst = lex_inst(22, 71, (DIST, VEH, LONG), (35, 0, 10))
    p = P(48, seed=13, population=8, candidates=128, epoch=3, stagnation_epochs=2, **ISLANDS[case])
    print(f"[lex islands] {case}", flush=True)
    h = gx.gx_instance_upload(ctx, inst)
    job = gx.gx_job_create(ctx, h, p)
    o = oracle.OracleInstance(inst)
    st = o.init(p)
    compare(ctx, job, p, inst.n, st, f"islands {case} init")
    for i, s in enumerate([7, 11, 30]):
        gx.gx_job_advance(ctx, job, s)
        o.run(p, st, s)
        compare(ctx, job, p, inst.n, st, f"islands {case} split {i}")
    gx.gx_job_free(ctx, job)
    gx.gx_instance_free(ctx, h)


def test_one_level_without_penalty_matches_the_scalar_kernel(ctx):
    """Distance alone, tolerance 0, no penalty possible: the lexicographic
    kernel and the weighted kernel run the same generations."""
    base = synth.vrptw_random(20, 4, key=70)
    b = base.b.copy()
    b[1, :] = 0
    b[2, :] = 10**5
    loose = dataclasses.replace(base, b=b, capacity=int(b[0].sum()) + 1, vehicles=20, horizon=10**5)
    lex = dataclasses.replace(loose, lex_order=(DIST, 0, 0), lex_tol=(0, 0, 0))
    p = P(40, seed=8, population=5, candidates=128, epoch=5)
    out = []
    for inst in (lex, loose):
        h = gx.gx_instance_upload(ctx, inst)
        job = gx.gx_job_create(ctx, h, p)
        gx.gx_job_advance(ctx, job, 40)
        out.append(gx.gx_snapshot(ctx, job, p.population, inst.n))
        gx.gx_job_free(ctx, job)
        gx.gx_instance_free(ctx, h)
    for k in KEYS:
        assert np.array_equal(np.asarray(out[0][k]), np.asarray(out[1][k])), k


def test_batch_mixing_modes(ctx):
    insts = [lex_inst(25, 80, (DIST, VEH, 0), (20, 0, 0)), synth.vrptw_random(25, 12, key=81),
             lex_inst(18, 82, (VEH, LONG, 0), (0, 10, 0))]
    params = [P(33, seed=1 + i, population=4 + i, candidates=128, epoch=5) for i in range(3)]
    hs = [gx.gx_instance_upload(ctx, i) for i in insts]
    jobs = gx.gx_solve_batch(ctx, hs, params)
    gx.gx_wait(ctx)
    for inst, p, job in zip(insts, params, jobs):
        o = oracle.OracleInstance(inst)
        fo, io = o.best_of(o.solve(p))
        sol, f = gx.gx_fetch_best(ctx, job, inst.n)
        assert f == fo, (inst.lex_order, f, fo)
    for j in jobs:
        gx.gx_job_free(ctx, j)
    for h in hs:
        gx.gx_instance_free(ctx, h)


def test_served_lex_request(ctx):
    reqs = [(lex_inst(22, 90, (DIST, VEH, LONG), (25, 0, 0)), P(40, seed=3, population=4)),
            (synth.vrptw_random(22, 13, key=91), P(40, seed=4, population=4))]
    srv = gx.gx_server_create(ctx, quantum_epochs=1)
    tickets = [gx.gx_server_submit(srv, i, p) for i, p in reqs]
    got = {}
    t_end = time.time() + 60
    while len(got) < len(reqs) and time.time() < t_end:
        for k, t in enumerate(tickets):
            if k not in got:
                r = gx.gx_server_poll(srv, t, reqs[k][0].n)
                if r is not None:
                    got[k] = r
        time.sleep(0.002)
    gx.gx_server_destroy(srv)
    assert len(got) == len(reqs)
    for k, (inst, p) in enumerate(reqs):
        o = oracle.OracleInstance(inst)
        fo, _ = o.best_of(o.solve(p))
        assert got[k][1] == fo, (k, got[k][1], fo)


def test_refusals(ctx):
    inst = lex_inst(15, 95, (DIST, 0, 0), (0, 0, 0))
    h = gx.gx_instance_upload(ctx, inst)
    with pytest.raises(gx.GxError):
        gx.gx_job_create(ctx, h, P(10, seed=1, population=4, aos_scope=1))
    job = gx.gx_job_create(ctx, h, P(10, seed=1, population=4))
    snap = gx.gx_snapshot(ctx, job, 4, inst.n)
    with pytest.raises(gx.GxError):
        gx.gx_job_restore(ctx, job, snap)
    gx.gx_job_free(ctx, job)
    gx.gx_instance_free(ctx, h)
    # a scalar job has no vectors
    s = synth.vrptw_random(15, 1, key=96)
    h = gx.gx_instance_upload(ctx, s)
    job = gx.gx_job_create(ctx, h, P(10, seed=1, population=4))
    with pytest.raises(gx.GxError):
        gx.gx_snapshot_lex(ctx, job, 4)
    gx.gx_job_free(ctx, job)
    gx.gx_instance_free(ctx, h)
    bad = [dict(lex_order=(DIST, DIST, 0)), dict(lex_order=(4, 0, 0)), dict(lex_order=(0, DIST, 0)),
           dict(lex_order=(DIST, 0, 0), lex_tol=(-1, 0, 0)), dict(lex_order=(DIST, 0, 0), lex_tol=(0, 5, 0)),
           dict(lex_order=(DIST, 0, 0), obj_weights=(1, 1, 0))]
    for kw in bad:
        with pytest.raises(gx.GxError):
            gx.gx_instance_upload(ctx, dataclasses.replace(s, **kw))
    with pytest.raises(gx.GxError):
        gx.gx_instance_upload(ctx, dataclasses.replace(synth.tsp_uniform(20, 1, key=97), lex_order=(DIST, 0, 0)))


def test_portfolio_compares_vectors(ctx):
    """Seeds of one lexicographic instance in one batch: the portfolio pick is
    the ordered scan, in job order, over the oracle's reported best vectors."""
    inst = lex_inst(24, 98, (VEH, DIST, LONG), (0, 40, 0))
    params = [P(36, seed=s, population=4, candidates=128, epoch=4) for s in (42, 123, 456, 789, 2024)]
    h = gx.gx_instance_upload(ctx, inst)
    jobs = gx.gx_solve_batch(ctx, [h] * len(params), params)
    gx.gx_wait(ctx)
    sol, f, idx = gx.gx_portfolio_best(ctx, jobs, inst.n)
    o = oracle.OracleInstance(inst)
    keep, kv, kf = 0, None, None
    for i, p in enumerate(params):
        st = o.solve(p)
        fo, io = o.best_of(st)
        v = st["best_v"][io]
        if i == 0 or o.lex_better(v, kv):
            keep, kv, kf = i, v, fo
    assert idx == keep and f == kf, (idx, keep, f, kf)
    assert list(o.lex_vector(sol)) == list(kv)
    for j in jobs:
        gx.gx_job_free(ctx, j)
    gx.gx_instance_free(ctx, h)
