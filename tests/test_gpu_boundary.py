"""GPU parity of the boundary's solve options and queries, through the C
interface: weights kept per solution (aos_scope 1) on every kind, caller
initial weights, the 3-opt operator alone on every permutation kernel and
TSP staging, run totals (gx_job_stats), the population query, resuming a job
from a snapshot (its own, or the oracle's state), and a served request with
a one-epoch scheduling quantum.  Every state field, the per-solution records
and the run totals are compared bit for bit with the oracle."""
import numpy as np
import pytest

import oracle
import synth
from paper_2603_19163_amd import gx

pytestmark = pytest.mark.gpu

KEYS = ["g", "stag", "T_q16", "epoch_ref", "accepted", "w_op", "w_k", "u_op", "v_op", "u_k", "v_k",
        "cur", "cur_f", "best", "best_f"]
TOT = [("u_op", "tot_u_op"), ("v_op", "tot_v_op"), ("u_k", "tot_u_k"), ("v_k", "tot_v_k")]


@pytest.fixture(scope="module")
def ctx():
    c = gx.gx_create(0)
    yield c
    gx.gx_destroy(c)


def compare(ctx, job, p, n, o_st, what):
    g = gx.gx_snapshot(ctx, job, p.population, n)
    for k in KEYS:
        a, b = np.asarray(g[k]), np.asarray(o_st[k])
        assert np.array_equal(a, b), f"{what}: {k} gpu {a.ravel()[:8]} oracle {b.ravel()[:8]}"
    s = gx.gx_job_stats(ctx, job)
    for gk, ok in TOT:
        assert np.array_equal(s[gk], o_st[ok]), f"{what}: run total {gk} gpu {s[gk]} oracle {o_st[ok]}"
    assert s["accepted"] == o_st["accepted"] and s["generations_done"] == o_st["g"]
    assert s["move_evals"] == p.population * p.candidates * o_st["g"]
    if p.aos_scope:
        r = gx.gx_snapshot_aos(ctx, job, p.population)
        assert r.tobytes() == o_st["saos"].tobytes(), f"{what}: per-solution records differ"


def run_both(ctx, inst, p, splits, what, threads=4):
    print(f"[boundary] {what} n={inst.n} P={p.population} splits={splits}", flush=True)
    h = gx.gx_instance_upload(ctx, inst)
    job = gx.gx_job_create(ctx, h, p)
    o = oracle.OracleInstance(inst)
    st = o.init(p)
    compare(ctx, job, p, inst.n, st, f"{what} init")
    for i, s in enumerate(splits):
        gx.gx_job_advance(ctx, job, s)
        o.run(p, st, s, threads=threads)
        compare(ctx, job, p, inst.n, st, f"{what} split {i}")
    gx.gx_job_free(ctx, job)
    gx.gx_instance_free(ctx, h)


def P(G, **kw):
    kw.setdefault("alpha_q32", synth.alpha_q32_for(G))
    return synth.Params(generations=G, **kw)


SCOPE = {
    "tsp-xy": (lambda: synth.tsp_uniform(37, 3, key=31), dict(staging=2)),
    "tsp-d16": (lambda: synth.tsp_clustered(64, 3, key=32), dict(staging=1)),
    "qap": (lambda: synth.qap_random(17, 3, key=33), dict()),
    "knap": (lambda: synth.knapsack_random(70, 3, key=34), dict()),
    "vrptw": (lambda: synth.vrptw_random(15, 3, key=35), dict()),
    "color": (lambda: synth.color_planted(30, 3, key=36), dict()),
}


@pytest.mark.parametrize("kind", list(SCOPE))
def test_solution_scope_parity(ctx, kind):
    make, kw = SCOPE[kind]
    p = P(57, seed=77, population=7, candidates=100, epoch=4, stagnation_epochs=2, aos_scope=1, **kw)
    run_both(ctx, make(), p, [9, 3, 25, 20], f"solution scope {kind}")


def test_solution_scope_with_islands(ctx):
    p = P(60, seed=5, population=8, candidates=64, epoch=3, aos_scope=1, islands=4, migrate_epochs=2,
          migrate_mode=2, migrate_n=1, elite_epochs=3)
    run_both(ctx, synth.tsp_clustered(50, 2, key=40), p, [60], "solution scope islands")


@pytest.mark.parametrize("credit", [0, 1])
def test_caller_initial_weights_and_run_totals(ctx, credit):
    w = [7000, 0, 30000, 1, 65536 * 4]             # 2-opt, swap (preset), insert, or-opt, 3-opt
    p = P(44, seed=12, population=5, candidates=128, op_mask=synth.PERM_OPS, credit=credit,
          init_weight_q16=tuple(w))
    run_both(ctx, synth.tsp_clustered(120, 4, key=41), p, [13, 31], f"initial weights credit {credit}")


@pytest.mark.parametrize("case", ["tsp1", "tsp2", "tsp3", "tsp4", "qap", "vrptw"])
def test_three_opt_alone(ctx, case):
    mask = 1 << synth.OP_3OPT
    if case.startswith("tsp"):
        inst = synth.tsp_clustered(90, 5, key=42)
        p = P(30, seed=3, population=5, candidates=128, op_mask=mask, staging=int(case[3]))
    elif case == "qap":
        inst = synth.qap_random(30, 5, key=43)
        p = P(30, seed=3, population=4, candidates=128, op_mask=mask)
    else:
        inst = synth.vrptw_random(25, 5, key=44)
        p = P(30, seed=3, population=4, candidates=128, op_mask=mask)
    run_both(ctx, inst, p, [11, 19], f"3-opt {case}")


def test_population_query(ctx):
    inst = synth.tsp_uniform(200, 1, key=45)
    h = gx.gx_instance_upload(ctx, inst)
    p = P(10, seed=1, population=0)
    auto = gx.gx_autosize_population(ctx, h, p)
    job = gx.gx_job_create(ctx, h, p)
    assert gx.gx_job_population(ctx, job) == auto >= 256
    gx.gx_job_free(ctx, job)
    job = gx.gx_job_create(ctx, h, p.with_(population=37))
    assert gx.gx_job_population(ctx, job) == 37
    gx.gx_job_free(ctx, job)
    gx.gx_instance_free(ctx, h)


@pytest.mark.parametrize("scope", [0, 1])
def test_restore_resumes_the_run(ctx, scope):
    inst = synth.qap_random(20, 6, key=46)
    p = P(70, seed=9, population=6, candidates=96, epoch=6, aos_scope=scope)
    h = gx.gx_instance_upload(ctx, inst)
    # uninterrupted
    a = gx.gx_job_create(ctx, h, p)
    gx.gx_job_advance(ctx, a, 33)
    snap = gx.gx_snapshot(ctx, a, p.population, inst.n)
    snap["saos"] = gx.gx_snapshot_aos(ctx, a, p.population)
    gx.gx_job_advance(ctx, a, 37)
    want = gx.gx_snapshot(ctx, a, p.population, inst.n)
    # a fresh job restored from the snapshot (its own initialisation discarded)
    b = gx.gx_job_create(ctx, h, p.with_(seed=p.seed))
    gx.gx_job_restore(ctx, b, snap)
    gx.gx_job_advance(ctx, b, 37)
    got = gx.gx_snapshot(ctx, b, p.population, inst.n)
    for k in KEYS:
        assert np.array_equal(np.asarray(got[k]), np.asarray(want[k])), k
    if scope:
        assert gx.gx_snapshot_aos(ctx, b, p.population).tobytes() == gx.gx_snapshot_aos(ctx, a, p.population).tobytes()
    # the oracle's own mid-run state, continued on the GPU
    o = oracle.OracleInstance(inst)
    st = o.init(p)
    o.run(p, st, 25)
    c = gx.gx_job_create(ctx, h, p)
    gx.gx_job_restore(ctx, c, st)
    gx.gx_job_advance(ctx, c, 17)
    o.run(p, st, 17)
    got = gx.gx_snapshot(ctx, c, p.population, inst.n)
    for k in KEYS:
        assert np.array_equal(np.asarray(got[k]), np.asarray(st[k])), ("from oracle", k)
    # a state that is not a solution is refused
    bad = dict(snap)
    bad["cur"] = snap["cur"].copy()
    bad["cur"][0, 0] = bad["cur"][0, 1]
    with pytest.raises(gx.GxError):
        gx.gx_job_restore(ctx, c, bad)
    for j in (a, b, c):
        gx.gx_job_free(ctx, j)
    gx.gx_instance_free(ctx, h)


def test_served_request_with_one_epoch_quanta(ctx):
    reqs = [(synth.tsp_uniform(33, 7, key=50), P(40, seed=4, population=4)),
            (synth.qap_random(14, 7, key=51), P(40, seed=5, population=3, aos_scope=1)),
            (synth.knapsack_random(90, 7, key=52), P(40, seed=6, population=5))]
    srv = gx.gx_server_create(ctx, quantum_epochs=1)
    tickets = [gx.gx_server_submit(srv, i, p) for i, p in reqs]
    got = {}
    import time
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
        fo, io = oracle.best_of(oracle.OracleInstance(inst).solve(p))
        assert got[k][1] == fo, (k, got[k][1], fo)
