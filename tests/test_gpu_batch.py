"""Batched solve: many instances of uneven size and kind in one persistent
launch per epoch.  Each job's final state must equal the oracle's solve of the
same instance and parameters, bit for bit (and therefore the plain solver's)."""
import numpy as np
import pytest

import oracle
import synth
from paper_2603_19163_amd import gx

pytestmark = pytest.mark.gpu

KEYS = ["g", "stag", "T_q16", "epoch_ref", "accepted", "w_op", "w_k", "u_op", "v_op", "u_k", "v_k",
        "cur", "cur_f", "best", "best_f"]


@pytest.fixture(scope="module")
def ctx():
    c = gx.gx_create(0)
    yield c
    gx.gx_destroy(c)


def mixed(count_tsp=6, count_qap=4, G=30):
    r = np.random.default_rng(17)
    insts, params = [], []
    for i in range(count_tsp):
        n = int(r.integers(20, 61))
        insts.append(synth.tsp_uniform(n, 100 + i, key=i))
        params.append(synth.Params(seed=10**6 + i, generations=G, population=int(r.integers(2, 7)),
                                   candidates=128, alpha_q32=synth.alpha_q32_for(G),
                                   staging=int(r.integers(1, 3))))
    for i in range(count_qap):
        n = int(r.integers(12, 21))
        insts.append(synth.qap_random(n, 200 + i, key=count_tsp + i))
        params.append(synth.Params(seed=10**6 + count_tsp + i, generations=G + 7 * i,
                                   population=int(r.integers(2, 6)), candidates=96,
                                   alpha_q32=synth.alpha_q32_for(G)))
    k = len(insts)
    insts.append(synth.knapsack_random(50, 300, key=k))
    params.append(synth.Params(seed=5, generations=G, population=3, alpha_q32=synth.alpha_q32_for(G)))
    insts.append(synth.vrptw_random(15, 301, key=k + 1))
    params.append(synth.Params(seed=6, generations=G - 4, population=3, alpha_q32=synth.alpha_q32_for(G)))
    insts.append(synth.color_planted(25, 3, inst_id=302, key=k + 2))
    params.append(synth.Params(seed=7, generations=G, population=4, alpha_q32=synth.alpha_q32_for(G)))
    return insts, params


def test_batch_equals_oracle_per_job(ctx):
    insts, params = mixed()
    handles = [gx.gx_instance_upload(ctx, i) for i in insts]
    print(f"[batch] {len(insts)} jobs", flush=True)
    jobs = gx.gx_solve_batch(ctx, handles, params)
    gx.gx_wait(ctx, jobs[0])
    for i, (inst, p, job) in enumerate(zip(insts, params, jobs)):
        g = gx.gx_snapshot(ctx, job, p.population, inst.n)
        o = oracle.OracleInstance(inst).solve(p)
        for k in KEYS:
            assert np.array_equal(np.asarray(g[k]), np.asarray(o[k])), (i, inst.kind, k)
        sol, f = gx.gx_fetch_best(ctx, job, inst.n)
        fo, io = oracle.best_of(o)
        assert f == fo and np.array_equal(sol, o["best"][io])
    for j in jobs:
        gx.gx_job_free(ctx, j)
    for h in handles:
        gx.gx_instance_free(ctx, h)


def test_batch_with_islands_equals_oracle(ctx):
    # jobs with island migration or elite injection next to jobs without:
    # the whole launch takes the migrating epoch kernel
    G = 40
    a = synth.alpha_q32_for(G)
    insts = [synth.tsp_uniform(30, 401, key=1), synth.qap_random(14, 402, key=2),
             synth.knapsack_random(60, 403, key=3), synth.tsp_uniform(22, 404, key=4)]
    params = [synth.Params(seed=11, generations=G, population=8, candidates=64, alpha_q32=a, islands=4,
                           migrate_epochs=1, migrate_mode=0, elite_epochs=2),
              synth.Params(seed=12, generations=G, population=6, candidates=96, alpha_q32=a, islands=2,
                           migrate_epochs=2, migrate_mode=1, migrate_n=2),
              synth.Params(seed=13, generations=G, population=4, candidates=64, alpha_q32=a, elite_epochs=1),
              synth.Params(seed=14, generations=G - 10, population=3, candidates=64, alpha_q32=a)]
    handles = [gx.gx_instance_upload(ctx, i) for i in insts]
    jobs = gx.gx_solve_batch(ctx, handles, params)
    gx.gx_wait(ctx, jobs[0])
    for i, (inst, p, job) in enumerate(zip(insts, params, jobs)):
        g = gx.gx_snapshot(ctx, job, p.population, inst.n)
        o = oracle.OracleInstance(inst).solve(p)
        for k in KEYS:
            assert np.array_equal(np.asarray(g[k]), np.asarray(o[k])), (i, inst.kind, k)
    for j in jobs:
        gx.gx_job_free(ctx, j)
    for h in handles:
        gx.gx_instance_free(ctx, h)


def test_batch_equals_plain_solver(ctx):
    # 700 generations: 70 epoch launches, the first 64 replayed from a captured
    # graph whose (kind, staging) groups run on side streams
    insts, params = mixed(3, 2, G=700)
    handles = [gx.gx_instance_upload(ctx, i) for i in insts]
    jobs = gx.gx_solve_batch(ctx, handles, params)
    batched = [gx.gx_fetch_best(ctx, j, i.n) for j, i in zip(jobs, insts)]
    for h, inst, p, (sol, f) in zip(handles, insts, params, batched):
        job = gx.gx_solve(ctx, h, p)
        s2, f2 = gx.gx_fetch_best(ctx, job, inst.n)
        assert f == f2 and np.array_equal(sol, s2)
        gx.gx_job_free(ctx, job)
    for j in jobs:
        gx.gx_job_free(ctx, j)
    for h in handles:
        gx.gx_instance_free(ctx, h)


def test_autotuner_choices_are_valid_and_result_neutral(ctx):
    """The tuner returns a supported staging per TSP bucket (0 for other
    kinds), and a batch solved with the tuned stagings gives the same results
    as with the default staging: the knob it turns never changes a trajectory."""
    from paper_2603_19163_amd import autotune
    insts = [synth.tsp_uniform(40, 31, key=1), synth.tsp_uniform(150, 32, key=2), synth.qap_random(20, 33, key=3)]
    samples = {autotune.bucket_of(i.kind, i.n): i for i in insts}
    alpha = synth.alpha_q32_for(200)
    staging = autotune.tune_buckets(ctx, samples, lambda i: synth.Params(seed=1, generations=50, alpha_q32=alpha),
                                    generations=20, cache=False)
    assert set(staging) == set(samples)
    for b, st in staging.items():
        assert st in ((1, 2, 3, 4) if b.startswith("1:") else (0,)), (b, st)
    hs = [gx.gx_instance_upload(ctx, i) for i in insts]
    out = []
    for tuned in (False, True):
        params = [synth.Params(seed=7 + k, generations=60, population=3, candidates=96, alpha_q32=alpha,
                               staging=staging[autotune.bucket_of(i.kind, i.n)] if tuned else 0)
                  for k, i in enumerate(insts)]
        jobs = gx.gx_solve_batch(ctx, hs, params)
        gx.gx_wait(ctx, jobs[0])
        res = [gx.gx_fetch_best(ctx, j, i.n) for j, i in zip(jobs, insts)]
        for j in jobs:
            gx.gx_job_free(ctx, j)
        out.append(res)
    for (s0, f0), (s1, f1) in zip(*out):
        assert f0 == f1 and np.array_equal(s0, s1)
    for h in hs:
        gx.gx_instance_free(ctx, h)


def test_portfolio_best_of_seeds(ctx):
    """Portfolio of independent solves of one instance (different seeds, one
    batch): the selection returns the smallest best objective (ties: the first
    job) and that job's solution, equal to the plain solves of the same seeds."""
    inst = synth.tsp_uniform(40, 77, key=7)
    G = 60
    params = [synth.Params(seed=500 + s, generations=G, population=4, candidates=64,
                           alpha_q32=synth.alpha_q32_for(G)) for s in range(6)]
    h = gx.gx_instance_upload(ctx, inst)
    jobs = gx.gx_solve_batch(ctx, [h] * len(params), params)
    sol, f, idx = gx.gx_portfolio_best(ctx, jobs, inst.n)
    plain = []
    for p in params:
        j = gx.gx_solve(ctx, h, p)
        plain.append(gx.gx_fetch_best(ctx, j, inst.n))
        gx.gx_job_free(ctx, j)
    fs = [pf for _, pf in plain]
    assert f == min(fs) and idx == fs.index(min(fs))
    assert np.array_equal(sol, plain[idx][0])
    other = gx.gx_instance_upload(ctx, synth.tsp_uniform(40, 78, key=8))
    j2 = gx.gx_solve(ctx, other, params[0])
    with pytest.raises(gx.GxError) as e:
        gx.gx_portfolio_best(ctx, [jobs[0], j2], inst.n)
    assert e.value.status == gx.GX_E_INVALID
    gx.gx_job_free(ctx, j2)
    gx.gx_instance_free(ctx, other)
    for j in jobs:
        gx.gx_job_free(ctx, j)
    gx.gx_instance_free(ctx, h)
