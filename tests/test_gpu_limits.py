"""Parity at the largest sizes each kernel accepts and at the full VRPTW
configuration (100 customers, P = 64): a short run from the start plus a
window resumed by the oracle from the GPU's own mid-run state."""
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


def same(g, o, what):
    for k in KEYS:
        assert np.array_equal(np.asarray(g[k]), np.asarray(o[k])), f"{what}: {k}"


def windowed(ctx, inst, p, warm, window, what):
    print(f"[limits] {what} n={inst.n} P={p.population} warm={warm} window={window}", flush=True)
    h = gx.gx_instance_upload(ctx, inst)
    job = gx.gx_job_create(ctx, h, p)
    o = oracle.OracleInstance(inst)
    same(gx.gx_snapshot(ctx, job, p.population, inst.n), o.init(p), f"{what} init")
    gx.gx_job_advance(ctx, job, warm)
    a = gx.gx_snapshot(ctx, job, p.population, inst.n)
    gx.gx_job_advance(ctx, job, window)
    b = gx.gx_snapshot(ctx, job, p.population, inst.n)
    gx.gx_job_free(ctx, job)
    gx.gx_instance_free(ctx, h)
    o.run(p, a, window)
    same(b, a, f"{what} window")


def P(G, **kw):
    return synth.Params(generations=G, alpha_q32=synth.alpha_q32_for(G), **kw)


@pytest.mark.parametrize("n", [1536, 1537])
def test_tsp_tour_buffer_boundary(ctx, n):
    # 1536: the longest tour rewritten through the candidate tables (up to the
    # byte below the run's counters); 1537: the shortest with a second buffer
    windowed(ctx, synth.tsp_uniform(n, 5, key=11), P(400, seed=9, population=8, staging=2), 30, 20, f"tsp{n}")


def test_tsp_2000_coordinates_in_lds(ctx):
    windowed(ctx, synth.tsp_uniform(2000, 3, key=1), P(1000, seed=3, population=16, staging=2), 40, 12, "tsp2000")


def test_qap_max_n(ctx):
    windowed(ctx, synth.qap_random(64, 1, key=2), P(500, seed=4, population=8), 30, 10, "qap64")


def test_vrptw_max_n(ctx):
    windowed(ctx, synth.vrptw_random(250, 1, key=3), P(500, seed=5, population=8), 30, 10, "vrptw250")


def test_knapsack_max_n(ctx):
    windowed(ctx, synth.knapsack_random(16384, 1, key=4), P(500, seed=6, population=4), 30, 10, "knap16384")


def test_vrptw_config_full_size(ctx):
    inst, p = synth.c3_vrptw(seed=42)
    windowed(ctx, inst, p, 1000, 20, "VRPTW 100 customers P=64")


def test_many_candidates(ctx):
    # three chunks of candidates (300 = 128 + 128 + 44)
    windowed(ctx, synth.tsp_clustered(120, 2, key=9), P(200, seed=8, population=4, candidates=300), 20, 10, "C=300")
    windowed(ctx, synth.qap_random(20, 2, key=9), P(200, seed=8, population=3, candidates=300), 20, 10, "qap C=300")
