"""Bit-exact parity at the configurations of the per-kind benchmark rows that
no other test runs at full size: QAP n = 50 at the autosized population, 0/1
knapsack n = 1000 and planted 3-colouring n = 1000 at P = 2048 (each operator
set the rows time), in 20-generation windows at the start, the quarters and
the end of the run, each resumed by the oracle from the GPU's own state; and
the multi-row lexicographic VRPTW row over its whole 5000-generation run with
a snapshot every 1000 generations."""
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
THREADS = max(1, min(16, os.cpu_count() or 1))


@pytest.fixture(scope="module")
def ctx():
    c = gx.gx_create(0)
    yield c
    gx.gx_destroy(c)


def same(g, o, what):
    for k in KEYS:
        a, b = np.asarray(g[k]), np.asarray(o[k])
        assert np.array_equal(a, b), f"{what}: {k} gpu {a.ravel()[:6]} oracle {b.ravel()[:6]}"


def params(P, G, **kw):
    return synth.Params(seed=42, generations=G, population=P, candidates=128, alpha_q32=synth.alpha_q32_for(G),
                        **kw)


ROWS = {
    "qap50": lambda: (synth.qap_random(50, 7), params(0, 2000)),
    "knapsack1000_flip": lambda: (synth.knapsack_random(1000, 7), params(2048, 5000, op_mask=1 << synth.OP_FLIP)),
    "knapsack1000_flip_segflip": lambda: (synth.knapsack_random(1000, 7), params(2048, 5000, op_mask=synth.BIN_OPS)),
    "color1000_reset": lambda: (synth.color_planted(1000, 3, inst_id=7),
                                params(2048, 5000, op_mask=1 << synth.OP_RESET)),
    "color1000_reset_segreset": lambda: (synth.color_planted(1000, 3, inst_id=7),
                                         params(2048, 5000, op_mask=synth.INT_OPS)),
}


@pytest.mark.parametrize("row", list(ROWS))
def test_kind_row_windows(ctx, row):
    inst, p = ROWS[row]()
    h = gx.gx_instance_upload(ctx, inst)
    if p.population == 0:
        p = p.with_(population=gx.gx_autosize_population(ctx, h, p))
    P, G = p.population, p.generations
    job = gx.gx_job_create(ctx, h, p)
    o = oracle.OracleInstance(inst)
    same(gx.gx_snapshot(ctx, job, P, inst.n), o.init(p), f"{row} init")
    g = 0
    for start in (0, G // 4, G // 2, 3 * G // 4, G - 20):
        gx.gx_job_advance(ctx, job, start - g)
        a = gx.gx_snapshot(ctx, job, P, inst.n)
        gx.gx_job_advance(ctx, job, 20)
        b = gx.gx_snapshot(ctx, job, P, inst.n)
        g = start + 20
        assert a["g"] == start and b["g"] == g
        t = time.perf_counter()
        o.run(p, a, 20, threads=THREADS)
        print(f"[kinds] {row} P={P} window {start}..{g}: best {int(b['best_f'].min())}, "
              f"oracle {time.perf_counter() - t:.1f} s", flush=True)
        same(b, a, f"{row} window {start}..{g}")
    gx.gx_job_free(ctx, job)
    gx.gx_instance_free(ctx, h)


def test_c3_rows_lexicographic_whole_run(ctx):
    """The multi-row VRPTW row in the lexicographic mode (routes, then distance
    within 20, then the longest route; 25 rows, P = 64, 5000 generations)."""
    base, p = synth.c3_vrptw_rows(seed=42)
    inst = dataclasses.replace(base, lex_order=(2, 1, 3), lex_tol=(0, 20, 0))
    N = synth.solution_len(inst)
    h = gx.gx_instance_upload(ctx, inst)
    job = gx.gx_job_create(ctx, h, p)
    o = oracle.OracleInstance(inst)
    st = o.init(p)
    same(gx.gx_snapshot(ctx, job, p.population, N), st, "C3 rows lexicographic init")
    for k in range(5):
        gx.gx_job_advance(ctx, job, 1000)
        t = time.perf_counter()
        o.run(p, st, 1000, threads=THREADS)
        print(f"[kinds] C3 rows lexicographic generations {1000 * k}..{1000 * (k + 1)}: "
              f"oracle {time.perf_counter() - t:.1f} s", flush=True)
        same(gx.gx_snapshot(ctx, job, p.population, N), st, f"C3 rows lexicographic generation {1000 * (k + 1)}")
        v = gx.gx_snapshot_lex(ctx, job, p.population)
        for key in ("cur_v", "best_v", "ref_v"):
            assert np.array_equal(v[key], st[key]), (key, 1000 * (k + 1))
    sol, f = gx.gx_fetch_best(ctx, job, N)
    fo, io = o.best_of(st)
    assert f == fo and np.array_equal(sol, st["best"][io])
    gx.gx_job_free(ctx, job)
    gx.gx_instance_free(ctx, h)
