"""Bit-exact parity where the benchmark times, beyond the early windows:
the 442-city configuration (autosized population, benchmark staging) in
20-generation windows at generations 10 000, 50 000, 100 000 and 199 980 of
one job advanced in this process, each window resumed by the oracle from the
GPU's own state; the island rows of the 442-city configuration (three
migration modes) in 100-generation windows that hold migrations and an elite
injection; and the VRPTW configuration (100 customers, P = 64) over its whole
5000-generation run with a snapshot every 1000 generations.  The oracle
runs threaded (pinned equal to its plain runner on the CPU)."""
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


def test_c2_late_windows(ctx):
    inst, p = synth.c2_tsp442(population=0, generations=200_000)
    h = gx.gx_instance_upload(ctx, inst)
    P = gx.gx_autosize_population(ctx, h, p)
    p = p.with_(population=P)
    job = gx.gx_job_create(ctx, h, p)
    o = oracle.OracleInstance(inst)
    g = 0
    for start in (10_000, 50_000, 100_000, 199_980):
        gx.gx_job_advance(ctx, job, start - g)
        a = gx.gx_snapshot(ctx, job, P, inst.n)
        gx.gx_job_advance(ctx, job, 20)
        b = gx.gx_snapshot(ctx, job, P, inst.n)
        g = start + 20
        assert a["g"] == start and b["g"] == g
        t = time.perf_counter()
        o.run(p, a, 20, threads=THREADS)
        print(f"[config parity] C2 P={P} window {start}..{g}: T_q16 {b['T_q16']}, best {int(b['best_f'].min())}, "
              f"oracle {time.perf_counter() - t:.1f} s", flush=True)
        same(b, a, f"C2 window {start}..{g}")
    gx.gx_job_free(ctx, job)
    gx.gx_instance_free(ctx, h)


def test_c3_whole_run(ctx):
    inst, p = synth.c3_vrptw(seed=42)
    h = gx.gx_instance_upload(ctx, inst)
    job = gx.gx_job_create(ctx, h, p)
    o = oracle.OracleInstance(inst)
    st = o.init(p)
    same(gx.gx_snapshot(ctx, job, p.population, inst.n), st, "C3 init")
    for k in range(5):
        gx.gx_job_advance(ctx, job, 1000)
        t = time.perf_counter()
        o.run(p, st, 1000, threads=THREADS)
        print(f"[config parity] C3 generations {1000 * k}..{1000 * (k + 1)}: oracle {time.perf_counter() - t:.1f} s",
              flush=True)
        same(gx.gx_snapshot(ctx, job, p.population, inst.n), st, f"C3 generation {1000 * (k + 1)}")
    sol, f = gx.gx_fetch_best(ctx, job, inst.n)
    fo, io = oracle.best_of(st)
    assert f == fo and np.array_equal(sol, st["best"][io])
    gx.gx_job_free(ctx, job)
    gx.gx_instance_free(ctx, h)


def test_c3_lexicographic_whole_run(ctx):
    """The VRPTW configuration in the lexicographic mode as the per-kind bench
    row runs it (routes, then distance within 20, then the longest route):
    the whole 5000-generation run, state and objective vectors compared with
    the oracle every 1000 generations."""
    import dataclasses
    base, p = synth.c3_vrptw(seed=42)
    inst = dataclasses.replace(base, lex_order=(2, 1, 3), lex_tol=(0, 20, 0))
    h = gx.gx_instance_upload(ctx, inst)
    job = gx.gx_job_create(ctx, h, p)
    o = oracle.OracleInstance(inst)
    st = o.init(p)
    for k in range(5):
        gx.gx_job_advance(ctx, job, 1000)
        t = time.perf_counter()
        o.run(p, st, 1000, threads=THREADS)
        print(f"[config parity] C3 lexicographic generations {1000 * k}..{1000 * (k + 1)}: "
              f"oracle {time.perf_counter() - t:.1f} s", flush=True)
        same(gx.gx_snapshot(ctx, job, p.population, inst.n), st, f"C3 lexicographic generation {1000 * (k + 1)}")
        v = gx.gx_snapshot_lex(ctx, job, p.population)
        for key in ("cur_v", "best_v", "ref_v"):
            assert np.array_equal(v[key], st[key]), (key, 1000 * (k + 1))
    sol, f = gx.gx_fetch_best(ctx, job, inst.n)
    fo, io = o.best_of(st)
    assert f == fo and np.array_equal(sol, st["best"][io])
    gx.gx_job_free(ctx, job)
    gx.gx_instance_free(ctx, h)


@pytest.mark.parametrize("mode,mig_n", [(0, 0), (1, 4), (2, 4)])
def test_c2_islands_windows(ctx, mode, mig_n):
    """The 442-city island rows of the per-kind bench (autosized population,
    16 islands, migration every 5 epochs, elite injection every 10, 20 000
    generations): 100-generation windows, each holding two migrations and an
    elite injection, at generations 9900 and 19 900 of one job, each resumed by
    the oracle from the GPU's state."""
    inst, p = synth.c2_tsp442(population=0, generations=20_000)
    p = p.with_(islands=16, migrate_epochs=5, elite_epochs=10, migrate_mode=mode, migrate_n=mig_n)
    h = gx.gx_instance_upload(ctx, inst)
    P = gx.gx_autosize_population(ctx, h, p)
    p = p.with_(population=P)
    job = gx.gx_job_create(ctx, h, p)
    o = oracle.OracleInstance(inst)
    g = 0
    for start in (9_900, 19_900):
        gx.gx_job_advance(ctx, job, start - g)
        a = gx.gx_snapshot(ctx, job, P, inst.n)
        gx.gx_job_advance(ctx, job, 100)
        b = gx.gx_snapshot(ctx, job, P, inst.n)
        g = start + 100
        assert a["g"] == start and b["g"] == g
        t = time.perf_counter()
        o.run(p, a, 100, threads=THREADS)
        print(f"[config parity] C2 islands mode {mode} P={P} window {start}..{g}: best {int(b['best_f'].min())}, "
              f"oracle {time.perf_counter() - t:.1f} s", flush=True)
        same(b, a, f"C2 islands mode {mode} window {start}..{g}")
    gx.gx_job_free(ctx, job)
    gx.gx_instance_free(ctx, h)
