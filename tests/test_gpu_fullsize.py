"""Parity at the full sizes of the systems workloads, in the launch
configurations the benchmark times: the whole 4096-instance batch (3072 TSP n
U[20,200] + 1024 QAP n U[12,40], population sized to fill the device, 5000
generations) and served requests of the mixed stream (TSP n U[20,500], QAP n
U[12,50], knapsack n U[100,1000], P = 4, 10 000 generations).  Every result is
checked for properties that hold at any size (a valid solution whose
objective, recomputed by the oracle, is the reported one); a sample is solved
by the oracle in full and must match bit for bit."""
import os
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import synth
from paper_2603_19163_amd import autotune, gx

pytestmark = pytest.mark.gpu

# oracle solves run side by side on the host's cores (the oracle call
# releases the interpreter lock); at most 16, the host share of one GPU
THREADS = max(1, min(16, os.cpu_count() or 1))


def oracle_solves(cases):
    """[(instance, params)] -> [(best objective, best solution)] by the oracle."""
    def one(c):
        o = oracle.OracleInstance(c[0]).solve(c[1])
        fo, io = oracle.best_of(o)
        return fo, o["best"][io].copy()
    with ThreadPoolExecutor(THREADS) as ex:
        return list(ex.map(one, cases))


@pytest.fixture(scope="module")
def ctx():
    c = gx.gx_create(0)
    yield c
    gx.gx_destroy(c)


def valid(inst, sol):
    if inst.kind in (synth.TSP, synth.QAP):
        return sorted(sol.tolist()) == list(range(inst.n))
    return bool(np.all((sol == 0) | (sol == 1)))


def test_c4_full_batch(ctx):
    insts = synth.c4_batched_instances(4096)
    G = 5000
    params, plan = autotune.tune_batch(ctx, insts, synth.c4_params_for(G), rule="tuned")
    print(f"[fullsize] C4 batch of {len(insts)}, populations per bucket "
          f"{ {b: v['population'] for b, v in plan.items()} }", flush=True)
    handles = [gx.gx_instance_upload(ctx, i) for i in insts]
    jobs = gx.gx_solve_batch(ctx, handles, params)
    gx.gx_wait(ctx, jobs[0])
    res = [gx.gx_fetch_best(ctx, j, i.n) for j, i in zip(jobs, insts)]
    for j in jobs:
        gx.gx_job_free(ctx, j)
    for h in handles:
        gx.gx_instance_free(ctx, h)
    for k in range(0, len(insts), 8):   # every eighth result: valid, objective as reported
        inst, (sol, f) = insts[k], res[k]
        assert valid(inst, sol), k
        assert oracle.OracleInstance(inst).objective(sol) == f, k
    # a 1/16 subsample stratified by kind and size: instances ordered by
    # (kind, n, index), every sixteenth, solved by the oracle in full
    order = sorted(range(len(insts)), key=lambda k: (insts[k].kind, insts[k].n, k))
    picks = order[::16]
    t = time.perf_counter()
    ref = oracle_solves([(insts[k], params[k]) for k in picks])
    print(f"[fullsize] C4 {len(picks)} instances by the oracle in {time.perf_counter() - t:.1f} s "
          f"({THREADS} threads)", flush=True)
    for k, (fo, so) in zip(picks, ref):
        assert res[k][1] == fo and np.array_equal(res[k][0], so), (k, insts[k].kind, insts[k].n)


def test_c5_served_full_size(ctx):
    reqs, _ = synth.c5_requests(400, 0.1)          # 40 requests of the mixed stream
    srv = gx.gx_server_create(ctx, hbm_budget_bytes=1 << 30, max_resident=256)
    tickets = [gx.gx_server_submit(srv, inst, p) for inst, p in reqs]
    print(f"[fullsize] C5 {len(tickets)} requests submitted", flush=True)
    res, t_end = {}, time.time() + 120
    while len(res) < len(tickets) and time.time() < t_end:
        for k, t in enumerate(tickets):
            if k not in res:
                r = gx.gx_server_poll(srv, t, reqs[k][0].n)
                if r is not None:
                    res[k] = r
        time.sleep(0.002)
    gx.gx_server_destroy(srv)
    assert len(res) == len(tickets)
    for k, (inst, p) in enumerate(reqs):
        sol, f = res[k][0], res[k][1]
        assert valid(inst, sol), k
        assert oracle.OracleInstance(inst).objective(sol) == f, k
    # every request (TSP n up to 500, QAP n up to 50, knapsack n up to 1000)
    # solved by the oracle in full
    t = time.perf_counter()
    ref = oracle_solves(reqs)
    kinds = sorted({inst.kind for inst, _ in reqs})
    print(f"[fullsize] C5 {len(reqs)} requests (kinds {kinds}, QAP n max "
          f"{max(i.n for i, _ in reqs if i.kind == synth.QAP)}) by the oracle in {time.perf_counter() - t:.1f} s",
          flush=True)
    assert len(kinds) == 3
    for k, (fo, so) in enumerate(ref):
        assert res[k][1] == fo and np.array_equal(res[k][0], so), (k, reqs[k][0].kind, reqs[k][0].n)
