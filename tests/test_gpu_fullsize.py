"""Parity at the full sizes of the systems workloads, in the launch
configurations the benchmark times: the whole 4096-instance batch (3072 TSP n
U[20,200] + 1024 QAP n U[12,40], population sized to fill the device, 5000
generations) and served requests of the mixed stream (TSP n U[20,500], QAP n
U[12,50], knapsack n U[100,1000], P = 4, 10 000 generations).  Every result is
checked for properties that hold at any size (a valid solution whose
objective, recomputed by the oracle, is the reported one); a sample is solved
by the oracle in full and must match bit for bit."""
import time

import numpy as np
import pytest

import oracle
import synth
from paper_2603_19163_amd import autotune, gx

pytestmark = pytest.mark.gpu


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
    P = autotune.fill_population(ctx, len(insts))
    G = 5000
    alpha = synth.alpha_q32_for(G)
    params = [synth.Params(seed=10**6 + i, generations=G, population=P, candidates=128, alpha_q32=alpha)
              for i in range(len(insts))]
    print(f"[fullsize] C4 batch of {len(insts)} P={P}", flush=True)
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
    # sample: first, middle and last TSP instance, first and last QAP instance
    for k in (0, 1535, 3071, 3072, 4095):
        t = time.perf_counter()
        o = oracle.OracleInstance(insts[k]).solve(params[k])
        fo, io = oracle.best_of(o)
        print(f"[fullsize] C4 instance {k} kind {insts[k].kind} n={insts[k].n}: oracle {time.perf_counter() - t:.1f} s",
              flush=True)
        assert res[k][1] == fo and np.array_equal(res[k][0], o["best"][io]), k


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
    # sample: the first request of each kind (QAP: the first with n <= 30, to
    # bound the oracle's O(n^2) recomputation per candidate)
    picks = {}
    for k, (inst, _) in enumerate(reqs):
        if inst.kind not in picks and (inst.kind != synth.QAP or inst.n <= 30):
            picks[inst.kind] = k
    assert len(picks) == 3
    for kind, k in sorted(picks.items()):
        inst, p = reqs[k]
        t = time.perf_counter()
        o = oracle.OracleInstance(inst).solve(p)
        fo, io = oracle.best_of(o)
        print(f"[fullsize] C5 request {k} kind {kind} n={inst.n}: oracle {time.perf_counter() - t:.1f} s", flush=True)
        assert res[k][1] == fo and np.array_equal(res[k][0], o["best"][io]), k
