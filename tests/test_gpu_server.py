"""Serving: requests of mixed kind and size arrive while others run, are
admitted by device footprint, share fused epoch launches, and each result
equals the same request solved alone (plain gx_solve) bit for bit."""
import threading
import time

import numpy as np
import pytest

import oracle
import synth
from paper_2603_19163_amd import gx

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = gx.gx_create(0)
    yield c
    gx.gx_destroy(c)


def requests(count=18, seed=5):
    r = np.random.default_rng(seed)
    out = []
    for i in range(count):
        kind = i % 3
        if kind == 0:
            inst = synth.tsp_uniform(int(r.integers(20, 61)), 500 + i, key=1000 + i)
        elif kind == 1:
            inst = synth.qap_random(int(r.integers(12, 21)), 600 + i, key=1000 + i)
        else:
            inst = synth.knapsack_random(int(r.integers(100, 201)), 700 + i, key=1000 + i)
        G = int(r.integers(30, 121))
        out.append((inst, synth.Params(seed=int(r.integers(0, 2**40)), generations=G, population=4,
                                       candidates=128, alpha_q32=synth.alpha_q32_for(G))))
    return out


def wait_all(srv, tickets, n_of, deadline_s=120):
    res = {}
    t_end = time.time() + deadline_s
    while len(res) < len(tickets) and time.time() < t_end:
        for t in tickets:
            if t in res:
                continue
            r = gx.gx_server_poll(srv, t, n_of[t])
            if r is not None:
                res[t] = r
        time.sleep(0.002)
    assert len(res) == len(tickets), f"only {len(res)} of {len(tickets)} finished"
    return res


def plain(ctx, inst, p):
    h = gx.gx_instance_upload(ctx, inst)
    job = gx.gx_solve(ctx, h, p)
    sol, f = gx.gx_fetch_best(ctx, job, inst.n)
    gx.gx_job_free(ctx, job)
    gx.gx_instance_free(ctx, h)
    return sol, f


def test_served_results_equal_alone(ctx):
    reqs = requests()
    srv = gx.gx_server_create(ctx, hbm_budget_bytes=256 << 20, max_resident=64)
    tickets, n_of = [], {}
    lock = threading.Lock()

    def submit(part):          # two client threads submitting while requests run
        for inst, p in part:
            t = gx.gx_server_submit(srv, inst, p)
            with lock:
                tickets.append((t, inst, p))
                n_of[t] = inst.n
            time.sleep(0.001)
    th = [threading.Thread(target=submit, args=(reqs[i::2],)) for i in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    print(f"[server] {len(tickets)} requests submitted", flush=True)
    res = wait_all(srv, [t for t, _, _ in tickets], n_of)
    stats = gx.gx_server_stats_get(srv)
    gx.gx_server_destroy(srv)
    assert stats["completed"] == len(reqs) and stats["quanta"] > 0
    for t, inst, p in tickets:
        sol, f, ts, td = res[t]
        s2, f2 = plain(ctx, inst, p)
        assert f == f2 and np.array_equal(sol, s2), (inst.kind, inst.n)
        assert td >= ts
    # two of them against the oracle directly
    for t, inst, p in tickets[:2]:
        o = oracle.OracleInstance(inst).solve(p)
        assert res[t][1] == oracle.best_of(o)[0]


def test_served_islands_equal_alone(ctx):
    # requests with island migration and elite injection share lane quanta
    # with requests without; each result equals the plain solve
    reqs = requests(9, seed=13)
    for i in range(0, 9, 2):
        inst, p = reqs[i]
        reqs[i] = (inst, p.with_(population=8, islands=4, migrate_epochs=1, migrate_mode=i % 3, migrate_n=1,
                                 elite_epochs=2))
    srv = gx.gx_server_create(ctx, hbm_budget_bytes=256 << 20, max_resident=64)
    tickets, n_of = [], {}
    for inst, p in reqs:
        t = gx.gx_server_submit(srv, inst, p)
        tickets.append((t, inst, p))
        n_of[t] = inst.n
    res = wait_all(srv, [t for t, _, _ in tickets], n_of)
    gx.gx_server_destroy(srv)
    for t, inst, p in tickets:
        sol, f, _, _ = res[t]
        s2, f2 = plain(ctx, inst, p)
        assert f == f2 and np.array_equal(sol, s2), (inst.kind, inst.n, p.islands)


def test_admission_backpressure_and_cancel(ctx):
    reqs = requests(8, seed=9)
    # an arena that holds only a few requests at a time forces queueing
    srv = gx.gx_server_create(ctx, hbm_budget_bytes=96 << 10, max_resident=8)
    long_inst = synth.tsp_uniform(50, 999, key=7)
    long_p = synth.Params(seed=1, generations=2_000_000, population=2, alpha_q32=synth.alpha_q32_for(10**6))
    t_long = gx.gx_server_submit(srv, long_inst, long_p)
    tickets = [gx.gx_server_submit(srv, i, p) for i, p in reqs]
    n_of = {t: i.n for t, (i, _) in zip(tickets, reqs)}
    time.sleep(0.05)
    gx.gx_server_cancel(srv, t_long)
    res = wait_all(srv, tickets, n_of)
    t_end = time.time() + 30
    cancelled = False
    while time.time() < t_end:
        try:
            if gx.gx_server_poll(srv, t_long, 50) is None:
                time.sleep(0.01)
                continue
        except gx.GxError as e:
            cancelled = e.status == gx.GX_E_CANCELLED
        break
    gx.gx_server_destroy(srv)
    assert cancelled
    for t, (inst, p) in zip(tickets, reqs):
        s2, f2 = plain(ctx, inst, p)
        assert res[t][1] == f2 and np.array_equal(res[t][0], s2)


def test_rejections(ctx):
    srv = gx.gx_server_create(ctx, hbm_budget_bytes=1 << 20, max_resident=4)
    with pytest.raises(gx.GxError):      # no population given
        gx.gx_server_submit(srv, synth.tsp_uniform(20, 0), synth.Params(population=0, alpha_q32=5))
    with pytest.raises(gx.GxError):      # never fits a 1 MiB arena (pool alone 1.6 MB)
        gx.gx_server_submit(srv, synth.tsp_uniform(400, 0),
                            synth.Params(population=256, generations=10, alpha_q32=5))
    gx.gx_server_destroy(srv)


def test_item_cap_queues_in_order(ctx):
    # at most 8 solutions resident: requests of P = 4 run two at a time
    reqs = requests(9, seed=13)
    srv = gx.gx_server_create(ctx, hbm_budget_bytes=256 << 20, max_resident=64, max_items=8)
    tickets = [gx.gx_server_submit(srv, i, p) for i, p in reqs]
    n_of = {t: i.n for t, (i, _) in zip(tickets, reqs)}
    res = wait_all(srv, tickets, n_of)
    stats = gx.gx_server_stats_get(srv)
    gx.gx_server_destroy(srv)
    assert stats["completed"] == len(reqs)
    for t, (inst, p) in zip(tickets, reqs):
        s2, f2 = plain(ctx, inst, p)
        assert res[t][1] == f2 and np.array_equal(res[t][0], s2), (inst.kind, inst.n)
