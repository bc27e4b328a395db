"""Oracle pins for the per-solution weight scope, the run totals and the
threaded runner.

- With one solution, weights kept per solution are the instance's weights:
  the two scopes give the same trajectory and the same weights.
- The run totals obey closed forms: every candidate credits one k and k
  operators (credit R1), or only the accepted moves do (credit R2); with the
  first epoch end beyond the run, the totals equal the epoch counts.
- The threaded runner reproduces the plain one bit for bit."""
import numpy as np
import pytest

import oracle
import synth

FIELDS = ["g", "stag", "T_q16", "epoch_ref", "accepted", "w_op", "w_k", "u_op", "v_op", "u_k", "v_k",
          "tot_u_op", "tot_v_op", "tot_u_k", "tot_v_k", "cur", "cur_f", "best", "best_f"]


def _same(a, b, what, scope=0):
    for k in FIELDS:
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), (what, k)
    if scope:
        assert a["saos"].tobytes() == b["saos"].tobytes(), (what, "saos")


CASES = {
    "tsp": lambda: synth.tsp_uniform(23, 4, key=3),
    "qap": lambda: synth.qap_random(13, 4, key=4),
    "knap": lambda: synth.knapsack_random(40, 4, key=5),
    "vrptw": lambda: synth.vrptw_random(14, 4, key=6),
    "color": lambda: synth.color_planted(18, 3, key=7),
}


@pytest.mark.parametrize("kind", list(CASES))
def test_one_solution_scopes_agree(kind):
    inst = CASES[kind]()
    o = oracle.OracleInstance(inst)
    base = synth.Params(seed=17, population=1, candidates=48, generations=73, epoch=4, stagnation_epochs=2,
                        alpha_q32=synth.alpha_q32_for(73))
    a = o.solve(base)
    b = o.solve(base.with_(aos_scope=1))
    for k in ("cur", "cur_f", "best", "best_f", "accepted", "T_q16", "tot_u_op", "tot_v_op", "tot_u_k", "tot_v_k"):
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k
    r = b["saos"][0]
    assert list(r["w_op"]) == list(a["w_op"]) and list(r["w_k"]) == list(a["w_k"])
    assert int(r["stag"]) == a["stag"] and int(r["epoch_ref"]) == a["epoch_ref"]
    # the instance record stays as initialised under per-solution weights
    init = o.init(base)
    assert list(b["w_op"]) == list(init["w_op"]) and int(b["u_op"].sum()) == 0


def test_solution_scope_weights_diverge_and_stay_normalised():
    inst = synth.tsp_uniform(40, 9, key=9)
    o = oracle.OracleInstance(inst)
    p = synth.Params(seed=3, population=6, candidates=64, generations=60, epoch=5,
                     alpha_q32=synth.alpha_q32_for(60), aos_scope=1)
    st = o.solve(p)
    w = st["saos"]["w_op"].astype(np.int64)
    assert len({tuple(r) for r in w}) > 1           # each solution learns from its own candidates
    for r in w:
        assert 65536 - 12 <= r.sum() <= 65536 and (r[:5] >= 1).all() and (r[5:] == 0).all()


@pytest.mark.parametrize("credit", [0, 1])
def test_run_totals_closed_forms(credit):
    inst = synth.tsp_uniform(30, 2, key=2)
    o = oracle.OracleInstance(inst)
    P, C, G = 5, 70, 40
    p = synth.Params(seed=8, population=P, candidates=C, generations=G, epoch=7, credit=credit,
                     alpha_q32=synth.alpha_q32_for(G))
    st = o.solve(p)
    ks = [int(x) for x in st["tot_u_k"]]
    assert sum(ks) == (P * C * G if credit == 0 else st["accepted"])
    assert int(st["tot_u_op"].sum()) == ks[0] + 2 * ks[1] + 3 * ks[2]
    assert (st["tot_v_op"] <= st["tot_u_op"]).all() and (st["tot_v_k"] <= st["tot_u_k"]).all()
    # one epoch longer than the run: the totals are the epoch's counts
    q = p.with_(epoch=1000)
    st2 = o.solve(q)
    for a, b in (("tot_u_op", "u_op"), ("tot_v_op", "v_op"), ("tot_u_k", "u_k"), ("tot_v_k", "v_k")):
        assert np.array_equal(st2[a], st2[b]), a


PAR = [
    ("tsp instance", lambda: synth.tsp_clustered(45, 3, key=1), dict()),
    ("qap solution", lambda: synth.qap_random(15, 2, key=2), dict(aos_scope=1)),
    ("knap islands", lambda: synth.knapsack_random(60, 3, key=3),
     dict(islands=3, migrate_epochs=1, migrate_mode=2, migrate_n=2, elite_epochs=2)),
    ("vrptw credit 1", lambda: synth.vrptw_random(16, 3, key=4), dict(credit=1)),
    ("color solution islands", lambda: synth.color_planted(25, 3, key=5),
     dict(aos_scope=1, islands=2, migrate_epochs=2)),
]


@pytest.mark.parametrize("what,make,kw", PAR, ids=[c[0] for c in PAR])
def test_threaded_runner_equals_plain(what, make, kw):
    inst = make()
    o = oracle.OracleInstance(inst)
    p = synth.Params(seed=21, population=6, candidates=40, generations=47, epoch=5,
                     alpha_q32=synth.alpha_q32_for(47), **kw)
    a = o.init(p)
    b = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in a.items()}
    for step in (3, 19, 25):                        # windows that start and end inside epochs
        o.run(p, a, step)
        o.run(p, b, step, threads=4)
        _same(a, b, what, kw.get("aos_scope", 0))
