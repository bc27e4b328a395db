"""Oracle pins for the lexicographic mode of the VRPTW objective (paper, Sec.
"Multi-Objective Optimization Modes", Tab. lexicographic_mode and Tab.
triobjective_mode: priorities over distance, vehicle count and longest route,
with tolerances).

- Comparisons worked by hand: the penalty decides first, then each level in
  priority order, values within a level's tolerance tie and pass the
  decision on, and a full tie is not an improvement.
- Objective vectors recomputed route by route for every tour of a small
  instance.
- Reductions: with no penalty possible and one level of tolerance 0, the
  mode is the scalar weighted mode (1, 0, 0) generation for generation; with
  dominating weights it makes the same greedy moves as the weighted mode;
  a tolerance wider than any difference hands every decision to the next level."""
import itertools

import numpy as np
import pytest

import oracle
import synth

DIST, VEH, LONG = 1, 2, 3


def vrptw(n, key, loose=False, **kw):
    base = synth.vrptw_random(n, 7, key=key)
    b = base.b.copy()
    cap, veh, hor = base.capacity, base.vehicles, base.horizon
    if loose:           # no lateness and no fleet excess possible: every penalty is 0
        b[1, :] = 0
        b[2, :] = 10**6
        cap, veh, hor = int(b[0].sum()) + 1, n, 10**6
    return synth.Instance(synth.VRPTW, n, base.a, b, capacity=cap, vehicles=veh, service_time=base.service_time,
                          horizon=hor, key=key, **kw)


def test_comparisons_worked_by_hand():
    o = oracle.OracleInstance(vrptw(6, 1, lex_order=(DIST, VEH, 0), lex_tol=(50, 0, 0)))
    B = o.lex_better
    # distance within 50: the vehicle count decides
    assert B([0, 820, 4, 0], [0, 800, 5, 0]) and not B([0, 800, 5, 0], [0, 820, 4, 0])
    # distance more than 50 apart decides, whatever the vehicles
    assert B([0, 780, 9, 0], [0, 840, 4, 0]) and not B([0, 840, 4, 0], [0, 780, 9, 0])
    # exactly 50 apart is within the tolerance
    assert B([0, 850, 4, 0], [0, 800, 5, 0])
    # the penalty comes first and has no tolerance
    assert B([0, 900, 9, 0], [100, 700, 3, 0]) and B([99, 900, 9, 0], [100, 700, 3, 0])
    # a full tie is not an improvement, either way
    assert not B([0, 810, 5, 0], [0, 800, 5, 0]) and not B([0, 800, 5, 0], [0, 810, 5, 0])
    # vehicles first, then distance with a tolerance of 100
    o2 = oracle.OracleInstance(vrptw(6, 1, lex_order=(VEH, DIST, 0), lex_tol=(0, 100, 0)))
    assert o2.lex_better([0, 5, 2000, 0], [0, 6, 700, 0])
    assert not o2.lex_better([0, 5, 760, 0], [0, 5, 700, 0]) and o2.lex_better([0, 5, 600, 0], [0, 5, 701, 0])


def test_vectors_route_by_route_for_every_tour():
    inst = vrptw(6, 3, lex_order=(LONG, VEH, DIST), lex_tol=(0, 0, 0))
    o = oracle.OracleInstance(inst)
    n = inst.n
    xy, dem, rdy, due = inst.a, inst.b[0], inst.b[1], inst.b[2]

    def d(i, j):
        return int(np.floor(np.hypot(*(xy[i] - xy[j])) + 0.5))
    for perm in itertools.permutations(range(n)):
        routes, cur, load = [], [], 0          # greedy split by capacity, written out here
        for c in (p + 1 for p in perm):
            if cur and load + dem[c] > inst.capacity:
                routes.append(cur)
                cur, load = [], 0
            cur.append(c)
            load += dem[c]
        routes.append(cur)
        dist = longest = late = 0
        for r in routes:
            t, prev, length = 0, 0, 0
            for c in r:
                t += d(prev, c)
                length += d(prev, c)
                t = max(t, rdy[c])
                late += max(0, t - due[c])
                t += inst.service_time
                prev = c
            t += d(prev, 0)
            length += d(prev, 0)
            late += max(0, t - inst.horizon)
            dist += length
            longest = max(longest, length)
        pen = 100 * late + 10000 * max(0, len(routes) - inst.vehicles)
        assert list(o.lex_vector(np.array(perm))) == [pen, longest, len(routes), dist], perm


def test_one_level_without_penalty_is_the_scalar_mode():
    lex = vrptw(14, 5, loose=True, lex_order=(DIST, 0, 0), lex_tol=(0, 0, 0))
    sca = vrptw(14, 5, loose=True)
    p = synth.Params(seed=9, population=5, candidates=64, generations=40, epoch=5, stagnation_epochs=2,
                     alpha_q32=synth.alpha_q32_for(40))
    a = oracle.OracleInstance(lex).solve(p)
    b = oracle.OracleInstance(sca).solve(p)
    for k in ("cur", "best", "cur_f", "best_f", "accepted", "T_q16", "w_op", "w_k", "stag", "epoch_ref",
              "tot_u_op", "tot_v_op"):
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k
    assert (a["cur_v"][:, 0] == 0).all() and np.array_equal(a["cur_v"][:, 1], a["cur_f"])


def test_dominating_weights_make_the_same_greedy_moves():
    # routes first, then distance, tolerance 0: the order of weights (1, 10^6, 0);
    # in the greedy limit only the order matters
    lex = vrptw(12, 6, loose=True, lex_order=(VEH, DIST, 0), lex_tol=(0, 0, 0))
    wtd = vrptw(12, 6, loose=True, obj_weights=(1, 10**6, 0))
    p = synth.Params(seed=3, population=4, candidates=64, generations=30, t0_q16=1, alpha_q32=2**31)
    a = oracle.OracleInstance(lex).solve(p)
    b = oracle.OracleInstance(wtd).solve(p)
    for k in ("cur", "best", "accepted"):
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k


def test_wide_tolerance_hands_the_decision_on():
    wide = vrptw(12, 8, lex_order=(DIST, VEH, 0), lex_tol=(10**7, 0, 0))
    veh = vrptw(12, 8, lex_order=(VEH, 0, 0), lex_tol=(0, 0, 0))
    p = synth.Params(seed=4, population=4, candidates=64, generations=30, epoch=4, t0_q16=1 << 16,
                     alpha_q32=synth.alpha_q32_for(30))
    a = oracle.OracleInstance(wide).solve(p)
    b = oracle.OracleInstance(veh).solve(p)
    for k in ("cur", "best", "accepted", "w_op", "w_k", "stag"):
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k


def test_run_invariants_and_threaded_runner():
    inst = vrptw(20, 9, lex_order=(DIST, VEH, LONG), lex_tol=(30, 0, 5))
    o = oracle.OracleInstance(inst)
    p = synth.Params(seed=11, population=6, candidates=64, generations=45, epoch=5,
                     alpha_q32=synth.alpha_q32_for(45))
    a = o.init(p)
    b = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in a.items()}
    o.run(p, a, 45)
    o.run(p, b, 45, threads=3)
    for k in a:
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k
    for s in range(p.population):
        assert sorted(a["cur"][s]) == list(range(inst.n))
        assert list(o.lex_vector(a["cur"][s])) == list(a["cur_v"][s])
        assert list(o.lex_vector(a["best"][s])) == list(a["best_v"][s])
        assert not o.lex_better(a["cur_v"][s], a["best_v"][s])   # the best is never beaten by the current
        assert a["cur_f"][s] == a["cur_v"][s][0] + a["cur_v"][s][1]
    f, i = o.best_of(a)
    assert f == a["best_f"][i]
    for s in range(i + 1, p.population):      # nothing after the kept index beats it
        assert not o.lex_better(a["best_v"][s], a["best_v"][i])


def test_solution_scope_is_refused():
    o = oracle.OracleInstance(vrptw(10, 2, lex_order=(DIST, 0, 0), lex_tol=(0, 0, 0)))
    with pytest.raises(ValueError):
        o.init(synth.Params(seed=1, population=4, candidates=64, generations=4, aos_scope=1))


def _lex_state(o, cur_v, best_v):
    """Six solutions of a small instance whose vectors are set by hand; the
    solution rows name their index (every copy can be traced)."""
    st = o.new_state(6)
    n = o.n
    base = np.arange(n, dtype=np.int32)
    for s in range(6):
        st["cur"][s] = np.roll(base, s)
        st["best"][s] = np.roll(base, s)
    st["cur_v"][:] = np.asarray(cur_v, np.int64)
    st["best_v"][:] = np.asarray(best_v, np.int64)
    st["cur_f"][:] = st["cur_v"][:, 0] + st["cur_v"][:, 1]
    st["best_f"][:] = st["best_v"][:, 0] + st["best_v"][:, 1]
    return st


def test_lexicographic_migration_by_hand():
    # distance first within 50, then routes; three islands of two
    o = oracle.OracleInstance(vrptw(6, 1, lex_order=(DIST, VEH, 0), lex_tol=(50, 0, 0)))
    best_v = [[0, 800, 5, 0], [0, 830, 4, 0],     # island 0: s1 is better (tie on distance, fewer routes)
              [0, 700, 6, 0], [0, 760, 5, 0],     # island 1: s2 (more than 50 shorter)
              [100, 500, 3, 0], [0, 900, 7, 0]]   # island 2: s5 (penalty first)
    cur_v = [[0, 900, 6, 0], [0, 920, 6, 0],      # island 0: tie within 50 on distance and routes -> s1 worst (later)
             [0, 850, 5, 0], [0, 820, 9, 0],      # island 1: s3 is not better than s2 (within 50, more routes) -> s3
             [0, 800, 4, 0], [200, 100, 1, 0]]    # island 2: s5 (penalty)
    st = o.migrate(synth.Params(population=6, islands=3, migrate_epochs=1, migrate_mode=0),
                   _lex_state(o, cur_v, best_v), 1)
    # ring: s1's best -> island 1's worst s3; s2's best -> island 2's worst s5; s5's best -> island 0's worst s1
    assert st["cur"][3].tolist() == np.roll(np.arange(o.n), 1).tolist() and st["cur_v"][3].tolist() == best_v[1]
    assert st["cur"][5].tolist() == np.roll(np.arange(o.n), 2).tolist() and st["cur_v"][5].tolist() == best_v[2]
    assert st["cur"][1].tolist() == np.roll(np.arange(o.n), 5).tolist() and st["cur_v"][1].tolist() == best_v[5]
    # a target's best changes only when the elite is strictly better than it
    assert st["best_v"][3].tolist() == best_v[3]          # [0,830,4] vs [0,760,5]: 830 > 760 + 50, not better
    assert st["best_v"][5].tolist() == best_v[2]          # [0,700,6] vs [0,900,7]: better
    assert st["best_v"][1].tolist() == best_v[1]          # penalty 100 vs 0: not better
    assert st["cur_f"][3] == 830 and st["best_f"][5] == 700
    for s in (0, 2, 4):
        assert st["cur_v"][s].tolist() == cur_v[s]


def test_lexicographic_elite_injection_by_hand():
    o = oracle.OracleInstance(vrptw(6, 1, lex_order=(VEH, DIST, 0), lex_tol=(0, 30, 0)))
    best_v = [[0, 5, 700, 0], [0, 4, 900, 0], [0, 4, 880, 0], [0, 6, 500, 0], [0, 4, 860, 0], [0, 5, 100, 0]]
    # best: s1 (4 routes), s2 ties s1 within 30, s4 beats s1 by more than 30? 860 + 30 < 900: yes -> s4
    cur_v = [[0, 5, 100, 0]] * 6
    st = o.migrate(synth.Params(population=6, elite_epochs=1), _lex_state(o, cur_v, best_v), 1)
    # every current vector ties: the worst is the last one, s5, which takes s4's best
    assert st["cur_v"][5].tolist() == best_v[4] and st["cur_f"][5] == 4
    assert st["best_v"][5].tolist() == best_v[4]          # 4 routes beat 5
    assert [s for s in range(6) if st["cur_v"][s].tolist() != cur_v[s]] == [5]


def test_islands_run_invariants():
    inst = vrptw(16, 12, lex_order=(DIST, VEH, 0), lex_tol=(25, 0, 0))
    o = oracle.OracleInstance(inst)
    for mode in (0, 1, 2):
        p = synth.Params(seed=5, population=8, candidates=64, generations=30, epoch=3, islands=2,
                         migrate_epochs=2, migrate_mode=mode, migrate_n=2, elite_epochs=3,
                         alpha_q32=synth.alpha_q32_for(30))
        a = o.init(p)
        b = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in a.items()}
        o.run(p, a, 30)
        o.run(p, b, 30, threads=3)
        for k in a:
            assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), (mode, k)
        for s in range(p.population):
            assert list(o.lex_vector(a["cur"][s])) == list(a["cur_v"][s])
            assert list(o.lex_vector(a["best"][s])) == list(a["best_v"][s])
            assert not o.lex_better(a["cur_v"][s], a["best_v"][s])
