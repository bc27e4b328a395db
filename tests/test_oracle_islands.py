"""Island model and elite injection in the oracle (paper, Sec. "Island Model
and Elite Injection"; readings in the design notes): migrations and
injections worked by hand on a six-solution population, ties, intervals, and
the invariants of whole runs with islands."""
import numpy as np
import pytest

import oracle
import synth


def _state(o):
    """Six solutions of a 3-city instance in three islands of two: current
    objectives, best objectives, and best vectors that name their solution
    (b[s] = [s, s, s]) so that every copy can be traced."""
    st = o.new_state(6)
    st["cur"][:] = np.array([[0, 1, 2], [0, 2, 1], [1, 0, 2], [1, 2, 0], [2, 0, 1], [2, 1, 0]], np.int32)
    st["cur_f"][:] = [10, 30, 20, 25, 40, 15]
    st["best_f"][:] = [8, 30, 20, 12, 35, 15]
    st["best"][:] = np.repeat(np.arange(6, dtype=np.int32)[:, None], 3, axis=1)
    return st


def _params(**kw):
    return synth.Params(population=6, **kw)


@pytest.fixture(scope="module")
def o():
    return oracle.OracleInstance(synth.tsp_uniform(3, 0))


def _row(v):
    return [v, v, v]


def test_ring_migration_by_hand(o):
    # island bests: s0 (8), s3 (12), s5 (15); island worsts: s1 (30), s3 (25), s4 (40)
    # s0 -> island 1's worst s3, s3 -> island 2's worst s4, s5 -> island 0's worst s1;
    # s3 is a source and a target: s4 receives s3's best from before the copies
    st = o.migrate(_params(islands=3, migrate_epochs=1, migrate_mode=0), _state(o), 1)
    assert st["cur"][3].tolist() == _row(0) and st["cur_f"][3] == 8 and st["best_f"][3] == 8
    assert st["best"][3].tolist() == _row(0)
    assert st["cur"][4].tolist() == _row(3) and st["cur_f"][4] == 12 and st["best_f"][4] == 12
    assert st["cur"][1].tolist() == _row(5) and st["cur_f"][1] == 15 and st["best_f"][1] == 15
    for s in (0, 2, 5):   # untouched
        assert st["cur_f"][s] == _state(o)["cur_f"][s]
        assert st["best"][s].tolist() == _row(s)


def test_top_n_migration_by_hand(o):
    # the two best: s0 (8), s3 (12); each island's two worst, worst first:
    # (s1, s0), (s3, s2), (s4, s5); the best replaces the worst, the second the second
    st = o.migrate(_params(islands=3, migrate_epochs=1, migrate_mode=1, migrate_n=2), _state(o), 1)
    for s, src, f in ((1, 0, 8), (3, 0, 8), (4, 0, 8), (0, 3, 12), (2, 3, 12), (5, 3, 12)):
        assert st["cur"][s].tolist() == _row(src) and st["cur_f"][s] == f, s
    # a solution keeps its own best unless the elite improves it
    assert st["best_f"].tolist() == [8, 8, 12, 8, 8, 12]
    assert st["best"][0].tolist() == _row(0) and st["best"][2].tolist() == _row(3)


def test_hybrid_alternates_ring_and_top_n(o):
    ring = o.migrate(_params(islands=3, migrate_epochs=1, migrate_mode=0), _state(o), 1)
    topn = o.migrate(_params(islands=3, migrate_epochs=1, migrate_mode=1, migrate_n=1), _state(o), 1)
    p = _params(islands=3, migrate_epochs=2, migrate_mode=2, migrate_n=1)
    odd = o.migrate(p, _state(o), 2)      # e / 2 = 1: ring
    even = o.migrate(p, _state(o), 4)     # e / 2 = 2: top-N
    skip = o.migrate(p, _state(o), 3)     # not a multiple of the interval
    for k in ("cur", "cur_f", "best", "best_f"):
        assert np.array_equal(odd[k], ring[k]) and np.array_equal(even[k], topn[k])
        assert np.array_equal(skip[k], _state(o)[k])


def test_elite_injection_by_hand(o):
    # population best s0 (8) replaces its worst s4 (40); islands play no part
    for isl in (0, 3):
        st = o.migrate(_params(islands=isl, elite_epochs=2), _state(o), 2)
        assert st["cur"][4].tolist() == _row(0) and st["cur_f"][4] == 8 and st["best_f"][4] == 8
        changed = [s for s in range(6) if st["cur_f"][s] != _state(o)["cur_f"][s]]
        assert changed == [4]


def test_ties_take_the_lowest_best_and_the_highest_worst(o):
    st = _state(o)
    st["best_f"][:] = [5, 5, 9, 9, 9, 9]
    st["cur_f"][:] = [7, 7, 7, 7, 7, 7]
    st = o.migrate(_params(elite_epochs=1), st, 1)
    assert st["cur"][5].tolist() == _row(0)          # best: s0 of {s0, s1}; worst: s5 of all


def test_no_migration_without_islands_or_interval(o):
    for p in (_params(islands=0, migrate_epochs=1), _params(islands=3, migrate_epochs=0),
              _params(islands=1, migrate_epochs=1, elite_epochs=0)):
        st = o.migrate(p, _state(o), 1)
        for k in ("cur", "cur_f", "best", "best_f"):
            assert np.array_equal(st[k], _state(o)[k])


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_runs_with_islands_keep_the_invariants(mode):
    inst = synth.tsp_uniform(14, 3, key=4)
    o = oracle.OracleInstance(inst)
    p = synth.Params(seed=5, generations=60, population=8, candidates=32, alpha_q32=synth.alpha_q32_for(60),
                     islands=4, migrate_epochs=2, migrate_mode=mode, migrate_n=1, elite_epochs=3)
    st = o.init(p)
    prev = None
    for _ in range(6):
        st = o.run(p, st, 10)
        for s in range(8):
            assert sorted(st["cur"][s]) == list(range(14))
            assert o.objective(st["cur"][s]) == st["cur_f"][s]
            assert o.objective(st["best"][s]) == st["best_f"][s]
            assert st["best_f"][s] <= st["cur_f"][s]
        # a migration never loses the population's best
        ib = int(st["best_f"].min())
        assert prev is None or ib <= prev
        prev = ib
    # and it changes the trajectory
    plain = o.solve(p.with_(islands=0, migrate_epochs=0, elite_epochs=0))
    assert not np.array_equal(plain["cur"], st["cur"])
