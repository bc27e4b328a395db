"""Oracle pins for the multi-row solution form (paper, Sec. "Solution
Structure": row-organised solutions with a length per row; Tab. operators,
row level: row_swap, row_split, row_merge; Tab. generality: CVRP and VRPTW as
multi-row permutations; Sec. "Partition Encoding Heuristic Initialization").

A solution of n customers and R rows holds n + R entries: entry c < n is
customer node c + 1, entries n .. n + R - 1 are row markers, each row's
customers are followed by its marker and the final entry is a marker.

- The objective recomputed here route by route from the definition, on
  random solutions with binding capacities and windows, in the weighted and
  lexicographic modes.
- Brute force: over every solution of a small instance the best objective
  equals the best over every way to split the customers into at most R
  ordered routes, enumerated here without the encoding.
- Reductions: one row with loose constraints is a TSP tour through the depot
  (the oracle's TSP objective); rows that are the capacity split of a giant
  tour cost what the giant tour costs.
- Row operators and the sweep initialisation worked by hand; invariants of
  every operator under random draws; the random initial solutions keep the
  final marker and shuffle the rest uniformly."""
import itertools
from collections import Counter

import numpy as np
import pytest

import oracle
import synth

DIST, VEH, LONG = 1, 2, 3


def rows_inst(n, R, key, cap=None, loose=False, **kw):
    base = synth.vrptw_random(n, 11, key=key)
    b = base.b.copy()
    hor = base.horizon
    if loose:
        b[1, :] = 0
        b[2, :] = 10**6
        hor = 10**6
    return synth.Instance(synth.VRPTW_ROWS, n, base.a, b, capacity=base.capacity if cap is None else cap,
                          vehicles=R, service_time=base.service_time, horizon=hor, key=key, **kw)


def d(xy, u, v):
    """nearest-integer Euclidean distance, computed here in exact integers"""
    s = int((xy[u][0] - xy[v][0]) ** 2 + (xy[u][1] - xy[v][1]) ** 2)
    r = int(np.floor(np.sqrt(s)))
    while r * r > s:
        r -= 1
    while (r + 1) ** 2 <= s:
        r += 1
    # round half up: r + 1 when s >= (r + 1/2)^2, i.e. 4 s >= (2 r + 1)^2
    return r + (4 * s >= (2 * r + 1) ** 2)


def route_costs(inst, routes):
    """(distance, routes, longest, lateness, load above capacity) of a list of
    routes (lists of customer nodes), from the definition"""
    xy = [tuple(map(int, p)) for p in inst.a]
    dem, rdy, due = inst.b
    dist = late = longest = over = 0
    used = 0
    for r in routes:
        if not r:
            continue
        used += 1
        t = load = ln = 0
        prev = 0
        for c in r:
            dd = d(xy, prev, c)
            dist += dd
            ln += dd
            t = max(t + dd, int(rdy[c]))
            late += max(0, t - int(due[c]))
            t += inst.service_time
            load += int(dem[c])
            prev = c
        back = d(xy, prev, 0)
        dist += back
        ln += back
        late += max(0, t + back - inst.horizon)
        longest = max(longest, ln)
        over += max(0, load - inst.capacity)
    return dist, used, longest, late, over


def rows_of(inst, x):
    """the routes of a solution (customer nodes per row)"""
    out, cur = [], []
    for e in x:
        if e < inst.n:
            cur.append(int(e) + 1)
        else:
            out.append(cur)
            cur = []
    assert not cur, "the final entry must be a marker"
    return out


def objective_here(inst, x):
    dist, used, longest, late, over = route_costs(inst, rows_of(inst, x))
    w = inst.obj_weights if any(inst.obj_weights) else (1, 0, 0)
    return w[0] * dist + w[1] * used + w[2] * longest + 100 * late + 100 * over


def random_rows_solution(inst, rng):
    N = inst.n + inst.vehicles
    x = np.concatenate([rng.permutation(N - 1), [N - 1]]).astype(np.int32)
    return x


@pytest.mark.parametrize("weights", [(0, 0, 0), (6, 2, 2), (1, 1000, 0)])
def test_objective_route_by_route(weights):
    rng = np.random.default_rng(5)
    for key, (n, R, cap) in enumerate([(12, 4, 60), (20, 5, 90), (9, 3, 200), (15, 1, 10**6)]):
        inst = rows_inst(n, R, key, cap=cap, obj_weights=weights)
        o = oracle.OracleInstance(inst)
        assert o.n == n + R
        for _ in range(60):
            x = random_rows_solution(inst, rng)
            assert o.objective(x) == objective_here(inst, x)


def test_lexicographic_vector_route_by_route():
    rng = np.random.default_rng(6)
    inst = rows_inst(14, 4, 3, cap=70, lex_order=(VEH, DIST, LONG), lex_tol=(0, 30, 0))
    o = oracle.OracleInstance(inst)
    for _ in range(80):
        x = random_rows_solution(inst, rng)
        dist, used, longest, late, over = route_costs(inst, rows_of(inst, x))
        assert list(o.lex_vector(x)) == [100 * late + 100 * over, used, dist, longest]


def test_brute_force_best_matches_route_enumeration():
    n, R = 5, 2
    inst = rows_inst(n, R, 9, cap=60)
    o = oracle.OracleInstance(inst)
    N = n + R
    best_enc = min(o.objective(np.array(list(p) + [N - 1], np.int32)) for p in itertools.permutations(range(N - 1)))
    # every split of the customers into R ordered routes (some possibly empty)
    best_direct = None
    for assign in itertools.product(range(R), repeat=n):
        groups = [[c + 1 for c in range(n) if assign[c] == r] for r in range(R)]
        for orders in itertools.product(*[list(itertools.permutations(g)) for g in groups]):
            dist, used, longest, late, over = route_costs(inst, [list(r) for r in orders])
            f = dist + 100 * late + 100 * over
            best_direct = f if best_direct is None else min(best_direct, f)
    assert best_enc == best_direct


def test_one_loose_row_is_a_tsp_tour_through_the_depot():
    n = 10
    inst = rows_inst(n, 1, 4, cap=10**6, loose=True)
    o = oracle.OracleInstance(inst)
    tsp = oracle.OracleInstance(synth.Instance(synth.TSP, n + 1, inst.a, a_is_coords=1, key=4))
    rng = np.random.default_rng(2)
    for _ in range(30):
        perm = rng.permutation(n)
        x = np.concatenate([perm, [n]]).astype(np.int32)
        tour = np.concatenate([[0], perm + 1]).astype(np.int32)
        late_free = o.objective(x)
        assert late_free == tsp.objective(tour)


def test_rows_of_a_capacity_split_cost_the_giant_tour():
    n, R = 16, 8
    rows = rows_inst(n, R, 5, cap=80)
    giant = synth.Instance(synth.VRPTW, n, rows.a, rows.b, capacity=80, vehicles=R,
                           service_time=rows.service_time, horizon=rows.horizon, key=5)
    og, orr = oracle.OracleInstance(giant), oracle.OracleInstance(rows)
    rng = np.random.default_rng(8)
    checked = 0
    for _ in range(50):
        perm = rng.permutation(n)
        # the greedy capacity split, written here
        routes, cur, load = [], [], 0
        for e in perm:
            c = int(e) + 1
            if cur and load + int(rows.b[0][c]) > rows.capacity:
                routes.append(cur)
                cur, load = [], 0
            cur.append(e)
            load += int(rows.b[0][c])
        routes.append(cur)
        if len(routes) > R:
            continue
        x = []
        for r, rt in enumerate(routes):
            x += list(rt) + [n + r]
        x += [n + r for r in range(len(routes), R)]
        assert orr.objective(np.array(x, np.int32)) == og.objective(perm.astype(np.int32))
        checked += 1
    assert checked >= 20


# ------------------------------------------------------------ row operators
SOL = np.array([0, 9, 3, 2, 1, 5, 12, 6, 7, 11, 10, 8, 4, 13, 14, 15], np.int32)   # n = 12, R = 4


def w_for(p, N):
    """a draw w1 with floor(w1 (N - 1) / 2^32) = p"""
    w = -(-(p << 32) // (N - 1))
    assert (w * (N - 1)) >> 32 == p
    return w


@pytest.mark.parametrize("op,p,expect", [
    # row_swap: rows 0 and 1 trade places, markers with them
    (5, 0, [6, 7, 11, 10, 8, 4, 13, 0, 9, 3, 2, 1, 5, 12, 14, 15]),
    (5, 6, [6, 7, 11, 10, 8, 4, 13, 0, 9, 3, 2, 1, 5, 12, 14, 15]),
    # row 1 and the empty row 2
    (5, 7, [0, 9, 3, 2, 1, 5, 12, 14, 6, 7, 11, 10, 8, 4, 13, 15]),
    # the empty row 2 and the empty last row
    (5, 14, [0, 9, 3, 2, 1, 5, 12, 6, 7, 11, 10, 8, 4, 13, 15, 14]),
    # row_split: the empty last row's marker moves to p
    (6, 3, [0, 9, 3, 14, 2, 1, 5, 12, 6, 7, 11, 10, 8, 4, 13, 15]),
    (6, 0, [14, 0, 9, 3, 2, 1, 5, 12, 6, 7, 11, 10, 8, 4, 13, 15]),
    (6, 14, list(SOL)),                       # p = N - 2: nothing
    # row_merge: row 0 takes row 1's customers, an empty row closes the sequence
    (7, 2, [0, 9, 3, 2, 1, 5, 6, 7, 11, 10, 8, 4, 13, 14, 12, 15]),
    (7, 13, [0, 9, 3, 2, 1, 5, 12, 6, 7, 11, 10, 8, 4, 14, 13, 15]),
    (7, 14, list(SOL)),                       # the next row is the empty last row
])
def test_row_operators_by_hand(op, p, expect):
    inst = synth.Instance(synth.VRPTW_ROWS, 12, np.zeros((13, 2), np.int32), np.zeros((3, 13), np.int32),
                          capacity=10, vehicles=4, horizon=100)
    o = oracle.OracleInstance(inst)
    assert list(o.apply_op(SOL, op, w_for(p, 16), 0, 0)) == expect


def test_row_split_needs_an_empty_last_row():
    inst = synth.Instance(synth.VRPTW_ROWS, 4, np.zeros((5, 2), np.int32), np.zeros((3, 5), np.int32),
                          capacity=10, vehicles=2, horizon=100)
    o = oracle.OracleInstance(inst)
    x = np.array([0, 1, 4, 2, 3, 5], np.int32)
    for p in range(5):
        assert list(o.apply_op(x, 6, w_for(p, 6), 0, 0)) == list(x)
    # the last row is empty here: split row 0 before its second customer
    y = np.array([0, 1, 2, 3, 4, 5], np.int32)
    assert list(o.apply_op(y, 6, w_for(1, 6), 0, 0)) == [0, 4, 1, 2, 3, 5]


def test_element_operators_keep_the_final_marker():
    inst = rows_inst(10, 3, 2)
    o = oracle.OracleInstance(inst)
    rng = np.random.default_rng(3)
    x = random_rows_solution(inst, rng)
    for _ in range(400):
        op = int(rng.integers(0, 8))
        w = [int(v) for v in rng.integers(0, 2**32, size=3)]
        y = o.apply_op(x, op, *w)
        assert sorted(y) == list(range(13)) and y[-1] >= 10
        ry, rx = rows_of(inst, y), rows_of(inst, x)
        if op == 5:      # the same routes, two of them in the other order
            assert Counter(map(tuple, ry)) == Counter(map(tuple, rx))
        elif op == 7 and ry != rx:    # two neighbouring routes joined, an empty one at the end
            assert ry[-1] == [] and len([r for r in ry if r]) >= len([r for r in rx if r]) - 1
            joined = {tuple(rx[i] + rx[i + 1]) for i in range(len(rx) - 1)}
            assert any(tuple(r) in joined for r in ry)
        elif op == 6:    # one route cut in two, at most
            assert len([r for r in ry if r]) <= len([r for r in rx if r]) + 1
            assert [c for r in ry for c in r] == [c for r in rx for c in r]
        x = y


def test_sweep_initialisation_by_hand():
    # depot (50, 50); customers at angles 0 (twice), 45, 90, 180 and 270 degrees
    xy = np.array([[50, 50], [60, 50], [50, 60], [40, 50], [50, 40], [70, 50], [60, 60]], np.int32)
    dem = [0, 3, 2, 6, 1, 4, 5]
    rdy = [0, 0, 10, 5, 5, 0, 20]
    due = [1000, 300, 100, 50, 50, 200, 100]
    b = np.array([dem, rdy, due], np.int32)
    # sweep order 1, 5, 6, 2, 3, 4; capacity 10 closes a row at 6 and at 3
    inst = synth.Instance(synth.VRPTW_ROWS, 6, xy, b, capacity=10, vehicles=3, horizon=1000)
    h = oracle.OracleInstance(inst).heuristic_perms()
    assert h.shape == (1, 9)
    # rows {1,5} by due: 5, 1; {6,2}: due tie, by ready: 2, 6; {3,4}: due and ready tie: 3, 4
    assert list(h[0]) == [4, 0, 6, 1, 5, 7, 2, 3, 8]
    # two rows: the last takes every customer left, ordered by (due, ready, index)
    inst2 = synth.Instance(synth.VRPTW_ROWS, 6, xy, b, capacity=10, vehicles=2, horizon=1000)
    assert list(oracle.OracleInstance(inst2).heuristic_perms()[0]) == [4, 0, 6, 2, 3, 1, 5, 7]


def test_random_initial_solutions_keep_the_marker_and_are_uniform():
    inst = synth.Instance(synth.VRPTW_ROWS, 2, np.zeros((3, 2), np.int32), np.zeros((3, 3), np.int32),
                          capacity=10, vehicles=2, horizon=100, key=3)
    o = oracle.OracleInstance(inst)
    p = synth.Params(seed=77, generations=1, population=1, candidates=1)
    seen = Counter()
    for q in range(6000):
        x = o.random_solution(p, q)
        assert x[-1] == 3
        seen[tuple(x[:3])] += 1
    assert len(seen) == 6
    # chi-square over the 6 orders of the first three entries, 5 degrees of freedom, p ~ 0.001
    chi2 = sum((v - 1000) ** 2 / 1000 for v in seen.values())
    assert chi2 < 20.5


def test_presets_and_default_operator_set():
    inst = rows_inst(20, 4, 1)
    o = oracle.OracleInstance(inst)
    assert o.effective_mask(0) == synth.ROWS_ALL_OPS
    w = o.initial_weights(0)
    # raw: 1.0 for the O(1) and row operators, or-opt 0.8 and 3-opt 0.5 at 24 entries
    raw = [65536, 65536, 65536, 52429, 32768, 65536, 65536, 65536]
    s = sum(raw)
    assert list(w[:8]) == [max(1, (r << 16) // s) for r in raw] and not any(w[8:])


@pytest.mark.parametrize("lex", [False, True])
def test_run_invariants_and_threaded_runner(lex):
    kw = dict(lex_order=(VEH, DIST, 0), lex_tol=(0, 25, 0)) if lex else {}
    inst = rows_inst(18, 5, 6, cap=70, **kw)
    o = oracle.OracleInstance(inst)
    p = synth.Params(seed=4, generations=60, population=6, candidates=24, op_mask=synth.ROWS_ALL_OPS,
                     alpha_q32=synth.alpha_q32_for(60))
    st = o.init(p)
    a = o.run(p, {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in st.items()}, 60)
    b = o.run(p, {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in st.items()}, 60, threads=3)
    for key in ("cur", "best", "cur_f", "best_f", "w_op", "u_op", "tot_u_op"):
        assert np.array_equal(a[key], b[key]), key
    for s in range(p.population):
        for arr, fa in ((a["cur"], a["cur_f"]), (a["best"], a["best_f"])):
            x = arr[s]
            assert sorted(x) == list(range(23)) and x[-1] >= 18
            if lex:
                v = o.lex_vector(x)
                assert fa[s] == v[0] + v[1]
            else:
                assert fa[s] == objective_here(inst, x)
    assert int(a["tot_u_op"][5:8].sum()) > 0 and not a["tot_u_op"][8:].any()
