"""Pins of the CPU oracle against values that do not come from the oracle:
published known-answer vectors, worked values computed by hand (tests/golden),
closed forms, brute force, textbook routines and invariants."""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def gold(name):
    with open(os.path.join(GOLD, name)) as fh:
        return json.load(fh)


# ------------------------------------------------------------------ RNG
def test_philox_known_answers():
    for v in gold("philox_kat.json")["vectors"]:
        ctr = [int(x, 16) for x in v["ctr"]]
        key = [int(x, 16) for x in v["key"]]
        out = [int(x, 16) for x in v["out"]]
        assert list(oracle.philox(ctr, key)) == out


def test_philox_uniformity_chi_square():
    # 64 bins over 4096 blocks x 4 words; chi-square with 63 dof stays well below 120
    words = np.concatenate([oracle.philox([i, 7, 3, 1], [42, 0]) for i in range(4096)])
    hist = np.bincount(words >> 26, minlength=64)
    exp = len(words) / 64
    chi2 = float(((hist - exp) ** 2 / exp).sum())
    assert chi2 < 120


# ------------------------------------------------------------------ distance
def test_nint_distance_worked_values():
    for x1, y1, x2, y2, d in gold("worked_values.json")["nint_distance"]["cases"]:
        assert oracle.nint_dist(x1, y1, x2, y2) == d


def test_nint_distance_matches_float_rounding():
    # an integer square sum is never (k + 1/2)^2, so float64 rounding is exact here
    r = np.random.default_rng(5)
    for _ in range(2000):
        x1, y1, x2, y2 = (int(v) for v in r.integers(0, 10001, 4))
        ref = int(math.floor(math.hypot(x1 - x2, y1 - y2) + 0.5))
        assert oracle.nint_dist(x1, y1, x2, y2) == ref


def test_isqrt_matches_python():
    r = np.random.default_rng(1)
    for v in list(r.integers(0, 2**62, 500)) + [0, 1, 2, 3, 4, 15, 16, 17, 2**62 - 1]:
        assert oracle.isqrt(int(v)) == math.isqrt(int(v))


# ------------------------------------------------------------------ acceptance, cooling
def test_exp_threshold_worked_values():
    for c in gold("worked_values.json")["exp_tables"]["threshold_cases"]:
        thr, rej = oracle.accept_threshold(c["delta"], c["t_q16"])
        if c.get("reject"):
            assert rej
        else:
            assert not rej and thr == c["p"]


def test_exp_threshold_close_to_exp():
    # p / 2^31 approximates e^{-delta/T} to within table rounding (relative 1e-8)
    for delta in (1, 2, 3, 7, 10, 33, 100):
        for t_q16 in (65536, 3 * 65536 + 17, 20 * 65536, 500 * 65536):
            z = (delta << 24) // t_q16
            thr, rej = oracle.accept_threshold(delta, t_q16)
            if z >= 4096:
                assert rej
                continue
            want = 2**31 * math.exp(-z / 256.0)
            assert abs(thr - want) <= 2 + want * 1e-8


def test_exp_threshold_wide_deltas_exact():
    # z = floor(2^24 delta / T) in Python big integers: the quotient must not
    # wrap for delta >= 2^40 (Alg. 1, rand() < e^{-delta/T})
    cases = [(2**40 + 5, 65536, None), (2**41, 2**62, 2081412522)]   # reject; z = 8
    for delta, t_q16, p in cases:
        thr, rej = oracle.accept_threshold(delta, t_q16)
        assert rej if p is None else (not rej and thr == p)
    deltas = [2**39, 2**39 + 3, 2**40 - 1, 2**40 + 5, 2**41, 2**44, 2**52 - 1, 2**52, 2**62 + 11]
    temps = [2**16, 3 * 2**20 + 7, 2**40 + 17, 2**53 + 1, 2**62, 2**64 - 1]
    r = np.random.default_rng(9)
    for _ in range(400):
        deltas.append(int(r.integers(1, 2**62)))
        temps.append(int(r.integers(1, 2**63)) * 2 + 1)
    for delta in deltas:
        for t_q16 in temps + [delta << 12, (delta << 12) + 1, (delta << 12) - 1]:
            if not 0 < t_q16 < 2**64:
                continue
            z = (delta << 24) // t_q16
            thr, rej = oracle.accept_threshold(delta, t_q16)
            if z >= 4096:
                assert rej, (delta, t_q16)
            else:
                want = 2**31 * math.exp(-z / 256.0)
                assert not rej and abs(thr - want) <= 2 + want * 1e-8, (delta, t_q16, z, thr)


def test_cooling_exact_and_sequence():
    g = gold("worked_values.json")["cooling"]
    assert synth.alpha_q32_for(g["generations"]) == g["alpha_q32"]
    t = g["sequence"][0]
    for want in g["sequence"][1:]:
        t = oracle.cool(t, g["alpha_q32"])
        assert t == want
    r = np.random.default_rng(3)
    for _ in range(2000):
        t = int(r.integers(0, 2**63)) * 2 + int(r.integers(0, 2))
        a = int(r.integers(1, 2**32))
        assert oracle.cool(t, a) == (t * a) >> 32   # exact 128-bit product


# ------------------------------------------------------------------ AOS arithmetic
def test_aos_update_worked_example():
    g = gold("worked_values.json")["aos_update"]
    inst, p = synth.c1_small_tsp(0)
    o = oracle.OracleInstance(inst)
    st = o.new_state(1)
    for op, w, u, v in zip(g["ops"], g["w_before"], g["u"], g["v"]):
        st["w_op"][op], st["u_op"][op], st["v_op"][op] = w, u, v
    st["w_k"][:] = [52429, 9830, 3277]
    st["epoch_ref"] = 100
    o.aos_update(p, st, 100)
    assert [int(st["w_op"][i]) for i in g["ops"]] == g["w_after"]
    assert st["stag"] == 1                       # instance best did not improve
    assert int(st["u_op"].sum()) == 0 and int(st["v_op"].sum()) == 0   # windowed counts


def test_aos_single_op_and_bounds():
    inst = synth.knapsack_random(30)
    o = oracle.OracleInstance(inst)
    p = synth.Params(population=1, op_mask=1 << synth.OP_FLIP)
    st = o.new_state(1)
    st["w_op"][4] = 65536
    st["w_k"][:] = [52429, 9830, 3277]
    r = np.random.default_rng(0)
    for _ in range(50):
        st["u_op"][4] = int(r.integers(0, 10**6)); st["v_op"][4] = int(r.integers(0, 1 + st["u_op"][4]))
        u = r.integers(0, 10**6, 3); st["u_k"][:] = u
        st["v_k"][:] = [int(r.integers(0, 1 + x)) for x in u]
        o.aos_update(p, st, 0)
        assert st["w_op"][4] == 65536                      # one enabled op always holds all mass
        assert 3 <= int(st["w_k"].sum()) <= 65536 and int(st["w_k"].min()) >= 1


def test_stagnation_resets_k_weights():
    inst, p = synth.c1_small_tsp(0)
    o = oracle.OracleInstance(inst)
    st = o.new_state(1)
    st["w_op"][[0, 1, 3]] = [23405, 23405, 18724]
    st["w_k"][:] = [60000, 4000, 1536]
    st["epoch_ref"] = 50
    for e in range(5):
        st["u_k"][:] = [100, 0, 0]; st["v_k"][:] = [100, 0, 0]
        o.aos_update(p, st, 50)
    assert list(st["w_k"]) == gold("worked_values.json")["k_defaults"]["w_k"]
    assert st["stag"] == 0


def test_initial_weights_presets():
    for c in gold("worked_values.json")["initial_weights"]["cases"]:
        o = oracle.OracleInstance(synth.tsp_uniform(c["n"], 1))
        assert list(o.initial_weights(c["mask"], c.get("init_w"))) == c["w"], c


# ------------------------------------------------------------------ operators
def test_operator_worked_examples():
    names = {n: i for i, n in enumerate(synth.OP_NAMES)}
    for c in gold("operators.json")["cases"]:
        n = c["n"]
        if c.get("zeros"):
            if c["op"] in ("flip", "segflip"):
                inst = synth.Instance(synth.KNAPSACK, n, np.ones(n), np.ones(n), capacity=n)
            else:
                inst = synth.Instance(synth.INTCOLOR, n, np.array([[0, 1]]), lb=c["lb"], ub=c["ub"], n_edges=1)
            x = np.zeros(n, np.int32)
        else:
            inst = synth.tsp_uniform(n, 0)
            x = np.arange(n, dtype=np.int32)
        o = oracle.OracleInstance(inst)
        w = [int(v, 16) for v in c["w"]]
        assert list(o.apply_op(x, names[c["op"]], *w)) == c["out"], c


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 12])
def test_permutation_ops_keep_validity_and_shape(n):
    o = oracle.OracleInstance(synth.tsp_uniform(n, 0))
    r = np.random.default_rng(n)
    for _ in range(300):
        x = r.permutation(n).astype(np.int32)
        op = int(r.integers(0, 4))
        w = [int(v) for v in r.integers(0, 2**32, 3, dtype=np.uint64)]
        y = o.apply_op(x, op, *w)
        assert sorted(y) == list(range(n))
        if n < 2:
            assert list(y) == list(x)
            continue
        diff = np.nonzero(x != y)[0]
        if op == 1:                     # swap: exactly two positions exchanged
            assert len(diff) == 2 and x[diff[0]] == y[diff[1]] and x[diff[1]] == y[diff[0]]
        elif op == 0 and len(diff):     # reversal: the changed range is reversed
            lo, hi = diff[0], diff[-1]
            assert list(y[lo:hi + 1]) == list(x[lo:hi + 1][::-1])
        elif op == 2:                   # insert: a rotation by one of the changed range
            lo, hi = diff[0], diff[-1]
            seg_x, seg_y = list(x[lo:hi + 1]), list(y[lo:hi + 1])
            assert seg_y == seg_x[1:] + seg_x[:1] or seg_y == seg_x[-1:] + seg_x[:-1]


# ------------------------------------------------------------------ objectives
def _tsp_len_float(xy, perm):
    tot = 0
    for a, b in zip(perm, list(perm[1:]) + [perm[0]]):
        tot += int(math.floor(math.hypot(*(xy[a] - xy[b])) + 0.5))
    return tot


def test_tsp_objective_exhaustive_n7():
    inst = synth.tsp_uniform(7, 3)
    o = oracle.OracleInstance(inst)
    xy = inst.a.astype(np.int64)
    for perm in itertools.permutations(range(7)):
        assert o.objective(np.array(perm)) == _tsp_len_float(xy, perm)


def test_tsp_circle_planted_optimum_brute_force():
    inst = synth.tsp_circle(9)
    o = oracle.OracleInstance(inst)
    best = min(o.objective(np.array((0,) + p)) for p in itertools.permutations(range(1, 9)))
    assert best == o.objective(np.arange(9))


def test_tsp_matrix_and_coords_agree():
    inst = synth.tsp_uniform(20, 2)
    o = oracle.OracleInstance(inst)
    D = np.array([[o.dist(i, j) for j in range(20)] for i in range(20)], np.int32)
    om = oracle.OracleInstance(synth.tsp_matrix(D))
    r = np.random.default_rng(0)
    for _ in range(50):
        x = r.permutation(20)
        assert o.objective(x) == om.objective(x)


def test_qap_reduces_to_tsp_with_cycle_flow():
    # flow = adjacency of the cycle 0-1-..-(n-1)-0, distance = a TSP matrix:
    # then sum_ij F_ij D_{p_i p_j} = 2 x tour length of p
    n = 7
    t = oracle.OracleInstance(synth.tsp_uniform(n, 4))
    D = np.array([[t.dist(i, j) for j in range(n)] for i in range(n)], np.int32)
    F = np.zeros((n, n), np.int32)
    for i in range(n):
        F[i, (i + 1) % n] = F[(i + 1) % n, i] = 1
    q = oracle.OracleInstance(synth.Instance(synth.QAP, n, F, D))
    for perm in itertools.permutations(range(n)):
        p = np.array(perm)
        assert q.objective(p) == 2 * t.objective(p)


def test_qap_path_on_line_brute_force():
    n = 7
    F = np.zeros((n, n), np.int32)
    for i in range(n - 1):
        F[i, i + 1] = F[i + 1, i] = 1
    D = np.abs(np.arange(n)[:, None] - np.arange(n)[None, :]).astype(np.int32)
    q = oracle.OracleInstance(synth.Instance(synth.QAP, n, F, D))
    vals = [q.objective(np.array(p)) for p in itertools.permutations(range(n))]
    assert min(vals) == 2 * (n - 1) == q.objective(np.arange(n))


def _knap_dp(w, v, cap):
    best = [0] * (cap + 1)                 # textbook 0/1 knapsack DP
    for wi, vi in zip(w, v):
        for c in range(cap, wi - 1, -1):
            best[c] = max(best[c], best[c - wi] + vi)
    return best[cap]


def test_knapsack_brute_force_equals_dp():
    for seed in range(3):
        inst = synth.knapsack_random(14, seed)
        o = oracle.OracleInstance(inst)
        fmin = min(o.objective(np.array(bits)) for bits in itertools.product((0, 1), repeat=14))
        assert fmin == -_knap_dp(list(inst.a), list(inst.b), inst.capacity)


def test_knapsack_feasible_value_and_penalty():
    inst = synth.knapsack_random(10, 7)
    o = oracle.OracleInstance(inst)
    ones = np.ones(10, np.int32)
    over = int(inst.a.sum()) - inst.capacity
    assert o.objective(ones) == -int(inst.b.sum()) + (int(inst.b.max()) + 1) * over
    assert o.objective(np.zeros(10, np.int32)) == 0


def test_vrptw_worked_examples():
    g = gold("vrptw_small.json")
    for c in g["cases"]:
        b = np.array([g["demand"], g["ready"], g["due"][:1] and [c["horizon"]] + g["due"][1:]], np.int32)
        inst = synth.Instance(synth.VRPTW, 3, np.array(g["coords"]), b, capacity=g["capacity"],
                              vehicles=g["vehicles"], service_time=g["service_time"],
                              horizon=c["horizon"])
        o = oracle.OracleInstance(inst)
        assert o.objective(np.array(c["tour"])) == c["f"], c


def test_vrptw_weighted_objectives_worked_examples():
    g = gold("vrptw_small.json")
    for c in g["weighted_cases"]:
        b = np.array([g["demand"], g["ready"], [c["horizon"]] + g["due"][1:]], np.int32)
        inst = synth.Instance(synth.VRPTW, 3, np.array(g["coords"]), b, capacity=g["capacity"],
                              vehicles=g["vehicles"], service_time=g["service_time"],
                              horizon=c["horizon"], obj_weights=tuple(c["weights"]))
        assert oracle.OracleInstance(inst).objective(np.array(c["tour"])) == c["f"], c


def test_vrptw_weighted_loose_reduces_to_tsp_through_depot():
    # one route that never waits or runs late: distance = longest route = the
    # closed tour through the depot, one route, so f = (wD + wM) tour + wR
    inst = synth.vrptw_random(8, 3)
    b = inst.b.copy()
    b[1, :] = 0
    b[2, :] = 10**6
    t = oracle.OracleInstance(synth.Instance(synth.TSP, 9, inst.a, a_is_coords=1))
    r = np.random.default_rng(5)
    for w in [(6, 2, 2), (0, 1000, 1), (1, 0, 0), (3, 0, 7)]:
        loose = synth.Instance(synth.VRPTW, 8, inst.a, b, capacity=10**6, vehicles=1, service_time=10,
                               horizon=10**6, obj_weights=w)
        o = oracle.OracleInstance(loose)
        for _ in range(10):
            x = r.permutation(8)
            tour = t.objective(np.concatenate([[0], x + 1]))
            assert o.objective(x) == (w[0] + w[2]) * tour + w[1], w


def test_vrptw_loose_reduces_to_tsp_through_depot():
    # unlimited capacity, one vehicle, windows never binding: f = closed tour depot -> tour -> depot
    inst = synth.vrptw_random(8, 1)
    b = inst.b.copy()
    b[1, :] = 0
    b[2, :] = 10**6
    loose = synth.Instance(synth.VRPTW, 8, inst.a, b, capacity=10**6, vehicles=1,
                           service_time=10, horizon=10**6)
    o = oracle.OracleInstance(loose)
    t = oracle.OracleInstance(synth.Instance(synth.TSP, 9, inst.a, a_is_coords=1))
    r = np.random.default_rng(2)
    for _ in range(30):
        x = r.permutation(8)
        assert o.objective(x) == t.objective(np.concatenate([[0], x + 1]))


def test_color_brute_force():
    inst = synth.color_planted(9, 3, 14, 0)
    o = oracle.OracleInstance(inst)
    vals = [o.objective(np.array(c)) for c in itertools.product(range(3), repeat=9)]
    assert min(vals) == 0
    k4 = synth.Instance(synth.INTCOLOR, 4, np.array([[i, j] for i in range(4) for j in range(i + 1, 4)]),
                        lb=0, ub=2, n_edges=6)
    o4 = oracle.OracleInstance(k4)
    assert min(o4.objective(np.array(c)) for c in itertools.product(range(3), repeat=4)) == 1


# ------------------------------------------------------------------ init
def test_heuristic_perms_sorted_by_row_sums():
    inst = synth.tsp_uniform(30, 5)
    o = oracle.OracleInstance(inst)
    D = np.array([[o.dist(i, j) for j in range(30)] for i in range(30)], np.int64)
    H = o.heuristic_perms()
    assert H.shape == (4, 30)
    rs, cs = D.sum(1), D.sum(0)
    for h, s, sign in ((H[0], rs, 1), (H[1], rs, -1), (H[2], cs, 1), (H[3], cs, -1)):
        assert sorted(h) == list(range(30))
        keys = [(sign * s[i], i) for i in h]
        assert keys == sorted(keys)
    q = oracle.OracleInstance(synth.qap_random(12, 0))
    assert q.heuristic_perms().shape == (8, 12)
    assert oracle.OracleInstance(synth.knapsack_random(12)).heuristic_perms().shape[0] == 0


@pytest.mark.parametrize("kind", ["tsp", "qap", "knap", "vrptw", "color"])
def test_init_selects_best_of_pool(kind):
    inst = {"tsp": lambda: synth.tsp_uniform(25, 1), "qap": lambda: synth.qap_random(14, 1),
            "knap": lambda: synth.knapsack_random(40, 1), "vrptw": lambda: synth.vrptw_random(20, 1),
            "color": lambda: synth.color_planted(20, 3)}[kind]()
    o = oracle.OracleInstance(inst)
    p = synth.Params(population=8, generations=0, alpha_q32=synth.alpha_q32_for(100))
    st = o.init(p)
    assert list(st["cur_f"]) == sorted(st["cur_f"])
    for s in range(8):
        assert o.objective(st["cur"][s]) == st["cur_f"][s]
    H = o.heuristic_perms()
    if len(H):
        assert st["cur_f"][0] <= min(o.objective(h) for h in H)
    assert st["T_q16"] == ((abs(int(st["cur_f"][0])) << 16) // inst.n) >> 2


# ------------------------------------------------------------------ whole runs
def _small(kind, seed=42, P=6, G=25, C=32, **kw):
    inst = {"tsp": lambda: synth.tsp_uniform(17, 2), "qap": lambda: synth.qap_random(11, 2),
            "knap": lambda: synth.knapsack_random(33, 2), "vrptw": lambda: synth.vrptw_random(12, 2),
            "color": lambda: synth.color_planted(15, 3)}[kind]()
    kw.setdefault("alpha_q32", synth.alpha_q32_for(max(G, 1)))
    p = synth.Params(seed=seed, population=P, generations=G, candidates=C, **kw)
    return oracle.OracleInstance(inst), p


def _valid(o, x):
    if o.inst.encoding == "perm":
        return sorted(x) == list(range(o.n))
    if o.inst.encoding == "binary":
        return set(np.unique(x)) <= {0, 1}
    return x.min() >= o.inst.lb and x.max() <= o.inst.ub


@pytest.mark.parametrize("kind", ["tsp", "qap", "knap", "vrptw", "color"])
def test_run_invariants(kind):
    o, p = _small(kind)
    st = o.init(p)
    prev_best = st["best_f"].copy()
    for _ in range(p.generations):
        o.run(p, st, 1)
        assert (st["best_f"] <= prev_best).all() and (st["best_f"] <= st["cur_f"]).all()
        prev_best = st["best_f"].copy()
    for s in range(p.population):
        assert _valid(o, st["cur"][s]) and _valid(o, st["best"][s])
        assert o.objective(st["cur"][s]) == st["cur_f"][s]
        assert o.objective(st["best"][s]) == st["best_f"][s]
    # mid-epoch: the counts cover 25 mod 10 = 5 generations of P*C candidates
    assert int(st["u_k"].sum()) == 5 * p.population * p.candidates
    assert int(st["u_op"].sum()) == sum((k + 1) * int(st["u_k"][k]) for k in range(3))
    w = st["w_op"][st["w_op"] > 0]
    assert 1 <= int(w.sum()) <= 65536 + len(w)


def test_determinism_and_seed_sensitivity():
    o, p = _small("tsp")
    a = o.solve(p)
    b = o.solve(p)
    c = o.solve(p.with_(seed=43))
    for k in ("cur", "best", "cur_f", "best_f", "w_op", "w_k"):
        assert np.array_equal(a[k], b[k])
    assert not np.array_equal(a["cur"], c["cur"])


def test_resume_equals_uninterrupted():
    o, p = _small("qap", G=40)
    full = o.solve(p)
    st = o.init(p)
    o.run(p, st, 20)
    snap = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in st.items()}
    o.run(p, snap, 20)
    for k in full:
        assert np.array_equal(np.asarray(full[k]), np.asarray(snap[k])), k


def test_greedy_limit_never_worsens():
    o, p = _small("tsp", t0_q16=1)            # T = 1/65536: every delta >= 1 has z >= 4096
    st = o.init(p)
    for _ in range(p.generations):
        before = st["cur_f"].copy()
        o.run(p, st, 1)
        assert (st["cur_f"] <= before).all()


def test_random_walk_limit_accepts_everything():
    o, p = _small("knap", t0_q16=2**62, alpha_q32=2**32 - 1)
    st = o.solve(p)
    assert st["accepted"] == p.population * p.generations


def test_credit_accepted_only_counts_accepts():
    o, p = _small("color", credit=1, G=7)
    st = o.solve(p)
    assert int(st["u_k"].sum()) == st["accepted"]


def test_planted_circle_is_found():
    inst = synth.tsp_circle(24)
    o = oracle.OracleInstance(inst)
    p = synth.Params(seed=7, population=8, generations=600, candidates=64,
                     alpha_q32=synth.alpha_q32_for(600))
    st = o.solve(p)
    assert oracle.best_of(st)[0] == o.objective(np.arange(24))


@pytest.mark.parametrize("kind", ["knap", "color"])
def test_segment_ops_keep_encoding_and_shape(kind):
    n = 12
    inst = (synth.knapsack_random(n, 0) if kind == "knap"
            else synth.Instance(synth.INTCOLOR, n, np.array([[0, 1]]), lb=-2, ub=3, n_edges=1))
    o = oracle.OracleInstance(inst)
    op = synth.OP_SEGFLIP if kind == "knap" else synth.OP_SEGRESET
    r = np.random.default_rng(3)
    for _ in range(300):
        x = (r.integers(0, 2, n) if kind == "knap" else r.integers(-2, 4, n)).astype(np.int32)
        w = [int(v) for v in r.integers(0, 2**32, 3, dtype=np.uint64)]
        y = o.apply_op(x, op, *w)
        L = min(2 + (w[2] * 6 >> 32), n)
        a = w[0] * (n - L + 1) >> 32
        changed = np.nonzero(x != y)[0]
        assert set(changed) <= set(range(a, a + L))
        if kind == "knap":
            assert list(changed) == list(range(a, a + L)) and set(y) <= {0, 1}
        else:
            assert len(set(y[a:a + L])) == 1 and -2 <= y.min() and y.max() <= 3
