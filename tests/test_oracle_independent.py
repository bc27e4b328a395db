"""Independent pins of oracle parts that GPU agreement alone would otherwise
fix: the Q16 roulette (exact counts from the closed form, and its use in a
run), one generation worked by hand from known-answer-pinned Philox words
(the k / operator bit fields, positions, the argmin tie to the lowest
candidate, the acceptance draw), Fisher-Yates random starts (hand trace and
uniformity), TSP optima by Held-Karp dynamic programming, the VRPTW split
against an evaluation written here route by route, and the device's float
distance path modelled with a one-ulp square root over every rounding
boundary."""
import itertools
import math

import numpy as np
import pytest

import oracle
import synth


# ------------------------------------------------------------------ roulette
def _roulette_counts(w):
    """How many of the 65536 16-bit draws pick each index: u = floor(u16 S / 2^16)
    lies below the cumulative sum c exactly when u16 < c 2^16 / S, i.e. for
    ceil(c 2^16 / S) values of u16."""
    w = [int(x) for x in w]
    S = sum(w)
    c = np.cumsum([0] + w)
    below = [-(-int(x) * 65536 // S) for x in c]
    return [below[i + 1] - below[i] for i in range(len(w))]


@pytest.mark.parametrize("w", [[23405, 23405, 18726], [52429, 9830, 3277], [1, 65534, 1],
                               [19859, 19859, 19859, 5957], [7, 3, 11, 2], [65536], [1, 1]])
def test_roulette_exhaustive_counts(w):
    got = [0] * len(w)
    for u16 in range(65536):
        got[oracle.wpick(u16, w)] += 1
    assert got == _roulette_counts(w)
    if sum(w) == 65536:          # normalised weights: each index gets exactly w_i draws
        assert got == list(w)


def test_roulette_frequencies_in_a_run():
    # weights frozen (the first AOS update lies beyond the run): the operator
    # and k counts of the run follow the roulette's exact probabilities
    inst = synth.tsp_uniform(50, 8)
    o = oracle.OracleInstance(inst)
    p = synth.Params(seed=5, population=8, candidates=128, generations=60, epoch=1000,
                     alpha_q32=synth.alpha_q32_for(60))
    st = o.solve(p)
    w_op = list(o.initial_weights(0)[:5])
    for counts, w in ((st["u_op"][:5], w_op), (st["u_k"], [52429, 9830, 3277])):
        n = int(sum(counts))
        prob = np.array(_roulette_counts(w)) / 65536
        chi2 = float((((np.asarray(counts, float) - n * prob) ** 2) / (n * prob)).sum())
        assert chi2 < 20, (counts, w, chi2)     # 2-3 degrees of freedom


# ------------------------------------------------------------------ one generation by hand
def _rmap(w, m):
    return (int(w) * m) >> 32


def _tour_len(D, x):
    return int(sum(D[x[i], x[(i + 1) % len(x)]] for i in range(len(x))))


def _hand_generation(o, D, x, f, p, w_op, w_k, T, key):
    """One generation of one solution (P = 1, g = 0) traced from the Philox
    words: k from bits 31..16 of word 0 of block (g, sol, 4t, key), the
    operator of step m from bits 15..0 of word 0 of block (g, sol, 4t + m, key)
    and its positions from words 1..3; the lowest delta wins, ties to the
    lowest t; a worse move is accepted when word 0 of block
    (g, sol, 2^32 - 1, key), shifted right by one, is below the threshold."""
    seed = [p.seed & 0xFFFFFFFF, p.seed >> 32]
    ids = [i for i in range(len(w_op)) if w_op[i]]
    wl = [w_op[i] for i in ids]
    cands = []
    for t in range(p.candidates):
        y = np.array(x, np.int32)
        r = oracle.philox([0, 0, 4 * t, key], seed)
        k = 1 + oracle.wpick(int(r[0]) >> 16, w_k)
        ops = []
        for m in range(k):
            if m:
                r = oracle.philox([0, 0, 4 * t + m, key], seed)
            op = ids[oracle.wpick(int(r[0]) & 0xFFFF, wl)]
            y = o.apply_op(y, op, int(r[1]), int(r[2]), int(r[3]))
            ops.append(op)
        cands.append((_tour_len(D, y) - f, t, k, ops, y))
    best = min(cands, key=lambda c: (c[0], c[1]))
    d = best[0]
    if d <= 0:
        acc = True
    else:
        thr, rej = oracle.accept_threshold(d, T)
        draw = int(oracle.philox([0, 0, 0xFFFFFFFF, key], seed)[0]) >> 1
        acc = (not rej) and draw < thr
    return cands, best, acc


def test_one_generation_with_planted_tie():
    # every tour of the all-ones matrix has length 6: all deltas are 0 and the
    # lowest candidate index must win
    n = 6
    D = np.ones((n, n), np.int32) - np.eye(n, dtype=np.int32)
    inst = synth.tsp_matrix(D, key=21)
    o = oracle.OracleInstance(inst)
    for seed in range(40):
        p = synth.Params(seed=seed, population=1, candidates=3, generations=1, op_mask=synth.PERM_OPS,
                         alpha_q32=2**31)
        st = o.init(p)
        x, f = st["cur"][0].copy(), int(st["cur_f"][0])
        cands, best, acc = _hand_generation(o, D, x, f, p, list(st["w_op"]), list(st["w_k"]),
                                            st["T_q16"], 21)
        if len({tuple(c[4]) for c in cands}) < 3:
            continue                                  # need three distinct candidate tours
        assert best[1] == 0 and acc
        o.run(p, st, 1)
        assert list(st["cur"][0]) == list(cands[0][4])
        # every candidate credits its operators and its k (reading R1); none improves
        want_u = np.zeros(len(st["u_op"]), np.int64)
        for c in cands:
            for op in c[3]:
                want_u[op] += 1
        assert list(st["u_op"]) == list(want_u) and int(st["v_op"].sum()) == 0
        assert list(st["u_k"]) == [sum(1 for c in cands if c[2] == kk) for kk in (1, 2, 3)]
        return
    pytest.fail("no seed gave three distinct candidates")


def test_one_generation_acceptance_draw():
    n = 6
    r = np.random.default_rng(4)
    A = r.integers(50, 500, (n, n))
    D = ((A + A.T) // 2).astype(np.int32)
    np.fill_diagonal(D, 0)
    inst = synth.tsp_matrix(D, key=5)
    o = oracle.OracleInstance(inst)
    outcomes = {"improve": 0, "worse_acc": 0, "worse_rej": 0}
    for seed in range(200):
        p = synth.Params(seed=seed, population=1, candidates=1, generations=1, op_mask=synth.PERM_OPS,
                         t0_q16=300 << 16, alpha_q32=2**31)
        st = o.init(p)
        x, f = st["cur"][0].copy(), int(st["cur_f"][0])
        cands, best, acc = _hand_generation(o, D, x, f, p, list(st["w_op"]), list(st["w_k"]),
                                            st["T_q16"], 5)
        o.run(p, st, 1)
        assert int(st["cur_f"][0]) == (f + best[0] if acc else f)
        assert list(st["cur"][0]) == list(best[4] if acc else x)
        assert st["accepted"] == int(acc)
        outcomes["improve" if best[0] <= 0 else ("worse_acc" if acc else "worse_rej")] += 1
    assert min(outcomes.values()) >= 10, outcomes


# ------------------------------------------------------------------ random starts
def test_fisher_yates_hand_trace():
    inst = synth.tsp_uniform(6, 1, key=33)
    o = oracle.OracleInstance(inst)
    p = synth.Params(seed=0x1234567890ABCDEF)
    seed = [p.seed & 0xFFFFFFFF, p.seed >> 32]
    for q in (4, 5, 77, 2**20 + 3):
        x = list(range(6))
        for i in range(5, 0, -1):
            w = oracle.philox([0xFFFFFFFF, q, i >> 2, 33], seed)[i & 3]
            j = _rmap(w, i + 1)
            x[i], x[j] = x[j], x[i]
        assert list(o.random_solution(p, q)) == x
    kn = oracle.OracleInstance(synth.knapsack_random(9, 0, key=34))
    bits = [int(oracle.philox([0xFFFFFFFF, 7, i >> 2, 34], seed)[i & 3]) >> 31 for i in range(9)]
    assert list(kn.random_solution(p, 7)) == bits
    col = synth.Instance(synth.INTCOLOR, 5, np.array([[0, 1]]), lb=-3, ub=4, n_edges=1, key=35)
    vals = [-3 + _rmap(oracle.philox([0xFFFFFFFF, 9, i >> 2, 35], seed)[i & 3], 8) for i in range(5)]
    assert list(oracle.OracleInstance(col).random_solution(p, 9)) == vals


@pytest.mark.parametrize("n", [3, 4])
def test_fisher_yates_uniform(n):
    o = oracle.OracleInstance(synth.tsp_uniform(n, 2, key=3))
    p = synth.Params(seed=99)
    perms = {pp: i for i, pp in enumerate(itertools.permutations(range(n)))}
    m = 24000
    counts = np.zeros(len(perms))
    for q in range(m):
        counts[perms[tuple(o.random_solution(p, q))]] += 1
    exp = m / len(perms)
    chi2 = float(((counts - exp) ** 2 / exp).sum())
    assert chi2 < (25 if n == 3 else 55), chi2      # 5 / 23 degrees of freedom, far tail


# ------------------------------------------------------------------ TSP optima by Held-Karp
def _held_karp(D):
    """Textbook dynamic programme over subsets (Held and Karp, 1962): optimal
    closed tour length and one optimal tour starting at city 0."""
    n = len(D)
    if n <= 3:
        t = list(range(n))
        return _tour_len(D, t), t
    m = n - 1                                   # cities 1..n-1 as bits 0..m-1
    INF = np.iinfo(np.int64).max // 4
    dp = np.full((1 << m, m), INF, np.int64)
    par = np.full((1 << m, m), -1, np.int64)
    for j in range(m):
        dp[1 << j, j] = D[0, j + 1]
    Dm = D[1:, 1:].astype(np.int64)
    for mask in range(1, 1 << m):
        for j in range(m):
            if not (mask >> j) & 1 or mask == (1 << j):
                continue
            prev = mask ^ (1 << j)
            cand = dp[prev] + Dm[:, j]
            cand[[i for i in range(m) if not (prev >> i) & 1]] = INF
            i = int(np.argmin(cand))
            dp[mask, j], par[mask, j] = cand[i], i
    full = (1 << m) - 1
    tot = dp[full] + D[1:, 0]
    j = int(np.argmin(tot))
    best = int(tot[j])
    tour, mask = [], full
    while j >= 0:
        tour.append(j + 1)
        pj = int(par[mask, j])
        mask ^= 1 << j
        j = pj
    return best, [0] + tour[::-1]


def _dist_matrix(o, n):
    return np.array([[o.dist(i, j) for j in range(n)] for i in range(n)], np.int64)


def test_held_karp_agrees_with_brute_force_n8():
    inst = synth.tsp_uniform(8, 6)
    o = oracle.OracleInstance(inst)
    D = _dist_matrix(o, 8)
    best, tour = _held_karp(D)
    assert best == min(o.objective(np.array((0,) + pp)) for pp in itertools.permutations(range(1, 8)))
    assert o.objective(np.array(tour)) == best


@pytest.mark.parametrize("n", [10, 12, 13])
def test_circle_planted_optimum_by_held_karp(n):
    inst = synth.tsp_circle(n)
    o = oracle.OracleInstance(inst)
    best, tour = _held_karp(_dist_matrix(o, n))
    assert sorted(tour) == list(range(n))
    assert o.objective(np.array(tour)) == best == o.objective(np.arange(n))


@pytest.mark.parametrize("n", [11, 12])
def test_uniform_optimum_by_held_karp(n):
    inst = synth.tsp_uniform(n, 40 + n)
    o = oracle.OracleInstance(inst)
    best, tour = _held_karp(_dist_matrix(o, n))
    assert o.objective(np.array(tour)) == best
    r = np.random.default_rng(n)
    for _ in range(300):                       # no random tour beats the optimum
        assert o.objective(r.permutation(n)) >= best


# ------------------------------------------------------------------ VRPTW split by routes
def _vrptw_by_routes(xy, dem, ready, due, cap, veh, svc, hor, w, perm):
    """Evaluate a giant tour route by route: cut it greedily wherever the next
    customer's demand would overload the vehicle, then drive each route from
    the depot and back, waiting for windows to open and charging lateness."""
    def d(a, b):
        s = int((xy[a][0] - xy[b][0]) ** 2 + (xy[a][1] - xy[b][1]) ** 2)
        return (math.isqrt(4 * s) + 1) // 2
    routes, cur, load = [], [], 0
    for c in (int(v) + 1 for v in perm):
        if cur and load + dem[c] > cap:
            routes.append(cur)
            cur, load = [], 0
        cur.append(c)
        load += dem[c]
    if cur:
        routes.append(cur)
    dist = late = longest = 0
    for rt in routes:
        clock, length, here = 0, 0, 0
        for c in rt:
            clock += d(here, c)
            length += d(here, c)
            clock = max(clock, ready[c])
            late += max(0, clock - due[c])
            clock += svc
            here = c
        clock += d(here, 0)
        length += d(here, 0)
        late += max(0, clock - hor)
        dist += length
        longest = max(longest, length)
    f = w[0] * dist + w[1] * len(routes) + w[2] * longest + 100 * late + 10000 * max(0, len(routes) - veh)
    return f, len(routes), late


@pytest.mark.parametrize("weights", [(0, 0, 0), (3, 50, 2)])
def test_vrptw_brute_force_with_binding_capacity_and_windows(weights):
    r = np.random.default_rng(12)
    n = 8
    xy = r.integers(0, 101, (n + 1, 2))
    xy[0] = (50, 50)
    dem = np.concatenate([[0], r.integers(10, 31, n)])
    ready = np.concatenate([[0], r.integers(0, 120, n)])
    due = ready + np.concatenate([[400], r.integers(15, 60, n)])
    cap, veh, svc, hor = 60, 2, 10, 400
    inst = synth.Instance(synth.VRPTW, n, xy, np.stack([dem, ready, due]), capacity=cap, vehicles=veh,
                          service_time=svc, horizon=hor, obj_weights=weights)
    o = oracle.OracleInstance(inst)
    w = weights if any(weights) else (1, 0, 0)
    routes, lates = set(), set()
    for perm in itertools.permutations(range(n)):
        want, nr, late = _vrptw_by_routes(xy, dem, ready, due, cap, veh, svc, hor, w, perm)
        assert o.objective(np.array(perm)) == want, perm
        routes.add(nr)
        lates.add(late > 0)
    # capacity splits every tour into more routes than the fleet, in varying
    # numbers; some orders are late and some are not
    assert min(routes) > veh and len(routes) >= 2 and lates == {True, False}


# ------------------------------------------------------------------ device float distance model
def _ulp_neighbours(v):
    v = np.asarray(v, np.float32)
    return [np.nextafter(v, np.float32(-np.inf)), v, np.nextafter(v, np.float32(np.inf))]


def test_float_distance_path_exact_under_one_ulp_sqrt():
    """The device computes nint(sqrt(s)) as k0 + (s > k0 (k0 + 1)) with
    k0 = trunc(fma(sqrt(float(s)), 1 - 2^-19, 1/2)) in float32.  With
    float(s) rounded to nearest, a square root anywhere within one ulp of the
    correctly rounded one, and a correctly rounded fma, this equals the exact
    nearest integer at both sides of every rounding boundary k(k+1) (and of
    k^2 and k(k-1)) for every k the coordinate range reaches, and on random s."""
    k = np.arange(1, 23171, dtype=np.int64)
    ss = [k * (k + 1) + o for o in (-2, -1, 0, 1, 2)] + [k * k + o for o in (-1, 0, 1)] + \
         [k * (k - 1) + o for o in (0, 1)]
    ss.append(np.random.default_rng(6).integers(0, 2 * 16383**2 + 1, 2_000_000))
    s = np.unique(np.concatenate(ss))
    s = s[(s >= 0) & (s <= 2 * 16383**2)]
    want = np.floor(np.sqrt(s.astype(np.float64)) + 0.5).astype(np.int64)
    fs = s.astype(np.float32)                                  # round to nearest
    c = np.float64(np.float32(0.99999809265136719))
    for r in _ulp_neighbours(np.sqrt(fs)):
        y = (r.astype(np.float64) * c + 0.5).astype(np.float32)   # exact product + 1/2, one rounding
        k0 = np.floor(y).astype(np.int64)
        got = k0 + (s > k0 * k0 + k0)
        bad = np.nonzero(got != want)[0]
        assert len(bad) == 0, (s[bad[:5]], got[bad[:5]], want[bad[:5]])
