"""Oracle pins for the LNS operators (paper, Sec. "Built-in Operator
Hierarchy": segment shuffle, scatter shuffle and guided rebuild, the destroyed
part following the problem size; Tab. weight_preset: the LNS weight and the
LNS cap by scale).

- Each operator recomputed here from its stated reading, with the extra
  draws taken from the Philox4x32-10 function that the known-answer vectors
  pin, a Fisher-Yates, Floyd's sampling and a sort written in this file.
- Distributions: a segment shuffle is a uniform permutation of its segment,
  the scattered positions a uniform subset, guided rebuilds sorted by the
  heuristic key in the drawn direction.
- Presets and the cap of the EMA clamp worked by hand; the LNS operators
  are opt-in, belong to the single-row permutations only, and keep runs
  valid (threaded runner equal to the plain one)."""
from collections import Counter

import numpy as np
import pytest

import oracle
import synth

KEY = (0x4C4E5331, 0x4C4E5332)


def rmap(w, m):
    return (int(w) * m) >> 32


def word(w1, w2, w3, i):
    return int(oracle.philox([w1, w2, w3, i >> 2], KEY)[i & 3])


def L_of(n):
    return min(n, 2 + n // 16, 64)


def fisher_yates(vals, w, base):
    v = list(vals)
    L = len(v)
    for i in range(L - 1, 0, -1):
        j = rmap(word(*w, base + L - 1 - i), i + 1)
        v[i], v[j] = v[j], v[i]
    return v


def floyd(n, L, w):
    s = []
    for j in range(n - L, n):
        r = rmap(word(*w, j - n + L), j + 1)
        s.append(j if r in s else r)
    return sorted(s)


def hkey(inst, o):
    n = inst.n
    if inst.kind == synth.TSP:
        return [sum(o.dist(i, j) for j in range(n)) for i in range(n)]
    if inst.kind == synth.QAP:
        return [int(inst.a[i].sum()) for i in range(n)]
    return [sum(o.dist(i + 1, j + 1) for j in range(n)) for i in range(n)]


def expected(inst, o, x, op, w):
    n = len(x)
    L = L_of(n)
    y = list(x)
    if L < 2:
        return y
    if op == synth.OP_LNS_SCATTER:
        pos = floyd(n, L, w)
    else:
        a = rmap(w[0], n - L + 1)
        pos = list(range(a, a + L))
    vals = [y[p] for p in pos]
    if op == synth.OP_LNS_GUIDED:
        k = hkey(inst, o)
        sign = -1 if (w[1] >> 31) else 1
        vals = sorted(vals, key=lambda e: (sign * k[e], e))
    else:
        vals = fisher_yates(vals, w, L if op == synth.OP_LNS_SCATTER else 0)
    for p, v in zip(pos, vals):
        y[p] = v
    return y


def test_destroyed_part_follows_the_size():
    for n, L in [(1, 1), (2, 2), (5, 2), (15, 2), (16, 3), (50, 5), (100, 8), (442, 29), (991, 63), (2000, 64)]:
        assert oracle.lns_len(n) == L == L_of(n)


INSTS = [synth.tsp_uniform(40, 3, key=5), synth.qap_random(33, 2, key=6), synth.vrptw_random(50, 4, key=7),
         synth.tsp_clustered(442, 1, key=8)]


@pytest.mark.parametrize("which", range(len(INSTS)))
@pytest.mark.parametrize("op", [synth.OP_LNS_SEG, synth.OP_LNS_SCATTER, synth.OP_LNS_GUIDED])
def test_operators_recomputed_here(which, op):
    inst = INSTS[which]
    o = oracle.OracleInstance(inst)
    rng = np.random.default_rng(100 + op + 10 * which)
    for _ in range(12):
        x = rng.permutation(inst.n).astype(np.int32)
        w = [int(v) for v in rng.integers(0, 2**32, size=3)]
        assert list(o.apply_op(x, op, *w)) == expected(inst, o, x, op, w)


def test_segment_shuffle_is_uniform():
    inst = synth.tsp_uniform(48, 1, key=9)          # L = 5
    o = oracle.OracleInstance(inst)
    x = np.arange(48, dtype=np.int32)
    rng = np.random.default_rng(1)
    seen = Counter()
    N = 24000
    for _ in range(N):
        w = [0] + [int(v) for v in rng.integers(0, 2**32, size=2)]     # a = 0
        seen[tuple(o.apply_op(x, synth.OP_LNS_SEG, *w)[:5])] += 1
    assert len(seen) == 120
    chi2 = sum((c - N / 120) ** 2 / (N / 120) for c in seen.values())
    assert chi2 < 180          # 119 degrees of freedom, p ~ 3e-4


def test_scatter_positions_are_a_uniform_subset():
    inst = synth.tsp_uniform(8, 1, key=10)          # L = 2
    o = oracle.OracleInstance(inst)
    x = np.arange(8, dtype=np.int32)
    rng = np.random.default_rng(2)
    seen = Counter()
    N = 14000
    for _ in range(N):
        w = [int(v) for v in rng.integers(0, 2**32, size=3)]
        y = o.apply_op(x, synth.OP_LNS_SCATTER, *w)
        moved = tuple(sorted(int(p) for p in np.flatnonzero(y != x)))
        if moved:
            seen[moved] += 1
        # with two positions the shuffle swaps them or keeps them: either way a subset of size 0 or 2
        assert len(moved) in (0, 2)
    assert len(seen) == 28
    chi2 = sum((c - sum(seen.values()) / 28) ** 2 / (sum(seen.values()) / 28) for c in seen.values())
    assert chi2 < 60           # 27 degrees of freedom


def test_guided_rebuild_orders_by_the_heuristic_key():
    inst = synth.tsp_uniform(64, 4, key=11)
    o = oracle.OracleInstance(inst)
    k = hkey(inst, o)
    rng = np.random.default_rng(3)
    L = L_of(64)
    for desc in (0, 1):
        x = rng.permutation(64).astype(np.int32)
        w = [int(rng.integers(0, 2**32)), (desc << 31) | 12345, 777]
        y = o.apply_op(x, synth.OP_LNS_GUIDED, *w)
        a = rmap(w[0], 64 - L + 1)
        seg = [int(v) for v in y[a:a + L]]
        assert sorted(seg) == sorted(int(v) for v in x[a:a + L])
        keys = [k[e] for e in seg]
        assert keys == sorted(keys, reverse=bool(desc))
        assert np.array_equal(np.delete(y, range(a, a + L)), np.delete(x, range(a, a + L)))


def test_presets_caps_and_masks():
    small, mid, big = synth.tsp_uniform(90, 1), synth.tsp_uniform(200, 1), synth.tsp_uniform(300, 1)
    for inst, lns, cap in ((small, 393, 1311), (mid, 262, 655), (big, 66, 328)):
        o = oracle.OracleInstance(inst)
        assert o.lns_cap() == cap
        n = inst.n
        raw = [65536, 65536, 65536, 52429 if n <= 100 else (45875 if n <= 250 else 19661),
               32768 if n <= 100 else (19661 if n <= 250 else 3277), lns, lns, lns]
        s = sum(raw)
        w = o.initial_weights(synth.PERM_LNS_OPS)
        assert list(w[:8]) == [max(1, (r << 16) // s) for r in raw]
    o = oracle.OracleInstance(small)
    assert o.effective_mask(0) == synth.PERM_OPS                 # opt-in
    assert o.effective_mask(synth.PERM_LNS_OPS) == synth.PERM_LNS_OPS
    kn = oracle.OracleInstance(synth.knapsack_random(20, 1))
    assert kn.effective_mask(synth.LNS_OPS) == 0 and kn.lns_cap() == 0
    rows = oracle.OracleInstance(synth.vrptw_rows(12, 1, vehicles=3))
    assert rows.lns_cap() == 0                                   # ids 5-7 are the row operators there


def test_ema_clamp_caps_lns_weights():
    inst = synth.tsp_uniform(90, 2)                 # cap 0.02 (1311), floor 1024
    o = oracle.OracleInstance(inst)
    p = synth.Params(seed=1, generations=10, population=2, candidates=8, op_mask=synth.PERM_LNS_OPS,
                     alpha_q32=synth.alpha_q32_for(10))
    st = o.init(p)
    st["w_op"][:] = 0
    st["w_op"][:8] = [20000, 20000, 10000, 5000, 5000, 393, 393, 393]
    st["u_op"][:] = 0
    st["v_op"][:] = 0
    st["u_op"][:8] = [100, 100, 100, 100, 100, 10, 10, 10]
    st["v_op"][:8] = [10, 0, 50, 0, 0, 9, 0, 1]
    w0, u0, v0 = st["w_op"].copy(), st["u_op"].copy(), st["v_op"].copy()
    out = o.aos_update(p, st, st["epoch_ref"], op_mask=synth.PERM_LNS_OPS)
    A, FL = 49152, 1024
    raw = []
    for i in range(8):
        r = (int(v0[i]) << 16) // (int(u0[i]) + 1)
        nw = (A * int(w0[i]) + (65536 - A) * (r + FL)) >> 16
        lo, hi = (min(FL, 1311), 1311) if i >= 5 else (FL, 65536)
        raw.append(min(max(nw, lo), hi))
    s = sum(raw)
    assert list(out["w_op"][:8]) == [max(1, (r << 16) // s) for r in raw]
    assert raw[5] == 1311 and raw[6] == 1024            # capped above, floored below


@pytest.mark.parametrize("which", [0, 1, 2])
def test_runs_with_lns_stay_valid(which):
    inst = INSTS[which]
    o = oracle.OracleInstance(inst)
    p = synth.Params(seed=5, generations=40, population=5, candidates=32, op_mask=synth.PERM_LNS_OPS,
                     alpha_q32=synth.alpha_q32_for(40), init_weight_q16=[0, 0, 0, 0, 0, 8000, 8000, 8000])
    st = o.init(p)
    a = o.run(p, {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in st.items()}, 40)
    b = o.run(p, {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in st.items()}, 40, threads=3)
    for key in ("cur", "best", "cur_f", "best_f", "w_op", "tot_u_op"):
        assert np.array_equal(a[key], b[key]), key
    for s in range(p.population):
        assert sorted(a["cur"][s]) == list(range(inst.n))
        assert a["cur_f"][s] == o.objective(a["cur"][s]) and a["best_f"][s] == o.objective(a["best"][s])
    assert int(a["tot_u_op"][5:8].sum()) > 0


def test_per_sequence_caps_by_hand():
    """Caller caps (Sec. "Two-Level Weight Structure": the clamp is [w_floor,
    min(w_cap, cap_i)]): a cap above the floor bounds the weight, a cap below
    it pins the weight to the cap, 0 keeps the default (1.0, or the LNS cap)."""
    inst = synth.tsp_uniform(90, 5)
    o = oracle.OracleInstance(inst)
    caps = [20000, 500, 0, 0, 0, 0, 900, 0]
    p = synth.Params(seed=1, generations=10, population=2, candidates=8, op_mask=synth.PERM_LNS_OPS,
                     alpha_q32=synth.alpha_q32_for(10), weight_cap_q16=caps)
    st = o.init(p)
    st["w_op"][:] = 0
    st["w_op"][:8] = [30000, 20000, 10000, 5000, 5000, 393, 393, 393]
    st["u_op"][:] = 0
    st["v_op"][:] = 0
    st["u_op"][:8] = [100, 100, 100, 100, 100, 10, 10, 10]
    st["v_op"][:8] = [90, 30, 50, 0, 0, 9, 5, 1]
    w0, u0, v0 = st["w_op"].copy(), st["u_op"].copy(), st["v_op"].copy()
    out = o.aos_update(p, st, st["epoch_ref"], op_mask=synth.PERM_LNS_OPS)
    A, FL = 49152, 1024
    raw = []
    for i in range(8):
        r = (int(v0[i]) << 16) // (int(u0[i]) + 1)
        nw = (A * int(w0[i]) + (65536 - A) * (r + FL)) >> 16
        hi = caps[i] or (1311 if i >= 5 else 65536)
        raw.append(min(max(nw, min(FL, hi)), hi))
    s = sum(raw)
    assert list(out["w_op"][:8]) == [max(1, (r << 16) // s) for r in raw]
    assert raw[0] == 20000 and raw[1] == 500 and raw[6] == 900 and raw[5] == 1311
