"""Device primitives against independent implementations, through the C
interface's gx_device_check: Philox4x32-10 in both device forms against the
oracle's block (itself pinned by published known-answer vectors) on a million
counters; the nearest-integer distance at every coordinate difference whose
squared norm lies within two of a rounding boundary k(k+1) (or of k^2),
against exact integer arithmetic; the acceptance threshold at every table
index z < 4096 and its boundaries, and for deltas up to 2^62, against Python
big integers and the exact-decimal tables.  Then a whole-run parity case
whose worse moves all have deltas above 2^40 (the range where a 64-bit
2^24 delta numerator would wrap)."""
import math
import os

import numpy as np
import pytest

import oracle
import synth
from paper_2603_19163_amd import gx

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def ctx():
    c = gx.gx_create(0)
    yield c
    gx.gx_destroy(c)


def test_philox_both_forms_on_a_million_counters(ctx):
    rng = np.random.default_rng(20260319)
    m = 1 << 20
    ctr = rng.integers(0, 2**32, (m, 4), dtype=np.uint64).astype(np.uint32)
    # the counter layout of the candidate draws for part of them: (g, sol, 4t + slot, key)
    ctr[: m // 2, 0] = np.arange(m // 2) // 4096
    ctr[: m // 2, 1] = (np.arange(m // 2) // 512) % 8
    ctr[: m // 2, 2] = np.arange(m // 2) % 512
    ctr[m // 4: m // 4 + 16, 2] = 0xFFFFFFFF          # the acceptance-draw slot
    for key in (0, 42, 0xFFFFFFFFFFFFFFFF, 0x0123456789ABCDEF):
        k = (key & 0xFFFFFFFF, key >> 32)
        want = oracle.philox_many(ctr, k)
        words = ctr.astype(np.uint64)
        packed = np.stack([words[:, 0] | words[:, 1] << np.uint64(32), words[:, 2] | words[:, 3] << np.uint64(32)], 1)
        out = gx.gx_device_check(ctx, gx.GX_CHECK_PHILOX, packed, key)
        for form in (0, 1):
            got = np.stack([out[:, 2 * form] & np.uint64(0xFFFFFFFF), out[:, 2 * form] >> np.uint64(32),
                            out[:, 2 * form + 1] & np.uint64(0xFFFFFFFF), out[:, 2 * form + 1] >> np.uint64(32)],
                           1).astype(np.uint32)
            bad = np.nonzero((got != want).any(1))[0]
            assert len(bad) == 0, (hex(key), form, ctr[bad[:3]], got[bad[:3]], want[bad[:3]])


def _exact_nint(s):
    """nint(sqrt(s)) = (isqrt(4 s) + 1) >> 1, with an exact integer square root."""
    r = np.floor(np.sqrt(4.0 * s.astype(np.float64))).astype(np.int64)
    r -= (r * r > 4 * s)
    r += ((r + 1) * (r + 1) <= 4 * s)
    assert np.all(r * r <= 4 * s) and np.all((r + 1) * (r + 1) > 4 * s)
    return (r + 1) >> 1


def _near_boundary_differences():
    """Every (dx, dy) with 0 <= dx <= dy < 2^14 whose squared norm is within
    two of k(k+1) or of k^2 for k = floor(sqrt(s)) - 1 .. floor(sqrt(s)) + 1."""
    out = []
    dy = np.arange(16384, dtype=np.int64)[None, :]
    for x0 in range(0, 16384, 256):
        dx = np.arange(x0, x0 + 256, dtype=np.int64)[:, None]
        s = dx * dx + dy * dy
        k = np.floor(np.sqrt(s.astype(np.float64))).astype(np.int64)
        near = np.zeros(s.shape, bool)
        for kk in (k - 1, k, k + 1):
            near |= np.abs(s - kk * (kk + 1)) <= 2
            near |= np.abs(s - kk * kk) <= 2
        near &= dy >= dx
        i, j = np.nonzero(near)
        out.append(np.stack([i + x0, j], 1))
    return np.concatenate(out)


def test_distance_at_every_rounding_boundary(ctx):
    dd = _near_boundary_differences()
    rng = np.random.default_rng(5)
    dd = np.concatenate([dd, rng.integers(0, 16384, (200_000, 2))])
    # place the differences at coordinates, with both signs of each difference
    x0 = rng.integers(0, 16384, len(dd))
    y0 = rng.integers(0, 16384, len(dd))
    x1 = np.where(x0 + dd[:, 0] < 16384, x0, dd[:, 0])
    x2 = np.where(x0 + dd[:, 0] < 16384, x0 + dd[:, 0], 0)
    y1 = np.where(y0 + dd[:, 1] < 16384, y0 + dd[:, 1], 0)
    y2 = np.where(y0 + dd[:, 1] < 16384, y0, dd[:, 1])
    pts = np.stack([x1, y1, x2, y2], 1).astype(np.uint64)
    packed = pts[:, 0] | pts[:, 1] << np.uint64(16) | pts[:, 2] << np.uint64(32) | pts[:, 3] << np.uint64(48)
    out = gx.gx_device_check(ctx, gx.GX_CHECK_DIST, packed)
    s = (x1 - x2) ** 2 + (y1 - y2) ** 2
    want = _exact_nint(s.astype(np.int64))
    for path in (0, 1):
        bad = np.nonzero(out[:, path].astype(np.int64) != want)[0]
        assert len(bad) == 0, (path, pts[bad[:5]], out[bad[:5], path], want[bad[:5]])
    for i in rng.choice(len(pts), 2000, replace=False):    # the oracle's routine on a sample
        assert oracle.nint_dist(*[int(v) for v in pts[i]]) == int(want[i])
    print(f"[device checks] {len(pts)} coordinate pairs, {len(dd) - 200_000} near a rounding boundary", flush=True)


def _threshold(delta, t):
    """Threshold by Python big integers and the exact-decimal tables (None: reject)."""
    if t == 0:
        return None
    z = (delta << 24) // t
    if z >= 4096:
        return None
    hi, lo = _tables()
    return (hi[z >> 8] * lo[z & 255]) >> 31


_TAB = []


def _tables():
    if not _TAB:
        import re
        src = open(os.path.join(ROOT, "oracle", "exp_tables.h")).read()
        nums = [int(x) for x in re.findall(r"(\d+)u", src)]
        _TAB.extend([nums[:16], nums[16:]])
    return _TAB


def test_acceptance_threshold_every_index_and_wide_deltas(ctx):
    rng = np.random.default_rng(11)
    cases = []
    for z in range(1, 4097):                        # 2^24 d = z t exactly, and t one above and below
        m = int(rng.integers(1, 1 << 20))
        t, d = m << 24, z * m
        cases += [(d, t), (d, t + 1), (d, t - 1)]
    for e in range(1, 63):                          # deltas up to 2^62 against temperatures of every scale
        for _ in range(40):
            d = int(rng.integers(1, 1 << 62)) >> (62 - e)
            d = max(d, 1)
            t = int(rng.integers(1, 1 << 63)) >> int(rng.integers(0, 63))
            cases.append((d, max(t, 0)))
            cases.append((d, (d << 8) // max(1, int(rng.integers(1, 4200)))))   # z near the table range
    cases += [(2**39, 2**16), (2**40 + 5, 2**16), (2**44, 2**16), (2**39, 2**62), (2**40 + 5, 2**62),
              (2**44, 2**62), (2**41, 2**62), (1, 0), (2**62, 2**64 - 1), (2**52 - 1, 2**64 - 1), (2**52, 2**64 - 1)]
    cases = [(d, t) for d, t in cases if 0 < d < 2**63 and 0 <= t < 2**64]
    inp = np.array(cases, dtype=np.uint64)
    out = gx.gx_device_check(ctx, gx.GX_CHECK_ACCEPT, inp)[:, 0]
    for (d, t), got in zip(cases, out):
        want = _threshold(d, t)
        assert int(got) == (2**64 - 1 if want is None else want), (d, t, int(got), want)
        thr, rej = oracle.accept_threshold(d, t)
        assert (None if rej else thr) == want, (d, t)
    print(f"[device checks] {len(cases)} acceptance cases", flush=True)


def test_wide_delta_run_parity(ctx):
    """0/1 knapsack with capacity 0, every weight 2^20 and values up to 2^20:
    the empty set is optimal and every move from it costs 2^40 + 2^20 - v,
    so from the moment a solution empties, each generation's decision is an
    acceptance test on a delta above 2^40 (T0 puts delta / T near 1..10)."""
    n = 7
    w = np.full(n, 1 << 20, np.int32)
    v = np.array([1 << 20, 3, 77, 1 << 19, 12345, 999_999, 1], np.int32)
    inst = synth.Instance(synth.KNAPSACK, n, w, v, capacity=0, key=41)
    G = 120
    p = synth.Params(seed=2024, generations=G, population=8, candidates=64, alpha_q32=synth.alpha_q32_for(G),
                     t0_q16=(1 << 40) << 14)     # T = 2^38 at the start
    h = gx.gx_instance_upload(ctx, inst)
    job = gx.gx_job_create(ctx, h, p)
    o = oracle.OracleInstance(inst)
    st = o.init(p)
    keys = ["g", "stag", "T_q16", "epoch_ref", "accepted", "w_op", "w_k", "u_op", "v_op", "u_k", "v_k",
            "cur", "cur_f", "best", "best_f"]
    for step in (20, 40, 60):
        gx.gx_job_advance(ctx, job, step)
        o.run(p, st, step)
        g = gx.gx_snapshot(ctx, job, p.population, n)
        for k in keys:
            assert np.array_equal(np.asarray(g[k]), np.asarray(st[k])), (step, k, g[k], st[k])
    # the run really took decisions on wide deltas: accepted worse moves from the empty set
    assert st["accepted"] > 0 and int(st["best_f"].min()) == 0
    gx.gx_job_free(ctx, job)
    gx.gx_instance_free(ctx, h)
