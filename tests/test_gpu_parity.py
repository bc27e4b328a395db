"""Parity of the HIP engine with the CPU oracle, element by element and bit for
bit: initial populations, whole trajectories (every state field: solutions,
objectives, best-so-far, weights, statistics, temperature, stagnation, accept
count), every problem kind and TSP staging, ragged candidate counts, edge
sizes, and a windowed check at the full 442-city configuration the benchmark
times.  Every call goes through the C interface (libgx.so)."""
import numpy as np
import pytest

import oracle
import synth
from paper_2603_19163_amd import gx

pytestmark = pytest.mark.gpu

KEYS = ["g", "stag", "T_q16", "epoch_ref", "accepted", "w_op", "w_k", "u_op", "v_op", "u_k", "v_k",
        "cur", "cur_f", "best", "best_f"]


@pytest.fixture(scope="module")
def ctx():
    c = gx.gx_create(0)
    yield c
    gx.gx_destroy(c)


def assert_same(g, o, what=""):
    for k in KEYS:
        a, b = np.asarray(g[k]), np.asarray(o[k])
        if not np.array_equal(a, b):
            bad = np.argwhere(a != b)[:5] if a.shape == b.shape else "shape"
            raise AssertionError(f"{what}: state field {k} differs at {bad}: gpu {a.ravel()[:8]} oracle {b.ravel()[:8]}")


def gpu_states(ctx, inst, p, splits):
    """GPU job: snapshot after init and after each advance in `splits`."""
    h = gx.gx_instance_upload(ctx, inst)
    job = gx.gx_job_create(ctx, h, p)
    out = [gx.gx_snapshot(ctx, job, p.population, inst.n)]
    for s in splits:
        gx.gx_job_advance(ctx, job, s)
        out.append(gx.gx_snapshot(ctx, job, p.population, inst.n))
    sol, f = gx.gx_fetch_best(ctx, job, inst.n)
    out[-1]["stats"] = gx.gx_job_stats(ctx, job)
    gx.gx_job_free(ctx, job)
    gx.gx_instance_free(ctx, h)
    return out, (sol, f)


def oracle_states(inst, p, splits):
    o = oracle.OracleInstance(inst)
    st = o.init(p)
    out = [{k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in st.items()}]
    for s in splits:
        o.run(p, st, s)
        out.append({k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in st.items()})
    return out


def check(ctx, inst, p, splits, what):
    print(f"[parity] {what} n={inst.n} P={p.population} C={p.candidates} splits={splits}", flush=True)
    gs, (sol, f) = gpu_states(ctx, inst, p, splits)
    os_ = oracle_states(inst, p, splits)
    for i, (g, o) in enumerate(zip(gs, os_)):
        assert_same(g, o, f"{what} snapshot {i}")
    stats = gs[-1]["stats"]
    for gk, ok in (("u_op", "tot_u_op"), ("v_op", "tot_v_op"), ("u_k", "tot_u_k"), ("v_k", "tot_v_k")):
        assert np.array_equal(stats[gk], os_[-1][ok]), f"{what}: run total {gk}"
    fo, io = oracle.best_of(os_[-1])
    assert f == fo and np.array_equal(sol, os_[-1]["best"][io])


def P(**kw):
    G = kw.pop("G", 25)
    kw.setdefault("alpha_q32", synth.alpha_q32_for(max(G, 1)))
    return synth.Params(generations=G, **kw)


SMALL = {
    "tsp": lambda: synth.tsp_uniform(17, 2, key=11),
    "qap": lambda: synth.qap_random(11, 2, key=12),
    "knap": lambda: synth.knapsack_random(33, 2, key=13),
    "vrptw": lambda: synth.vrptw_random(12, 2, key=14),
    "color": lambda: synth.color_planted(15, 3, key=15),
}


@pytest.mark.parametrize("kind", list(SMALL))
def test_small_trajectory_parity(ctx, kind):
    inst = SMALL[kind]()
    p = P(seed=42, population=6, candidates=100, G=25)     # 100 = one full round + a ragged one
    check(ctx, inst, p, [7, 3, 15], kind)


@pytest.mark.parametrize("staging", [1, 2, 3, 4])
def test_tsp_staging_modes_agree_with_oracle(ctx, staging):
    inst = synth.tsp_clustered(60, 1, key=5)
    p = P(seed=123, population=5, candidates=128, G=30, op_mask=synth.PERM_OPS, staging=staging)
    check(ctx, inst, p, [30], f"tsp staging {staging}")


def test_tsp_distance_matrix_input(ctx):
    o = oracle.OracleInstance(synth.tsp_uniform(23, 9))
    D = np.array([[o.dist(i, j) for j in range(23)] for i in range(23)], np.int32)
    inst = synth.tsp_matrix(D, key=77)
    check(ctx, inst, P(seed=5, population=4, candidates=64, G=20), [20], "tsp matrix")


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_tiny_permutations(ctx, n):
    for inst in (synth.tsp_uniform(n, 1, key=n), synth.qap_random(n, 1, key=n)):
        check(ctx, inst, P(seed=7, population=3, candidates=65, G=12), [12], f"tiny perm kind {inst.kind}")


def test_tiny_other_encodings(ctx):
    check(ctx, synth.knapsack_random(1, 0, key=1), P(seed=3, population=2, candidates=3, G=11), [11], "knap n=1")
    check(ctx, synth.vrptw_random(2, 0, key=2), P(seed=3, population=2, candidates=64, G=11), [11], "vrptw n=2")
    e = synth.Instance(synth.INTCOLOR, 2, np.array([[0, 1]]), lb=0, ub=1, n_edges=1, key=4)
    check(ctx, e, P(seed=3, population=2, candidates=64, G=11), [11], "color n=2")


def test_single_candidate_single_solution(ctx):
    check(ctx, synth.tsp_uniform(30, 4, key=2), P(seed=9, population=1, candidates=1, G=40), [40], "P=C=1")


def test_accepted_only_credit(ctx):
    check(ctx, synth.qap_random(14, 3, key=8), P(seed=11, population=4, candidates=64, G=30, credit=1),
          [30], "credit=1")


def _qap_wide(n, seed):
    """QAP with entries up to 2^14 - 1 and non-zero diagonals: the delta sums
    leave int32, so the 64-bit accumulation path runs."""
    r = np.random.default_rng([seed, n, 20260319])
    F = r.integers(0, 16384, (n, n))
    D = r.integers(0, 16384, (n, n))
    F = np.triu(F) + np.triu(F, 1).T
    D = np.triu(D) + np.triu(D, 1).T
    return synth.Instance(synth.QAP, n, F, D, key=seed)


def test_qap_wide_values(ctx):
    check(ctx, _qap_wide(21, 3), P(seed=6, population=4, candidates=128, G=30, op_mask=synth.PERM_OPS),
          [10, 20], "qap wide values")


def test_qap_medium_values(ctx):
    # n max F max D above 2^16 but 2 n max F max D below 2^31: 32-bit row sums H
    r = np.random.default_rng([7, 25, 20260319])
    F = r.integers(0, 1000, (25, 25))
    D = r.integers(0, 1000, (25, 25))
    inst = synth.Instance(synth.QAP, 25, np.triu(F) + np.triu(F, 1).T, np.triu(D) + np.triu(D, 1).T, key=31)
    check(ctx, inst, P(seed=9, population=4, candidates=128, G=30, op_mask=synth.PERM_OPS), [15, 15], "qap medium values")


def test_qap_long_moves_in_windows(ctx):
    # reversals and block moves on a short permutation change most positions:
    # a round's entries exceed the 24n list and are evaluated in several windows
    ops = (1 << synth.OP_2OPT) | (1 << synth.OP_OROPT)
    check(ctx, synth.qap_random(9, 4, key=9), P(seed=3, population=3, candidates=200, G=20, op_mask=ops), [20],
          "qap windows")


@pytest.mark.parametrize("n", [37, 48])
def test_qap_ragged_rows(ctx, n):
    # rows padded to a multiple of 8 (37 -> 40) and an exact multiple (48)
    check(ctx, synth.qap_random(n, 5, key=n), P(seed=n, population=3, candidates=128, G=25, op_mask=synth.PERM_OPS),
          [25], f"qap n={n}")


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_island_migration_and_elite_injection(ctx, mode):
    # migrations every epoch (hybrid alternates), elite injection every second
    p = P(seed=17, population=12, candidates=64, G=60, islands=4, migrate_epochs=1, migrate_mode=mode,
          migrate_n=2, elite_epochs=2)
    check(ctx, synth.tsp_uniform(25, 6, key=21), p, [20, 20, 20], f"islands mode {mode}")


@pytest.mark.parametrize("islands,mode,mig_n", [(32, 0, 1), (20, 1, 2), (24, 2, 1)])
def test_more_islands_than_epoch_waves(ctx, islands, mode, mig_n):
    # more islands than the 16 waves of the epoch kernel's workgroup: each
    # wave chooses for several islands; migrations and elite injection every epoch
    P_ = islands * (2 if islands == 32 else 3)
    p = P(seed=37, population=P_, candidates=64, G=30, islands=islands, migrate_epochs=1, migrate_mode=mode,
          migrate_n=mig_n, elite_epochs=1)
    check(ctx, synth.tsp_uniform(21, 9, key=25), p, [10, 20], f"{islands} islands mode {mode}")


def test_islands_on_two_wave_qap(ctx):
    p = P(seed=19, population=8, candidates=128, G=40, islands=2, migrate_epochs=1, migrate_mode=1,
          migrate_n=2, elite_epochs=1, op_mask=synth.PERM_OPS)
    check(ctx, synth.qap_random(16, 7, key=23), p, [20, 20], "qap islands")


@pytest.mark.parametrize("mask", ["segment", "both"])
def test_segment_operators(ctx, mask):
    # seg_flip / seg_reset alone and with the element operators, composite
    # moves of up to three overlapping segments
    kmask = (1 << synth.OP_SEGFLIP) | ((1 << synth.OP_FLIP) if mask == "both" else 0)
    cmask = (1 << synth.OP_SEGRESET) | ((1 << synth.OP_RESET) if mask == "both" else 0)
    check(ctx, synth.knapsack_random(40, 4, key=31), P(seed=23, population=4, candidates=128, G=30, op_mask=kmask),
          [15, 15], f"knapsack {mask}")
    check(ctx, synth.color_planted(24, 3, key=33), P(seed=29, population=4, candidates=128, G=30, op_mask=cmask),
          [15, 15], f"colouring {mask}")


def test_greedy_and_random_walk_limits(ctx):
    check(ctx, synth.tsp_uniform(25, 5, key=1), P(seed=2, population=3, candidates=64, G=20, t0_q16=1), [20], "greedy")
    check(ctx, synth.knapsack_random(40, 5, key=1),
          P(seed=2, population=3, candidates=64, G=20, t0_q16=2**62, alpha_q32=2**32 - 1), [20], "random walk")


def test_odd_epoch_and_stagnation(ctx):
    # epoch of 3 generations and a stagnation limit of 1 exercise the K-step reset often
    p = P(seed=4, population=4, candidates=64, G=40, epoch=3, stagnation_epochs=1)
    check(ctx, synth.color_planted(30, 3, key=6), p, [13, 27], "epoch 3")


@pytest.mark.parametrize("seed", [42, 123, 456, 789, 2024])   # the paper's five seeds
def test_c1_full_trajectory(ctx, seed):
    inst, p = synth.c1_small_tsp(0)
    p = p.with_(seed=seed)
    check(ctx, inst, p, [500, 500, 1000], f"TSP n=50 P=64 G=2000 seed {seed}")


def test_c2_full_size_windowed(ctx):
    """Full 442-city instance at the benchmark's launch configuration
    (autosized population, default staging): run 1000 generations on the GPU
    (graph-replayed launches), then compare a 20-generation window against the
    oracle resumed from the GPU's own state."""
    inst, p = synth.c2_tsp442(population=0, generations=200_000)
    h = gx.gx_instance_upload(ctx, inst)
    P_auto = gx.gx_autosize_population(ctx, h, p)
    p = p.with_(population=P_auto)
    print(f"[parity] C2 windowed P={P_auto}", flush=True)
    job = gx.gx_job_create(ctx, h, p)
    init = gx.gx_snapshot(ctx, job, P_auto, inst.n)
    o = oracle.OracleInstance(inst)
    ref_init = o.init(p)
    assert_same(init, ref_init, "C2 init")
    gx.gx_job_advance(ctx, job, 1000)
    a = gx.gx_snapshot(ctx, job, P_auto, inst.n)
    gx.gx_job_advance(ctx, job, 20)
    b = gx.gx_snapshot(ctx, job, P_auto, inst.n)
    gx.gx_job_free(ctx, job)
    gx.gx_instance_free(ctx, h)
    assert a["g"] == 1000 and b["g"] == 1020
    for s in range(P_auto):
        assert sorted(a["cur"][s]) == list(range(inst.n))
    o.run(p, a, 20)
    assert_same(b, a, "C2 window 1000..1020")


@pytest.mark.parametrize("w", [(6, 2, 2), (0, 1000, 1)])
def test_vrptw_weighted_objectives(ctx, w):
    # distance, route count and longest route weighted; (0, 1000, 1): routes
    # first, then the longest route
    base = synth.vrptw_random(30, 4, key=41)
    inst = synth.Instance(synth.VRPTW, base.n, base.a, base.b, capacity=base.capacity, vehicles=base.vehicles,
                          service_time=base.service_time, horizon=base.horizon, key=41, obj_weights=w)
    check(ctx, inst, P(seed=43, population=6, candidates=128, G=30), [10, 20], f"vrptw weights {w}")


def test_invalid_arguments_are_rejected(ctx):
    inst = synth.tsp_uniform(10, 0)
    h = gx.gx_instance_upload(ctx, inst)
    with pytest.raises(gx.GxError) as e:
        gx.gx_solve(ctx, h, P(seed=1, population=2, G=10, alpha_q32=0))
    assert e.value.status == gx.GX_E_INVALID
    with pytest.raises(gx.GxError):
        gx.gx_solve(ctx, h, P(seed=1, population=2, G=0))
    with pytest.raises(gx.GxError):
        gx.gx_solve(ctx, h, P(seed=1, population=2, G=10, op_mask=1 << synth.OP_FLIP))
    with pytest.raises(gx.GxError):
        gx.gx_solve(ctx, h, P(seed=1, population=2, G=10, candidates=70000))
    bad = synth.Instance(synth.TSP, 3, np.array([[0, 1, 2], [1, 0, 5], [3, 5, 0]]), key=0)
    with pytest.raises(gx.GxError):
        gx.gx_instance_upload(ctx, bad)          # not symmetric
    for bad_p in (P(seed=1, population=10, G=10, islands=4), P(seed=1, population=8, G=10, islands=4, migrate_mode=3),
                  P(seed=1, population=8, G=10, islands=4, migrate_n=2), P(seed=1, population=130, G=10, islands=65)):
        with pytest.raises(gx.GxError) as e:
            gx.gx_solve(ctx, h, bad_p)
        assert e.value.status == gx.GX_E_INVALID
    with pytest.raises(gx.GxError) as e:
        gx.gx_instance_upload(ctx, synth.qap_random(70, 0))
    assert e.value.status == gx.GX_E_UNSUPPORTED
    v = synth.vrptw_random(10, 0)
    for kind_inst in (synth.Instance(synth.TSP, 10, synth.tsp_uniform(10, 0).a, a_is_coords=1, obj_weights=(1, 1, 0)),
                      synth.Instance(synth.VRPTW, 10, v.a, v.b, capacity=v.capacity, vehicles=v.vehicles,
                                     service_time=v.service_time, horizon=v.horizon, obj_weights=(1, -1, 0)),
                      synth.Instance(synth.VRPTW, 10, v.a, v.b, capacity=v.capacity, vehicles=v.vehicles,
                                     service_time=v.service_time, horizon=v.horizon, obj_weights=(1 << 21, 0, 0))):
        with pytest.raises(gx.GxError) as e:
            gx.gx_instance_upload(ctx, kind_inst)
        assert e.value.status == gx.GX_E_INVALID
    gx.gx_instance_free(ctx, h)
