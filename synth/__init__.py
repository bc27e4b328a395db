"""Seeded synthetic workloads shared by the oracle and the HIP path.

This module only *makes inputs*: integer instance data, solve parameters and
request streams.  It holds none of the method's arithmetic (no objective, no
distance rule, no move, no acceptance test); each side computes those itself.

Problem kinds follow the paper's three encodings (Sec. "Encoding Types"):
permutation (TSP, QAP, VRPTW giant tour), binary (0/1 knapsack) and bounded
integer (graph colouring); VRPTW also in the multi-row form (Sec. "Solution
Structure": one route per row).  The benchmark datasets the paper evaluates on
(TSPLIB, QAPLIB, Solomon, Pisinger) are not available; the generators below
stand in for them with the shapes, sizes and value ranges of the workloads
this project measures.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from fractions import Fraction

import numpy as np

# ---- problem kinds and operator ids (shared vocabulary, no arithmetic) ----
TSP, QAP, KNAPSACK, VRPTW, INTCOLOR, VRPTW_ROWS = 1, 2, 3, 4, 5, 6
KIND_NAMES = {TSP: "tsp", QAP: "qap", KNAPSACK: "knapsack", VRPTW: "vrptw", INTCOLOR: "intcolor",
              VRPTW_ROWS: "vrptw_rows"}

# permutation 0-4; ids 5-7: the LNS operators on single-row permutations, the
# row operators on multi-row solutions; binary 8-9, integer 10-11
OP_2OPT, OP_SWAP, OP_INSERT, OP_OROPT, OP_3OPT = 0, 1, 2, 3, 4
OP_ROWSWAP, OP_ROWSPLIT, OP_ROWMERGE = 5, 6, 7
OP_LNS_SEG, OP_LNS_SCATTER, OP_LNS_GUIDED = 5, 6, 7
OP_FLIP, OP_SEGFLIP, OP_RESET, OP_SEGRESET = 8, 9, 10, 11
OP_NAMES = ["2opt", "swap", "insert", "oropt", "3opt", "rowswap", "rowsplit", "rowmerge", "flip", "segflip",
            "reset", "segreset"]
N_OPS = 12
PERM4_OPS = (1 << OP_2OPT) | (1 << OP_SWAP) | (1 << OP_INSERT) | (1 << OP_OROPT)
PERM_OPS = PERM4_OPS | (1 << OP_3OPT)
ROW_OPS = (1 << OP_ROWSWAP) | (1 << OP_ROWSPLIT) | (1 << OP_ROWMERGE)
ROWS_ALL_OPS = PERM_OPS | ROW_OPS
LNS_OPS = (1 << OP_LNS_SEG) | (1 << OP_LNS_SCATTER) | (1 << OP_LNS_GUIDED)
PERM_LNS_OPS = PERM_OPS | LNS_OPS
BIN_OPS = (1 << OP_FLIP) | (1 << OP_SEGFLIP)
INT_OPS = (1 << OP_RESET) | (1 << OP_SEGRESET)

ENCODING_OF = {TSP: "perm", QAP: "perm", VRPTW: "perm", KNAPSACK: "binary", INTCOLOR: "integer",
               VRPTW_ROWS: "perm_rows"}


@dataclass
class Instance:
    """One problem's integer data, laid out the way the C interfaces take it.

    TSP      a = coords (n,2) if a_is_coords else distance matrix (n,n); b unused
    QAP      a = flow F (n,n), b = distance D (n,n), both symmetric
    KNAPSACK a = weights (n,), b = values (n,), capacity
    VRPTW    n = customers; a = coords (n+1,2) with the depot at row 0;
             b = (3, n+1): demand, ready time, due time; capacity, vehicles,
             service_time, horizon
    VRPTW_ROWS  the VRPTW data, solved in the multi-row form with `vehicles`
             rows (a solution holds n + vehicles entries)
    INTCOLOR a = edge list (n_edges, 2); values in [lb, ub]
    """
    kind: int
    n: int
    a: np.ndarray
    b: np.ndarray | None = None
    a_is_coords: int = 0
    capacity: int = 0
    vehicles: int = 0
    service_time: int = 0
    horizon: int = 0
    lb: int = 0
    ub: int = 0
    n_edges: int = 0
    key: int = 0
    obj_weights: tuple = (0, 0, 0)   # VRPTW: weights of distance, routes, longest route
    lex_order: tuple = (0, 0, 0)     # VRPTW lexicographic mode: 1 distance, 2 routes, 3 longest; 0 ends
    lex_tol: tuple = (0, 0, 0)       # tolerance of each lexicographic level

    def __post_init__(self):
        self.a = np.ascontiguousarray(self.a, dtype=np.int32)
        if self.b is not None:
            self.b = np.ascontiguousarray(self.b, dtype=np.int32)

    @property
    def encoding(self) -> str:
        return ENCODING_OF[self.kind]


@dataclass
class Params:
    """Integer-only solve parameters (0 selects the documented default)."""
    seed: int = 42
    generations: int = 2000
    population: int = 64
    candidates: int = 128
    op_mask: int = 0
    t0_q16: int = 0
    alpha_q32: int = 0
    epoch: int = 10
    aos_alpha_q16: int = 49152
    w_floor_q16: int = 1024
    stagnation_epochs: int = 5
    credit: int = 0            # 0: every candidate credits its ops, 1: accepted move only
    oversample_k: int = 4
    staging: int = 0           # TSP distance staging (0 = library's choice)
    islands: int = 0           # island model: 0 or 1 = one population
    migrate_epochs: int = 0    # migration every this many epochs (0 = never)
    migrate_mode: int = 0      # 0 ring, 1 global top-N, 2 hybrid
    migrate_n: int = 0         # N of top-N (0 = 1)
    elite_epochs: int = 0      # elite injection every this many epochs (0 = never)
    aos_scope: int = 0         # 0 weights per instance, 1 per solution
    init_weight_q16: tuple = ()  # raw initial operator weights by id (0 = preset)
    weight_cap_q16: tuple = ()   # per-operator weight caps by id (0 = default)

    def with_(self, **kw) -> "Params":
        return replace(self, **kw)


def alpha_q32_for(generations: int, final_ratio: Fraction = Fraction(1, 1000)) -> int:
    """Cooling factor in Q32 so that T shrinks by ``final_ratio`` over the run.

    A schedule choice of the harness (the paper leaves alpha open), computed
    once here and handed to both sides as the same integer.
    """
    from decimal import Decimal, getcontext, ROUND_HALF_EVEN
    getcontext().prec = 60
    r = Decimal(final_ratio.numerator) / Decimal(final_ratio.denominator)
    a = (r.ln() / Decimal(generations)).exp() * (Decimal(2) ** 32)
    v = int(a.to_integral_value(rounding=ROUND_HALF_EVEN))
    return min(v, 2**32 - 1)


# ---------------------------------------------------------------- generators
def _rng(*ids) -> np.random.Generator:
    return np.random.default_rng([int(x) & 0xFFFFFFFF for x in ids] + [20260319])


def tsp_uniform(n: int, inst_id: int = 0, key: int | None = None) -> Instance:
    """TSP with integer coordinates uniform in [0,10000]^2."""
    r = _rng(1, n, inst_id)
    xy = r.integers(0, 10001, size=(n, 2))
    return Instance(TSP, n, xy, a_is_coords=1, key=inst_id if key is None else key)


def tsp_clustered(n: int, inst_id: int = 0, clusters: int = 20, sigma: float = 300.0,
                  key: int | None = None) -> Instance:
    """TSP with points drawn around ``clusters`` Gaussian centres (stand-in for pcb442)."""
    r = _rng(2, n, inst_id)
    centres = r.uniform(0, 10000, size=(clusters, 2))
    lab = r.integers(0, clusters, size=n)
    xy = np.clip(np.rint(centres[lab] + r.normal(0, sigma, size=(n, 2))), 0, 10000)
    return Instance(TSP, n, xy.astype(np.int32), a_is_coords=1,
                    key=inst_id if key is None else key)


def tsp_circle(n: int, radius: int = 4000, key: int = 0) -> Instance:
    """Planted TSP: points at equal angles on a circle; the angular order is optimal."""
    ang = 2.0 * np.pi * np.arange(n) / n
    xy = np.rint(np.stack([5000 + radius * np.cos(ang), 5000 + radius * np.sin(ang)], 1))
    return Instance(TSP, n, xy.astype(np.int32), a_is_coords=1, key=key)


def tsp_matrix(mat: np.ndarray, key: int = 0) -> Instance:
    mat = np.asarray(mat, dtype=np.int32)
    return Instance(TSP, mat.shape[0], mat, a_is_coords=0, key=key)


def qap_random(n: int, inst_id: int = 0, key: int | None = None) -> Instance:
    """QAP: symmetric flow U[0,9] and distance U[1,99], zero diagonals."""
    r = _rng(3, n, inst_id)
    F = r.integers(0, 10, size=(n, n))
    D = r.integers(1, 100, size=(n, n))
    F = np.triu(F, 1); F = F + F.T
    D = np.triu(D, 1); D = D + D.T
    return Instance(QAP, n, F, D, key=inst_id if key is None else key)


def knapsack_random(n: int, inst_id: int = 0, key: int | None = None) -> Instance:
    """0/1 knapsack: weights and values U[1,100], capacity half the total weight."""
    r = _rng(4, n, inst_id)
    w = r.integers(1, 101, size=n)
    v = r.integers(1, 101, size=n)
    return Instance(KNAPSACK, n, w, v, capacity=int(w.sum()) // 2,
                    key=inst_id if key is None else key)


def vrptw_random(n: int = 100, inst_id: int = 0, key: int | None = None,
                 capacity: int = 200, vehicles: int = 25, service: int = 10,
                 horizon: int = 1000) -> Instance:
    """VRPTW: depot at (50,50); half the customers uniform in [0,100]^2, half in
    5 Gaussian clusters; demand U[1,50]; windows of width U[30,120] that a
    direct depot round trip can serve.  (Stand-in for the Solomon sets.)"""
    r = _rng(5, n, inst_id)
    nu = n // 2
    uni = r.integers(0, 101, size=(nu, 2)).astype(float)
    cen = r.uniform(10, 90, size=(5, 2))
    lab = r.integers(0, 5, size=n - nu)
    clu = np.clip(np.rint(cen[lab] + r.normal(0, 5.0, size=(n - nu, 2))), 0, 100)
    xy = np.vstack([[50.0, 50.0], uni, clu]).astype(np.int32)
    demand = np.concatenate([[0], r.integers(1, 51, size=n)])
    width = r.integers(30, 121, size=n)
    # travel-time estimate used only to place the windows (generator-side,
    # rounded up so every window is reachable from the depot)
    far = np.ceil(np.hypot(xy[1:, 0] - 50.0, xy[1:, 1] - 50.0)).astype(np.int64)
    hi = np.maximum(far, horizon - service - far - width)
    ready = far + np.floor(r.uniform(0, 1, size=n) * (hi - far + 1)).astype(np.int64)
    due = ready + width
    b = np.stack([demand,
                  np.concatenate([[0], ready]),
                  np.concatenate([[horizon], due])]).astype(np.int32)
    return Instance(VRPTW, n, xy, b, capacity=capacity, vehicles=vehicles,
                    service_time=service, horizon=horizon,
                    key=inst_id if key is None else key)


def vrptw_rows(n: int = 100, inst_id: int = 0, key: int | None = None, vehicles: int = 25, **kw) -> Instance:
    """The VRPTW data of `vrptw_random`, for the multi-row form with `vehicles` rows."""
    return replace(vrptw_random(n, inst_id, key, vehicles=vehicles, **kw), kind=VRPTW_ROWS)


def solution_len(inst: Instance) -> int:
    """Entries of one solution of `inst` (customers plus one marker per row in the multi-row form)."""
    return inst.n + (inst.vehicles if inst.kind == VRPTW_ROWS else 0)


def color_planted(n: int, k: int = 3, m: int | None = None, inst_id: int = 0,
                  key: int | None = None) -> Instance:
    """Integer-encoding test problem: a random k-partite graph (so a proper
    colouring with f=0 exists), colours in [0, k-1]."""
    r = _rng(6, n, inst_id)
    part = r.integers(0, k, size=n)
    m = 3 * n if m is None else m
    edges = set()
    tries = 0
    while len(edges) < m and tries < 50 * m:
        tries += 1
        u, v = (int(x) for x in r.integers(0, n, size=2))
        if u == v or part[u] == part[v]:
            continue
        edges.add((min(u, v), max(u, v)))
    e = np.array(sorted(edges), dtype=np.int32).reshape(-1, 2)
    return Instance(INTCOLOR, n, e, lb=0, ub=k - 1, n_edges=e.shape[0],
                    key=inst_id if key is None else key)


# ------------------------------------------------------------ named workloads
PAPER_SEEDS = (42, 123, 456, 789, 2024)


def c1_small_tsp(inst_id: int = 0) -> tuple[Instance, Params]:
    """TSP n=50 uniform, P=64, C=128, 2000 generations, ops {2-opt, swap, or-opt}."""
    inst = tsp_uniform(50, inst_id)
    p = Params(seed=PAPER_SEEDS[inst_id % 5], generations=2000, population=64,
               candidates=128,
               op_mask=(1 << OP_2OPT) | (1 << OP_SWAP) | (1 << OP_OROPT),
               alpha_q32=alpha_q32_for(2000))
    return inst, p


def c2_tsp442(population: int, generations: int = 200_000, seed: int = 42) -> tuple[Instance, Params]:
    """Clustered TSP n=442 (20 clusters, sigma 300), the four element and
    or-opt permutation ops (2-opt, swap, insert, or-opt)."""
    inst = tsp_clustered(442, 0)
    p = Params(seed=seed, generations=generations, population=population, candidates=128,
               op_mask=PERM4_OPS, alpha_q32=alpha_q32_for(generations))
    return inst, p


def c4_batched_instances(count: int = 4096) -> list[Instance]:
    """Batched workload: the first three quarters TSP n U[20,200] (uniform
    coordinates), the rest QAP n U[12,40]; instance key = index."""
    r = np.random.default_rng([4, count, 20260319])
    n_tsp = count * 3 // 4
    out = []
    for i in range(count):
        if i < n_tsp:
            out.append(tsp_uniform(int(r.integers(20, 201)), 10_000 + i, key=i))
        else:
            out.append(qap_random(int(r.integers(12, 41)), 20_000 + i, key=i))
    return out


def c4_params_for(generations: int = 5000):
    """Parameters of batched instance `index` (seed 10^6 + index, C = 128,
    cooling to 0.001 over the run) at a given population and staging."""
    alpha = alpha_q32_for(generations)

    def make(inst, index, population, staging):
        return Params(seed=10**6 + index, generations=generations, population=population, candidates=128,
                      alpha_q32=alpha, staging=staging)
    return make


def c5_requests(rate: float, duration: float, kinds=(0, 1, 2), generations: int = 10_000,
                population: int = 4):
    """Served workload: int(rate * duration) requests with exponential gaps
    (Poisson arrivals at `rate`), each of a kind drawn from `kinds` (0 TSP n
    U[20,500], 1 QAP n U[12,50], 2 knapsack n U[100,1000]) with its own seed.
    Returns (requests [(instance, params)], gaps in seconds)."""
    r = np.random.default_rng([5, 789, 20260319])
    n_req = int(rate * duration)
    gaps = r.exponential(1.0 / rate, size=n_req)
    alpha = alpha_q32_for(generations)
    reqs = []
    for i in range(n_req):
        kind = kinds[int(r.integers(0, len(kinds)))]
        if kind == 0:
            inst = tsp_uniform(int(r.integers(20, 501)), 30_000 + i, key=i)
        elif kind == 1:
            inst = qap_random(int(r.integers(12, 51)), 40_000 + i, key=i)
        else:
            inst = knapsack_random(int(r.integers(100, 1001)), 50_000 + i, key=i)
        reqs.append((inst, Params(seed=int(r.integers(0, 2**40)), generations=generations, population=population,
                                  candidates=128, alpha_q32=alpha)))
    return reqs, gaps


def c3_vrptw(seed: int = 42, generations: int = 5000, population: int = 64) -> tuple[Instance, Params]:
    inst = vrptw_random(100, 0)
    p = Params(seed=seed, generations=generations, population=population, candidates=128,
               op_mask=PERM_OPS, alpha_q32=alpha_q32_for(generations))
    return inst, p


def c3_vrptw_rows(seed: int = 42, generations: int = 5000, population: int = 64) -> tuple[Instance, Params]:
    """The C3 customers in the multi-row form (25 rows), every operator of the form."""
    inst = vrptw_rows(100, 0)
    p = Params(seed=seed, generations=generations, population=population, candidates=128,
               op_mask=ROWS_ALL_OPS, alpha_q32=alpha_q32_for(generations))
    return inst, p
