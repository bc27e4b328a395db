"""Python access to the CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use it; the product package never imports it.  The oracle is
a plain, slow transcription of the paper's definitions (Alg. 1, Alg. 2,
Eq. ema, Sec. "Population Management"), with every objective recomputed in
full on a real copy of each candidate.

Parity is pinned for every function here (tests/test_oracle_*.py): objectives
by brute force and closed forms, Philox by published known-answer vectors, the
exp tables by exact regeneration, the AOS arithmetic by a worked example, and
whole runs by invariants (delta == full recompute, validity, determinism,
greedy / random-walk limits, snapshot-resume equivalence).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
N_OPS = 12


def build(force: bool = False) -> str:
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < max(
            os.path.getmtime(src), os.path.getmtime(os.path.join(_HERE, "oracle.h"))):
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-shared", "-fPIC", "-pthread",
                               "-o", _SO + ".tmp", src])
        os.replace(_SO + ".tmp", _SO)
    return _SO


class _Desc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n", C.c_int32),
                ("a", C.POINTER(C.c_int32)), ("b", C.POINTER(C.c_int32)),
                ("a_is_coords", C.c_int32), ("capacity", C.c_int32), ("vehicles", C.c_int32),
                ("service_time", C.c_int32), ("horizon", C.c_int32), ("lb", C.c_int32),
                ("ub", C.c_int32), ("n_edges", C.c_int32), ("key", C.c_uint32),
                ("obj_w", C.c_int32 * 3), ("lex_order", C.c_int32 * 3), ("lex_tol", C.c_int32 * 3)]


class _Params(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("generations", C.c_uint32), ("population", C.c_uint32),
                ("candidates", C.c_uint32), ("op_mask", C.c_uint32), ("t0_q16", C.c_uint64),
                ("alpha_q32", C.c_uint32), ("epoch", C.c_uint32), ("aos_alpha_q16", C.c_uint32),
                ("w_floor_q16", C.c_uint32), ("stagnation_epochs", C.c_uint32),
                ("credit", C.c_uint32), ("oversample_k", C.c_uint32), ("islands", C.c_uint32),
                ("migrate_epochs", C.c_uint32), ("migrate_mode", C.c_uint32), ("migrate_n", C.c_uint32),
                ("elite_epochs", C.c_uint32), ("aos_scope", C.c_uint32), ("init_w", C.c_uint32 * N_OPS),
                ("cap_w", C.c_uint32 * N_OPS)]


# per-solution AOS state (or_sol_aos), as a numpy record
SOL_AOS = np.dtype([("w_op", np.uint32, N_OPS), ("w_k", np.uint32, 3), ("stag", np.uint32),
                    ("epoch_ref", np.int64), ("u_op", np.uint32, N_OPS), ("v_op", np.uint32, N_OPS),
                    ("u_k", np.uint32, 3), ("v_k", np.uint32, 3)])
assert SOL_AOS.itemsize == 192


class _State(C.Structure):
    _fields_ = [("g", C.c_uint32), ("stag", C.c_uint32), ("T_q16", C.c_uint64),
                ("epoch_ref", C.c_int64), ("w_op", C.c_uint32 * N_OPS), ("w_k", C.c_uint32 * 3),
                ("pad_", C.c_uint32),
                ("u_op", C.c_uint64 * N_OPS), ("v_op", C.c_uint64 * N_OPS),
                ("u_k", C.c_uint64 * 3), ("v_k", C.c_uint64 * 3), ("accepted", C.c_uint64),
                ("tot_u_op", C.c_uint64 * N_OPS), ("tot_v_op", C.c_uint64 * N_OPS),
                ("tot_u_k", C.c_uint64 * 3), ("tot_v_k", C.c_uint64 * 3),
                ("cur", C.POINTER(C.c_int32)), ("cur_f", C.POINTER(C.c_int64)),
                ("best", C.POINTER(C.c_int32)), ("best_f", C.POINTER(C.c_int64)), ("saos", C.c_void_p),
                ("cur_v", C.c_void_p), ("best_v", C.c_void_p), ("ref_v", C.c_int64 * 4)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        P32, P64 = C.POINTER(C.c_uint32), C.POINTER(C.c_int32)
        L.or_philox4x32_10.argtypes = [P32, P32, P32]
        L.or_philox_many.argtypes = [C.c_void_p, C.c_int64, P32, C.c_void_p]
        L.or_nint_dist.argtypes = [C.c_int32] * 4
        L.or_nint_dist.restype = C.c_int32
        L.or_isqrt.argtypes = [C.c_uint64]
        L.or_isqrt.restype = C.c_uint64
        L.or_accept_threshold.argtypes = [C.c_uint64, C.c_uint64, C.POINTER(C.c_int)]
        L.or_accept_threshold.restype = C.c_uint32
        L.or_cool.argtypes = [C.c_uint64, C.c_uint32]
        L.or_cool.restype = C.c_uint64
        L.or_inst_new.argtypes = [C.POINTER(_Desc)]
        L.or_inst_new.restype = C.c_void_p
        L.or_inst_free.argtypes = [C.c_void_p]
        L.or_objective.argtypes = [C.c_void_p, P64]
        L.or_objective.restype = C.c_int64
        L.or_dist.argtypes = [C.c_void_p, C.c_int32, C.c_int32]
        L.or_dist.restype = C.c_int32
        L.or_apply_op.argtypes = [C.c_void_p, P64, C.c_int, C.c_uint32, C.c_uint32, C.c_uint32]
        L.or_initial_weights.argtypes = [C.c_void_p, C.c_uint32, C.c_void_p, P32]
        L.or_aos_update.argtypes = [C.c_void_p, C.POINTER(_Params), C.c_uint32, C.POINTER(_State), C.c_int64]
        L.or_lns_len.argtypes = [C.c_int]
        L.or_lns_len.restype = C.c_int
        L.or_lns_cap.argtypes = [C.c_void_p]
        L.or_lns_cap.restype = C.c_uint32
        L.or_migrate.argtypes = [C.c_void_p, C.POINTER(_Params), C.c_int, C.POINTER(_State), C.c_uint32]
        L.or_heuristic_perms.argtypes = [C.c_void_p, P64, C.c_int]
        L.or_heuristic_perms.restype = C.c_int
        L.or_init.argtypes = [C.c_void_p, C.POINTER(_Params), C.POINTER(_State)]
        L.or_random_solution.argtypes = [C.c_void_p, C.POINTER(_Params), C.c_uint32, P64]
        L.or_wpick.argtypes = [C.c_uint32, P32, C.c_int]
        L.or_wpick.restype = C.c_int
        L.or_run.argtypes = [C.c_void_p, C.POINTER(_Params), C.POINTER(_State), C.c_uint32]
        L.or_run_par.argtypes = [C.c_void_p, C.POINTER(_Params), C.POINTER(_State), C.c_uint32, C.c_int]
        L.or_effective_mask.argtypes = [C.c_void_p, C.c_uint32]
        L.or_effective_mask.restype = C.c_uint32
        L.or_lex_mode.argtypes = [C.c_void_p]
        L.or_lex_mode.restype = C.c_int
        L.or_lex_vector.argtypes = [C.c_void_p, P64, C.c_void_p]
        L.or_lex_better.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.or_lex_better.restype = C.c_int
        L.or_lex_best.argtypes = [C.c_void_p, C.POINTER(_State), C.c_int]
        L.or_lex_best.restype = C.c_int
        _lib = L
    return _lib


def _i32p(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


# ------------------------------------------------------------------ helpers
def lns_len(n: int) -> int:
    return int(lib().or_lns_len(n))


def philox(ctr, key) -> np.ndarray:
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (C.c_uint32 * 4)()
    lib().or_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def philox_many(ctr, key) -> np.ndarray:
    """Philox4x32-10 blocks for an (m, 4) array of counters -> (m, 4) uint32."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    out = np.zeros_like(c)
    lib().or_philox_many(c.ctypes.data, len(c), k, out.ctypes.data)
    return out


def wpick(u16: int, w) -> int:
    """Index the Q16 roulette picks for the 16-bit draw u16 over weights w."""
    arr = (C.c_uint32 * len(w))(*[int(x) for x in w])
    return int(lib().or_wpick(u16, arr, len(w)))


def nint_dist(x1, y1, x2, y2) -> int:
    return int(lib().or_nint_dist(x1, y1, x2, y2))


def isqrt(v: int) -> int:
    return int(lib().or_isqrt(v))


def accept_threshold(delta: int, t_q16: int):
    """(threshold, rejected_outright) for a positive delta."""
    rej = C.c_int(0)
    thr = lib().or_accept_threshold(delta, t_q16, C.byref(rej))
    return int(thr), bool(rej.value)


def cool(t_q16: int, alpha_q32: int) -> int:
    return int(lib().or_cool(t_q16, alpha_q32))


def _params(p) -> _Params:
    return _Params(seed=p.seed & 0xFFFFFFFFFFFFFFFF, generations=p.generations,
                   population=p.population, candidates=p.candidates or 128,
                   op_mask=p.op_mask, t0_q16=p.t0_q16, alpha_q32=p.alpha_q32,
                   epoch=p.epoch or 10, aos_alpha_q16=p.aos_alpha_q16 or 49152,
                   w_floor_q16=p.w_floor_q16 or 1024,
                   stagnation_epochs=p.stagnation_epochs or 5, credit=p.credit,
                   oversample_k=p.oversample_k or 4, islands=p.islands,
                   migrate_epochs=p.migrate_epochs, migrate_mode=p.migrate_mode,
                   migrate_n=p.migrate_n, elite_epochs=p.elite_epochs,
                   aos_scope=getattr(p, "aos_scope", 0),
                   init_w=(C.c_uint32 * N_OPS)(*_init_w(p)),
                   cap_w=(C.c_uint32 * N_OPS)(*_per_op(p, "weight_cap_q16")))


def _per_op(p, name):
    w = list(getattr(p, name, ()) or ())
    return [int(x) for x in w] + [0] * (N_OPS - len(w))


def _init_w(p):
    return _per_op(p, "init_weight_q16")


class OracleInstance:
    """Owns the oracle's copy of an instance (the caller's arrays stay referenced)."""

    def __init__(self, inst):
        self.inst = inst
        self._a = np.ascontiguousarray(inst.a, dtype=np.int32)
        self._b = None if inst.b is None else np.ascontiguousarray(inst.b, dtype=np.int32)
        d = _Desc(kind=inst.kind, n=inst.n, a=_i32p(self._a),
                  b=_i32p(self._b) if self._b is not None else C.POINTER(C.c_int32)(),
                  a_is_coords=inst.a_is_coords, capacity=inst.capacity, vehicles=inst.vehicles,
                  service_time=inst.service_time, horizon=inst.horizon, lb=inst.lb, ub=inst.ub,
                  n_edges=inst.n_edges, key=inst.key & 0xFFFFFFFF,
                  obj_w=(C.c_int32 * 3)(*getattr(inst, "obj_weights", (0, 0, 0))),
                  lex_order=(C.c_int32 * 3)(*getattr(inst, "lex_order", (0, 0, 0))),
                  lex_tol=(C.c_int32 * 3)(*getattr(inst, "lex_tol", (0, 0, 0))))
        self._desc = d
        self.h = lib().or_inst_new(C.byref(d))
        if not self.h:
            raise ValueError("oracle rejected the instance")

    def __del__(self):
        if getattr(self, "h", None):
            lib().or_inst_free(self.h)
            self.h = None

    @property
    def n(self):
        """Entries of a solution: n, or n customers plus one marker per row in the multi-row VRPTW form."""
        return self.inst.n + (self.inst.vehicles if self.inst.kind == 6 else 0)

    def objective(self, x) -> int:
        x = np.ascontiguousarray(x, dtype=np.int32)
        assert x.shape == (self.n,)
        return int(lib().or_objective(self.h, _i32p(x)))

    def dist(self, u, v) -> int:
        return int(lib().or_dist(self.h, u, v))

    def apply_op(self, x, op, w1, w2, w3):
        x = np.array(x, dtype=np.int32, copy=True)
        lib().or_apply_op(self.h, _i32p(x), op, w1 & 0xFFFFFFFF, w2 & 0xFFFFFFFF, w3 & 0xFFFFFFFF)
        return x

    def initial_weights(self, op_mask, init_w=None) -> np.ndarray:
        w = (C.c_uint32 * N_OPS)()
        iw = None if init_w is None else (C.c_uint32 * N_OPS)(*(list(init_w) + [0] * (N_OPS - len(init_w))))
        lib().or_initial_weights(self.h, op_mask, iw, w)
        return np.array(list(w), dtype=np.uint32)

    def lns_cap(self) -> int:
        return int(lib().or_lns_cap(self.h))

    def effective_mask(self, op_mask) -> int:
        return int(lib().or_effective_mask(self.h, op_mask))

    def random_solution(self, params, pool_index: int) -> np.ndarray:
        """The random member of the initial pool at `pool_index`."""
        x = np.zeros(self.n, np.int32)
        pp = _params(params)
        lib().or_random_solution(self.h, C.byref(pp), pool_index, _i32p(x))
        return x

    def heuristic_perms(self) -> np.ndarray:
        out = np.zeros((8, self.n), dtype=np.int32)
        c = lib().or_heuristic_perms(self.h, _i32p(out), 8)
        return out[:c]

    # -------------------------------------------------------------- solve
    def _state_struct(self, st: dict) -> _State:
        s = _State(g=st["g"], stag=st["stag"], T_q16=st["T_q16"], epoch_ref=st["epoch_ref"],
                   accepted=st["accepted"])
        for name in ("w_op", "w_k", "u_op", "v_op", "u_k", "v_k", "tot_u_op", "tot_v_op", "tot_u_k", "tot_v_k"):
            arr = getattr(s, name)
            for i, v in enumerate(st[name]):
                arr[i] = int(v)
        s.cur = _i32p(st["cur"])
        s.cur_f = st["cur_f"].ctypes.data_as(C.POINTER(C.c_int64))
        s.best = _i32p(st["best"])
        s.best_f = st["best_f"].ctypes.data_as(C.POINTER(C.c_int64))
        s.saos = st["saos"].ctypes.data
        s.cur_v = st["cur_v"].ctypes.data
        s.best_v = st["best_v"].ctypes.data
        for i, v in enumerate(st["ref_v"]):
            s.ref_v[i] = int(v)
        return s

    @staticmethod
    def _read_back(s: _State, st: dict):
        st["g"], st["stag"], st["T_q16"] = int(s.g), int(s.stag), int(s.T_q16)
        st["epoch_ref"], st["accepted"] = int(s.epoch_ref), int(s.accepted)
        for name, dt in (("w_op", np.uint32), ("w_k", np.uint32), ("u_op", np.uint64),
                         ("v_op", np.uint64), ("u_k", np.uint64), ("v_k", np.uint64),
                         ("tot_u_op", np.uint64), ("tot_v_op", np.uint64), ("tot_u_k", np.uint64),
                         ("tot_v_k", np.uint64)):
            st[name] = np.array(list(getattr(s, name)), dtype=dt)
        st["ref_v"] = np.array(list(s.ref_v), dtype=np.int64)

    def new_state(self, P: int) -> dict:
        n = self.n
        return {"g": 0, "stag": 0, "T_q16": 0, "epoch_ref": 0, "accepted": 0,
                "w_op": np.zeros(N_OPS, np.uint32), "w_k": np.zeros(3, np.uint32),
                "u_op": np.zeros(N_OPS, np.uint64), "v_op": np.zeros(N_OPS, np.uint64),
                "u_k": np.zeros(3, np.uint64), "v_k": np.zeros(3, np.uint64),
                "tot_u_op": np.zeros(N_OPS, np.uint64), "tot_v_op": np.zeros(N_OPS, np.uint64),
                "tot_u_k": np.zeros(3, np.uint64), "tot_v_k": np.zeros(3, np.uint64),
                "cur": np.zeros((P, n), np.int32), "cur_f": np.zeros(P, np.int64),
                "best": np.zeros((P, n), np.int32), "best_f": np.zeros(P, np.int64),
                "saos": np.zeros(P, SOL_AOS), "cur_v": np.zeros((P, 4), np.int64),
                "best_v": np.zeros((P, 4), np.int64), "ref_v": np.zeros(4, np.int64)}

    def init(self, params) -> dict:
        st = self.new_state(params.population)
        s = self._state_struct(st)
        pp = _params(params)
        if lib().or_init(self.h, C.byref(pp), C.byref(s)) != 0:
            raise ValueError("the lexicographic mode takes instance-level weights")
        self._read_back(s, st)
        return st

    def run(self, params, st: dict, n_gens: int, threads: int = 1) -> dict:
        """Advance ``st`` (modified in place and returned) by ``n_gens``
        generations; ``threads`` > 1 takes the threaded runner (same result)."""
        for k in ("cur", "best"):
            st[k] = np.ascontiguousarray(st[k], dtype=np.int32)
        for k in ("cur_f", "best_f"):
            st[k] = np.ascontiguousarray(st[k], dtype=np.int64)
        if "saos" not in st or len(st["saos"]) != len(st["cur_f"]):
            st["saos"] = np.zeros(len(st["cur_f"]), SOL_AOS)
        st["saos"] = np.ascontiguousarray(st["saos"], dtype=SOL_AOS)
        for k in ("tot_u_op", "tot_v_op", "tot_u_k", "tot_v_k"):
            st.setdefault(k, np.zeros(N_OPS if k.endswith("op") else 3, np.uint64))
        P = len(st["cur_f"])
        for k in ("cur_v", "best_v"):
            st[k] = np.ascontiguousarray(st.get(k, np.zeros((P, 4), np.int64)), dtype=np.int64)
        st.setdefault("ref_v", np.zeros(4, np.int64))
        s = self._state_struct(st)
        pp = _params(params)
        if threads > 1:
            lib().or_run_par(self.h, C.byref(pp), C.byref(s), n_gens, threads)
        else:
            lib().or_run(self.h, C.byref(pp), C.byref(s), n_gens)
        self._read_back(s, st)
        return st

    def aos_update(self, params, st: dict, inst_best_now: int, op_mask=None) -> dict:
        s = self._state_struct(st)
        pp = _params(params)
        m = self.effective_mask(params.op_mask if op_mask is None else op_mask)
        lib().or_aos_update(self.h, C.byref(pp), m, C.byref(s), inst_best_now)
        self._read_back(s, st)
        return st

    def migrate(self, params, st: dict, epoch: int) -> dict:
        """Migration and elite injection at the end of epoch `epoch` (1-based)."""
        s = self._state_struct(st)
        pp = _params(params)
        lib().or_migrate(self.h, C.byref(pp), self.n, C.byref(s), epoch)
        self._read_back(s, st)
        return st

    @property
    def lex(self) -> bool:
        return bool(lib().or_lex_mode(self.h))

    def lex_vector(self, x) -> np.ndarray:
        """(penalty, level 1, level 2, level 3) of a solution in the lexicographic mode."""
        x = np.ascontiguousarray(x, dtype=np.int32)
        v = np.zeros(4, np.int64)
        lib().or_lex_vector(self.h, _i32p(x), v.ctypes.data)
        return v

    def lex_better(self, a, b) -> bool:
        a = np.ascontiguousarray(a, dtype=np.int64)
        b = np.ascontiguousarray(b, dtype=np.int64)
        return bool(lib().or_lex_better(self.h, a.ctypes.data, b.ctypes.data))

    def best_of(self, st: dict):
        """(reported objective, index) of the best solution: the minimum of
        (best_f, index), or in the lexicographic mode the ordered scan of the
        best vectors."""
        if not self.lex:
            return best_of(st)
        s = self._state_struct(st)
        i = int(lib().or_lex_best(self.h, C.byref(s), len(st["best_f"])))
        return int(st["best_f"][i]), i

    def solve(self, params, threads: int = 1) -> dict:
        st = self.init(params)
        return self.run(params, st, params.generations, threads)


def best_of(st: dict):
    """(objective, index) of the best solution: min over (best_f, index)."""
    i = int(np.argmin(st["best_f"]))   # argmin returns the first minimum
    return int(st["best_f"][i]), i
