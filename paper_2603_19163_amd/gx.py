"""ctypes binding of the gx C interface (include/gx.h), same names as the C
entry points.  Argument marshalling only: every step of the solve runs in the
HIP kernels of libgx.so.  There is no CPU fallback: importing works anywhere,
but any call that needs the library raises if libgx.so is missing, and
gx_create fails without a gfx950 device."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgx.so")

GX_OK, GX_E_INVALID, GX_E_UNSUPPORTED, GX_E_NOMEM, GX_E_DEVICE, GX_E_NOT_READY, GX_E_BUSY, GX_E_CANCELLED = \
    0, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "GX_OK", -1: "GX_E_INVALID", -2: "GX_E_UNSUPPORTED", -3: "GX_E_NOMEM",
                -4: "GX_E_DEVICE", -5: "GX_E_NOT_READY", -6: "GX_E_BUSY", -7: "GX_E_CANCELLED"}
STAGE_AUTO, STAGE_LDS_D16, STAGE_LDS_XY, STAGE_GLB_D16, STAGE_GLB_D32 = 0, 1, 2, 3, 4
N_OPS = 12

EXPORTED = ["gx_create", "gx_destroy", "gx_last_error", "gx_get_device_info", "gx_instance_upload",
            "gx_instance_free", "gx_autosize_population", "gx_job_create", "gx_job_advance", "gx_solve",
            "gx_solve_static", "gx_wait", "gx_poll", "gx_fetch_best", "gx_portfolio_best", "gx_job_info_get", "gx_job_stats",
            "gx_job_population", "gx_snapshot", "gx_snapshot_aos", "gx_snapshot_lex", "gx_job_restore", "gx_job_free",
            "gx_solve_batch", "gx_exp_tables", "gx_device_check", "gx_measure_peaks", "gx_server_create", "gx_server_submit", "gx_server_poll",
            "gx_server_cancel", "gx_server_stats_get", "gx_server_destroy"]


class GxError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class gx_instance_desc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n", C.c_int32), ("is_device_ptr", C.c_int32),
                ("a", C.c_void_p), ("b", C.c_void_p),
                ("a_is_coords", C.c_int32), ("capacity", C.c_int32), ("vehicles", C.c_int32),
                ("service_time", C.c_int32), ("horizon", C.c_int32), ("lb", C.c_int32),
                ("ub", C.c_int32), ("n_edges", C.c_int32), ("instance_key", C.c_uint32),
                ("obj_weights", C.c_int32 * 3), ("lex_order", C.c_int32 * 3), ("lex_tol", C.c_int32 * 3)]


class gx_solve_params(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("generations", C.c_uint32), ("population", C.c_uint32),
                ("candidates", C.c_uint32), ("op_mask", C.c_uint32), ("t0_q16", C.c_uint64),
                ("alpha_q32", C.c_uint32), ("aos_epoch", C.c_uint32), ("aos_alpha_q16", C.c_uint32),
                ("w_floor_q16", C.c_uint32), ("stagnation_epochs", C.c_uint32),
                ("aos_credit", C.c_uint32), ("oversample_k", C.c_uint32), ("staging", C.c_uint32),
                ("islands", C.c_uint32), ("migrate_epochs", C.c_uint32), ("migrate_mode", C.c_uint32),
                ("migrate_n", C.c_uint32), ("elite_epochs", C.c_uint32), ("aos_scope", C.c_uint32),
                ("init_weight_q16", C.c_uint32 * N_OPS), ("weight_cap_q16", C.c_uint32 * N_OPS)]


class gx_device_info(C.Structure):
    _fields_ = [("cus", C.c_int32), ("lds_per_block", C.c_int32), ("wave_size", C.c_int32),
                ("l2_bytes", C.c_int32), ("arch", C.c_char * 64)]


class gx_job_info(C.Structure):
    _fields_ = [("population", C.c_uint32), ("candidates", C.c_uint32),
                ("generations_done", C.c_uint32), ("staging", C.c_uint32),
                ("move_evals", C.c_uint64), ("accepted", C.c_uint64),
                ("evolve_launches", C.c_uint32), ("evolve_ms", C.c_float),
                ("op_steps", C.c_uint64 * N_OPS), ("k_count", C.c_uint64 * 3)]


class gx_peaks(C.Structure):
    _fields_ = [("lds_gather_bytes_per_s", C.c_double), ("philox_blocks_per_s", C.c_double),
                ("valu_lane_ops_per_s", C.c_double), ("valu_instr_per_s", C.c_double),
                ("l2_gather_bytes_per_s", C.c_double), ("hbm_read_bytes_per_s", C.c_double),
                ("cus", C.c_int32), ("pad_", C.c_int32)]


class gx_run_stats(C.Structure):
    _fields_ = [("move_evals", C.c_uint64), ("accepted", C.c_uint64),
                ("u_op", C.c_uint64 * N_OPS), ("v_op", C.c_uint64 * N_OPS),
                ("u_k", C.c_uint64 * 3), ("v_k", C.c_uint64 * 3),
                ("generations_done", C.c_uint32), ("population", C.c_uint32)]


class gx_sol_aos(C.Structure):
    _fields_ = [("w_op", C.c_uint32 * N_OPS), ("w_k", C.c_uint32 * 3), ("stag", C.c_uint32),
                ("epoch_ref", C.c_int64), ("u_op", C.c_uint32 * N_OPS), ("v_op", C.c_uint32 * N_OPS),
                ("u_k", C.c_uint32 * 3), ("v_k", C.c_uint32 * 3)]


# the same record as a numpy dtype (arrays of P records)
SOL_AOS = np.dtype([("w_op", np.uint32, N_OPS), ("w_k", np.uint32, 3), ("stag", np.uint32),
                    ("epoch_ref", np.int64), ("u_op", np.uint32, N_OPS), ("v_op", np.uint32, N_OPS),
                    ("u_k", np.uint32, 3), ("v_k", np.uint32, 3)])


class gx_server_cfg(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_uint64), ("max_resident", C.c_uint32), ("max_lds_bytes", C.c_uint32),
                ("max_items", C.c_uint32), ("quantum_epochs", C.c_uint32), ("reserved", C.c_uint32)]


class gx_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("admitted", C.c_uint64), ("completed", C.c_uint64),
                ("cancelled", C.c_uint64), ("quanta", C.c_uint64), ("move_evals", C.c_uint64),
                ("resident", C.c_uint32), ("pending", C.c_uint32), ("arena_used_bytes", C.c_uint64),
                ("arena_bytes", C.c_uint64), ("busy_seconds", C.c_double)]


class gx_state_scalars(C.Structure):
    _fields_ = [("g", C.c_uint32), ("stag", C.c_uint32), ("T_q16", C.c_uint64),
                ("epoch_ref", C.c_int64), ("w_op", C.c_uint32 * N_OPS), ("w_k", C.c_uint32 * 3),
                ("pad_", C.c_uint32), ("u_op", C.c_uint64 * N_OPS), ("v_op", C.c_uint64 * N_OPS),
                ("u_k", C.c_uint64 * 3), ("v_k", C.c_uint64 * 3), ("accepted", C.c_uint64)]


_lib = None


def lib():
    """Load libgx.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it (python -m paper_2603_19163_amd.build)")
        L = C.CDLL(LIB_PATH)
        vp, i32, u32 = C.c_void_p, C.c_int32, C.c_uint32
        pp = C.POINTER(C.c_void_p)
        sig = {
            "gx_create": ([C.c_int, vp, pp], i32),
            "gx_destroy": ([vp], i32),
            "gx_last_error": ([vp], C.c_char_p),
            "gx_get_device_info": ([vp, C.POINTER(gx_device_info)], i32),
            "gx_instance_upload": ([vp, C.POINTER(gx_instance_desc), pp], i32),
            "gx_instance_free": ([vp, vp], i32),
            "gx_autosize_population": ([vp, vp, C.POINTER(gx_solve_params), C.POINTER(u32)], i32),
            "gx_job_create": ([vp, vp, C.POINTER(gx_solve_params), pp], i32),
            "gx_job_advance": ([vp, vp, u32], i32),
            "gx_solve": ([vp, vp, C.POINTER(gx_solve_params), pp], i32),
            "gx_solve_static": ([vp, vp, C.POINTER(gx_solve_params), vp, vp], i32),
            "gx_wait": ([vp, vp], i32),
            "gx_poll": ([vp, vp], i32),
            "gx_fetch_best": ([vp, vp, vp, i32, C.POINTER(C.c_int64)], i32),
            "gx_portfolio_best": ([vp, pp, i32, vp, i32, C.POINTER(C.c_int64), C.POINTER(C.c_int32)], i32),
            "gx_job_info_get": ([vp, vp, C.POINTER(gx_job_info)], i32),
            "gx_job_stats": ([vp, vp, C.POINTER(gx_run_stats)], i32),
            "gx_job_population": ([vp, vp, C.POINTER(u32)], i32),
            "gx_snapshot": ([vp, vp, C.POINTER(gx_state_scalars), vp, vp, vp, vp], i32),
            "gx_snapshot_aos": ([vp, vp, vp], i32),
            "gx_snapshot_lex": ([vp, vp, vp, vp, vp], i32),
            "gx_job_restore": ([vp, vp, C.POINTER(gx_state_scalars), vp, vp, vp, vp, vp], i32),
            "gx_job_free": ([vp, vp], i32),
            "gx_solve_batch": ([vp, pp, C.POINTER(gx_solve_params), i32, pp], i32),
            "gx_exp_tables": ([C.POINTER(u32), C.POINTER(u32)], i32),
            "gx_device_check": ([vp, i32, C.c_uint64, vp, vp, C.c_int64], i32),
            "gx_measure_peaks": ([vp, C.POINTER(gx_peaks)], i32),
            "gx_server_create": ([vp, C.POINTER(gx_server_cfg), pp], i32),
            "gx_server_submit": ([vp, C.POINTER(gx_instance_desc), C.POINTER(gx_solve_params),
                                  C.POINTER(C.c_uint64)], i32),
            "gx_server_poll": ([vp, C.c_uint64, vp, i32, C.POINTER(C.c_int64), C.POINTER(C.c_uint64),
                                C.POINTER(C.c_uint64)], i32),
            "gx_server_cancel": ([vp, C.c_uint64], i32),
            "gx_server_stats_get": ([vp, C.POINTER(gx_server_stats)], i32),
            "gx_server_destroy": ([vp], i32),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes, f.restype = args, res
        _lib = L
    return _lib


def _check(ctx, status):
    if status != GX_OK:
        msg = lib().gx_last_error(ctx).decode() if ctx else ""
        raise GxError(status, msg)


# ------------------------------------------------------------------ wrappers
def gx_exp_tables():
    hi = (C.c_uint32 * 16)()
    lo = (C.c_uint32 * 256)()
    _check(None, lib().gx_exp_tables(hi, lo))
    return np.array(list(hi), np.uint32), np.array(list(lo), np.uint32)


GX_CHECK_PHILOX, GX_CHECK_DIST, GX_CHECK_ACCEPT = 1, 2, 3
_CHECK_WIDTH = {GX_CHECK_PHILOX: (2, 4), GX_CHECK_DIST: (1, 2), GX_CHECK_ACCEPT: (2, 1)}


def gx_device_check(ctx, what: int, inputs, key: int = 0) -> np.ndarray:
    """Device arithmetic on `inputs` (uint64, `in` words per element as in
    include/gx.h); returns the (count, out words) uint64 results."""
    w_in, w_out = _CHECK_WIDTH[what]
    x = np.ascontiguousarray(inputs, dtype=np.uint64).reshape(-1, w_in)
    out = np.zeros((len(x), w_out), np.uint64)
    _check(ctx, lib().gx_device_check(ctx, what, key & 0xFFFFFFFFFFFFFFFF, x.ctypes.data, out.ctypes.data, len(x)))
    return out


def gx_measure_peaks(ctx) -> dict:
    """Measured device ceilings (include/gx.h, gx_measure_peaks)."""
    r = gx_peaks()
    _check(ctx, lib().gx_measure_peaks(ctx, C.byref(r)))
    return {k: getattr(r, k) for k, _ in gx_peaks._fields_ if k != "pad_"}


def gx_create(device: int = 0, stream=None):
    """Context on `device`; `stream` is a hipStream_t handle (int) or a
    torch.cuda.Stream, or None for a stream the context owns."""
    if stream is not None and not isinstance(stream, int):
        stream = int(stream.cuda_stream)
    out = C.c_void_p()
    st = lib().gx_create(device, C.c_void_p(stream or None), C.byref(out))
    if st != GX_OK:
        raise GxError(st, "gx_create failed (no usable gfx950 device?)")
    return out


def gx_destroy(ctx):
    _check(None, lib().gx_destroy(ctx))


def gx_last_error(ctx) -> str:
    return lib().gx_last_error(ctx).decode()


def gx_get_device_info(ctx) -> dict:
    info = gx_device_info()
    _check(ctx, lib().gx_get_device_info(ctx, C.byref(info)))
    return {"cus": info.cus, "lds_per_block": info.lds_per_block, "wave_size": info.wave_size,
            "l2_bytes": info.l2_bytes, "arch": info.arch.decode()}


def _desc(inst, keep):
    """gx_instance_desc from an object with the fields of include/gx.h (kind, n, a, b, ...).
    Arrays may be numpy (host) or torch tensors (host or device)."""
    def ptr(x):
        if x is None:
            return None, 0
        if hasattr(x, "data_ptr"):          # torch tensor
            import torch
            t = x.to(torch.int32).contiguous()
            keep.append(t)
            return t.data_ptr(), int(t.is_cuda)
        arr = np.ascontiguousarray(x, dtype=np.int32)
        keep.append(arr)
        return arr.ctypes.data, 0
    pa, da = ptr(inst.a)
    pb, db = ptr(getattr(inst, "b", None))
    if pb is not None and db != da:
        raise ValueError("arrays a and b must both be host or both be device memory")
    return gx_instance_desc(kind=inst.kind, n=inst.n, is_device_ptr=da, a=pa, b=pb,
                            a_is_coords=getattr(inst, "a_is_coords", 0),
                            capacity=getattr(inst, "capacity", 0), vehicles=getattr(inst, "vehicles", 0),
                            service_time=getattr(inst, "service_time", 0),
                            horizon=getattr(inst, "horizon", 0), lb=getattr(inst, "lb", 0),
                            ub=getattr(inst, "ub", 0), n_edges=getattr(inst, "n_edges", 0),
                            instance_key=getattr(inst, "key", 0) & 0xFFFFFFFF,
                            obj_weights=(C.c_int32 * 3)(*getattr(inst, "obj_weights", (0, 0, 0))),
                            lex_order=(C.c_int32 * 3)(*getattr(inst, "lex_order", (0, 0, 0))),
                            lex_tol=(C.c_int32 * 3)(*getattr(inst, "lex_tol", (0, 0, 0))))


def gx_instance_upload(ctx, inst):
    keep = []
    d = _desc(inst, keep)
    out = C.c_void_p()
    _check(ctx, lib().gx_instance_upload(ctx, C.byref(d), C.byref(out)))
    return out


def gx_instance_free(ctx, inst):
    _check(ctx, lib().gx_instance_free(ctx, inst))


def _params(p) -> gx_solve_params:
    return gx_solve_params(seed=p.seed & 0xFFFFFFFFFFFFFFFF, generations=p.generations,
                           population=p.population, candidates=p.candidates, op_mask=p.op_mask,
                           t0_q16=p.t0_q16, alpha_q32=p.alpha_q32, aos_epoch=p.epoch,
                           aos_alpha_q16=p.aos_alpha_q16, w_floor_q16=p.w_floor_q16,
                           stagnation_epochs=p.stagnation_epochs, aos_credit=p.credit,
                           oversample_k=p.oversample_k, staging=getattr(p, "staging", 0),
                           islands=getattr(p, "islands", 0), migrate_epochs=getattr(p, "migrate_epochs", 0),
                           migrate_mode=getattr(p, "migrate_mode", 0), migrate_n=getattr(p, "migrate_n", 0),
                           elite_epochs=getattr(p, "elite_epochs", 0), aos_scope=getattr(p, "aos_scope", 0),
                           init_weight_q16=(C.c_uint32 * N_OPS)(*_init_w(p)),
                           weight_cap_q16=(C.c_uint32 * N_OPS)(*_per_op(p, "weight_cap_q16")))


def _per_op(p, name):
    w = [int(x) for x in (getattr(p, name, ()) or ())]
    if len(w) > N_OPS:
        raise ValueError(f"at most {N_OPS} entries in {name}")
    return w + [0] * (N_OPS - len(w))


def _init_w(p):
    return _per_op(p, "init_weight_q16")


def gx_autosize_population(ctx, inst, params) -> int:
    out = C.c_uint32()
    pp = _params(params)
    _check(ctx, lib().gx_autosize_population(ctx, inst, C.byref(pp), C.byref(out)))
    return int(out.value)


def gx_job_create(ctx, inst, params):
    out = C.c_void_p()
    pp = _params(params)
    _check(ctx, lib().gx_job_create(ctx, inst, C.byref(pp), C.byref(out)))
    return out


def gx_job_advance(ctx, job, n_generations: int):
    _check(ctx, lib().gx_job_advance(ctx, job, n_generations))


def gx_solve(ctx, inst, params):
    out = C.c_void_p()
    pp = _params(params)
    _check(ctx, lib().gx_solve(ctx, inst, C.byref(pp), C.byref(out)))
    return out


def gx_solve_static(ctx, inst, params, best_solution, best_objective):
    """Solve into caller-owned device buffers without allocating: best_solution
    (n int32) and best_objective (one int64) are device pointers (ints) or
    torch tensors on the context's device.  Asynchronous on the context's stream."""
    def dptr(x):
        return int(x.data_ptr()) if hasattr(x, "data_ptr") else int(x)
    pp = _params(params)
    _check(ctx, lib().gx_solve_static(ctx, inst, C.byref(pp), C.c_void_p(dptr(best_solution)),
                                      C.c_void_p(dptr(best_objective))))


def gx_wait(ctx, job=None):
    _check(ctx, lib().gx_wait(ctx, job))


def gx_poll(ctx, job=None) -> bool:
    st = lib().gx_poll(ctx, job)
    if st == GX_E_NOT_READY:
        return False
    _check(ctx, st)
    return True


def gx_fetch_best(ctx, job, n: int):
    sol = np.zeros(n, np.int32)
    f = C.c_int64()
    _check(ctx, lib().gx_fetch_best(ctx, job, sol.ctypes.data, n, C.byref(f)))
    return sol, int(f.value)


def gx_portfolio_best(ctx, jobs, n: int):
    arr = (C.c_void_p * len(jobs))(*[j.value if isinstance(j, C.c_void_p) else j for j in jobs])
    sol = np.zeros(n, np.int32)
    f, i = C.c_int64(), C.c_int32()
    _check(ctx, lib().gx_portfolio_best(ctx, C.cast(arr, C.POINTER(C.c_void_p)), len(jobs), sol.ctypes.data, n,
                                        C.byref(f), C.byref(i)))
    return sol, int(f.value), int(i.value)


def gx_job_info_get(ctx, job) -> dict:
    i = gx_job_info()
    _check(ctx, lib().gx_job_info_get(ctx, job, C.byref(i)))
    out = {k: getattr(i, k) for k, _ in gx_job_info._fields_}
    out["op_steps"] = [int(x) for x in i.op_steps]
    out["k_count"] = [int(x) for x in i.k_count]
    return out


def gx_job_stats(ctx, job) -> dict:
    r = gx_run_stats()
    _check(ctx, lib().gx_job_stats(ctx, job, C.byref(r)))
    return {"move_evals": int(r.move_evals), "accepted": int(r.accepted),
            "u_op": np.array(list(r.u_op), np.uint64), "v_op": np.array(list(r.v_op), np.uint64),
            "u_k": np.array(list(r.u_k), np.uint64), "v_k": np.array(list(r.v_k), np.uint64),
            "generations_done": int(r.generations_done), "population": int(r.population)}


def gx_job_population(ctx, job) -> int:
    out = C.c_uint32()
    _check(ctx, lib().gx_job_population(ctx, job, C.byref(out)))
    return int(out.value)


def gx_snapshot_aos(ctx, job, P: int) -> np.ndarray:
    """The P per-solution AOS records (numpy array of SOL_AOS)."""
    out = np.zeros(P, SOL_AOS)
    _check(ctx, lib().gx_snapshot_aos(ctx, job, out.ctypes.data))
    return out


def gx_snapshot_lex(ctx, job, P: int) -> dict:
    """Objective vectors of a job in the VRPTW lexicographic mode: "cur_v" and
    "best_v" (P x 4 int64), "ref_v" (4 int64)."""
    cur_v = np.zeros((P, 4), np.int64)
    best_v = np.zeros((P, 4), np.int64)
    ref_v = np.zeros(4, np.int64)
    _check(ctx, lib().gx_snapshot_lex(ctx, job, cur_v.ctypes.data, best_v.ctypes.data, ref_v.ctypes.data))
    return {"cur_v": cur_v, "best_v": best_v, "ref_v": ref_v}


def gx_job_restore(ctx, job, st: dict):
    """Overwrite a job's state with ``st`` (the dict gx_snapshot returns, plus
    "saos" records for per-solution weights)."""
    sc = gx_state_scalars(g=st["g"], stag=st["stag"], T_q16=st["T_q16"], epoch_ref=st["epoch_ref"],
                          accepted=st["accepted"])
    for name in ("w_op", "w_k", "u_op", "v_op", "u_k", "v_k"):
        arr = getattr(sc, name)
        for i, v in enumerate(st[name]):
            arr[i] = int(v)
    cur = np.ascontiguousarray(st["cur"], np.int32)
    best = np.ascontiguousarray(st["best"], np.int32)
    cur_f = np.ascontiguousarray(st["cur_f"], np.int64)
    best_f = np.ascontiguousarray(st["best_f"], np.int64)
    aos = st.get("saos")
    aos = None if aos is None else np.ascontiguousarray(aos, SOL_AOS)
    _check(ctx, lib().gx_job_restore(ctx, job, C.byref(sc), cur.ctypes.data, cur_f.ctypes.data, best.ctypes.data,
                                     best_f.ctypes.data, None if aos is None else aos.ctypes.data))


def gx_snapshot(ctx, job, P: int, n: int) -> dict:
    """Job state in the oracle's state layout (dict of numpy arrays and ints)."""
    sc = gx_state_scalars()
    cur = np.zeros((P, n), np.int32)
    best = np.zeros((P, n), np.int32)
    cur_f = np.zeros(P, np.int64)
    best_f = np.zeros(P, np.int64)
    _check(ctx, lib().gx_snapshot(ctx, job, C.byref(sc), cur.ctypes.data, cur_f.ctypes.data,
                                  best.ctypes.data, best_f.ctypes.data))
    return {"g": int(sc.g), "stag": int(sc.stag), "T_q16": int(sc.T_q16),
            "epoch_ref": int(sc.epoch_ref), "accepted": int(sc.accepted),
            "w_op": np.array(list(sc.w_op), np.uint32), "w_k": np.array(list(sc.w_k), np.uint32),
            "u_op": np.array(list(sc.u_op), np.uint64), "v_op": np.array(list(sc.v_op), np.uint64),
            "u_k": np.array(list(sc.u_k), np.uint64), "v_k": np.array(list(sc.v_k), np.uint64),
            "cur": cur, "cur_f": cur_f, "best": best, "best_f": best_f}


def gx_job_free(ctx, job):
    _check(ctx, lib().gx_job_free(ctx, job))


def gx_solve_batch(ctx, insts, params_list):
    count = len(insts)
    arr = (C.c_void_p * count)(*[i.value if isinstance(i, C.c_void_p) else i for i in insts])
    pars = (gx_solve_params * count)(*[_params(p) for p in params_list])
    jobs = (C.c_void_p * count)()
    _check(ctx, lib().gx_solve_batch(ctx, C.cast(arr, C.POINTER(C.c_void_p)), pars, count,
                                     C.cast(jobs, C.POINTER(C.c_void_p))))
    return [C.c_void_p(j) for j in jobs]


# ------------------------------------------------------------------ serving
def gx_server_create(ctx, hbm_budget_bytes=0, max_resident=0, max_lds_bytes=0, max_items=0, quantum_epochs=0):
    cfg = gx_server_cfg(hbm_budget_bytes=hbm_budget_bytes, max_resident=max_resident,
                        max_lds_bytes=max_lds_bytes, max_items=max_items, quantum_epochs=quantum_epochs)
    out = C.c_void_p()
    _check(ctx, lib().gx_server_create(ctx, C.byref(cfg), C.byref(out)))
    return out


def gx_server_submit(srv, inst, params) -> int:
    """Thread-safe; returns the ticket.  Raises GxError on a rejected request."""
    keep = []
    d = _desc(inst, keep)
    pp = _params(params)
    t = C.c_uint64()
    st = lib().gx_server_submit(srv, C.byref(d), C.byref(pp), C.byref(t))
    if st != GX_OK:
        raise GxError(st, "request rejected")
    return int(t.value)


def gx_server_poll(srv, ticket: int, n: int):
    """None while not ready; otherwise (solution, objective, t_submit_ns, t_done_ns).
    Raises GxError(GX_E_CANCELLED) for a cancelled request."""
    sol = np.zeros(n, np.int32)
    f, ts, td = C.c_int64(), C.c_uint64(), C.c_uint64()
    st = lib().gx_server_poll(srv, ticket, sol.ctypes.data, n, C.byref(f), C.byref(ts), C.byref(td))
    if st == GX_E_NOT_READY:
        return None
    if st != GX_OK:
        raise GxError(st, f"ticket {ticket}")
    return sol, int(f.value), int(ts.value), int(td.value)


def gx_server_cancel(srv, ticket: int):
    st = lib().gx_server_cancel(srv, ticket)
    if st != GX_OK:
        raise GxError(st, f"ticket {ticket}")


def gx_server_stats_get(srv) -> dict:
    s = gx_server_stats()
    st = lib().gx_server_stats_get(srv, C.byref(s))
    if st != GX_OK:
        raise GxError(st, "stats")
    return {k: getattr(s, k) for k, _ in gx_server_stats._fields_}


def gx_server_destroy(srv):
    st = lib().gx_server_destroy(srv)
    if st != GX_OK:
        raise GxError(st, "destroy")
