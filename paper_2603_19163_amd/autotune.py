"""Launch-schedule autotuner.

Picks, per size bucket, the knobs that do not change results (TSP distance
staging) by timing short runs of the evolve kernels on the device, and sizes
the population of a batch so that the batch fills the GPU.  Choices that would
change a trajectory (P, C) are never made silently: they are returned and
recorded by the caller.  Timings come from the library's own HIP events
(gx_job_info.evolve_ms), so nothing here depends on host timers.
"""
from __future__ import annotations

import json
import os

from . import gx

STAGES_TSP = (gx.STAGE_LDS_D16, gx.STAGE_LDS_XY, gx.STAGE_GLB_D16, gx.STAGE_GLB_D32)
_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_autotune_cache.json")


def _rate(ctx, inst_handle, params, generations):
    """Move evaluations per second of the evolve launches for `generations`."""
    job = gx.gx_job_create(ctx, inst_handle, params)
    try:
        gx.gx_job_advance(ctx, job, generations)
        info = gx.gx_job_info_get(ctx, job)
        return params.population * params.candidates * generations / (info["evolve_ms"] / 1e3)
    finally:
        gx.gx_job_free(ctx, job)


def tune_tsp_staging(ctx, inst, params, generations: int = 200, stages=STAGES_TSP, population: int = 0,
                     repeats: int = 2):
    """Time every TSP staging the instance supports with the device full of
    this instance's workgroups (population, default 20 per CU: a batch or a
    server keeps the device that full, and a staging's LDS footprint decides
    how many workgroups a CU holds); each staging keeps the best of `repeats`
    passes taken round-robin over the stagings, so that one slow pass (a
    first launch, a clock change) does not decide.  Returns (best stage,
    {stage: evals/s})."""
    h = gx.gx_instance_upload(ctx, inst)
    table = {}
    P = population or 20 * gx.gx_get_device_info(ctx)["cus"]
    try:
        for _ in range(repeats):
            for st in stages:
                p = params.with_(staging=st, generations=generations, population=P)
                try:
                    r = _rate(ctx, h, p, generations)
                except gx.GxError as e:
                    if e.status != gx.GX_E_UNSUPPORTED:
                        raise
                    continue
                table[st] = max(table.get(st, 0.0), r)
    finally:
        gx.gx_instance_free(ctx, h)
    best = max(table, key=table.get)
    return best, table


def bucket_of(kind: int, n: int) -> str:
    edges = (32, 64, 96, 128, 192, 256, 384, 512, 768, 1024)
    for e in edges:
        if n <= e:
            return f"{kind}:{e}"
    return f"{kind}:big"


def tune_buckets(ctx, samples, params_for, generations: int = 200, cache: bool = True):
    """samples: {bucket: representative instance}; params_for(inst) -> Params.
    Returns {bucket: staging} for TSP buckets (other kinds have one staging)."""
    known = {}
    if cache and os.path.exists(_CACHE):
        with open(_CACHE) as fh:
            known = json.load(fh)
    dev = gx.gx_get_device_info(ctx)["arch"]
    out = {}
    for b, inst in samples.items():
        key = f"{dev}|{b}"
        if inst.kind != 1:
            out[b] = 0
            continue
        if key in known:
            out[b] = known[key]
            continue
        best, _ = tune_tsp_staging(ctx, inst, params_for(inst), generations)
        out[b] = known[key] = best
    if cache:
        with open(_CACHE, "w") as fh:
            json.dump(known, fh, indent=1)
    return out


def fill_population(ctx, count: int, blocks_per_cu: int = 20, p_min: int = 1, p_max: int = 64) -> int:
    """Population per instance so that `count` instances fill the device with
    about `blocks_per_cu` resident 64-lane workgroups per CU (the evolve
    kernels hold 20 per CU at their register and LDS use)."""
    cus = gx.gx_get_device_info(ctx)["cus"]
    want = cus * blocks_per_cu
    p = max(p_min, min(p_max, (want + count - 1) // count))
    return p
