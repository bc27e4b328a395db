"""Launch-schedule autotuner.

Picks, per (kind, size) bucket, the knobs that do not change results (TSP
distance staging) and the population of every instance of a batch, by timing
short runs of the evolve kernels on the device.  Choices that change a
trajectory (P) are never made silently: they are returned and recorded by the
caller.  Timings come from the library's own HIP events (gx_job_info.evolve_ms),
so nothing here depends on host timers.  Measurements are cached per device
architecture and kernel source (SHA-256 of the HIP sources), so a changed
kernel is timed again.
"""
from __future__ import annotations

import glob
import hashlib
import json
import math
import os

from . import gx

STAGES_TSP = (gx.STAGE_LDS_D16, gx.STAGE_LDS_XY, gx.STAGE_GLB_D16, gx.STAGE_GLB_D32)
_HERE = os.path.dirname(os.path.abspath(__file__))
_CACHE = os.path.join(_HERE, "_autotune_cache.json")


def kernel_source_hash() -> str:
    """SHA-256 over the HIP sources the library is built from."""
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(_HERE, "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def _load_cache() -> dict:
    try:
        with open(_CACHE) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _save_cache(known: dict):
    tmp = _CACHE + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(known, fh, indent=1)
    os.replace(tmp, _CACHE)


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
    known = _load_cache() if cache else {}
    dev = gx.gx_get_device_info(ctx)["arch"]
    src = kernel_source_hash()
    out = {}
    for b, inst in samples.items():
        key = f"staging|{dev}|{src}|{b}"
        if inst.kind != 1:
            out[b] = 0
            continue
        if key in known:
            out[b] = known[key]
            continue
        best, _ = tune_tsp_staging(ctx, inst, params_for(inst), generations)
        out[b] = known[key] = best
    if cache:
        _save_cache(known)
    return out


def bucket_costs(ctx, samples, params_for, generations: int = 100, cache: bool = True):
    """Device time of one solution-generation per bucket: each bucket's
    representative instance run with the device full of its workgroups
    (20 per CU), timed by the library's events, best of two passes.
    samples: {bucket: instance}; params_for(inst) -> Params (its staging and
    operator set).  Returns {bucket: seconds per solution-generation}."""
    known = _load_cache() if cache else {}
    dev = gx.gx_get_device_info(ctx)
    src = kernel_source_hash()
    P = 20 * dev["cus"]
    out = {}
    for b, inst in samples.items():
        key = f"cost|{dev['arch']}|{src}|{b}"
        if key not in known:
            h = gx.gx_instance_upload(ctx, inst)
            try:
                p = params_for(inst).with_(population=P, generations=generations)
                best = max(_rate(ctx, h, p, generations) for _ in range(2))
            finally:
                gx.gx_instance_free(ctx, h)
            known[key] = p.candidates / best   # seconds per solution-generation at full occupancy
        out[b] = known[key]
    if cache:
        _save_cache(known)
    return out


def plan_populations(counts, costs, total: int, p_min: int = 1, p_max: int = 64):
    """Population per bucket for a batch: every instance gets about the same
    device time per generation (P_b proportional to 1 / cost_b) and the batch
    holds about `total` solutions; P_b is rounded to the nearest power of two
    in log space and clamped to [p_min, p_max].
    counts: {bucket: instances}; costs: {bucket: seconds per
    solution-generation}.  Returns {bucket: P}."""
    k = total / sum(c / costs[b] for b, c in counts.items())
    out = {}
    for b in counts:
        ideal = max(k / costs[b], 1e-9)
        p = 2 ** round(math.log2(ideal))
        out[b] = int(min(p_max, max(p_min, p)))
    return out


def fill_population(ctx, count: int, blocks_per_cu: int = 20, p_min: int = 1, p_max: int = 64) -> int:
    """Population per instance so that `count` instances fill the device with
    about `blocks_per_cu` resident 64-lane workgroups per CU (the evolve
    kernels hold 20 per CU at their register and LDS use)."""
    cus = gx.gx_get_device_info(ctx)["cus"]
    want = cus * blocks_per_cu
    p = max(p_min, min(p_max, (want + count - 1) // count))
    return p


def tune_batch(ctx, insts, make_params, rule: str = "tuned", blocks_per_cu: int = 20):
    """Parameters of a batch: per bucket the fastest TSP staging and the
    population, by `rule`: "fill" gives every instance the population that
    fills the device (fill_population); "tuned" spreads the same total number
    of solutions over the buckets by their measured cost (plan_populations).
    make_params(inst, index, population, staging) -> Params.  Returns
    (params per instance, {bucket: {"instances", "population", "staging",
    "cost_s"}})."""
    if rule not in ("fill", "tuned"):
        raise ValueError(f"unknown population rule {rule!r}")
    samples, counts = {}, {}
    for inst in insts:
        b = bucket_of(inst.kind, inst.n)
        samples.setdefault(b, inst)
        counts[b] = counts.get(b, 0) + 1
    p_fill = fill_population(ctx, len(insts), blocks_per_cu)
    staging = tune_buckets(ctx, samples, lambda i: make_params(i, 0, p_fill, 0))
    costs = {}
    if rule == "fill":
        pops = {b: p_fill for b in counts}
    else:
        costs = bucket_costs(ctx, samples,
                             lambda i: make_params(i, 0, p_fill, staging[bucket_of(i.kind, i.n)]))
        pops = plan_populations(counts, costs, p_fill * len(insts))
    params = []
    for i, inst in enumerate(insts):
        b = bucket_of(inst.kind, inst.n)
        params.append(make_params(inst, i, pops[b], staging[b]))
    plan = {b: {"instances": counts[b], "population": pops[b], "staging": staging[b], "cost_s": costs.get(b)}
            for b in sorted(counts)}
    return params, plan
