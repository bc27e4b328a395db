"""Benchmark: move evaluations per second of the population-parallel local
search on a 442-city clustered TSP, on one MI355X.

One step = one whole solve through the C interface: initialisation
(oversampled pool, heuristics, selection), all generations (sampling, delta
evaluation, argmin, acceptance, application, AOS statistics and epoch weight
updates, cooling) and the fetch of the best tour.  The instance is uploaded to
HBM before the timed region.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps 3] [--warmup 1] [--generations 200000]
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "move evals/s on 442-node TSP; mixed-stream solves/s + p50/p99 vs plain"

# LDS bytes one operator step reads during delta evaluation, per staging of the
# distances: tour entries are 2 bytes; a distance is one int16 matrix entry
# (LDS_D16) or two 8-byte coordinate pairs (LDS_XY); for GLB_* the distances
# come through L2 and only the tour is LDS traffic.
#   2-opt: 4 tour + 4 distances; swap: 6 tour + 8 distances;
#   insert / or-opt: 6 tour + 6 distances.
_TOUR = {0: 4, 1: 6, 2: 6, 3: 6}
_DIST = {0: 4, 1: 8, 2: 6, 3: 6}
_DIST_BYTES = {1: 2, 2: 16, 3: 0, 4: 0}
STAGE_NAMES = {1: "int16 distances in LDS", 2: "coordinates in LDS, exact distance recomputed",
               3: "int16 distances through L2", 4: "int32 distances through L2"}

LDS_PEAK_GBS = 256 * 128 * 2.4   # 256 CUs x 128 B/clk x 2.4 GHz = 78,643 GB/s
# 32-bit vector ALU: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39,322 G lane-ops/s
ALU_PEAK_GOPS = 256 * 4 * 16 * 2.4

# Algorithmic integer/float operations (per lane) of one move evaluation:
#   per operator step: one Philox4x32-10 block (10 rounds x (2 widening multiplies
#   + 4 xors) = 60), sampling of the operator and its positions (12), and the
#   delta: per distance 14 ops for the exact recomputation from coordinates
#   (2 sub, 2 mul, add, shift, 2 convert, sqrt, 2 x (mul, compare), add+shift)
#   or 1 (address) for a stored matrix, plus one add per distance and one
#   address per tour read;
#   per candidate: k choice 3, key and running min 4.
_PHILOX_OPS, _SAMPLE_OPS, _CAND_OPS = 60, 12, 7
_DIST_OPS = {1: 1, 2: 14, 3: 1, 4: 1}


def lds_bytes(op_steps, stage):
    return sum(op_steps[o] * (2 * _TOUR[o] + _DIST_BYTES[stage] * _DIST[o]) for o in range(4))


def alu_ops(op_steps, evals, stage):
    per_step = {o: _PHILOX_OPS + _SAMPLE_OPS + _DIST[o] * (_DIST_OPS[stage] + 1) + _TOUR[o] for o in range(4)}
    return sum(op_steps[o] * per_step[o] for o in range(4)) + _CAND_OPS * evals


def measured_traffic(path=os.path.join(ROOT, "profiles", "k_evolve_tsp442_traffic.md")):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel source (else None)."""
    import hashlib
    src = os.path.join(ROOT, "paper_2603_19163_amd", "csrc", "gx_kernels.hip")
    try:
        with open(path) as fh:
            lines = dict(l.strip().split(": ", 1) for l in fh if ": " in l and l.startswith("- "))
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
        if lines.get("- kernel_source_sha256") != sha:
            return None
        return float(lines["- hbm_bytes_per_launch"]), int(lines["- population"])
    except (OSError, KeyError, ValueError):
        return None


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(inst, params, seconds: float):
    """The oracle as it stands on a bounded sample: the full population of
    the same solve from its initial state for as many generations as fit in
    about seconds / 2 on one thread, then the same generations from the same
    state on all host threads (at most 16, the host share of one GPU), whose
    result must equal the one-thread run's bit for bit.  `value` is the
    all-thread rate, `single_core` the one-thread rate."""
    import numpy as np
    import oracle
    o = oracle.OracleInstance(inst)
    st0 = o.init(params)

    def copy(st):
        return {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in st.items()}
    probe = copy(st0)
    t = time.perf_counter()
    o.run(params, probe, 1)
    t1 = time.perf_counter() - t
    g = max(1, int(seconds / 2 / max(t1, 1e-6)))
    one = copy(st0)
    t = time.perf_counter()
    o.run(params, one, g)
    dt1 = time.perf_counter() - t
    threads = max(1, min(16, os.cpu_count() or 1))
    many = copy(st0)
    t = time.perf_counter()
    o.run(params, many, g, threads=threads)
    dtn = time.perf_counter() - t
    same = all(np.array_equal(np.asarray(one[k]), np.asarray(many[k])) for k in one)
    evals = params.population * params.candidates * g
    return {"value": evals / dtn, "unit": "move evals/s", "cores": threads, "kind": "oracle",
            "single_core": evals / dt1, "nproc": os.cpu_count(), "cpu_model": _cpu_model(),
            "threads_equal_one_thread": bool(same),
            "sample": f"same instance and population P={params.population}, C={params.candidates}, "
                      f"generations 0..{g} of the solve from its initial state ({evals} move evals), once on "
                      f"one thread ({dt1:.1f} s) and once on {threads} threads ({dtn:.1f} s); "
                      f"full-recompute objective per candidate"}


def bench_peaks(args):
    """Measured device ceilings (gx_measure_peaks) beside the nominal ones."""
    import torch
    from paper_2603_19163_amd import gx
    ctx = gx.gx_create(0, torch.cuda.Stream())
    pk = gx.gx_measure_peaks(ctx)
    gx.gx_destroy(ctx)
    return {"metric": "device ceilings", "measured": pk,
            "nominal": {"hbm_read_bytes_per_s": 8e12, "valu_lane_ops_per_s_1_per_clk": ALU_PEAK_GOPS * 1e9,
                        "lds_bytes_per_s_128B_per_clk": LDS_PEAK_GBS * 1e9}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--generations", type=int, default=200_000)
    ap.add_argument("--population", type=int, default=0, help="0: autosized")
    ap.add_argument("--staging", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-peaks", action="store_true",
                    help="tsp442: skip the device-ceiling microbenchmarks after the timed region")
    ap.add_argument("--workload", choices=["tsp442", "batched", "served", "kinds", "peaks"], default="tsp442",
                    help="tsp442: the benchmark line; batched / served: the systems patterns; "
                         "kinds: one solve per encoding, operator set and island setting")
    ap.add_argument("--instances", type=int, default=4096, help="batched: number of instances")
    ap.add_argument("--batch-generations", type=int, default=5000)
    ap.add_argument("--population-rule", choices=["tuned", "fill"], default="tuned",
                    help="batched: population per size bucket from measured costs (tuned) or the same "
                         "device-filling population for every instance (fill)")
    ap.add_argument("--plain-sample", type=int, default=32, help="batched/served: requests solved alone")
    ap.add_argument("--rate", type=float, default=2000.0, help="served: offered requests/s")
    ap.add_argument("--duration", type=float, default=10.0, help="served: seconds of arrivals")
    ap.add_argument("--served-generations", type=int, default=10000)
    ap.add_argument("--served-population", type=int, default=4)
    ap.add_argument("--served-kinds", default="tsp,qap,knapsack",
                    help="served: request kinds drawn uniformly (subset of tsp,qap,knapsack)")
    ap.add_argument("--no-mixed", action="store_true",
                    help="tsp442: skip the batched and served measurements appended to the line")
    ap.add_argument("--sustained-rate", type=float, default=800.0,
                    help="tsp442: offered rate of the second served measurement (below capacity)")
    ap.add_argument("--mixed-duration", type=float, default=3.0,
                    help="tsp442: seconds of served arrivals measured for the line")
    ap.add_argument("--kinds-rows", default="",
                    help="kinds: comma-separated row names to run (default: all)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n}))
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; "
                          "instances and requests shard across GPUs without exchange, "
                          "so N > 1 is not measured here"}))
        sys.exit(2)

    if args.workload == "batched":
        print(json.dumps(bench_batched(args)), flush=True)
        return
    if args.workload == "served":
        print(json.dumps(bench_served(args)), flush=True)
        return
    if args.workload == "kinds":
        print(json.dumps(bench_kinds(args)), flush=True)
        return
    if args.workload == "peaks":
        print(json.dumps(bench_peaks(args)), flush=True)
        return

    import torch
    import synth
    from paper_2603_19163_amd import gx

    inst, p = synth.c2_tsp442(population=0, generations=args.generations)
    p = p.with_(staging=args.staging)
    stream = torch.cuda.Stream()
    ctx = gx.gx_create(0, stream)
    dev = gx.gx_get_device_info(ctx)
    h = gx.gx_instance_upload(ctx, inst)
    P = args.population or gx.gx_autosize_population(ctx, h, p)
    p = p.with_(population=P)

    def step():
        job = gx.gx_solve(ctx, h, p)
        sol, f = gx.gx_fetch_best(ctx, job, inst.n)
        info = gx.gx_job_info_get(ctx, job)
        gx.gx_job_free(ctx, job)
        return f, info

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos, best = [], None
    for _ in range(args.steps):
        best, info = step()
        infos.append(info)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    evals = sum(i["move_evals"] for i in infos)
    value = evals / dt
    # the instance handed over in host buffers: upload (coordinates over PCIe,
    # device-side preparation) timed on its own, added once per solve
    up = []
    for _ in range(5):
        torch.cuda.synchronize()
        t = time.perf_counter()
        h2 = gx.gx_instance_upload(ctx, inst)
        torch.cuda.synchronize()
        up.append(time.perf_counter() - t)
        gx.gx_instance_free(ctx, h2)
    upload_s = sorted(up)[len(up) // 2]
    stage = infos[-1]["staging"]
    launches = sum(i["evolve_launches"] for i in infos)
    ev_ms = sum(i["evolve_ms"] for i in infos)
    avg_launch_s = ev_ms / 1e3 / launches
    bytes_total = sum(lds_bytes(i["op_steps"], stage) for i in infos)
    lds_achieved = bytes_total / launches / avg_launch_s / 1e9
    ops_total = sum(alu_ops(i["op_steps"], i["move_evals"], stage) for i in infos)
    achieved = ops_total / launches / avg_launch_s / 1e9
    tr = measured_traffic()
    traffic = tr[0] if tr and tr[1] == P else None
    # device ceilings measured on this device after the timed region
    # (gx_measure_peaks: random LDS gather, full-rate VALU issue, Philox, L2 gather, HBM read)
    pk = None if args.no_peaks else gx.gx_measure_peaks(ctx)
    k_tot = [sum(i["k_count"][k] for i in infos) for k in range(3)]
    steps_per_eval = sum((k + 1) * k_tot[k] for k in range(3)) / max(1, sum(k_tot))
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "move evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {
            "workload": f"TSP n=442, 20 Gaussian clusters (sigma 300) in [0,10000]^2; population "
                        f"P={P} (autosized, one 64-lane workgroup each), C=128 candidates, "
                        f"{args.generations} generations, ops 2-opt/swap/insert/or-opt, "
                        f"AOS epoch 10; {STAGE_NAMES.get(stage, stage)}",
            "population": P, "candidates": p.candidates, "generations": args.generations,
            "staging": stage, "device": dev["arch"], "cus": dev["cus"],
            "best_tour": best, "op_steps_per_eval": round(steps_per_eval, 4),
        },
        "roofline": {
            "bound": "alu",
            "kernel": "k_evolve<TSP>",
            "achieved": achieved,
            "peak": ALU_PEAK_GOPS,
            "unit": "G lane-ops/s",
            "frac": achieved / ALU_PEAK_GOPS,
            "traffic": traffic,
            "avg_launch_ms": avg_launch_s * 1e3,
            "launches": launches,
            "algorithmic_ops_per_launch": ops_total / launches,
            "peak_measured": pk["valu_instr_per_s"] / 1e9 if pk else None,
            "frac_measured": achieved / (pk["valu_instr_per_s"] / 1e9) if pk else None,
        },
        "roofline_lds": {
            "achieved": lds_achieved, "peak": LDS_PEAK_GBS, "unit": "GB/s",
            "frac": lds_achieved / LDS_PEAK_GBS, "algorithmic_bytes_per_launch": bytes_total / launches,
            "peak_measured": pk["lds_gather_bytes_per_s"] / 1e9 if pk else None,
            "frac_measured": lds_achieved / (pk["lds_gather_bytes_per_s"] / 1e9) if pk else None,
        },
        "peaks_measured": pk,
        "pcie_inclusive": {"upload_s": upload_s, "value": evals / (dt + args.steps * upload_s),
                           "note": "instance uploaded from host buffers once per solve"},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(inst, p, args.cpu_seconds)
    gx.gx_instance_free(ctx, h)
    gx.gx_destroy(ctx)
    if not args.no_mixed:
        # the second half of the metric: the batched configuration (4096
        # instances) and the served stream (2000 requests/s, a shorter window),
        # each against the plain solver on a sample of the same requests
        mixed = argparse.Namespace(**vars(args))
        mixed.plain_sample = 8
        mixed.duration = args.mixed_duration
        line["batched"] = bench_batched(mixed)
        line["mixed_stream"] = bench_served(mixed)
        # the same stream at a rate this device sustains for the mix, so that
        # p50/p99 show service time rather than a growing backlog
        sustained = argparse.Namespace(**vars(mixed))
        sustained.rate = args.sustained_rate
        line["mixed_stream_sustained"] = bench_served(sustained)
    print(json.dumps(line), flush=True)


def _pct(v, q):
    import numpy as np
    return float(np.percentile(np.asarray(v), q)) if len(v) else None


def bench_batched(args):
    """Batched pattern: TSP n U[20,200] (3/4) and QAP n U[12,40] (1/4) in one
    gx_solve_batch (persistent fused launch per epoch, graph-replayed), against
    the plain solver on a sample of the same instances."""
    import numpy as np
    import torch
    import synth
    from paper_2603_19163_amd import autotune, gx

    ctx = gx.gx_create(0, torch.cuda.Stream())
    cus = gx.gx_get_device_info(ctx)["cus"]
    count, G = args.instances, args.batch_generations
    n_tsp = count * 3 // 4
    insts = synth.c4_batched_instances(count)
    params, plan = autotune.tune_batch(ctx, insts, synth.c4_params_for(G), rule=args.population_rule)
    handles = [gx.gx_instance_upload(ctx, i) for i in insts]
    # one untimed batch of the same shape first (first-call costs of the
    # runtime: code-object loading, graph instantiation, allocator growth)
    warm = [p.with_(generations=min(G, 100)) for p in params]
    for j in gx.gx_solve_batch(ctx, handles, warm):
        gx.gx_wait(ctx, j)
        gx.gx_job_free(ctx, j)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    jobs = gx.gx_solve_batch(ctx, handles, params)
    gx.gx_wait(ctx, jobs[0])
    dt = time.perf_counter() - t0
    device_s = gx.gx_job_info_get(ctx, jobs[0])["evolve_ms"] / 1e3
    results = [gx.gx_fetch_best(ctx, j, i.n) for j, i in zip(jobs, insts)]
    evals = sum(p.population * p.candidates * p.generations for p in params)
    # plain solver: the same requests one at a time, on an evenly spaced sample
    idx = np.linspace(0, count - 1, min(args.plain_sample, count)).astype(int)
    t1 = time.perf_counter()
    same = 0
    for i in idx:
        job = gx.gx_solve(ctx, handles[i], params[i])
        sol, f = gx.gx_fetch_best(ctx, job, insts[i].n)
        same += int(f == results[i][1] and np.array_equal(sol, results[i][0]))
        gx.gx_job_free(ctx, job)
    plain_dt = (time.perf_counter() - t1) / len(idx)
    for j in jobs:
        gx.gx_job_free(ctx, j)
    gx.gx_destroy(ctx)
    return {
        "metric": "batched solves/s", "value": count / dt, "unit": "solves/s",
        "move_evals_per_s": evals / dt, "seconds": dt, "device_seconds": device_s,
        "plain_solves_per_s": 1.0 / plain_dt, "speedup_vs_plain": plain_dt * count / dt,
        "plain_sample": int(len(idx)), "plain_identical": same,
        "config": {"workload": f"{count} instances: {n_tsp} TSP n U[20,200] + {count - n_tsp} QAP n "
                               f"U[12,40]; population per size bucket by the '{args.population_rule}' rule "
                               f"({sum(p.population for p in params)} solutions on {cus} CUs), C=128, "
                               f"{G} generations; TSP staging per bucket tuned",
                   "population_rule": args.population_rule, "generations": G, "plan": plan,
                   "solutions": sum(p.population for p in params)},
    }


def bench_kinds(args):
    """Plain-solver throughput of every problem kind and encoding, with and
    without the segment operators, and of the 442-city TSP with the island
    model on (ring, global top-N and hybrid migration plus elite injection)
    against the same solve with one population.  One timed solve per row
    after one untimed solve of the same row."""
    import torch
    import synth
    from paper_2603_19163_amd import gx

    ctx = gx.gx_create(0, torch.cuda.Stream())
    g442 = 20_000

    def tsp442(**kw):
        inst, p = synth.c2_tsp442(population=0, generations=g442)
        return inst, p.with_(**kw)

    def one(inst, p, G):
        return inst, synth.Params(seed=42, generations=G, population=p, candidates=128,
                                  alpha_q32=synth.alpha_q32_for(G))

    isl = dict(islands=16, migrate_epochs=5, elite_epochs=10)
    rows = [
        ("tsp442", "TSP n=442 clustered, 2-opt/swap/insert/or-opt, one population", tsp442()),
        ("tsp442_islands_ring", "same, 16 islands, ring migration every 5 epochs, elite every 10",
         tsp442(**isl, migrate_mode=0)),
        ("tsp442_islands_topn", "same, 16 islands, global top-4 migration every 5 epochs, elite every 10",
         tsp442(**isl, migrate_mode=1, migrate_n=4)),
        ("tsp442_islands_hybrid", "same, 16 islands, hybrid migration every 5 epochs, elite every 10",
         tsp442(**isl, migrate_mode=2, migrate_n=4)),
        ("tsp442_lns", "same, one population, with the three LNS operators at their preset weights",
         tsp442(op_mask=synth.PERM4_OPS | synth.LNS_OPS)),
        ("tsp442_lns_capped", "same, the LNS operators' weights capped at 1/65536 (the LNS kernel, almost no LNS step)",
         tsp442(op_mask=synth.PERM4_OPS | synth.LNS_OPS, weight_cap_q16=(0, 0, 0, 0, 0, 1, 1, 1))),
        ("tsp442_3opt", "same, 2-opt/swap/insert/or-opt and 3-opt (the kernel the LNS one extends)",
         tsp442(op_mask=synth.PERM4_OPS | (1 << synth.OP_3OPT))),
        ("tsp50", "TSP n=50 uniform, P=64, 2-opt/swap/or-opt, 2000 generations", synth.c1_small_tsp(0)),
        ("vrptw100", "VRPTW 100 customers, giant tour + split, P=64, 5000 generations", synth.c3_vrptw()),
        ("vrptw100_weighted", "same, weighted objectives 6 distance + 2 routes + 2 longest route",
         (dataclasses.replace(synth.c3_vrptw()[0], obj_weights=(6, 2, 2)), synth.c3_vrptw()[1])),
        ("vrptw100_lex", "same, lexicographic: routes, then distance within 20, then longest route",
         (dataclasses.replace(synth.c3_vrptw()[0], lex_order=(2, 1, 3), lex_tol=(0, 20, 0)), synth.c3_vrptw()[1])),
        ("vrptw100_rows", "same customers in the multi-row form: 25 rows, every permutation and row operator",
         synth.c3_vrptw_rows()),
        ("vrptw100_rows_lex", "same, multi-row, lexicographic: routes, then distance within 20, then longest route",
         (dataclasses.replace(synth.c3_vrptw_rows()[0], lex_order=(2, 1, 3), lex_tol=(0, 20, 0)),
          synth.c3_vrptw_rows()[1])),
        ("qap50", "QAP n=50, P autosized, 2000 generations", one(synth.qap_random(50, 7), 0, 2000)),
        ("vrptw100_lns", "VRPTW 100 customers, giant tour, every permutation operator and the LNS operators",
         (synth.c3_vrptw()[0], synth.c3_vrptw()[1].with_(op_mask=synth.PERM_LNS_OPS))),
    ]
    kp_inst, kp = one(synth.knapsack_random(1000, 7), 2048, 5000)
    rows += [("knapsack1000_flip", "0/1 knapsack n=1000, P=2048, flip only, 5000 generations",
              (kp_inst, kp.with_(op_mask=1 << synth.OP_FLIP))),
             ("knapsack1000_flip_segflip", "same, flip + seg_flip", (kp_inst, kp.with_(op_mask=synth.BIN_OPS)))]
    co_inst, co = one(synth.color_planted(1000, 3, inst_id=7), 2048, 5000)
    rows += [("color1000_reset", "planted 3-colouring n=1000 (integer encoding), P=2048, reset only, 5000 generations",
              (co_inst, co.with_(op_mask=1 << synth.OP_RESET))),
             ("color1000_reset_segreset", "same, reset + seg_reset", (co_inst, co.with_(op_mask=synth.INT_OPS)))]
    if args.kinds_rows:
        keep = set(args.kinds_rows.split(","))
        rows = [r for r in rows if r[0] in keep]
    out = []
    for name, what, (inst, p) in rows:
        h = gx.gx_instance_upload(ctx, inst)
        if p.population == 0:
            p = p.with_(population=gx.gx_autosize_population(ctx, h, p))
        for rep in range(2):
            job = gx.gx_solve(ctx, h, p)
            _, f = gx.gx_fetch_best(ctx, job, synth.solution_len(inst))
            info = gx.gx_job_info_get(ctx, job)
            gx.gx_job_free(ctx, job)
        gx.gx_instance_free(ctx, h)
        s = info["evolve_ms"] / 1e3
        names = list(synth.OP_NAMES)
        if inst.kind != synth.VRPTW_ROWS:   # ids 5-7 are the LNS operators on single-row permutations
            names[5:8] = ["lns_segment", "lns_scatter", "lns_guided"]
        out.append({"row": name, "workload": what, "population": p.population,
                    "move_evals_per_s": info["move_evals"] / s, "avg_launch_us": s * 1e6 / info["evolve_launches"],
                    "best": int(f), "op_steps": {names[o]: int(info["op_steps"][o])
                                                 for o in range(len(names)) if info["op_steps"][o]}})
    gx.gx_destroy(ctx)
    return {"metric": "move evals/s per problem kind", "unit": "move evals/s", "rows": out}


def bench_served(args):
    """Served pattern: Poisson arrivals of mixed TSP n U[20,500], QAP n U[12,50]
    and knapsack n U[100,1000] requests into gx_server; p50/p99 latency and
    completed solves/s, against the plain solver on a sample."""
    import numpy as np
    import torch
    import synth
    from paper_2603_19163_amd import gx

    ctx = gx.gx_create(0, torch.cuda.Stream())
    G, P = args.served_generations, args.served_population
    names = {"tsp": 0, "qap": 1, "knapsack": 2}
    kinds = [names[k] for k in args.served_kinds.split(",")]
    reqs, gaps = synth.c5_requests(args.rate, args.duration, kinds, G, P)
    n_req = len(reqs)
    srv = gx.gx_server_create(ctx, hbm_budget_bytes=8 << 30, max_resident=8192)
    tickets = []
    t0 = time.perf_counter()
    t_next = t0
    t_note = t0 + 10
    for (inst, p), gap in zip(reqs, gaps):
        t_next += gap
        while time.perf_counter() < t_next:
            pass
        tickets.append(gx.gx_server_submit(srv, inst, p))
        if t_next >= t_note:   # a progress line every 10 s of a long stream
            print(f"[served] {len(tickets)} of {n_req} submitted", file=sys.stderr, flush=True)
            t_note += 10
    t_sub_end = time.perf_counter()
    lat, done, results = [], 0, {}
    deadline = time.perf_counter() + 600
    pending = set(range(n_req))
    while pending and time.perf_counter() < deadline:
        if time.perf_counter() >= t_note:
            print(f"[served] {n_req - len(pending)} of {n_req} done", file=sys.stderr, flush=True)
            t_note += 10
        for k in list(pending):
            res = gx.gx_server_poll(srv, tickets[k], reqs[k][0].n)
            if res is not None:
                results[k] = res
                lat.append((res[3] - res[2]) * 1e-9)
                pending.discard(k)
        time.sleep(0.001)
    t_end = time.perf_counter()
    stats = gx.gx_server_stats_get(srv)
    gx.gx_server_destroy(srv)
    idx = [k for k in np.linspace(0, n_req - 1, min(args.plain_sample, n_req)).astype(int) if k in results]
    same, plain_lat = 0, []
    for k in idx:
        inst, p = reqs[k]
        h = gx.gx_instance_upload(ctx, inst)
        t = time.perf_counter()
        job = gx.gx_solve(ctx, h, p)
        sol, f = gx.gx_fetch_best(ctx, job, inst.n)
        plain_lat.append(time.perf_counter() - t)
        same += int(f == results[k][1] and np.array_equal(sol, results[k][0]))
        gx.gx_job_free(ctx, job)
        gx.gx_instance_free(ctx, h)
    gx.gx_destroy(ctx)
    offered = args.rate * args.served_population * 128 * G
    return {
        "metric": "served solves/s", "value": len(results) / (t_end - t0), "unit": "solves/s",
        "offered_move_evals_per_s": offered,
        "offered_rate": args.rate, "submitted": n_req, "completed": len(results),
        "arrival_seconds": t_sub_end - t0, "drain_seconds": t_end - t_sub_end,
        "p50_s": _pct(lat, 50), "p99_s": _pct(lat, 99),
        "move_evals_per_s": stats["move_evals"] / max(stats["busy_seconds"], 1e-9),
        "plain_p50_s": _pct(plain_lat, 50), "plain_p99_s": _pct(plain_lat, 99),
        "plain_solves_per_s_sequential": len(plain_lat) / max(sum(plain_lat), 1e-9),
        "plain_identical": same, "plain_sample": len(idx),
        "server": stats,
        "config": {"workload": f"Poisson {args.rate}/s for {args.duration}s: TSP n U[20,500], QAP n "
                               f"U[12,50], knapsack n U[100,1000] (kinds {args.served_kinds}); P={P}, C=128, "
                               f"{G} generations each"},
    }


if __name__ == "__main__":
    main()
