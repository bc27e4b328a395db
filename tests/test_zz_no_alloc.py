"""gx_solve_static (the entry point that allocates nothing: its device state
lives in the library's static workspace) against gx_solve on the same
requests: five calls in a row, each smaller than the one before (a VRPTW
instance in the lexicographic mode, whose objective vectors live in the
workspace too, a multi-row VRPTW and a TSP with the LNS operators among
them), each equal to the plain solve in its best solution and objective; a
solve larger than the workspace is refused on the host."""
import dataclasses

import numpy as np
import pytest
import torch

import synth
from paper_2603_19163_amd import gx

pytestmark = pytest.mark.gpu


def _plain(ctx, h, inst, p):
    job = gx.gx_solve(ctx, h, p)
    sol, f = gx.gx_fetch_best(ctx, job, synth.solution_len(inst))
    gx.gx_job_free(ctx, job)
    return sol, f


def test_static_solves_equal_plain_solves():
    ctx = gx.gx_create(0)
    try:
        reqs = [(synth.tsp_clustered(150, 3, key=61),
                 synth.Params(seed=42, generations=120, population=48, alpha_q32=synth.alpha_q32_for(120))),
                (synth.qap_random(18, 3, key=62),
                 synth.Params(seed=7, generations=60, population=6, alpha_q32=synth.alpha_q32_for(60), aos_scope=1)),
                # a VRPTW instance in the lexicographic mode: its objective vectors in the workspace too
                (dataclasses.replace(synth.vrptw_random(16, 3, key=64), vehicles=2, lex_order=(2, 1, 0),
                                     lex_tol=(0, 15, 0)),
                 synth.Params(seed=9, generations=40, population=4, alpha_q32=synth.alpha_q32_for(40))),
                # the multi-row form (rows closed by markers) and the LNS operators' kernels
                (synth.vrptw_rows(12, 3, key=65, vehicles=3),
                 synth.Params(seed=11, generations=30, population=3, alpha_q32=synth.alpha_q32_for(30))),
                (synth.tsp_uniform(20, 3, key=66),
                 synth.Params(seed=13, generations=30, population=2, alpha_q32=synth.alpha_q32_for(30),
                              op_mask=synth.PERM_LNS_OPS, init_weight_q16=[0, 0, 0, 0, 0, 20000, 20000, 20000]))]
        for inst, p in reqs:                      # each call smaller than the one before
            print(f"[static] kind {inst.kind} n={inst.n} P={p.population}", flush=True)
            h = gx.gx_instance_upload(ctx, inst)
            sol_d = torch.full((synth.solution_len(inst),), -1, dtype=torch.int32, device="cuda")
            obj_d = torch.zeros(1, dtype=torch.int64, device="cuda")
            torch.cuda.synchronize()
            gx.gx_solve_static(ctx, h, p, sol_d, obj_d)
            gx.gx_wait(ctx, None)
            sol, f = _plain(ctx, h, inst, p)
            assert int(obj_d.cpu()[0]) == f
            assert np.array_equal(sol_d.cpu().numpy(), sol)
            gx.gx_instance_free(ctx, h)
        big = synth.tsp_uniform(2000, 1, key=63)
        h = gx.gx_instance_upload(ctx, big)
        sol_d = torch.zeros(big.n, dtype=torch.int32, device="cuda")
        obj_d = torch.zeros(1, dtype=torch.int64, device="cuda")
        with pytest.raises(gx.GxError) as e:
            gx.gx_solve_static(ctx, h, synth.Params(seed=1, generations=10, population=2048,
                                                    alpha_q32=synth.alpha_q32_for(10)), sol_d, obj_d)
        assert e.value.status == gx.GX_E_UNSUPPORTED
        gx.gx_instance_free(ctx, h)
    finally:
        gx.gx_destroy(ctx)
