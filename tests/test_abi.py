"""The C ABI library loads and exports every declared symbol; the binding's structs match the
header's layout (CPU only: no compute call is made)."""

import ctypes
import os
import subprocess
import tempfile

import pytest

from paper_2112_03370_amd import mapmaker

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    if not os.path.exists(mapmaker.LIB_PATH):
        pytest.skip("libmm.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(mapmaker.LIB_PATH)
    names = mapmaker.exported_symbols()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    mapmaker.load()
    assert lib.mm_status_string  # callable without a device


def test_status_strings_without_device():
    if not os.path.exists(mapmaker.LIB_PATH):
        pytest.skip("libmm.so not built")
    lib = mapmaker.load()
    assert lib.mm_status_string(0) == b"MM_OK"
    assert lib.mm_status_string(-2) == b"MM_ERR_NOT_SPD"
    # argument validation happens before any device call
    assert lib.mm_plan(None, None, None) == -1
    assert lib.mm_plan_destroy(None) == 0
    # serving calls validate their handles before touching a device
    assert lib.mm_server_create(None, None) == -1
    assert lib.mm_server_destroy(None) == 0
    t = ctypes.c_uint64()
    assert lib.mm_submit(None, 1, None, 1, 0, None, None, ctypes.byref(t)) == -1
    assert lib.mm_poll(None, 1, None, None) == -1
    assert lib.mm_wait(None, 1, None, None) == -1
    assert lib.mm_server_stats(None, None) == -1
    assert lib.mm_server_plan(None, None, 1, None) == -1
    assert lib.mm_deflation_build(None, None, 8, None) == -1
    assert lib.mm_deflation_clear(None) == -1
    assert lib.mm_precond_2lvl(None, None, None, 1, None) == -1


def test_struct_layout_matches_header():
    src = r"""
#include <stddef.h>
#include <stdio.h>
#include "mm.h"
#define P(T, f) printf(#T "." #f " %zu\n", offsetof(T, f));
int main(void) {
  printf("mm_geometry %zu\n", sizeof(mm_geometry));
  printf("mm_plan_info_t %zu\n", sizeof(mm_plan_info_t));
  printf("mm_solve_opts %zu\n", sizeof(mm_solve_opts));
  printf("mm_solve_info %zu\n", sizeof(mm_solve_info));
  P(mm_geometry, n_pix_global) P(mm_geometry, band_coef) P(mm_geometry, cond_max)
  P(mm_geometry, fft_size) P(mm_geometry, flags) P(mm_plan_info_t, lambda_max)
  P(mm_plan_info_t, n_chunks) P(mm_plan_info_t, fused)
  P(mm_solve_info, relres) P(mm_solve_info, ms) P(mm_solve_opts, use_graph)
  P(mm_solve_opts, block) P(mm_solve_info, block)
  printf("mm_server_opts %zu\n", sizeof(mm_server_opts));
  printf("mm_request_times %zu\n", sizeof(mm_request_times));
  printf("mm_server_stats_t %zu\n", sizeof(mm_server_stats_t));
  P(mm_server_opts, max_bypass) P(mm_request_times, slot) P(mm_server_stats_t, queued)
  P(mm_server_stats_t, n_plans) P(mm_server_opts, large_work) P(mm_server_opts, large_slots)
  P(mm_server_stats_t, peak_large)
  printf("mm_deflation_info_t %zu\n", sizeof(mm_deflation_info_t));
  P(mm_deflation_info_t, build_ms) P(mm_deflation_info_t, device_bytes) P(mm_solve_opts, precond)
  P(mm_geometry, precision) P(mm_geometry, n_poly) P(mm_geometry, n_baselines)
  P(mm_geometry, base_len) P(mm_plan_info_t, precision) P(mm_plan_info_t, n_baselines)
  P(mm_solve_opts, refine) P(mm_solve_opts, check_fp64) P(mm_solve_info, refine_steps)
  P(mm_solve_info, true_relres64) P(mm_solve_info, inner_iterations)
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "layout.c")
        exe = os.path.join(d, "layout")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), c, "-o", exe],
                       check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    got = dict(line.rsplit(" ", 1) for line in out.strip().splitlines())
    M = mapmaker
    exp = {
        "mm_geometry": ctypes.sizeof(M.Geometry), "mm_plan_info_t": ctypes.sizeof(M.PlanInfo),
        "mm_solve_opts": ctypes.sizeof(M.SolveOpts), "mm_solve_info": ctypes.sizeof(M.SolveInfo),
        "mm_geometry.n_pix_global": M.Geometry.n_pix_global.offset,
        "mm_geometry.band_coef": M.Geometry.band_coef.offset,
        "mm_geometry.cond_max": M.Geometry.cond_max.offset,
        "mm_geometry.fft_size": M.Geometry.fft_size.offset,
        "mm_geometry.flags": M.Geometry.flags.offset,
        "mm_plan_info_t.lambda_max": M.PlanInfo.lambda_max.offset,
        "mm_plan_info_t.n_chunks": M.PlanInfo.n_chunks.offset,
        "mm_plan_info_t.fused": M.PlanInfo.fused.offset,
        "mm_solve_info.relres": M.SolveInfo.relres.offset,
        "mm_solve_info.ms": M.SolveInfo.ms.offset,
        "mm_solve_opts.use_graph": M.SolveOpts.use_graph.offset,
        "mm_solve_opts.block": M.SolveOpts.block.offset,
        "mm_solve_info.block": M.SolveInfo.block.offset,
        "mm_server_opts": ctypes.sizeof(M.ServerOpts),
        "mm_request_times": ctypes.sizeof(M.RequestTimes),
        "mm_server_stats_t": ctypes.sizeof(M.ServerStats),
        "mm_server_opts.max_bypass": M.ServerOpts.max_bypass.offset,
        "mm_request_times.slot": M.RequestTimes.slot.offset,
        "mm_server_stats_t.queued": M.ServerStats.queued.offset,
        "mm_server_stats_t.n_plans": M.ServerStats.n_plans.offset,
        "mm_server_opts.large_work": M.ServerOpts.large_work.offset,
        "mm_server_opts.large_slots": M.ServerOpts.large_slots.offset,
        "mm_server_stats_t.peak_large": M.ServerStats.peak_large.offset,
        "mm_deflation_info_t": ctypes.sizeof(M.DeflationInfo),
        "mm_deflation_info_t.build_ms": M.DeflationInfo.build_ms.offset,
        "mm_deflation_info_t.device_bytes": M.DeflationInfo.device_bytes.offset,
        "mm_solve_opts.precond": M.SolveOpts.precond.offset,
        "mm_geometry.precision": M.Geometry.precision.offset,
        "mm_geometry.n_poly": M.Geometry.n_poly.offset,
        "mm_geometry.n_baselines": M.Geometry.n_baselines.offset,
        "mm_geometry.base_len": M.Geometry.base_len.offset,
        "mm_plan_info_t.precision": M.PlanInfo.precision.offset,
        "mm_plan_info_t.n_baselines": M.PlanInfo.n_baselines.offset,
        "mm_solve_opts.refine": M.SolveOpts.refine.offset,
        "mm_solve_opts.check_fp64": M.SolveOpts.check_fp64.offset,
        "mm_solve_info.refine_steps": M.SolveInfo.refine_steps.offset,
        "mm_solve_info.true_relres64": M.SolveInfo.true_relres64.offset,
        "mm_solve_info.inner_iterations": M.SolveInfo.inner_iterations.offset,
    }
    assert {k: int(v) for k, v in got.items()} == exp
