"""mm_pcg_solve_noalloc (static device scratch, no allocation) against mm_pcg_solve.

Two calls in a row through the C ABI, the second on a smaller plan (the scratch keeps the first
call's contents), each compared with mm_pcg_solve on the same plan and data: the same kernels
run in the same order, so the iteration counts agree and the maps differ only by the order of
FP64 atomic additions in the pointing sums (bound 1e-9 relative L2, far below the 1e-6 map
tolerance against the oracle, which both also meet)."""

import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu


def _case(gpu_lib, prob):
    import torch
    plan = gpu_lib.Plan.from_problem(prob, device="cuda")
    d = torch.from_numpy(prob.d[0]).cuda()
    x_ref, info_ref = plan.pcg_solve(d, tol=1e-8)
    x = torch.full((plan.n_kept, 3), float("nan"), dtype=torch.float64, device="cuda")
    x, info = plan.pcg_solve_noalloc(d, x, tol=1e-8)
    torch.cuda.synchronize()
    a, b = x.cpu().numpy(), x_ref.cpu().numpy()
    assert info["converged"] == 1 and info_ref["converged"] == 1
    assert abs(info["iterations"] - info_ref["iterations"]) <= 1
    assert np.linalg.norm(a - b) / np.linalg.norm(b) <= 1e-9
    ref = O.plan_from_problem(prob)
    res = O.pcg(ref, O.rhs(ref, prob.d[0]), tol=1e-8)
    assert np.linalg.norm(a - res.x) / np.linalg.norm(res.x) <= 1e-6
    plan.close()
    return info


def test_noalloc_matches_pcg_solve_twice_second_smaller(gpu_lib):
    big = synth.make_raster(cfg_id=0)  # 4 detectors x 65,536 samples, lambda 1024
    small = synth.make_raster(cfg_id=91, n_dets=2, side=24, dwell=8, lam=256)
    i1 = _case(gpu_lib, big)
    i2 = _case(gpu_lib, small)
    print("noalloc iterations", i1["iterations"], i2["iterations"], flush=True)


def test_noalloc_rejects_what_it_cannot_hold(gpu_lib):
    import torch
    prob = synth.make_raster(cfg_id=92, n_dets=2, side=16, dwell=8, lam=64)
    plan = gpu_lib.Plan.from_problem(prob, device="cuda", flags=gpu_lib.FLAG_UNFUSED)
    d = torch.from_numpy(prob.d[0]).cuda()
    x = torch.zeros((plan.n_kept, 3), dtype=torch.float64, device="cuda")
    _, info = plan.pcg_solve_noalloc(d, x, raise_on_error=False)
    assert info["status"] == "MM_ERR_UNSUPPORTED"
