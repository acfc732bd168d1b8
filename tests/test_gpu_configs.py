"""Map parity at the shapes of the ground-like and satellite-like workloads (GPU vs FP64 oracle).

Each case keeps every per-detector dimension of its workload and slices the focal plane:
  * ground-like: 16 of the 256 detectors, each 2^20 samples in 16 intervals of 2^16, 512 x 512
    patch, lambda 8192 (FFT length 2^15, the register-resident fused product);
  * satellite-like: 2 of the 32 detectors, each 2^23 samples in 8 intervals of 2^20, 786,432
    pixels, HWP, lambda 2^15 (FFT length 2^17, the four-step long-band product).
The slice keeps the oracle's full PCG solve (its FP64 products take ~1 s per 16.8 M samples on
the host cores) inside a couple of minutes per case.

Checks, with tolerances derived from the arithmetic:
  * kept pixel ids and hit counts: bit-exact;
  * the refined GPU map (FP64 true residual < 1e-8, the standard the oracle's map meets with its
    recursive 1e-8) against the oracle's FP64 map at 1e-8: relative L2 <= 1e-6; two maps with
    FP64 residuals <= 1e-8 differ by at most 2 kappa_eff 1e-8, and kappa_eff (map error over
    residual) is ~16 on the 16-detector ground slice (143 iterations);
  * the plain GPU map (recursive 1e-8, FP64 true residual ~6e-8: the FP32 product floor)
    against the same oracle map: relative L2 <= 3e-6, the same bound with its ~6x larger
    residual; iteration counts within 2;
  * the GPU map's FP64 true residual ||b - A x|| / ||b|| recomputed by the oracle: below 2e-7
    (the FP32 product floor, ~5e-8 measured), and equal to the library's own FP64 exit check to
    1e-4 relative;
  * with one refinement step: the oracle's FP64 true residual of the refined map < 1e-8.
"""

import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.timeout(900)
@pytest.mark.parametrize("name,n_dets", [("ground", 16), ("satellite", 2)])
def test_workload_slice_map_parity(gpu_lib, name, n_dets):
    prob = synth.make_config(name, n_dets=n_dets)
    print(f"[{name}] {prob.n_samples} samples, {n_dets} detectors", flush=True)
    plan = gpu_lib.Plan.from_problem(prob)
    ids, hits = plan.pixels()
    ref = O.plan_from_problem(prob)
    assert np.array_equal(ids, ref.kept) and np.array_equal(hits, ref.hits)
    d = _dev(prob.d[0])
    x, info = plan.pcg_solve(d, tol=1e-8, check_fp64=True)
    xr, info_r = plan.pcg_solve(d, tol=1e-8, refine=2)
    m, mr = x.cpu().numpy(), xr.cpu().numpy()
    print(f"[{name}] GPU: {info['iterations']} iterations, FP64 true {info['true_relres64']:.2e}; "
          f"refined +{info_r['inner_iterations']}, FP64 true {info_r['true_relres64']:.2e}",
          flush=True)
    b = O.rhs(ref, prob.d[0])
    nb = np.linalg.norm(b)
    r_gpu = np.linalg.norm(b - O.apply_A(ref, m)) / nb
    r_ref = np.linalg.norm(b - O.apply_A(ref, mr)) / nb
    print(f"[{name}] oracle FP64 residuals: plain {r_gpu:.2e}, refined {r_ref:.2e}", flush=True)
    assert r_gpu < 2e-7 and abs(info["true_relres64"] - r_gpu) <= 1e-4 * r_gpu
    assert r_ref < 1e-8 and info_r["converged"] == 1
    res = O.pcg(ref, b, tol=1e-8)
    err = np.linalg.norm(m - res.x) / np.linalg.norm(res.x)
    err_r = np.linalg.norm(mr - res.x) / np.linalg.norm(res.x)
    print(f"[{name}] oracle: {res.iterations} iterations; map rel L2 plain {err:.2e}, "
          f"refined {err_r:.2e}", flush=True)
    assert res.converged and abs(info["iterations"] - res.iterations) <= 2
    assert err_r <= 1e-6
    assert err <= 3e-6
