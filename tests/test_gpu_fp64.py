"""GPU parity of the FP64 product, the FP64 exit check (Eq. CGresidual) and refinement.

Tolerances (derived from the arithmetic):
  * FP64 product (MM_PRECISION_FP64 plans, every Toeplitz length and the direct and diagonal
    products): every step in FP64 -> per element |y_gpu - y_oracle| <= 1e-12 * (|P|^T |N^-1| |P|
    |x|)_i, i.e. FP64 rounding of the sums that form the element (FFT depth <= 17 passes);
  * PCG on an FP64 plan: the same Alg. 1 with products equal to FP64 rounding -> map within
    1e-9 of the oracle's map at the same tolerance and the same iteration count +-1;
  * FP64 true residual reported by the library: the oracle recomputes ||b - A x|| / ||b|| of the
    returned map in FP64; both are FP64 products of the same vectors, and the residual is ~1e-8
    of ||b|| -> agreement to 1e-4 relative;
  * refinement: the oracle's FP64 residual of the returned map must be < tol = 1e-8.
"""

import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _abs_bound(ref, x):
    """(|P|^T |N^-1| |P| |x|) per unknown: the magnitude each element's roundings scale with."""
    import dataclasses
    ok = ref.lpix >= 0
    lp = np.where(ok, ref.lpix, 0)
    ax = np.abs(np.asarray(x, np.float64))
    t = np.where(ok, ax[lp, 0] + np.abs(ref.wq) * ax[lp, 1] + np.abs(ref.wu) * ax[lp, 2], 0.0)
    absplan = dataclasses.replace(ref, bands=[np.abs(b) for b in ref.bands])
    u = O.noise_weight(t, absplan, "fft" if max(len(b) for b in ref.bands) > 65 else "direct")
    p = ref.lpix[ok]
    out = np.zeros((ref.n_kept, 3))
    out[:, 0] = np.bincount(p, weights=u[ok], minlength=ref.n_kept)
    out[:, 1] = np.bincount(p, weights=np.abs(ref.wq[ok]) * u[ok], minlength=ref.n_kept)
    out[:, 2] = np.bincount(p, weights=np.abs(ref.wu[ok]) * u[ok], minlength=ref.n_kept)
    return out


CASES = {
    # (problem, plan keyword arguments)
    "direct_lam24": (lambda: synth.make_random_small(seed=11, n_samples=4001, n_pix=50, n_dets=3,
                                                     lam_max=24, flag_frac=0.05, gap_frac=0.2,
                                                     dwell=4), {}),
    "diag": (lambda: synth.make_raster(cfg_id=93, n_dets=2, side=16, dwell=8, lam=0,
                                       noise="white"), {}),
    "fft_2e11": (lambda: synth.make_random_small(seed=12, n_samples=9001, n_pix=70, n_dets=3,
                                                 lam_max=300, flag_frac=0.05, gap_frac=0.15,
                                                 dwell=5), {"fft_size": 1 << 11}),
    "fft_2e13": (lambda: synth.make_raster(cfg_id=94, n_dets=2, side=24, dwell=16, lam=1500),
                 {"fft_size": 1 << 13}),
    "fft_2e15": (lambda: synth.make_ground(cfg_id=95, n_dets=2, samples_per_det=1 << 17,
                                           interval=1 << 16, side=32, lam=8192), {}),
    "fft_2e17": (lambda: synth.make_ground(cfg_id=96, n_dets=2, samples_per_det=1 << 18,
                                           interval=3 << 16, side=32, lam=20000), {}),
    # the batched transform's scatter with one sample per pixel: more runs per wavefront than
    # its 64-run list holds
    "fft_2e17_dwell1": (lambda: synth.make_ground(cfg_id=102, n_dets=2, samples_per_det=1 << 18,
                                                  interval=3 << 16, side=32, dwell=1, lam=20000,
                                                  flag_frac=0.01), {}),
    # 2^16 points: one radix-256 pass, one radix-16 pass and one radix-8 pass per transform
    "fft_2e16": (lambda: synth.make_ground(cfg_id=100, n_dets=2, samples_per_det=150001,
                                           interval=70001, side=32, lam=12001, flag_frac=0.01),
                 {"fft_size": 1 << 16}),
    # one workgroup per segment with the FP64 transform in registers (N = 2^12 .. 2^15, at most
    # N/2 outputs per segment): odd lambda, ragged intervals, flags
    "fused_2e12": (lambda: synth.make_ground(cfg_id=97, n_dets=3, samples_per_det=30011,
                                             interval=10007, side=24, lam=1025,
                                             flag_frac=0.02), {"fft_size": 1 << 12}),
    "fused_2e13": (lambda: synth.make_ground(cfg_id=98, n_dets=2, samples_per_det=40009,
                                             interval=20011, side=24, lam=2048,
                                             flag_frac=0.01), {}),
    "fused_2e14": (lambda: synth.make_ground(cfg_id=99, n_dets=2, samples_per_det=70001,
                                             interval=30011, side=24, lam=4097),
                   {"fft_size": 1 << 14}),
    # one sample per pixel: every wavefront round overflows the 64-run list of the scatter
    "fused_2e15_dwell1": (lambda: synth.make_ground(cfg_id=101, n_dets=2, samples_per_det=70001,
                                                    interval=65536, side=24, dwell=1, lam=8192,
                                                    flag_frac=0.01), {}),
}

_cache = {}


def case(name):
    if name not in _cache:
        mk, kw = CASES[name]
        prob = mk()
        _cache[name] = (prob, O.plan_from_problem(prob), kw)
    return _cache[name]


@pytest.mark.parametrize("name", list(CASES))
def test_fp64_product_elementwise(gpu_lib, name):
    prob, ref, kw = case(name)
    plan = gpu_lib.Plan.from_problem(prob, precision=gpu_lib.PRECISION_FP64, **kw)
    x = np.random.default_rng(5).standard_normal((ref.n_kept, 3))
    y = plan.apply_A(_dev(x)).cpu().numpy()
    want = O.apply_A(ref, x)
    bound = _abs_bound(ref, x)
    assert np.all(np.abs(y - want) <= 1e-12 * bound + 1e-300), np.max(np.abs(y - want) / bound)
    b = plan.rhs(_dev(prob.d[0])).cpu().numpy()
    bw = O.rhs(ref, prob.d[0])
    assert np.linalg.norm(b - bw) / np.linalg.norm(bw) <= 1e-12


@pytest.mark.parametrize("name", ["direct_lam24", "fft_2e13", "fft_2e15", "fused_2e12"])
def test_fp64_plan_pcg_matches_oracle(gpu_lib, name):
    prob, ref, kw = case(name)
    plan = gpu_lib.Plan.from_problem(prob, precision=gpu_lib.PRECISION_FP64, **kw)
    x, info = plan.pcg_solve(_dev(prob.d[0]), tol=1e-8, check_fp64=True)
    res = O.pcg(ref, O.rhs(ref, prob.d[0]), tol=1e-8)
    m = x.cpu().numpy()
    assert abs(info["iterations"] - res.iterations) <= 1
    assert np.linalg.norm(m - res.x) / np.linalg.norm(res.x) <= 1e-9
    assert info["true_relres64"] < 1e-8 * 1.5


@pytest.mark.parametrize("name", ["fft_2e13", "fft_2e15"])
def test_fp64_exit_check_matches_oracle_residual(gpu_lib, name):
    prob, ref, kw = case(name)
    plan = gpu_lib.Plan.from_problem(prob, **kw)  # mixed precision
    x, info = plan.pcg_solve(_dev(prob.d[0]), tol=1e-8, check_fp64=True)
    m = x.cpu().numpy()
    b = O.rhs(ref, prob.d[0])
    r = np.linalg.norm(b - O.apply_A(ref, m)) / np.linalg.norm(b)
    assert info["true_relres64"] > 0
    assert abs(info["true_relres64"] - r) <= 1e-4 * r
    print(f"{name}: recursive {info['relres']:.2e}, FP32-product true {info['true_relres']:.2e}, "
          f"FP64 true {info['true_relres64']:.2e} (oracle {r:.2e})", flush=True)


@pytest.mark.parametrize("name", ["fft_2e13", "fft_2e15", "fft_2e17", "fused_2e14"])
def test_refinement_reaches_fp64_tolerance(gpu_lib, name):
    prob, ref, kw = case(name)
    plan = gpu_lib.Plan.from_problem(prob, **kw)  # mixed precision
    x, info = plan.pcg_solve(_dev(prob.d[0]), tol=1e-8, refine=3)
    m = x.cpu().numpy()
    b = O.rhs(ref, prob.d[0])
    r = np.linalg.norm(b - O.apply_A(ref, m)) / np.linalg.norm(b)
    assert info["converged"] == 1 and info["true_relres64"] < 1e-8
    assert r < 1e-8, r
    res = O.pcg(ref, b, tol=1e-10)
    assert np.linalg.norm(m - res.x) / np.linalg.norm(res.x) <= 1e-6
    print(f"{name}: {info['iterations']} + {info['inner_iterations']} inner iterations, "
          f"{info['refine_steps']} step(s), FP64 true {info['true_relres64']:.2e} "
          f"(oracle {r:.2e})", flush=True)
