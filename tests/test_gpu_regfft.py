"""GPU register-resident FFT segment kernel (2^15-sample segments with at most 2^14 outputs,
i.e. lambda >= 2^13) through the C ABI.

It computes the same system product as the LDS-resident fused kernel, so the bars are the same:
relative L2 3e-6 against the FP64 oracle for A x and b = P^T N^-1 d (FP32 time domain), the two
kernels within that bound of each other, and the PCG map within 1e-6 of the oracle's map.
Cases: lambda 8192 with the automatic 2^15 length, odd lambda 8193 with the length forced
(odd output offset, 16,382 outputs per segment), lambda 12000 (8,768 outputs), odd block
lengths (ragged last segments), flagged samples (zero rows of P), and two columns at once.
Also blocks of exactly four segments back to back (a window's halo must not reach into the
neighbouring block) and 13-segment blocks.
"""

import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


CASES = {
    "lam8192": (dict(cfg_id=41, n_dets=3, samples_per_det=120001, interval=50021, side=40,
                     lam=8192, flag_frac=0.02), {}),
    "lam8193_forced": (dict(cfg_id=42, n_dets=2, samples_per_det=100003, interval=65536, side=40,
                            lam=8193, flag_frac=0.01), dict(fft_size=32768)),
    "lam12000": (dict(cfg_id=43, n_dets=2, samples_per_det=90007, interval=45001, side=32,
                      lam=12000, flag_frac=0.0), {}),
    # blocks of exactly four segments, back to back: halos stop at each block edge
    "lam8192_exact_blocks": (dict(cfg_id=46, n_dets=2, samples_per_det=196608, interval=65536,
                                  side=40, lam=8192, flag_frac=0.01), {}),
    # 13 segments per block, the last one ragged
    "lam8192_long_blocks": (dict(cfg_id=47, n_dets=2, samples_per_det=200003, interval=200003,
                                 side=40, lam=8192, flag_frac=0.01), {}),
    # one and three samples per pixel: 170 to 512 runs per wavefront and scatter round, more than
    # the 64 the run list holds (the rest are flushed directly)
    "lam8192_dwell1": (dict(cfg_id=49, n_dets=2, samples_per_det=100003, interval=50021, side=40,
                            dwell=1, lam=8192, flag_frac=0.01), {}),
    "lam8192_dwell3": (dict(cfg_id=50, n_dets=2, samples_per_det=100003, interval=50021, side=40,
                            dwell=3, lam=8192, flag_frac=0.01), {}),
}

_cache = {}


def case(name):
    if name not in _cache:
        gkw, pkw = CASES[name]
        prob = synth.make_ground(n_rhs=2, **gkw)
        _cache[name] = (prob, O.plan_from_problem(prob), pkw)
    return _cache[name]


@pytest.mark.parametrize("name", list(CASES))
def test_register_kernel_products_match_oracle(gpu_lib, name):
    prob, ref, pkw = case(name)
    plan = gpu_lib.Plan.from_problem(prob, **pkw)
    assert plan.info["fused"] == 2 and plan.info["fft_size"] == 32768, plan.info
    lds = gpu_lib.Plan.from_problem(prob, flags=gpu_lib.FLAG_LDS_FFT, **pkw)
    assert lds.info["fused"] == 1
    x = np.random.default_rng(11).standard_normal((2, ref.n_kept, 3))
    y = plan.apply_A(_dev(x)).cpu().numpy()
    y_lds = lds.apply_A(_dev(x)).cpu().numpy()
    for j in range(2):
        want = O.apply_A(ref, x[j])
        err = float(_rel(y[j], want))
        assert err <= 3e-6, (j, err)
        assert float(_rel(y[j], y_lds[j])) <= 3e-6
    for j in range(2):
        b = plan.rhs(_dev(prob.d[j])).cpu().numpy()
        err = float(_rel(b, O.rhs(ref, prob.d[j])))
        assert err <= 3e-6, (j, err)


def test_register_kernel_pcg_map(gpu_lib):
    prob, ref, pkw = case("lam8192")
    plan = gpu_lib.Plan.from_problem(prob, **pkw)
    want = O.pcg(ref, O.rhs(ref, prob.d[0]), tol=1e-8)
    x, info = plan.pcg_solve(_dev(prob.d[0]), tol=1e-8)
    assert info["converged"] == 1 and info["true_relres"] < 1e-7, info
    err = float(_rel(x.cpu().numpy(), want.x))
    assert err <= 1e-6, err
    assert abs(info["iterations"] - want.iterations) <= 3, (info["iterations"], want.iterations)


def test_register_kernel_mixed_band_lengths(gpu_lib):
    # the segments use the plan's longest band as halo; a detector with a short band keeps its
    # own symbol in the table
    prob = synth.make_ground(cfg_id=45, n_dets=3, samples_per_det=80001, interval=40001, side=24,
                             lam=8192, flag_frac=0.01)
    k = np.arange(51, dtype=np.float64)
    tail = -0.3 * np.exp(-k[1:] / 6.0)
    short = np.concatenate([[1.0 + 2.0 * np.abs(tail).sum() + 0.2], tail]).astype(np.float32)
    prob.bands[1] = short
    ref = O.plan_from_problem(prob)
    plan = gpu_lib.Plan.from_problem(prob)
    assert plan.info["fused"] == 2 and plan.info["lambda_max"] == 8192, plan.info
    x = np.random.default_rng(14).standard_normal((ref.n_kept, 3))
    err = float(_rel(plan.apply_A(_dev(x)).cpu().numpy(), O.apply_A(ref, x)))
    assert err <= 3e-6, err
    err = float(_rel(plan.rhs(_dev(prob.d[0])).cpu().numpy(), O.rhs(ref, prob.d[0])))
    assert err <= 3e-6, err


def test_lds_flag_keeps_other_shapes(gpu_lib):
    # lambda < 2^13 at length 2^15 has more than 2^14 outputs per segment: LDS kernel
    prob = synth.make_ground(cfg_id=44, n_dets=2, samples_per_det=70001, interval=40001, side=24,
                             lam=5000)
    plan = gpu_lib.Plan.from_problem(prob)
    assert plan.info["fft_size"] == 32768 and plan.info["fused"] == 1, plan.info


def test_kernel_timing_counts_working_launches(gpu_lib):
    # with per-kernel timing on, launches queued past convergence are dropped from the counts:
    # one fused product for b, one per iteration, one for the true residual
    prob, ref, pkw = case("lam8192")
    plan = gpu_lib.Plan.from_problem(prob, **pkw)
    d = _dev(prob.d[0])
    x0, info0 = plan.pcg_solve(d, tol=1e-8)
    plan.set_timing(True)
    x1, info1 = plan.pcg_solve(d, tol=1e-8)
    ms, n = plan.kernel_time(1)
    plan.set_timing(False)
    assert info1["iterations"] == info0["iterations"]
    assert n == info1["iterations"] + 2, (n, info1["iterations"])
    assert ms > 0.0
    # the scatter's FP64 atomics commit in a different order on every run
    assert float(_rel(x1.cpu().numpy(), x0.cpu().numpy())) <= 1e-8


@pytest.mark.parametrize("flags", [0, "lds"])
def test_segment_order_does_not_change_products(gpu_lib, flags):
    # With detector offsets the plan runs segments by time inside their detector, then by
    # detector; without them, in block order.  Only the order of the FP64 atomics differs.
    prob = synth.make_ground(cfg_id=48, n_dets=6, samples_per_det=131072, interval=32768, side=40,
                             lam=8192, flag_frac=0.01)
    f = gpu_lib.FLAG_LDS_FFT if flags == "lds" else 0
    args = (_dev(prob.pix), _dev(prob.wq), _dev(prob.wu), prob.n_pix_global, prob.blk_start,
            prob.blk_len, prob.blk_band, prob.bands)
    timed = gpu_lib.Plan(*args, det_offset=prob.det_offset, flags=f)
    plain = gpu_lib.Plan(*args, flags=f)
    assert timed.info["fused"] == (1 if f else 2)
    x = np.random.default_rng(15).standard_normal((timed.n_kept, 3))
    y1 = timed.apply_A(_dev(x)).cpu().numpy()
    y2 = plain.apply_A(_dev(x)).cpu().numpy()
    assert float(_rel(y1, y2)) <= 1e-12
    b1 = timed.rhs(_dev(prob.d[0])).cpu().numpy()
    b2 = plain.rhs(_dev(prob.d[0])).cpu().numpy()
    assert float(_rel(b1, b2)) <= 1e-12
