"""GPU parity: every step of the hot path, through the C ABI, against the FP64 oracle.

Tolerances (derived from the arithmetic):
  * integer work (hits, kept pixel ids, gap counts): bit-exact;
  * P x: FP64 sums rounded once to FP32 -> within 1 FP32 ulp of the oracle rounded to FP32;
  * P^T u: FP64 accumulation of identical FP32 products -> 1e-12 relative (summation order);
  * M_BD r: FP64 3x3 products -> 1e-12 relative;
  * N^-1 t: FP32 arithmetic; direct sums err ~ u32 * sum|c||t| and the FFT ~ u32 log2(N)
    relative to ||u|| -> relative L2 <= 2e-6, and per sample |du_i| <= 8 log2(N) u32
    sum_k|c_k| max|t| (so that an error confined to segment seams or block edges, of order
    |c_k t|, cannot hide in the L2 norm);
  * A x and b: FP32 time-domain storage + FP32 Toeplitz -> relative L2 <= 3e-6, and per unknown
    the per-sample bound (plus the rounding of P x) pointed back with |P|^T;
  * PCG maps: relative L2 <= 1e-6 against the oracle's FP64 map at the same tolerance 1e-8
    (the FP32 floor measured with the oracle's single-precision emulation is ~1.3e-7).
"""

import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _dev(a):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _plan(lib, prob, **kw):
    return lib.Plan.from_problem(prob, **kw)


def _rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


U32 = 2.0 ** -24


def _band_l1(ref):
    return max(float(np.abs(b[0]) + 2.0 * np.abs(b[1:]).sum()) for b in ref.bands)


def _depth(plan):
    """Rounding depth of the Toeplitz step: log2(N) for the FFT product, the number of
    accumulated terms (lambda + 1 folded pairs) for the direct sum."""
    n = plan.info["fft_size"]
    if n:
        return float(np.log2(n))
    return float(plan.info["lambda_max"] + 1)


def _nw_bound(plan, ref, t):
    """Per-sample bound on |N^-1 t (GPU) - N^-1 t (oracle)|: FP32 rounding of the stored input
    and of the transform, 8 log2(N) u32 sum_k |c_k| max|t| (a seam or block-edge slip moves an
    element by O(|c_k| |t|), far above it)."""
    return 8.0 * _depth(plan) * U32 * _band_l1(ref) * float(np.abs(t).max())


def _A_bound(plan, ref, t):
    """Per-unknown bound on the product error: the per-sample bound of the Toeplitz step, plus
    the FP32 rounding of P x, pointed back with |P|^T."""
    per = _nw_bound(plan, ref, t) + 2.0 * U32 * _band_l1(ref) * float(np.abs(t).max())
    ok = ref.lpix >= 0
    p = ref.lpix[ok]
    out = np.zeros((ref.n_kept, 3))
    out[:, 0] = np.bincount(p, minlength=ref.n_kept) * per
    out[:, 1] = np.bincount(p, weights=np.abs(ref.wq[ok]), minlength=ref.n_kept) * per
    out[:, 2] = np.bincount(p, weights=np.abs(ref.wu[ok]), minlength=ref.n_kept) * per
    return out


CASES = {
    "tiny": lambda: synth.make_config("tiny"),
    "random_flags_gaps": lambda: synth.make_random_small(seed=3, n_samples=5003, n_pix=60,
                                                         n_dets=4, lam_max=40, flag_frac=0.1,
                                                         gap_frac=0.2, dwell=5),
    "ground_mini": lambda: synth.make_ground(cfg_id=21, n_dets=6, samples_per_det=40000,
                                             interval=9000, side=32, lam=700, flag_frac=0.02),
    "ground_lam8192": lambda: synth.make_ground(cfg_id=22, n_dets=4, samples_per_det=1 << 17,
                                                interval=1 << 16, side=48, lam=8192),
}

_cache = {}


def case(name):
    if name not in _cache:
        prob = CASES[name]()
        _cache[name] = (prob, O.plan_from_problem(prob))
    return _cache[name]


@pytest.mark.parametrize("name", list(CASES))
def test_plan_pixels_and_hits_bit_exact(gpu_lib, name):
    prob, ref = case(name)
    plan = _plan(gpu_lib, prob)
    ids, hits = plan.pixels()
    assert np.array_equal(ids, ref.kept)
    assert np.array_equal(hits, ref.hits)
    info = plan.info
    assert info["n_obs"] == ref.n_kept + ref.n_excised
    assert info["n_excised"] == ref.n_excised
    assert info["n_gap_samples"] == int(np.sum(ref.lpix < 0))


@pytest.mark.parametrize("name", ["tiny", "random_flags_gaps", "ground_mini"])
def test_unpoint_within_one_ulp(gpu_lib, name):
    prob, ref = case(name)
    plan = _plan(gpu_lib, prob)
    x = np.random.default_rng(1).standard_normal((ref.n_kept, 3))
    t = plan.unpoint(_dev(x)).cpu().numpy()
    want = O.unpoint(ref, x).astype(np.float32)
    ulp = np.spacing(np.abs(want).astype(np.float32))
    assert np.all(np.abs(t - want) <= ulp)


@pytest.mark.parametrize("name", ["tiny", "random_flags_gaps", "ground_mini", "ground_lam8192"])
def test_point_parity(gpu_lib, name):
    prob, ref = case(name)
    plan = _plan(gpu_lib, prob)
    u = np.random.default_rng(2).standard_normal(ref.n_samples).astype(np.float32)
    y = plan.point(_dev(u)).cpu().numpy()
    want = O.point(ref, u.astype(np.float64))
    scale = np.abs(want).max()
    assert np.abs(y - want).max() <= 1e-12 * max(scale, 1.0)


@pytest.mark.parametrize("dwell", [1, 2, 3, 40])
def test_point_parity_short_runs(gpu_lib, dwell):
    # The scatter lists the runs each wavefront completes before flushing them, one per lane;
    # short runs (many runs inside one lane's 8 samples) fill the list and a random pixel per
    # sample overflows it (more than 128 runs per 512 samples: direct flushes).
    prob = synth.make_random_small(seed=20 + dwell, n_samples=200003, n_pix=3000, n_dets=5,
                                   lam_max=8, dwell=dwell)
    ref = O.plan_from_problem(prob)
    plan = _plan(gpu_lib, prob)
    u = np.random.default_rng(dwell).standard_normal(ref.n_samples).astype(np.float32)
    y = plan.point(_dev(u)).cpu().numpy()
    want = O.point(ref, u.astype(np.float64))
    scale = np.abs(want).max()
    assert np.abs(y - want).max() <= 1e-12 * max(scale, 1.0)


@pytest.mark.parametrize("name", ["tiny", "random_flags_gaps", "ground_mini", "ground_lam8192"])
@pytest.mark.parametrize("algo", ["auto", "direct", "fft"])
def test_noise_weight_parity(gpu_lib, name, algo):
    prob, ref = case(name)
    if algo == "direct" and prob.lam_max > 4096:
        pytest.skip("direct product limited to lambda <= 4096")
    a = {"auto": gpu_lib.TOEPLITZ_AUTO, "direct": gpu_lib.TOEPLITZ_DIRECT,
         "fft": gpu_lib.TOEPLITZ_FFT}[algo]
    plan = _plan(gpu_lib, prob, toeplitz_algo=a)
    t = np.random.default_rng(3).standard_normal(ref.n_samples).astype(np.float32)
    u = plan.noise_weight(_dev(t)).cpu().numpy()
    want = O.noise_weight(t.astype(np.float64), ref)
    err = float(_rel(u, want))
    assert err <= 2e-6, err
    assert np.all(np.abs(u - want) <= _nw_bound(plan, ref, t))
    # samples outside every block pass through unchanged (bit-exact copy)
    cov = np.zeros(ref.n_samples, bool)
    for s, L in zip(ref.blk_start, ref.blk_len):
        cov[s:s + L] = True
    assert np.array_equal(u[~cov], t[~cov])


@pytest.mark.parametrize("fft_size", [2048, 4096, 8192, 16384, 32768])
def test_noise_weight_every_fft_size(gpu_lib, fft_size):
    lam = min(900, fft_size // 2 - 1)
    prob = synth.make_ground(cfg_id=23, n_dets=2, samples_per_det=50001, interval=20011,
                             side=16, lam=lam)
    ref = O.plan_from_problem(prob)
    plan = _plan(gpu_lib, prob, toeplitz_algo=gpu_lib.TOEPLITZ_FFT, fft_size=fft_size)
    assert plan.info["fft_size"] == fft_size
    t = np.random.default_rng(4).standard_normal(ref.n_samples).astype(np.float32)
    u = plan.noise_weight(_dev(t)).cpu().numpy()
    want = O.noise_weight(t.astype(np.float64), ref)
    err = float(_rel(u, want))
    assert err <= 2e-6, err
    assert np.all(np.abs(u - want) <= _nw_bound(plan, ref, t))


@pytest.mark.parametrize("fft_size", [2048, 4096, 8192, 16384, 32768])
@pytest.mark.parametrize("flags", [0, 1])
def test_apply_A_every_fft_size(gpu_lib, fft_size, flags):
    # odd lambda and odd interval lengths: unaligned windows, ragged last segments
    lam = min(901, fft_size // 2 - 1)
    prob = synth.make_ground(cfg_id=24, n_dets=2, samples_per_det=50001, interval=20011,
                             side=16, lam=lam, flag_frac=0.01)
    ref = O.plan_from_problem(prob)
    plan = _plan(gpu_lib, prob, toeplitz_algo=gpu_lib.TOEPLITZ_FFT, fft_size=fft_size,
                 flags=flags)
    x = np.random.default_rng(7).standard_normal((ref.n_kept, 3))
    y, want = plan.apply_A(_dev(x)).cpu().numpy(), O.apply_A(ref, x)
    err = float(_rel(y, want))
    assert err <= 3e-6, err
    assert np.all(np.abs(y - want) <= _A_bound(plan, ref, O.unpoint(ref, x)))
    b, bw = plan.rhs(_dev(prob.d[0])).cpu().numpy(), O.rhs(ref, prob.d[0])
    err = float(_rel(b, bw))
    assert err <= 3e-6, err
    dm = np.where(ref.lpix >= 0, prob.d[0].astype(np.float64), 0.0)
    assert np.all(np.abs(b - bw) <= _A_bound(plan, ref, dm))


def test_fft_length_tuning(gpu_lib):
    # lambda 901: the rule's length is 4096; the tuner times 4096, 8192 and 16384 and keeps one,
    # and a second plan of the same shape takes the remembered length without tuning
    prob = synth.make_ground(cfg_id=28, n_dets=2, samples_per_det=50001, interval=20011,
                             side=16, lam=901, flag_frac=0.01)
    ref = O.plan_from_problem(prob)
    plan = _plan(gpu_lib, prob, toeplitz_algo=gpu_lib.TOEPLITZ_FFT, fft_size=-1)
    n = plan.info["fft_size"]
    assert n in (4096, 8192, 16384), plan.info
    x = np.random.default_rng(12).standard_normal((ref.n_kept, 3))
    y, want = plan.apply_A(_dev(x)).cpu().numpy(), O.apply_A(ref, x)
    assert float(_rel(y, want)) <= 3e-6
    assert np.all(np.abs(y - want) <= _A_bound(plan, ref, O.unpoint(ref, x)))
    again = _plan(gpu_lib, prob, toeplitz_algo=gpu_lib.TOEPLITZ_FFT, fft_size=-1)
    assert again.info["fft_size"] == n
    with pytest.raises(gpu_lib.MMError):
        _plan(gpu_lib, prob, toeplitz_algo=gpu_lib.TOEPLITZ_FFT, fft_size=-2)


@pytest.mark.parametrize("name", ["tiny", "random_flags_gaps", "ground_mini"])
def test_precond_parity(gpu_lib, name):
    prob, ref = case(name)
    plan = _plan(gpu_lib, prob)
    r = np.random.default_rng(5).standard_normal((ref.n_kept, 3))
    z = plan.precond_bj(_dev(r)).cpu().numpy()
    want = O.precond_bj(ref, r)
    assert np.abs(z - want).max() <= 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("mode", ["auto", "fft_fused", "fft_unfused"])
def test_apply_A_and_rhs_parity(gpu_lib, name, mode):
    prob, ref = case(name)
    kw = {}
    if mode != "auto":
        flags = {"fft_fused": 0, "fft_unfused": gpu_lib.FLAG_UNFUSED}[mode]
        kw = dict(toeplitz_algo=gpu_lib.TOEPLITZ_FFT, flags=flags)
    plan = _plan(gpu_lib, prob, **kw)
    x = np.random.default_rng(6).standard_normal((ref.n_kept, 3))
    y = plan.apply_A(_dev(x)).cpu().numpy()
    want = O.apply_A(ref, x)
    err = float(_rel(y, want))
    assert err <= 3e-6, err
    assert np.all(np.abs(y - want) <= _A_bound(plan, ref, O.unpoint(ref, x)))
    b = plan.rhs(_dev(prob.d[0])).cpu().numpy()
    bw = O.rhs(ref, prob.d[0])
    err = float(_rel(b, bw))
    assert err <= 3e-6, err
    dm = np.where(ref.lpix >= 0, prob.d[0].astype(np.float64), 0.0)
    assert np.all(np.abs(b - bw) <= _A_bound(plan, ref, dm))


@pytest.mark.parametrize("name", ["tiny", "random_flags_gaps", "ground_mini"])
@pytest.mark.parametrize("unfused", [False, True])
def test_pcg_map_parity(gpu_lib, name, unfused):
    prob, ref = case(name)
    plan = _plan(gpu_lib, prob, flags=gpu_lib.FLAG_UNFUSED if unfused else 0)
    x, info = plan.pcg_solve(_dev(prob.d[0]), tol=1e-8)
    res = O.pcg(ref, O.rhs(ref, prob.d[0]), tol=1e-8)
    m = x.cpu().numpy()
    assert info["converged"] == 1 and res.converged
    err = float(_rel(m, res.x))
    assert err <= 1e-6, err
    assert abs(info["iterations"] - res.iterations) <= 2
    assert info["relres"] < 1e-8
    assert info["true_relres"] < 1e-7


def test_pcg_graph_and_eager_agree(gpu_lib):
    prob, ref = case("tiny")
    plan = _plan(gpu_lib, prob)
    torch = _torch()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        d = _dev(prob.d[0])
        xg, ig = plan.pcg_solve(d, use_graph=True, stream=s)
        xe, ie = plan.pcg_solve(d, use_graph=False, stream=s)
        xg2, ig2 = plan.pcg_solve(d, use_graph=True, check_every=8, stream=s)
    s.synchronize()
    # The FP64 atomic adds of P^T land in a run-dependent order (last-bit differences per
    # product), which CG carries through its iterations: two solves agree to ~1e-10, far
    # inside the 1e-6 map tolerance; the replay mode itself changes nothing.
    assert ig["iterations"] == ie["iterations"] == ig2["iterations"]
    err = float(_rel(xg.cpu().numpy(), xe.cpu().numpy()))
    assert err <= 1e-8, err
    err = float(_rel(xg2.cpu().numpy(), xe.cpu().numpy()))
    assert err <= 1e-8, err


def test_cached_graphs_replay_across_solves(gpu_lib):
    # The iteration graphs stay in the plan's workspace and are replayed by later solves into
    # the same map buffer: other right-hand sides, and a two-level solve after the deflation
    # space was rebuilt (its graph must be captured anew).  Every replay is compared with an
    # eager solve run between the replays.
    prob, ref = case("tiny")
    plan = _plan(gpu_lib, prob)
    torch = _torch()
    d0 = prob.d[0]
    d1 = (0.5 * d0 + np.random.default_rng(5).standard_normal(d0.size)).astype(np.float32)
    X = torch.zeros(ref.n_kept, 3, dtype=torch.float64, device="cuda")
    for d in (d0, d1, d0, d1):
        xg, ig = plan.pcg_solve(_dev(d), x=X)
        xg = xg.cpu().numpy().copy()
        xe, ie = plan.pcg_solve(_dev(d), use_graph=False)
        assert ig["converged"] == 1 and ig["iterations"] == ie["iterations"]
        err = float(_rel(xg, xe.cpu().numpy()))
        assert err <= 1e-8, err
    for m in (8, 12):
        plan.deflation_build(_dev(d0), m)
        for d in (d1, d0):
            xg, ig = plan.pcg_solve(_dev(d), x=X, precond=1)
            xg = xg.cpu().numpy().copy()
            xe, ie = plan.pcg_solve(_dev(d), use_graph=False, precond=1)
            assert ig["converged"] == 1 and ig["iterations"] == ie["iterations"], (m, ig, ie)
            err = float(_rel(xg, xe.cpu().numpy()))
            assert err <= 1e-8, (m, err)


def test_cached_graphs_evicted_and_recaptured(gpu_lib):
    # Ten map buffers, each solved into twice: thirty (buffer, chunk) keys pass through the
    # workspace's eight graph slots, so graphs are evicted and captured again between solves;
    # every solve must still equal an eager one.
    prob, ref = case("tiny")
    plan = _plan(gpu_lib, prob)
    torch = _torch()
    d = _dev(prob.d[0])
    xe, ie = plan.pcg_solve(d, use_graph=False)
    xe = xe.cpu().numpy()
    bufs = [torch.zeros(ref.n_kept, 3, dtype=torch.float64, device="cuda") for _ in range(10)]
    for rep in range(2):
        for X in bufs:
            X.zero_()
            xg, ig = plan.pcg_solve(d, x=X)
            assert ig["converged"] == 1 and ig["iterations"] == ie["iterations"], (rep, ig)
            err = float(_rel(xg.cpu().numpy(), xe))
            assert err <= 1e-8, (rep, err)


def test_band_table_input_matches_band_list(gpu_lib):
    # A plan built from the band coefficients already in the ABI's table layout (BandTable)
    # holds the same operator as one built from the list of per-band arrays.
    prob, ref = case("ground_mini")
    torch = _torch()
    pix, wq, wu = _dev(prob.pix), _dev(prob.wq), _dev(prob.wu)
    table = gpu_lib.BandTable(*prob.band_table())
    p_list = gpu_lib.Plan(pix, wq, wu, prob.n_pix_global, prob.blk_start, prob.blk_len,
                          prob.blk_band, prob.bands, det_offset=prob.det_offset)
    p_tab = gpu_lib.Plan(pix, wq, wu, prob.n_pix_global, prob.blk_start, prob.blk_len,
                         prob.blk_band, table, det_offset=prob.det_offset)
    assert p_tab.info == p_list.info
    x = np.random.default_rng(13).standard_normal((ref.n_kept, 3))
    y_list = p_list.apply_A(_dev(x)).cpu().numpy()
    y_tab = p_tab.apply_A(_dev(x)).cpu().numpy()
    assert float(_rel(y_tab, y_list)) <= 1e-12
    bad = gpu_lib.BandTable(table.ncoef, table.offset[:-1], table.coef)
    with pytest.raises(ValueError):
        gpu_lib.Plan(pix, wq, wu, prob.n_pix_global, prob.blk_start, prob.blk_len,
                     prob.blk_band, bad, det_offset=prob.det_offset)


def test_white_noise_binned_map_in_one_iteration(gpu_lib):
    prob = synth.make_raster(cfg_id=52, n_dets=3, side=16, dwell=4, lam=0, noise="white")
    ref = O.plan_from_problem(prob)
    plan = _plan(gpu_lib, prob)
    x, info = plan.pcg_solve(_dev(prob.d[0]))
    assert info["iterations"] == 1
    err = float(_rel(x.cpu().numpy(), O.binned_map(ref, prob.d[0])))
    assert err <= 1e-7, err


def test_noiseless_recovers_sky(gpu_lib):
    prob = synth.make_raster(cfg_id=53, n_dets=4, side=32, dwell=8, lam=256, noise="none")
    ref = O.plan_from_problem(prob)
    plan = _plan(gpu_lib, prob)
    x, info = plan.pcg_solve(_dev(prob.d[0]), tol=1e-10)
    err = float(_rel(x.cpu().numpy(), prob.m_true[0][ref.kept]))
    assert err <= 1e-6, err


def test_multiple_rhs_and_restart(gpu_lib):
    prob = synth.make_raster(cfg_id=54, n_dets=2, side=16, dwell=8, lam=128, n_rhs=3)
    ref = O.plan_from_problem(prob)
    plan = _plan(gpu_lib, prob)
    x, infos = plan.pcg_solve(_dev(prob.d))
    for j in range(3):
        want = O.pcg(ref, O.rhs(ref, prob.d[j])).x
        err = float(_rel(x[j].cpu().numpy(), want))
        assert err <= 1e-6, err
    # restart from the solution: b - A x0 sits at the FP32 true-residual floor (a few 1e-8),
    # so a couple of iterations bring the recursive residual under 1e-8 again
    x0 = x[0].clone()
    x1, info = plan.pcg_solve(_dev(prob.d[0]), x=x0, use_x0=True)
    assert info["iterations"] <= 5
    err = float(_rel(x1.cpu().numpy(), x[0].cpu().numpy()))
    assert err <= 1e-6, err


def test_zero_data_and_empty_edges(gpu_lib):
    prob = synth.make_raster(cfg_id=55, n_dets=2, side=8, dwell=4, lam=16)
    plan = _plan(gpu_lib, prob)
    torch = _torch()
    d0 = torch.zeros(prob.n_samples, dtype=torch.float32, device="cuda")
    x, info = plan.pcg_solve(d0)
    assert info["iterations"] == 0 and info["converged"] == 1
    assert not torch.any(x)
    # a geometry with no blocks: N^-1 = identity, every sample passes through
    pix = _dev(prob.pix)
    p2 = gpu_lib.Plan(pix, _dev(prob.wq), _dev(prob.wu), prob.n_pix_global, [], [], [], [])
    t = torch.randn(prob.n_samples, device="cuda")
    assert torch.equal(p2.noise_weight(t), t)
    # every sample flagged: nothing observed, empty map, converged at once
    allflag = torch.full((prob.n_samples,), -1, dtype=torch.int32, device="cuda")
    p3 = gpu_lib.Plan(allflag, _dev(prob.wq), _dev(prob.wu), prob.n_pix_global,
                      prob.blk_start, prob.blk_len, prob.blk_band, prob.bands)
    assert p3.n_kept == 0
    x3, info3 = p3.pcg_solve(_dev(prob.d[0]))
    assert info3["iterations"] == 0


def test_invalid_inputs_are_rejected(gpu_lib):
    prob = synth.make_raster(cfg_id=56, n_dets=2, side=8, dwell=4, lam=16)
    torch = _torch()
    bad = prob.pix.copy()
    bad[7] = prob.n_pix_global  # out of range
    with pytest.raises(gpu_lib.MMError) as e:
        gpu_lib.Plan(_dev(bad), _dev(prob.wq), _dev(prob.wu), prob.n_pix_global,
                     prob.blk_start, prob.blk_len, prob.blk_band, prob.bands)
    assert e.value.status == -1
    with pytest.raises(gpu_lib.MMError) as e:  # overlapping blocks
        gpu_lib.Plan(_dev(prob.pix), _dev(prob.wq), _dev(prob.wu), prob.n_pix_global,
                     [0, 10], [20, 20], [0, 0], prob.bands)
    assert e.value.status == -1
    neg = [np.array([1.0, 0.9, 0.0], np.float32)]  # symbol 1 + 1.8 cos w < 0 at w = pi
    with pytest.raises(gpu_lib.MMError) as e:
        gpu_lib.Plan(_dev(prob.pix), _dev(prob.wq), _dev(prob.wu), prob.n_pix_global,
                     [0], [prob.n_samples], [0], neg)
    assert e.value.status == -2
    del torch


# ------------------------------------------------------------------------------------------
# Long bands: four-step segments of 2^16 and 2^17 samples
# ------------------------------------------------------------------------------------------

def test_noise_weight_long_band_unaligned_buffers(gpu_lib):
    # caller buffers at a 4-byte offset: the long kernel must take its scalar loads and stores
    import torch
    prob = synth.make_ground(cfg_id=26, n_dets=1, samples_per_det=200000, interval=200000,
                             side=16, lam=20000)
    plan = _plan(gpu_lib, prob, toeplitz_algo=gpu_lib.TOEPLITZ_FFT)
    assert plan.info["fft_size"] == 131072
    n = prob.n_samples
    t = np.random.default_rng(10).standard_normal(n).astype(np.float32)
    want = plan.noise_weight(_dev(t)).cpu().numpy()
    tb = torch.zeros(n + 1, dtype=torch.float32, device="cuda")
    ub = torch.zeros(n + 1, dtype=torch.float32, device="cuda")
    tb[1:] = _dev(t)
    got = plan.noise_weight(tb[1:], ub[1:]).cpu().numpy()
    assert np.array_equal(got, want)


@pytest.mark.parametrize("lam,fft_size", [(12001, 65536), (20000, 131072), (32768, 0)])
def test_noise_weight_long_band(gpu_lib, lam, fft_size):
    prob = synth.make_ground(cfg_id=25, n_dets=2, samples_per_det=300001, interval=200003,
                             side=16, lam=lam)
    ref = O.plan_from_problem(prob)
    plan = _plan(gpu_lib, prob, toeplitz_algo=gpu_lib.TOEPLITZ_FFT, fft_size=fft_size)
    assert plan.info["fft_size"] == (fft_size or 131072)
    t = np.random.default_rng(8).standard_normal(ref.n_samples).astype(np.float32)
    u = plan.noise_weight(_dev(t)).cpu().numpy()
    want = O.noise_weight(t.astype(np.float64), ref)
    err = float(_rel(u, want))
    assert err <= 2e-6, err
    assert np.all(np.abs(u - want) <= _nw_bound(plan, ref, t))
    x = np.random.default_rng(9).standard_normal((ref.n_kept, 3))
    err = float(_rel(plan.apply_A(_dev(x)).cpu().numpy(), O.apply_A(ref, x)))
    assert err <= 3e-6, err


@pytest.mark.parametrize("fft_size,lam", [(65536, 12001), (131072, 20001), (131072, 32768)])
@pytest.mark.parametrize("flags", [0, 1])
def test_apply_A_long_segments(gpu_lib, fft_size, lam, flags):
    # fused (gather and scatter inside the four-step kernel) and unfused long-segment products:
    # odd lambda and odd interval lengths (unaligned windows, ragged last segments), flagged
    # samples, a gap between intervals; per-unknown bounds on A x and b
    prob = synth.make_ground(cfg_id=27, n_dets=2, samples_per_det=300001, interval=200003,
                             side=24, lam=lam, flag_frac=0.01)
    ref = O.plan_from_problem(prob)
    plan = _plan(gpu_lib, prob, toeplitz_algo=gpu_lib.TOEPLITZ_FFT, fft_size=fft_size,
                 flags=flags)
    assert plan.info["fft_size"] == fft_size
    assert plan.info["fused"] == (0 if flags else 3), plan.info
    x = np.random.default_rng(11).standard_normal((ref.n_kept, 3))
    y, want = plan.apply_A(_dev(x)).cpu().numpy(), O.apply_A(ref, x)
    err = float(_rel(y, want))
    assert err <= 3e-6, err
    assert np.all(np.abs(y - want) <= _A_bound(plan, ref, O.unpoint(ref, x)))
    b, bw = plan.rhs(_dev(prob.d[0])).cpu().numpy(), O.rhs(ref, prob.d[0])
    err = float(_rel(b, bw))
    assert err <= 3e-6, err
    dm = np.where(ref.lpix >= 0, prob.d[0].astype(np.float64), 0.0)
    assert np.all(np.abs(b - bw) <= _A_bound(plan, ref, dm))


@pytest.mark.parametrize("dwell", [1, 3])
def test_apply_A_long_segments_short_runs(gpu_lib, dwell):
    # The long-segment scatter lists up to 64 runs per wavefront and drain round and flushes them
    # one value per lane; one or three samples per pixel (170 to 512 runs per 512 samples)
    # overflow the list, and the runs beyond it are flushed directly.
    prob = synth.make_ground(cfg_id=28, n_dets=2, samples_per_det=200003, interval=100003,
                             side=40, dwell=dwell, lam=12001, flag_frac=0.01)
    ref = O.plan_from_problem(prob)
    plan = _plan(gpu_lib, prob, toeplitz_algo=gpu_lib.TOEPLITZ_FFT, fft_size=65536)
    assert plan.info["fused"] == 3, plan.info
    x = np.random.default_rng(12).standard_normal((ref.n_kept, 3))
    y, want = plan.apply_A(_dev(x)).cpu().numpy(), O.apply_A(ref, x)
    err = float(_rel(y, want))
    assert err <= 3e-6, err
    assert np.all(np.abs(y - want) <= _A_bound(plan, ref, O.unpoint(ref, x)))


def test_satellite_long_band_pcg(gpu_lib):
    prob = synth.make_satellite(cfg_id=26, n_dets=2, samples_per_det=1 << 18, interval=1 << 17,
                                n_rings=32, n_phi=64, lam=1 << 14, fknee=0.05, fsample=20.0)
    ref = O.plan_from_problem(prob)
    plan = _plan(gpu_lib, prob)
    assert plan.info["fft_size"] == 65536 and plan.info["fused"] == 3
    x, info = plan.pcg_solve(_dev(prob.d[0]), tol=1e-8)
    res = O.pcg(ref, O.rhs(ref, prob.d[0]), tol=1e-8)
    err = float(_rel(x.cpu().numpy(), res.x))
    assert info["converged"] == 1 and err <= 1e-6, (err, info, res.iterations)
    assert abs(info["iterations"] - res.iterations) <= 2
