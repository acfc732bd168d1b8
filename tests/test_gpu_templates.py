"""GPU parity of template map-making (Eq. defFT with the Legendre baselines of Appendix A)
against the FP64 oracle, through the C ABI.

Tolerances (derived from the arithmetic): the template product is FP64 end to end, so
  * P^T F_T P x and P^T F_T d agree with the oracle elementwise to 1e-11 of the magnitude
    |P|^T W^-1 (|P x| + |T c|) that the element's sums are formed from (FP64 rounding of sums
    over one baseline of up to a few thousand samples);
  * PCG maps agree to 1e-8 relative L2 (the same Alg. 1 on products equal to FP64 rounding;
    the 1e-8 stop leaves map errors of kappa * 1e-8 against the exact solution, identical in
    both up to rounding); with every sample under a baseline the I monopole is a null direction
    of the system (Degeneracy section), so maps are compared with their mean I removed;
  * pixel ids and hits are bit-exact.
"""

import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _plan(lib, prob, n_poly=None):
    m = prob.meta
    return lib.Plan.from_problem(prob, n_poly=m["n_poly"] if n_poly is None else n_poly,
                                 base_start=m["base_start"], base_len=m["base_len"])


CASES = {
    "offsets_partial": lambda: synth.make_templates(cfg_id=61, n_dets=3, samples_per_det=1 << 14,
                                                    interval=1 << 13, side=24, dwell=8,
                                                    baseline=600, n_poly=1, cover=0.8,
                                                    flag_frac=0.02),
    "poly3_long_baselines": lambda: synth.make_templates(cfg_id=62, n_dets=2,
                                                         samples_per_det=1 << 15,
                                                         interval=1 << 14, side=24, dwell=8,
                                                         baseline=5000, n_poly=3, cover=0.9),
    "poly5_short": lambda: synth.make_templates(cfg_id=63, n_dets=4, samples_per_det=6000,
                                                interval=3000, side=16, dwell=4, baseline=97,
                                                n_poly=5, cover=0.85, flag_frac=0.05),
    # eight templates: the kernel blocks' rotations run in LDS (160-sample baselines keep the
    # blocks well conditioned, so the 1e-12 right-hand-side bound applies)
    "poly8": lambda: synth.make_templates(cfg_id=65, n_dets=3, samples_per_det=6000,
                                          interval=3000, side=16, dwell=4, baseline=160,
                                          n_poly=8, cover=0.85, flag_frac=0.05),
    "offsets_full_cover": lambda: synth.make_templates(cfg_id=64, n_dets=3,
                                                       samples_per_det=1 << 14,
                                                       interval=1 << 13, side=24, dwell=8,
                                                       baseline=1024, n_poly=1, cover=1.0),
}

_cache = {}


def case(name):
    if name not in _cache:
        prob = CASES[name]()
        _cache[name] = (prob, O.template_plan_from_problem(prob))
    return _cache[name]


def _magnitude(tp, x):
    """|P|^T W^-1 (|P x| + |T c|) per unknown, with c the oracle's template fit of W^-1 P x."""
    plan = tp.plan
    t = O.unpoint(plan, x)
    fit = np.zeros_like(t)
    u = tp.w * t
    for i, (s, L) in enumerate(zip(tp.base_start, tp.base_len)):
        s, L = int(s), int(L)
        T = O.legendre_templates(L, tp.n_poly)
        fit[s:s + L] = np.abs(T) @ np.abs(tp.Kinv[i] @ (T.T @ u[s:s + L]))
    a = tp.w * (np.abs(t) + fit)
    ok = plan.lpix >= 0
    p = plan.lpix[ok]
    out = np.zeros((plan.n_kept, 3))
    out[:, 0] = np.bincount(p, weights=a[ok], minlength=plan.n_kept)
    out[:, 1] = np.bincount(p, weights=np.abs(plan.wq[ok]) * a[ok], minlength=plan.n_kept)
    out[:, 2] = np.bincount(p, weights=np.abs(plan.wu[ok]) * a[ok], minlength=plan.n_kept)
    return out


@pytest.mark.parametrize("name", list(CASES))
def test_template_plan_pixels_and_product(gpu_lib, name):
    prob, tp = case(name)
    plan = _plan(gpu_lib, prob)
    ids, hits = plan.pixels()
    assert np.array_equal(ids, tp.plan.kept) and np.array_equal(hits, tp.plan.hits)
    assert plan.info["n_poly"] == tp.n_poly and plan.info["n_baselines"] == len(tp.base_start)
    x = np.random.default_rng(3).standard_normal((tp.plan.n_kept, 3))
    y = plan.apply_A(_dev(x)).cpu().numpy()
    want = O.template_apply_A(tp, x)
    mag = _magnitude(tp, x)
    assert np.all(np.abs(y - want) <= 1e-11 * mag + 1e-300), np.max(np.abs(y - want) / mag)
    b = plan.rhs(_dev(prob.d[0])).cpu().numpy()
    bw = O.template_rhs(tp, prob.d[0])
    assert np.linalg.norm(b - bw) / np.linalg.norm(bw) <= 1e-12


def _no_mono(m):
    m = np.array(m, copy=True)
    m[:, 0] -= m[:, 0].mean()
    return m


@pytest.mark.parametrize("name", list(CASES))
def test_template_pcg_map_matches_oracle(gpu_lib, name):
    prob, tp = case(name)
    plan = _plan(gpu_lib, prob)
    x, info = plan.pcg_solve(_dev(prob.d[0]), tol=1e-8)
    m = x.cpu().numpy()
    res = O.template_pcg(tp, O.template_rhs(tp, prob.d[0]), tol=1e-8)
    assert info["converged"] == 1 and res.converged
    assert abs(info["iterations"] - res.iterations) <= 2
    if name == "offsets_full_cover":
        a, b = _no_mono(m), _no_mono(res.x)
    else:
        a, b = m, res.x
    assert np.linalg.norm(a - b) / np.linalg.norm(b) <= 1e-8
    print(f"{name}: {info['iterations']} iterations (oracle {res.iterations}), "
          f"true relres {info['true_relres']:.2e}", flush=True)


def test_template_noiseless_drifts_recover_the_sky(gpu_lib):
    """d = P m + (polynomial drifts on the baselines), no noise: the GPU map is m."""
    prob = synth.make_templates(cfg_id=65, n_dets=3, samples_per_det=1 << 14, interval=1 << 13,
                                side=24, dwell=8, baseline=900, n_poly=3, cover=0.85)
    tp = O.template_plan_from_problem(prob)
    m = prob.m_true[0][tp.plan.kept]
    d = O.unpoint(tp.plan, m)
    rng = np.random.default_rng(1)
    for s, L in zip(tp.base_start, tp.base_len):
        c = 10.0 * rng.standard_normal(3)
        u = np.arange(L) / L
        d[s:s + L] += c[0] + c[1] * u + c[2] * u * u
    d32 = d.astype(np.float32)
    plan = _plan(gpu_lib, prob)
    x, info = plan.pcg_solve(_dev(d32), tol=1e-10)
    want = O.template_pcg(tp, O.template_rhs(tp, d32), tol=1e-10).x
    got = x.cpu().numpy()
    assert np.linalg.norm(got - want) / np.linalg.norm(want) <= 1e-8
    # the FP32 rounding of d is the only departure from the noiseless model
    assert np.linalg.norm(got - m) / np.linalg.norm(m) <= 1e-5


def test_template_geometry_is_validated(gpu_lib):
    import torch
    prob = CASES["poly5_short"]()
    m = prob.meta
    bs, bl = m["base_start"].copy(), m["base_len"].copy()
    lib = gpu_lib

    def status(**kw):
        try:
            lib.Plan.from_problem(prob, **kw)
            return "MM_OK"
        except lib.MMError as e:
            return lib.STATUS[e.status]

    assert status(n_poly=3, base_start=bs, base_len=bl) == "MM_OK"
    i = int(np.flatnonzero(bs[:-1] + bl[:-1] == bs[1:])[0])
    over = bl.copy()
    over[i] += 1  # runs into the next baseline
    assert status(n_poly=3, base_start=bs, base_len=over) == "MM_ERR_INVALID"
    j = int(np.flatnonzero((bs + bl) % 3000 == 0)[0])
    cross = bl.copy()
    cross[j] += 1  # runs past the end of its stationary interval
    if j + 1 < len(bs) and bs[j + 1] == bs[j] + bl[j]:
        bs2, cross = np.delete(bs, j + 1), np.delete(cross, j + 1)
    else:
        bs2 = bs
    assert status(n_poly=3, base_start=bs2, base_len=cross) == "MM_ERR_INVALID"
    past = bl.copy()
    past[-1] = prob.n_samples - bs[-1] + 1
    assert status(n_poly=3, base_start=bs, base_len=past) == "MM_ERR_INVALID"
    assert status(n_poly=9, base_start=bs, base_len=bl) == "MM_ERR_UNSUPPORTED"
    ml = synth.make_raster(cfg_id=97, n_dets=2, side=8, dwell=4, lam=16)
    try:
        lib.Plan.from_problem(ml, n_poly=2, base_start=[0], base_len=[64])
        st = "MM_OK"
    except lib.MMError as e:
        st = lib.STATUS[e.status]
    assert st == "MM_ERR_UNSUPPORTED"  # templates take diagonal weights
    torch.cuda.synchronize()
