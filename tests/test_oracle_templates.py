"""Pins of the template map-making oracle (Eq. defFT, Appendix A Eq. polytemplate; CPU only).

Each pin is independent of the oracle's code path: a dense T built entry by entry from the
Legendre series evaluated one point at a time, the dense definition of F_T with a library
pseudo-inverse, the projector identities F_T T = 0 and F_T W F_T = F_T, the unbiasedness of the
estimator on template-contaminated noiseless data, the binned map when there are no templates,
and the degeneracy between offsets and the I monopole that the paper describes.
"""

import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

import oracle as O
import synth


def _small(seed=0, n_poly=3, cover=0.8, baseline=37, flag_frac=0.05):
    prob = synth.make_templates(cfg_id=40 + seed, n_dets=2, samples_per_det=600, interval=300,
                                side=6, dwell=3, baseline=baseline, n_poly=n_poly, cover=cover,
                                flag_frac=flag_frac)
    return prob, O.template_plan_from_problem(prob)


def _dense_T(tp):
    """T column by column: degree k on baseline i, value sqrt((2k+1)/L) P_k((2j+1)/L - 1)."""
    n = tp.plan.n_samples
    cols = []
    for s, L in zip(tp.base_start, tp.base_len):
        for k in range(tp.n_poly):
            col = np.zeros(n)
            e = np.zeros(k + 1)
            e[k] = 1.0
            for j in range(int(L)):
                x = (2.0 * j + 1.0) / L - 1.0
                col[int(s) + j] = np.sqrt((2.0 * k + 1.0) / L) * npleg.legval(x, e)
            cols.append(col)
    return np.array(cols).T if cols else np.zeros((n, 0))


def _dense_F(tp):
    W = np.diag(tp.w)
    T = _dense_T(tp)
    K = T.T @ W @ T
    return W - W @ T @ np.linalg.pinv(K, rcond=1e-12, hermitian=True) @ T.T @ W


@pytest.mark.parametrize("seed,n_poly", [(0, 1), (1, 3), (2, 5)])
def test_filter_matches_dense_definition(seed, n_poly):
    _, tp = _small(seed, n_poly)
    F = _dense_F(tp)
    t = np.random.default_rng(seed).standard_normal(tp.plan.n_samples)
    np.testing.assert_allclose(O.template_filter(tp, t), F @ t, rtol=0,
                               atol=1e-11 * np.abs(F).sum(axis=1).max() * np.abs(t).max())


def test_filter_annihilates_templates_and_is_a_weighted_projector():
    _, tp = _small(3, 4)
    T = _dense_T(tp)
    a = np.random.default_rng(3).standard_normal(T.shape[1])
    Ta = T @ a
    assert np.abs(O.template_filter(tp, Ta)).max() <= 1e-11 * np.abs(Ta).max() * tp.w.max()
    n = tp.plan.n_samples
    F = np.array([O.template_filter(tp, e) for e in np.eye(n)]).T
    np.testing.assert_allclose(F, F.T, atol=1e-12)
    assert np.linalg.eigvalsh(0.5 * (F + F.T)).min() > -1e-10
    winv = np.where(tp.w > 0, 1.0 / np.where(tp.w > 0, tp.w, 1.0), 0.0)
    np.testing.assert_allclose(F @ (winv[:, None] * F), F, atol=1e-10 * np.abs(F).max())


def test_rank_deficient_kernel_blocks():
    # baselines shorter than the number of templates: the kernel block is singular and the
    # pseudo-inverse keeps only the directions the samples determine
    _, tp = _small(4, n_poly=4, baseline=3, cover=1.0)
    T = _dense_T(tp)
    a = np.random.default_rng(4).standard_normal(T.shape[1])
    assert np.abs(O.template_filter(tp, T @ a)).max() <= 1e-10 * np.abs(T @ a).max()
    F = _dense_F(tp)
    t = np.random.default_rng(5).standard_normal(tp.plan.n_samples)
    np.testing.assert_allclose(O.template_filter(tp, t), F @ t, rtol=0, atol=1e-10)


def test_legendre_templates_nearly_orthonormal_on_uniform_weights():
    L, n_poly = 1000, 6
    T = O.legendre_templates(L, n_poly)
    K = T.T @ T
    j, k = np.meshgrid(np.arange(n_poly), np.arange(n_poly), indexing="ij")
    assert np.abs(K[(j + k) % 2 == 1]).max() < 1e-13          # odd pairs vanish by symmetry
    # midpoint rule of the continuous orthonormality: error O(1 / L^2)
    assert np.abs(K - np.eye(n_poly)).max() < 50.0 / L ** 2 * n_poly ** 2
    for k in range(n_poly):   # values against the series evaluated point by point
        e = np.zeros(k + 1)
        e[k] = 1.0
        x = (2.0 * 17 + 1.0) / L - 1.0
        assert abs(T[17, k] - np.sqrt((2 * k + 1.0) / L) * npleg.legval(x, e)) < 1e-15


def test_noiseless_drifts_are_removed_exactly():
    """Unbiasedness (the identity after Eq. defFT): with d = P m + T x and no noise the estimate
    is m itself, whatever the template amplitudes."""
    prob = synth.make_templates(cfg_id=60, n_dets=3, samples_per_det=4096, interval=2048,
                                side=12, dwell=4, baseline=150, n_poly=3, cover=0.85)
    tp = O.template_plan_from_problem(prob)
    m = prob.m_true[0][tp.plan.kept]
    sky = O.unpoint(tp.plan, m)
    # noiseless data: the sky plus a quadratic drift of arbitrary amplitude on every baseline
    rng = np.random.default_rng(0)
    drift = np.zeros(prob.n_samples)
    for s, L in zip(tp.base_start, tp.base_len):
        c = rng.standard_normal(3) * 4.0
        u = np.arange(L) / L
        drift[s:s + L] = c[0] + c[1] * u + c[2] * u * u
    d = sky + drift
    res = O.template_pcg(tp, O.template_rhs(tp, d), tol=1e-11)
    assert res.converged
    assert np.linalg.norm(res.x - m) / np.linalg.norm(m) < 1e-7


def test_without_templates_the_map_is_the_weighted_binned_map():
    prob, _ = _small(5, n_poly=3)
    tp = O.template_plan_from_problem(prob, n_poly=0)
    b = O.template_rhs(tp, prob.d[0])
    res = O.template_pcg(tp, b, tol=1e-12)
    plan = tp.plan
    ok = plan.lpix >= 0
    p = plan.lpix[ok]
    w = [np.ones(p.size), plan.wq[ok], plan.wu[ok]]
    G = np.zeros((plan.n_kept, 3, 3))
    v = np.zeros((plan.n_kept, 3))
    ww = tp.w[ok]
    d = prob.d[0].astype(np.float64)[ok]
    for i in range(3):
        v[:, i] = np.bincount(p, weights=ww * w[i] * d, minlength=plan.n_kept)
        for j in range(3):
            G[:, i, j] = np.bincount(p, weights=ww * w[i] * w[j], minlength=plan.n_kept)
    want = np.linalg.solve(G, v[..., None])[..., 0]
    assert res.iterations == 1
    np.testing.assert_allclose(res.x, want, rtol=0, atol=1e-10 * np.abs(want).max())


def test_full_cover_offsets_leave_exactly_the_monopole():
    """Degeneracy of templates and sky (Degeneracy section): with every sample in some baseline,
    offsets absorb a constant I map, so the system has one null direction, the I monopole."""
    prob, tp = _small(6, n_poly=1, cover=1.0, flag_frac=0.0)
    n = 3 * tp.plan.n_kept
    A = np.array([O.template_apply_A(tp, e.reshape(-1, 3)).reshape(-1) for e in np.eye(n)]).T
    ev, V = np.linalg.eigh(0.5 * (A + A.T))
    assert abs(ev[0]) < 1e-10 * ev[-1] and ev[1] > 1e-6 * ev[-1]
    mono = np.zeros((tp.plan.n_kept, 3))
    mono[:, 0] = 1.0
    mono = mono.reshape(-1) / np.linalg.norm(mono)
    assert abs(abs(V[:, 0] @ mono) - 1.0) < 1e-8


@pytest.mark.parametrize("mistake", ["unweighted_projection", "unweighted_fit"])
def test_template_planted_mistakes_are_caught(monkeypatch, mistake):
    _, tp = _small(7, 3)
    T = _dense_T(tp)
    a = np.random.default_rng(7).standard_normal(T.shape[1])
    F = _dense_F(tp)
    t = np.random.default_rng(8).standard_normal(tp.plan.n_samples)
    good = O.templates.template_filter

    def bad(tp_, x):
        u = tp_.w * np.asarray(x, np.float64)
        out = u.copy()
        for i, (s, L) in enumerate(zip(tp_.base_start, tp_.base_len)):
            s, L = int(s), int(L)
            Tb = O.legendre_templates(L, tp_.n_poly)
            if mistake == "unweighted_projection":
                c = tp_.Kinv[i] @ (Tb.T @ np.asarray(x, np.float64)[s:s + L])
                out[s:s + L] -= tp_.w[s:s + L] * (Tb @ c)
            else:
                c = tp_.Kinv[i] @ (Tb.T @ u[s:s + L])
                out[s:s + L] -= Tb @ c
        return out

    assert np.abs(good(tp, T @ a)).max() <= 1e-10 * np.abs(T @ a).max()
    ok_dense = np.allclose(good(tp, t), F @ t, atol=1e-10)
    assert ok_dense
    caught = (np.abs(bad(tp, T @ a)).max() > 1e-6 * np.abs(T @ a).max()
              or not np.allclose(bad(tp, t), F @ t, atol=1e-10))
    assert caught
