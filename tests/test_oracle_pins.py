"""Pins of the FP64 oracle against what the paper and the mathematics fix (CPU only).

Each pin is independent of the oracle's own code path: brute-force dense matrices built here by
loops, closed forms (eigenfunctions of Toeplitz operators, binned maps by per-pixel least
squares, finite termination of CG), exact integer counts, and invariants (adjointness, symmetry,
positive definiteness).
"""

import collections

import numpy as np
import pytest

import oracle as O
import synth


def _tiny_problem(seed=0, n_samples=240, n_pix=9, lam_max=6, gap_frac=0.2, flag_frac=0.05,
                  noise_sigma=1.0):
    return synth.make_random_small(seed=seed, n_samples=n_samples, n_pix=n_pix, n_dets=3,
                                   lam_max=lam_max, flag_frac=flag_frac, gap_frac=gap_frac,
                                   noise_sigma=noise_sigma, dwell=3)


def _brute_noise_inverse(prob, n):
    """N^-1 from the definition, one entry at a time (identity outside blocks)."""
    M = np.eye(n)
    for s, L, b in zip(prob.blk_start, prob.blk_len, prob.blk_band):
        c = np.asarray(prob.bands[b], np.float64)
        for i in range(int(s), int(s + L)):
            for j in range(int(s), int(s + L)):
                M[i, j] = c[abs(i - j)] if abs(i - j) < c.size else 0.0
    return M


def _brute_pointing(plan):
    P = np.zeros((plan.n_samples, 3 * plan.n_kept))
    for s in range(plan.n_samples):
        p = plan.lpix[s]
        if p < 0:
            continue
        P[s, 3 * p:3 * p + 3] = (1.0, plan.wq[s], plan.wu[s])
    return P


# ------------------------------------------------------------------------------------------
# Toeplitz N^-1
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_noise_weight_matches_brute_force_dense(seed):
    prob = _tiny_problem(seed)
    plan = O.plan_from_problem(prob)
    x = np.random.default_rng(seed).standard_normal(plan.n_samples)
    ref = _brute_noise_inverse(prob, plan.n_samples) @ x
    np.testing.assert_allclose(O.noise_weight_direct(x, plan), ref, rtol=0, atol=1e-12)
    np.testing.assert_allclose(O.noise_weight_fft(x, plan), ref, rtol=0, atol=1e-12)


def test_noise_weight_long_band_fft_equals_direct():
    # several overlap-save segments per block, lambda not a power of two, ragged block ends
    rng = np.random.default_rng(7)
    lam = 37
    k = np.arange(lam + 1)
    c = np.exp(-k / 9.0) * np.cos(k / 5.0)
    c[0] = 1.0 + 2 * np.abs(c[1:]).sum()
    plan = O.build_plan(np.zeros(2000, np.int32), np.ones(2000), np.zeros(2000), 1,
                        [0, 700, 1505], [600, 805, 495], [0, 0, 0], [c])
    x = rng.standard_normal(2000)
    a = O.noise_weight_direct(x, plan)
    for nfft in (None, 128, 200):
        np.testing.assert_allclose(O.noise_weight_fft(x, plan, nfft=nfft), a, rtol=0, atol=1e-12)
    np.testing.assert_array_equal(a[600:700], x[600:700])  # uncovered samples pass unchanged


def test_noise_weight_impulse_and_edges():
    lam = 5
    c = np.array([3.0, -0.5, 0.25, -0.125, 0.0625, -0.03125])
    plan = O.build_plan(np.zeros(64, np.int32), np.ones(64), np.zeros(64), 1, [10], [40], [0], [c])
    e = np.zeros(64)
    e[30] = 1.0  # interior: the response is the band mirrored around the impulse
    y = O.noise_weight_direct(e, plan)
    np.testing.assert_array_equal(y[30 - lam:30 + lam + 1], np.r_[c[::-1], c[1:]])
    assert np.count_nonzero(y) == 2 * lam + 1
    e = np.zeros(64)
    e[10] = 1.0  # first sample of the block: truncated, nothing leaks before the block
    y = O.noise_weight_direct(e, plan)
    np.testing.assert_array_equal(y[10:16], c)
    assert np.all(y[:10] == 0) and np.all(y[16:] == 0)


def test_noise_weight_sinusoid_is_eigenfunction_away_from_edges():
    # away from block edges a Toeplitz operator maps cos(w n) to f(w) cos(w n), with the symbol
    # f(w) = c_0 + 2 sum_k c_k cos(k w)
    lam = 12
    k = np.arange(lam + 1)
    c = 0.3 ** k
    n = 400
    plan = O.build_plan(np.zeros(n, np.int32), np.ones(n), np.zeros(n), 1, [0], [n], [0], [c])
    w = 2 * np.pi * 0.0371
    x = np.cos(w * np.arange(n))
    f = c[0] + 2 * np.sum(c[1:] * np.cos(k[1:] * w))
    y = O.noise_weight_fft(x, plan)
    np.testing.assert_allclose(y[lam:n - lam], f * x[lam:n - lam], atol=1e-12)


def test_noise_weight_lambda_zero_is_diagonal():
    plan = O.build_plan(np.zeros(50, np.int32), np.ones(50), np.zeros(50), 1, [5, 30], [20, 10],
                        [0, 1], [np.array([2.5]), np.array([0.5])])
    x = np.arange(50.0)
    y = O.noise_weight(x, plan)
    expect = x.copy()
    expect[5:25] *= 2.5
    expect[30:40] *= 0.5
    np.testing.assert_array_equal(y, expect)


# ------------------------------------------------------------------------------------------
# Pointing
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 5])
def test_pointing_dense_and_adjoint(seed):
    prob = _tiny_problem(seed)
    plan = O.plan_from_problem(prob)
    rng = np.random.default_rng(seed)
    m = rng.standard_normal((plan.n_kept, 3))
    t = rng.standard_normal(plan.n_samples)
    P = _brute_pointing(plan)
    np.testing.assert_allclose(O.unpoint(plan, m), P @ m.reshape(-1), atol=1e-13)
    np.testing.assert_allclose(O.point(plan, t).reshape(-1), P.T @ t, atol=1e-12)
    lhs = np.dot(O.unpoint(plan, m), t)
    rhs = np.sum(m * O.point(plan, t))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_pointing_of_ones_counts_hits():
    prob = _tiny_problem(3)
    plan = O.plan_from_problem(prob)
    cnt = collections.Counter(int(p) for p in plan.lpix if p >= 0)
    got = O.point(plan, np.ones(plan.n_samples))[:, 0]
    assert [int(v) for v in got] == [cnt[i] for i in range(plan.n_kept)]


# ------------------------------------------------------------------------------------------
# Plan: hits, excision, BJ blocks
# ------------------------------------------------------------------------------------------

def test_hits_and_compaction_exact():
    prob = _tiny_problem(4, flag_frac=0.2)
    plan = O.plan_from_problem(prob)
    cnt = collections.Counter(int(p) for p in prob.pix if p >= 0)
    assert list(plan.kept) == sorted(plan.kept)
    for li, g in enumerate(plan.kept):
        assert plan.hits[li] == cnt[int(g)]
    for s in range(prob.n_samples):
        g = int(prob.pix[s])
        if g < 0 or g not in set(plan.kept.tolist()):
            assert plan.lpix[s] == -1
        else:
            assert plan.kept[plan.lpix[s]] == g


def test_excision_of_degenerate_pixels():
    # pixel 0: well-spread angles (kept); pixel 1: a single angle (singular, excised);
    # pixel 2: only two hits (excised); pixel 3: unobserved
    psi = np.r_[np.linspace(0, np.pi, 12, endpoint=False), np.full(8, 0.3), [0.1, 1.2]]
    pix = np.r_[np.zeros(12), np.ones(8), [2, 2]].astype(np.int32)
    plan = O.build_plan(pix, np.cos(2 * psi), np.sin(2 * psi), 4, [], [], [], [])
    assert plan.kept.tolist() == [0]
    assert plan.n_excised == 2
    assert np.all(plan.lpix[12:] == -1)


def test_bj_blocks_match_dense_and_condition_near_two():
    prob = _tiny_problem(2)
    plan = O.plan_from_problem(prob)
    P = _brute_pointing(plan)
    D = np.diag(np.diag(_brute_noise_inverse(prob, plan.n_samples)))
    dense = P.T @ D @ P
    for p in range(plan.n_kept):
        np.testing.assert_allclose(plan.B[p], dense[3 * p:3 * p + 3, 3 * p:3 * p + 3], atol=1e-12)
        np.testing.assert_allclose(plan.Minv[p] @ plan.B[p], np.eye(3), atol=1e-9)
    # a pixel observed many times with uniform angles: B/(h c0) -> diag(1, 1/2, 1/2), cond -> 2
    n = 20000
    psi = np.random.default_rng(1).uniform(0, np.pi, n)
    big = O.build_plan(np.zeros(n, np.int32), np.cos(2 * psi), np.sin(2 * psi), 1, [], [], [], [])
    np.testing.assert_allclose(big.B[0] / n, np.diag([1, 0.5, 0.5]), atol=0.02)
    assert abs(big.cond[0] - 2.0) < 0.1


# ------------------------------------------------------------------------------------------
# System matrix and solver
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1])
def test_system_matrix_symmetric_positive_definite(seed):
    prob = _tiny_problem(seed)
    plan = O.plan_from_problem(prob)
    n = 3 * plan.n_kept
    cols = [O.apply_A(plan, e.reshape(-1, 3), "direct").reshape(-1) for e in np.eye(n)]
    A = np.array(cols).T
    P = _brute_pointing(plan)
    ref = P.T @ _brute_noise_inverse(prob, plan.n_samples) @ P
    np.testing.assert_allclose(A, ref, atol=1e-11)
    np.testing.assert_allclose(A, A.T, atol=1e-11)
    assert np.linalg.eigvalsh(A).min() > 0


def test_pcg_finite_termination_textbook():
    # CG on an n x n SPD system terminates in at most n steps in exact arithmetic
    A = np.array([[4.0, 1.0, 0.5], [1.0, 3.0, 0.2], [0.5, 0.2, 2.0]])
    b = np.array([[1.0, 2.0, 3.0]])
    plan = O.build_plan(np.zeros(3, np.int32), np.ones(3), np.zeros(3), 1, [], [], [], [])
    res = O.pcg(plan, b, tol=1e-13, apply=lambda v: (A @ v.reshape(-1)).reshape(-1, 3),
                precond=lambda v: v)
    assert res.iterations <= 3
    np.testing.assert_allclose(res.x.reshape(-1), np.linalg.solve(A, b[0]), atol=1e-13)
    # the first step of unpreconditioned CG from 0 is the steepest-descent step
    res1 = O.pcg(plan, b, tol=0.0, max_iter=1, apply=lambda v: (A @ v.reshape(-1)).reshape(-1, 3),
                 precond=lambda v: v)
    r = b[0]
    np.testing.assert_allclose(res1.x.reshape(-1), (r @ r) / (r @ A @ r) * r, atol=1e-15)


def _per_pixel_lstsq(plan, d):
    out = np.zeros((plan.n_kept, 3))
    for p in range(plan.n_kept):
        idx = np.flatnonzero(plan.lpix == p)
        W = np.stack([np.ones(idx.size), plan.wq[idx], plan.wu[idx]], axis=1)
        out[p] = np.linalg.lstsq(W, np.asarray(d, np.float64)[idx], rcond=None)[0]
    return out


def test_white_noise_pcg_is_binned_map_in_one_iteration():
    prob = synth.make_raster(cfg_id=50, n_dets=2, side=8, dwell=4, lam=0, noise="white")
    plan = O.plan_from_problem(prob)
    b = O.rhs(plan, prob.d[0])
    res = O.pcg(plan, b, tol=1e-8)
    assert res.iterations == 1
    ref = _per_pixel_lstsq(plan, prob.d[0])
    np.testing.assert_allclose(res.x, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    np.testing.assert_allclose(O.binned_map(plan, prob.d[0]), ref, atol=1e-12 * np.abs(ref).max())


def test_noiseless_data_recovers_sky():
    prob = synth.make_raster(cfg_id=51, n_dets=3, side=8, dwell=4, lam=64, noise="none")
    plan = O.plan_from_problem(prob)
    res = O.pcg(plan, O.rhs(plan, prob.d[0]), tol=1e-12)
    truth = prob.m_true[0][plan.kept]
    # d is stored in float32: the recovered sky differs from the truth by that rounding only
    assert np.linalg.norm(res.x - truth) / np.linalg.norm(truth) < 1e-6


@pytest.mark.parametrize("seed", [0, 6])
def test_pcg_matches_dense_cholesky(seed):
    prob = _tiny_problem(seed)
    plan = O.plan_from_problem(prob)
    b = O.rhs(plan, prob.d[0], "direct")
    P = _brute_pointing(plan)
    Ninv = _brute_noise_inverse(prob, plan.n_samples)
    A = P.T @ Ninv @ P
    d0 = np.where(plan.lpix >= 0, prob.d[0].astype(np.float64), 0.0)
    np.testing.assert_allclose(b.reshape(-1), P.T @ Ninv @ d0, atol=1e-11)
    xs = np.linalg.solve(A, b.reshape(-1))
    res = O.pcg(plan, b, tol=1e-10, apply=lambda v: O.apply_A(plan, v, "direct"))
    kappa = np.linalg.cond(A)
    err = np.linalg.norm(res.x.reshape(-1) - xs) / np.linalg.norm(xs)
    assert res.converged and err <= kappa * 1e-10
    np.testing.assert_allclose(O.solve_dense(plan, b).reshape(-1), xs, rtol=1e-9, atol=1e-12)


def test_lanczos_extremes_bracket_dense_spectrum():
    prob = _tiny_problem(1)
    plan = O.plan_from_problem(prob)
    b = O.rhs(plan, prob.d[0])
    res = O.pcg(plan, b, tol=1e-14, max_iter=500)
    n = 3 * plan.n_kept
    A = np.array([O.apply_A(plan, e.reshape(-1, 3), "direct").reshape(-1) for e in np.eye(n)]).T
    Minv = np.zeros((n, n))
    for p in range(plan.n_kept):
        Minv[3 * p:3 * p + 3, 3 * p:3 * p + 3] = plan.Minv[p]
    ev = np.sort(np.linalg.eigvals(Minv @ A).real)
    lo, hi = O.lanczos_extremes(res.alphas, res.betas)
    assert ev[0] * (1 - 1e-6) <= lo and hi <= ev[-1] * (1 + 1e-6)
    assert abs(hi - ev[-1]) / ev[-1] < 1e-3


def test_zero_rhs_returns_zero_without_iterations():
    prob = _tiny_problem(0)
    plan = O.plan_from_problem(prob)
    res = O.pcg(plan, np.zeros((plan.n_kept, 3)))
    assert res.iterations == 0 and res.converged and not np.any(res.x)


# ------------------------------------------------------------------------------------------
# Planted mistakes: each plausible slip in the oracle must trip at least one pin above
# ------------------------------------------------------------------------------------------

def _pins_pass(plan, prob):
    rng = np.random.default_rng(11)
    m = rng.standard_normal((plan.n_kept, 3))
    t = rng.standard_normal(plan.n_samples)
    P = _brute_pointing(plan)
    N = _brute_noise_inverse(prob, plan.n_samples)
    ok = np.allclose(O.unpoint(plan, m), P @ m.reshape(-1), atol=1e-12)
    ok &= np.allclose(O.point(plan, t).reshape(-1), P.T @ t, atol=1e-11)
    ok &= np.allclose(O.noise_weight_direct(t, plan), N @ t, atol=1e-12)
    ok &= np.allclose(O.noise_weight_fft(t, plan), N @ t, atol=1e-12)
    return bool(ok)


@pytest.mark.parametrize("mistake", ["swap_qu", "drop_lower_band", "wrong_sign", "no_trunc"])
def test_planted_mistakes_are_caught(monkeypatch, mistake):
    prob = _tiny_problem(0)
    plan = O.plan_from_problem(prob)
    assert _pins_pass(plan, prob)
    mm = O.mapmaking
    if mistake == "swap_qu":
        good = mm.point
        monkeypatch.setattr(mm, "point", lambda pl, t: good(pl, t)[:, [0, 2, 1]])
        monkeypatch.setattr(O, "point", mm.point)
    elif mistake == "drop_lower_band":
        def bad(x, pl):
            y = np.asarray(x, np.float64).copy()
            for s, L, b in zip(pl.blk_start, pl.blk_len, pl.blk_band):
                c = pl.bands[int(b)]
                xb = y[s:s + L].copy()
                yb = c[0] * xb
                for k in range(1, min(c.size, L)):
                    yb[k:] += c[k] * xb[:-k]
                y[s:s + L] = yb
            return y
        monkeypatch.setattr(O, "noise_weight_direct", bad)
    elif mistake == "wrong_sign":
        good = mm.unpoint
        monkeypatch.setattr(O, "unpoint",
                            lambda pl, m: good(pl, np.asarray(m) * np.array([1.0, -1.0, 1.0])))
    elif mistake == "no_trunc":
        good_fft = mm.noise_weight_fft

        def bad(x, pl, nfft=None, single=False):
            y = good_fft(x, pl, nfft, single)
            for s, L, b in zip(pl.blk_start, pl.blk_len, pl.blk_band):
                c = pl.bands[int(b)]
                if c.size > 1 and L > 1:   # wrap the band around the block ends
                    y[s] += c[1] * x[s + L - 1]
            return y
        monkeypatch.setattr(O, "noise_weight_fft", bad)
    assert not _pins_pass(plan, prob)


# ------------------------------------------------------------------------------------------
# Stacked right-hand sides: enlarged-CG (Alg. 2, Orthomin) recurrences
# ------------------------------------------------------------------------------------------

def _stack(seed, k, lam=64):
    prob = synth.make_raster(cfg_id=70 + seed, n_dets=2, side=12, dwell=6, lam=lam, n_rhs=k)
    plan = O.plan_from_problem(prob)
    B = np.stack([O.rhs(plan, prob.d[j], "direct") for j in range(k)])
    return prob, plan, B


def test_block_ecg_with_one_column_is_alg1():
    _, plan, B = _stack(0, 1)
    r = O.block_ecg(plan, B)
    p = O.pcg(plan, B[0])
    assert r.block_iterations == p.iterations
    np.testing.assert_allclose(r.x[0], p.x, rtol=0, atol=1e-12 * np.abs(p.x).max())


def test_block_ecg_columns_solve_their_systems():
    _, plan, B = _stack(1, 6)
    n = 3 * plan.n_kept
    A = np.array([O.apply_A(plan, e.reshape(-1, 3), "direct").reshape(-1) for e in np.eye(n)]).T
    r = O.block_ecg(plan, B, tol=1e-10, apply=lambda v: O.apply_A(plan, v, "direct"))
    kappa = np.linalg.cond(A)
    for j in range(6):
        xs = np.linalg.solve(A, B[j].reshape(-1))
        err = np.linalg.norm(r.x[j].reshape(-1) - xs) / np.linalg.norm(xs)
        assert r.converged[j] and err <= kappa * 1e-10
    # the enlarged Krylov space never needs more iterations than the columns alone
    assert r.block_iterations <= O.block_pcg(plan, B, tol=1e-10).iterations.max()


def test_block_ecg_rank_deficient_and_zero_columns():
    _, plan, B = _stack(2, 2)
    B3 = np.stack([B[0], B[0], np.zeros_like(B[0]), B[1]])  # duplicated and zero columns
    r = O.block_ecg(plan, B3)
    ref = O.block_pcg(plan, B3)
    assert r.converged.all() and r.iterations[2] == 0 and not np.any(r.x[2])
    for j in (0, 1, 3):
        err = np.linalg.norm(r.x[j] - ref.x[j]) / np.linalg.norm(ref.x[j])
        assert err < 1e-6


def test_sym_pinv_drops_null_directions():
    rng = np.random.default_rng(3)
    V = np.linalg.qr(rng.standard_normal((5, 5)))[0]
    w = np.array([4.0, 2.0, 1.0, 1e-20, 0.0])
    G = (V * w) @ V.T
    want = (V[:, :3] / w[:3]) @ V[:, :3].T
    np.testing.assert_allclose(O.sym_pinv(G), want, atol=1e-10)


# ------------------------------------------------------------------------------------------
# Two-level a posteriori preconditioner (Eq. 2lvlDef, Alg. 3)
# ------------------------------------------------------------------------------------------

def _dense_A(plan):
    n = 3 * plan.n_kept
    return np.array([O.apply_A(plan, e.reshape(-1, 3), "direct").reshape(-1)
                     for e in np.eye(n)]).T


def test_lanczos_relation_and_orthonormal_basis():
    _, plan, B = _stack(3, 1)
    lz = O.lanczos(plan, B[0], 12, apply=lambda v: O.apply_A(plan, v, "direct"))
    V = lz.V.reshape(lz.m, -1).T
    AV = lz.AV.reshape(lz.m, -1).T
    A = _dense_A(plan)
    # the stored products are A v_k, and A V_m = V_m T_m + beta_(m+1) v_(m+1) e_m^T
    np.testing.assert_allclose(AV, A @ V, atol=1e-12 * np.abs(AV).max())
    resid = AV - V @ lz.T()
    resid[:, -1] -= lz.beta[lz.m] * lz.v_next.reshape(-1)
    assert np.abs(resid).max() <= 1e-12 * np.abs(AV).max()
    assert np.abs(V.T @ V - np.eye(lz.m)).max() < 1e-10
    np.testing.assert_allclose(V[:, 0], B[0].reshape(-1) / np.linalg.norm(B[0]), atol=1e-15)


def test_lanczos_ritz_values_inside_and_converging_to_spectrum():
    _, plan, B = _stack(4, 1)
    A = _dense_A(plan)
    ev = np.linalg.eigvalsh(0.5 * (A + A.T))
    lz = O.lanczos(plan, B[0], 60, apply=lambda v: O.apply_A(plan, v, "direct"))
    theta = np.linalg.eigvalsh(lz.T())
    assert theta[0] >= ev[0] * (1 - 1e-9) and theta[-1] <= ev[-1] * (1 + 1e-9)
    assert abs(theta[-1] - ev[-1]) / ev[-1] < 1e-8


def _deflation_from_Z(plan, Z, apply):
    Zp = np.stack([apply(z) for z in Z])
    E = Z.reshape(len(Z), -1) @ Zp.reshape(len(Z), -1).T
    return O.Deflation(Z, Zp, E, O.sym_pinv(0.5 * (E + E.T)), np.zeros(len(Z)))


def test_2lvl_maps_deflation_space_to_itself():
    # A-DEF1: (I - A Q) A Z = 0, so M_2lvl A Z = Q A Z = Z for any full-rank Z
    _, plan, _ = _stack(5, 1)
    apply = lambda v: O.apply_A(plan, v, "direct")  # noqa: E731
    Z = np.random.default_rng(5).standard_normal((7, plan.n_kept, 3))
    df = _deflation_from_Z(plan, Z, apply)
    for j in range(7):
        got = O.precond_2lvl(plan, df, apply(Z[j]))
        np.testing.assert_allclose(got, Z[j], atol=1e-9 * np.abs(Z[j]).max())


def test_2lvl_with_full_eigenbasis_is_the_inverse():
    _, plan, B = _stack(6, 1)
    apply = lambda v: O.apply_A(plan, v, "direct")  # noqa: E731
    A = _dense_A(plan)
    _, U = np.linalg.eigh(0.5 * (A + A.T))
    Z = U.T.reshape(-1, plan.n_kept, 3)
    df = _deflation_from_Z(plan, Z, apply)
    res = O.pcg(plan, B[0], tol=1e-10, apply=apply, precond=lambda r: O.precond_2lvl(plan, df, r))
    assert res.converged and res.iterations == 1
    xs = np.linalg.solve(A, B[0].reshape(-1))
    assert np.linalg.norm(res.x.reshape(-1) - xs) / np.linalg.norm(xs) < 1e-9


def test_2lvl_pcg_solves_the_system():
    prob, plan, B = _stack(7, 3)
    apply = lambda v: O.apply_A(plan, v, "direct")  # noqa: E731
    A = _dense_A(plan)
    kappa = np.linalg.cond(A)
    df = O.deflation_from_lanczos(O.lanczos(plan, B[0], 24, apply=apply))
    assert df.Z.shape[0] == 24
    for j in range(3):
        bd = O.pcg(plan, B[j], tol=1e-10, apply=apply)
        tl = O.pcg(plan, B[j], tol=1e-10, apply=apply,
                   precond=lambda r: O.precond_2lvl(plan, df, r))
        xs = np.linalg.solve(A, B[j].reshape(-1))
        assert tl.converged and np.linalg.norm(tl.x.reshape(-1) - xs) / np.linalg.norm(xs) <= kappa * 1e-10
        assert tl.iterations <= bd.iterations
    # the start vector's own system gains most: its Krylov space is the one already built
    own = O.pcg(plan, B[0], tol=1e-10, apply=apply, precond=lambda r: O.precond_2lvl(plan, df, r))
    assert own.iterations <= O.pcg(plan, B[0], tol=1e-10, apply=apply).iterations // 2


def test_2lvl_planted_swap_of_Z_and_AZ_is_caught():
    _, plan, _ = _stack(5, 1)
    apply = lambda v: O.apply_A(plan, v, "direct")  # noqa: E731
    Z = np.random.default_rng(8).standard_normal((5, plan.n_kept, 3))
    df = _deflation_from_Z(plan, Z, apply)
    bad = O.Deflation(df.Zp, df.Z, df.E, df.Einv, df.theta)
    got = O.precond_2lvl(plan, bad, apply(Z[0]))
    assert np.abs(got - Z[0]).max() > 1e-3 * np.abs(Z[0]).max()
