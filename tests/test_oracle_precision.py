"""Pins of the oracle's single-precision emulation and of its stacked-RHS recurrences (CPU only).

The emulation (``apply_A(emulate_fp32=True)``, ``noise_weight_fft(single=True)``) models FP32
time-domain storage and FP32 Toeplitz arithmetic, so that the precision floor of such a product
is measured on the CPU, independently of the GPU code.  It is pinned by what defines it: the
vectors it stores are exactly FP32-representable, its Toeplitz product is the dense product up
to an FP32-sized error (and not closer than FP64 would be), and its effect on the solve stays
within committed bounds.  The floor figures used for the GPU tolerances come from
``test_fp32_floor_of_the_solve``.

``block_ecg`` folds the inverse square roots of Alg. 2 into one pseudo-inverse; it is pinned
iterate by iterate against ``block_ecg_literal``, which takes Alg. 2's steps as written
(P_k = Z_k (Z_k^T A Z_k)^(-1/2), alpha_k = P_k^T R, Z_(k+1) = (I - P_k P_k^T A) M R), and the
literal form is pinned by Alg. 1 (t = 1) and the A-orthonormality of its search block.
"""

import numpy as np
import pytest

import oracle as O
import synth

U32 = 2.0 ** -24  # unit roundoff of float32


def _fp32_exact(v):
    v = np.asarray(v, np.float64)
    return np.array_equal(v, v.astype(np.float32).astype(np.float64))


def _dense_noise_inverse(prob, n):
    M = np.eye(n)
    for s, L, b in zip(prob.blk_start, prob.blk_len, prob.blk_band):
        c = np.asarray(prob.bands[b], np.float64)
        for i in range(int(s), int(s + L)):
            for j in range(max(int(s), i - c.size + 1), min(int(s + L), i + c.size)):
                M[i, j] = c[abs(i - j)]
    return M


# ------------------------------------------------------------------------------------------
# Single-precision Toeplitz product
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1])
def test_single_fft_is_dense_product_to_fp32_accuracy(seed):
    prob = synth.make_random_small(seed=seed, n_samples=600, n_pix=12, n_dets=3, lam_max=40,
                                   flag_frac=0.0, gap_frac=0.2, dwell=3)
    plan = O.plan_from_problem(prob)
    x = O.to_fp32(np.random.default_rng(seed).standard_normal(plan.n_samples))
    N = _dense_noise_inverse(prob, plan.n_samples)
    ref = N @ x
    got = O.noise_weight_fft(x, plan, single=True)
    # bound per sample: sum_j |N_ij x_j| times u32 and the transform depth
    scale = np.abs(N) @ np.abs(x)
    lam = max(len(b) - 1 for b in prob.bands)
    depth = np.log2(O.default_fft_size(lam))
    err = np.abs(got - ref)
    assert np.all(err <= 8.0 * depth * U32 * scale + 1e-300)
    # ... and really single precision: far above what FP64 would leave
    assert err.max() > 1e3 * np.finfo(np.float64).eps * scale.max()
    # the FP64 product of the same routine is exact to FP64 rounding
    assert np.abs(O.noise_weight_fft(x, plan) - ref).max() <= 1e-12 * scale.max()


# ------------------------------------------------------------------------------------------
# Emulated system product: what it stores, and how far it is from FP64
# ------------------------------------------------------------------------------------------

def _capture(monkeypatch):
    """Record the time-domain vectors that the emulated product hands to the Toeplitz step and
    to the pointing sums."""
    seen = {}
    mm = O.mapmaking
    nw, pt = mm.noise_weight, mm.point

    def nw_spy(x, plan, method="auto", single=False):
        seen["t"] = np.array(x, np.float64)
        seen["single"] = bool(single)
        return nw(x, plan, method, single=single)

    def pt_spy(plan, t):
        seen["u"] = np.array(t, np.float64)
        return pt(plan, t)

    monkeypatch.setattr(mm, "noise_weight", nw_spy)
    monkeypatch.setattr(mm, "point", pt_spy)
    return seen


def _emulation_pins_pass(monkeypatch, plan, x):
    seen = _capture(monkeypatch)
    y = O.apply_A(plan, x, emulate_fp32=True)
    monkeypatch.undo()
    y64 = O.apply_A(plan, x)
    rel = np.linalg.norm(y - y64) / np.linalg.norm(y64)
    # stored vectors are FP32, the Toeplitz step is the single-precision routine pinned above,
    # and the product sits an FP32-sized distance from the FP64 one
    return (_fp32_exact(seen["t"]) and _fp32_exact(seen["u"]) and seen["single"]
            and 1e-10 <= rel <= 1e-5)


def _raster_plan():
    prob = synth.make_raster(cfg_id=71, n_dets=2, side=16, dwell=8, lam=96)
    return O.plan_from_problem(prob)


def test_emulated_product_stores_fp32_and_differs_by_fp32_amounts(monkeypatch):
    plan = _raster_plan()
    x = np.random.default_rng(4).standard_normal((plan.n_kept, 3))
    assert _emulation_pins_pass(monkeypatch, plan, x)


@pytest.mark.parametrize("mistake", ["forgot_round_t", "forgot_round_u", "fp64_fft"])
def test_emulation_planted_mistakes_are_caught(monkeypatch, mistake):
    plan = _raster_plan()
    x = np.random.default_rng(4).standard_normal((plan.n_kept, 3))
    mm = O.mapmaking
    nw = mm.noise_weight
    if mistake == "forgot_round_t":
        # apply_A rounds twice: the un-pointed vector first, the Toeplitz output second
        calls = {"n": 0}
        real = mm.to_fp32

        def first_is_identity(v):
            calls["n"] += 1
            return np.asarray(v, np.float64) if calls["n"] % 2 == 1 else real(v)
        monkeypatch.setattr(mm, "to_fp32", first_is_identity)
    elif mistake == "forgot_round_u":
        calls = {"n": 0}
        real = mm.to_fp32

        def second_is_identity(v):
            calls["n"] += 1
            return np.asarray(v, np.float64) if calls["n"] % 2 == 0 else real(v)
        monkeypatch.setattr(mm, "to_fp32", second_is_identity)

        def nw_fp64_tail(x, plan, method="auto", single=False):
            # a product whose output is not FP32 (single transform, FP64 tail), as a product
            # that skipped the final rounding would leave on blocks with lambda = 0
            return nw(x, plan, method, single=single) * (1.0 + 1e-12)
        monkeypatch.setattr(mm, "noise_weight", nw_fp64_tail)
    elif mistake == "fp64_fft":
        # the transform ignores the single-precision switch
        fft = mm.noise_weight_fft
        monkeypatch.setattr(mm, "noise_weight_fft",
                            lambda x, plan, nfft=None, single=False: fft(x, plan, nfft, False))
    single_ok = _single_fft_above_fp64(plan)
    bad_pass = single_ok and _emulation_pins_pass(monkeypatch, plan, x)
    assert not bad_pass


def _single_fft_above_fp64(plan):
    """The single-precision Toeplitz routine leaves an error far above FP64 rounding."""
    x = O.to_fp32(np.random.default_rng(9).standard_normal(plan.n_samples))
    a = O.mapmaking.noise_weight_fft(x, plan, single=True)
    b = O.mapmaking.noise_weight_direct(x, plan)
    return np.abs(a - b).max() > 1e3 * np.finfo(np.float64).eps * np.abs(b).max()


def test_unplanted_emulation_passes_every_pin(monkeypatch):
    plan = _raster_plan()
    x = np.random.default_rng(4).standard_normal((plan.n_kept, 3))
    assert _single_fft_above_fp64(plan) and _emulation_pins_pass(monkeypatch, plan, x)


def test_fp32_floor_of_the_solve():
    """The precision floor of FP32 time-domain products, measured on the tiny raster (the
    4-detector, 65,536-sample configuration at full size) and on a ground-like scan (8
    detectors x 2^17 samples, intervals of 2^16, 64 x 64 patch, lambda 4096):
      * the map of a PCG that uses the emulated product for A and b, stopped at the recursive
        1e-8, lies 3e-8..5e-7 (rel. L2) from the FP64 map at 1e-8;
      * its FP64 true residual ||b64 - A64 x|| / ||b64|| lies 1e-8..2e-7, i.e. above 1e-8:
        FP32 Toeplitz arithmetic alone keeps the true residual from reaching the tolerance;
      * one step of refinement (FP64 residual, emulated inner solve to 0.05, FP64 update)
        brings the FP64 true residual below 1e-8.
    Measured when the test was written: maps 9.1e-8 / 2.2e-7, true residuals 6.0e-8 / 5.5e-8,
    after refinement 3-4e-9."""
    cases = [synth.make_raster(cfg_id=0),
             synth.make_ground(cfg_id=1, n_dets=8, samples_per_det=1 << 17, interval=1 << 16,
                               side=64, lam=4096)]
    for prob in cases:
        plan = O.plan_from_problem(prob)
        d = np.where(plan.lpix >= 0, prob.d[0].astype(np.float64), 0.0)
        b64 = O.rhs(plan, d)
        nb = np.linalg.norm(b64)
        A64 = lambda v: O.apply_A(plan, v)  # noqa: E731
        Aem = lambda v: O.apply_A(plan, v, emulate_fp32=True)  # noqa: E731
        bem = O.point(plan, O.to_fp32(O.noise_weight(O.to_fp32(d), plan, "fft", single=True)))
        ref = O.pcg(plan, b64, tol=1e-8)
        em = O.pcg(plan, bem, tol=1e-8, apply=Aem)
        assert ref.converged and em.converged
        dmap = np.linalg.norm(em.x - ref.x) / np.linalg.norm(ref.x)
        true64 = np.linalg.norm(b64 - A64(em.x)) / nb
        assert 3e-8 <= dmap <= 5e-7, dmap
        assert 1e-8 <= true64 <= 2e-7, true64
        r = b64 - A64(em.x)
        inner = O.pcg(plan, r, tol=0.05, apply=Aem)
        x1 = em.x + inner.x
        assert np.linalg.norm(b64 - A64(x1)) / nb < 1e-8


# ------------------------------------------------------------------------------------------
# Alg. 2 (Orthomin) as written, and the folded recurrences against it
# ------------------------------------------------------------------------------------------

def _stack(seed, k, lam=64):
    prob = synth.make_raster(cfg_id=80 + seed, n_dets=2, side=12, dwell=6, lam=lam, n_rhs=k)
    plan = O.plan_from_problem(prob)
    B = np.stack([O.rhs(plan, prob.d[j], "direct") for j in range(k)])
    apply = lambda v: O.apply_A(plan, v, "direct")  # noqa: E731
    return plan, B, apply


def test_literal_ecg_with_one_column_is_alg1():
    plan, B, apply = _stack(0, 1)
    lit = O.block_ecg_literal(plan, B, apply=apply)
    p = O.pcg(plan, B[0], apply=apply)
    assert lit.block_iterations == p.iterations
    np.testing.assert_allclose(lit.x[0], p.x, rtol=0, atol=1e-11 * np.abs(p.x).max())


def test_literal_ecg_search_block_is_A_orthonormal():
    plan, B, apply = _stack(1, 4)
    seen = []

    def grab(k, X, R):
        seen.append((X.copy(), R.copy()))
    O.block_ecg_literal(plan, B, tol=1e-10, apply=apply, on_iter=grab)
    # X_k - X_(k-1) = P_k alpha_k lies in span(P_k); with P_k^T A P_k = I the residual update
    # is A-orthogonal to every earlier step: <dX_i, A dX_j> = 0 for i != j (block CG property)
    dX = [seen[0][0]] + [seen[i][0] - seen[i - 1][0] for i in range(1, min(len(seen), 6))]
    for i in range(len(dX)):
        for j in range(i):
            for a in range(B.shape[0]):
                for c in range(B.shape[0]):
                    u, v = dX[i][a], dX[j][c]
                    num = abs(np.sum(u * apply(v)))
                    den = np.sqrt(np.sum(u * apply(u)) * np.sum(v * apply(v))) + 1e-300
                    assert num <= 1e-6 * den


@pytest.mark.parametrize("seed,k", [(2, 3), (3, 6)])
def test_folded_ecg_equals_literal_iterate_by_iterate(seed, k):
    plan, B, apply = _stack(seed, k)
    lit, fold = [], []
    r1 = O.block_ecg_literal(plan, B, tol=1e-9, apply=apply,
                             on_iter=lambda i, X, R: lit.append(X.copy()))
    r2 = O.block_ecg(plan, B, tol=1e-9, apply=apply,
                     on_iter=lambda i, X, R: fold.append(X.copy()))
    assert r1.block_iterations == r2.block_iterations
    np.testing.assert_array_equal(r1.iterations, r2.iterations)
    for a, b in zip(lit, fold):
        scale = np.abs(a).max()
        assert np.abs(a - b).max() <= 1e-9 * scale


def test_literal_ecg_planted_missing_projection_is_caught():
    """Dropping the (I - P P^T A) projection turns the search block into the bare
    preconditioned residual: the iterates then leave the literal Alg. 2 sequence."""
    plan, B, apply = _stack(4, 3)
    good = []
    O.block_ecg_literal(plan, B, tol=1e-9, apply=apply,
                        on_iter=lambda i, X, R: good.append(X.copy()))
    assert len(good) >= 3
    # planted: the same block steps with the projection dropped (Z <- M R)
    Bf = B.reshape(B.shape[0], -1)
    X = np.zeros_like(Bf)
    R = Bf.copy()
    shape = B.shape[1:]
    M = lambda v: O.precond_bj(plan, v)  # noqa: E731
    Z = np.stack([M(r.reshape(shape)).reshape(-1) for r in R])
    planted = []
    for _ in range(3):
        AZ = np.stack([apply(z.reshape(shape)).reshape(-1) for z in Z])
        S = O.mapmaking._sym_inv_sqrt(Z @ AZ.T, 1e-12)
        P, AP = S @ Z, S @ AZ
        al = P @ R.T
        X += (P.T @ al).T
        R -= (AP.T @ al).T
        planted.append(X.reshape(B.shape).copy())
        Z = np.stack([M(r.reshape(shape)).reshape(-1) for r in R])
    # the first step agrees (no projection yet); later steps leave the Alg. 2 sequence
    assert np.abs(planted[0] - good[0]).max() <= 1e-9 * np.abs(good[0]).max()
    diff = max(np.abs(planted[i] - good[i]).max() / np.abs(good[i]).max() for i in (1, 2))
    assert diff > 1e-3
