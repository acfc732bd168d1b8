"""FP64 reference for the maximum-likelihood map-maker solved by block-Jacobi PCG.

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the benchmark's CPU baseline;
never by the library.  Plain NumPy/SciPy in float64, written from the paper (arXiv:2112.03370):

  system      (P^T N^-1 P) m = P^T N^-1 d        Eq. genMapEstimator with F_T = W^-1 = N^-1
  pointing    one pixel and weights (1, cos2psi, sin2psi) per sample   Eq. dataModelSingleSlot
  noise       block-diagonal banded Toeplitz N^-1, identity outside blocks  Eq. MADCAP, stbmm
  BJ          M_BD = (P^T diag(N^-1) P)^-1, 3x3 per pixel, condition-number excision
  solver      PCG as in Alg. 1 (x0 = 0, stop on ||r|| < eps ||b||)

Readings where the paper is silent (each also listed in the design notes):
  * band coefficients c_0..c_lambda inclusive (Eq. MADCAP keeps |t - t'| <= lambda);
  * Toeplitz products are truncated at block edges (no wrap); uncovered samples pass unchanged;
  * flagged (pix = -1) and excised samples behave as gaps: their P rows and data are zero;
  * diag(N^-1) of a sample is c_0 of its block's band, 1 outside blocks;
  * a pixel is kept when it has >= 3 hits and its 3x3 BJ block has condition number <= cond_max
    (default 1e3; the paper sets a threshold without a value);
  * a zero right-hand side (or an exactly converged start) returns after 0 iterations.

Two-level a posteriori preconditioner (Eq. 2lvlDef, A-DEF1; Alg. 3):
  * Lanczos runs on A itself (not on M_BD A), from r0 = b (x0 = 0), storing V_m and A V_m;
  * the deflation space takes all m Ritz vectors Z = V_m X of the tridiagonal T_m = X Theta X^T,
    with Z' = (A V_m) X and E = Z^T Z' formed explicitly, as the paper does;
  * E^-1 is a pseudo-inverse (the paper uses a least-squares SVD solver): E is symmetrized and
    its eigen-directions with eigenvalues <= 1e-12 of the largest are dropped.
"""

from __future__ import annotations

import dataclasses
import os
from typing import Optional

import numpy as np
import scipy.fft as sfft
import scipy.linalg as sla

__all__ = [
    "OraclePlan", "build_plan", "plan_from_problem", "sample_diagonal", "hits_global",
    "bj_blocks_global", "condition_numbers", "noise_weight_direct",
    "noise_weight_fft", "noise_weight", "unpoint", "point", "rhs", "apply_A", "precond_bj",
    "PCGResult", "pcg", "lanczos_extremes", "binned_map", "dense_pointing",
    "dense_noise_inverse", "dense_A", "solve_dense", "default_fft_size", "block_pcg",
    "BlockPCGResult", "block_ecg", "sym_pinv", "LanczosResult", "lanczos", "Deflation",
    "deflation_from_lanczos", "precond_2lvl", "to_fp32", "block_ecg_literal",
]

DEFAULT_COND_MAX = 1.0e3
MIN_HITS = 3


def _threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return max(1, os.cpu_count() or 1)


# --------------------------------------------------------------------------------------------
# Plan: hits, block-Jacobi blocks, excision, compaction  (MAPMAT local pixels; BJ section)
# --------------------------------------------------------------------------------------------

@dataclasses.dataclass
class OraclePlan:
    n_samples: int
    n_pix_global: int
    lpix: np.ndarray          # int64 [N_s], local pixel (rank among kept global ids) or -1
    wq: np.ndarray            # float64 [N_s]
    wu: np.ndarray            # float64 [N_s]
    kept: np.ndarray          # int64 [n_kept], ascending global ids
    hits: np.ndarray          # int64 [n_kept]
    n_excised: int            # observed pixels dropped by the hit / condition test
    blk_start: np.ndarray
    blk_len: np.ndarray
    blk_band: np.ndarray
    bands: list               # float64 arrays c_0..c_lambda
    diag: np.ndarray          # float64 [N_s] diag(N^-1)
    B: np.ndarray             # float64 [n_kept, 3, 3]  P^T diag(N^-1) P blocks
    Minv: np.ndarray          # float64 [n_kept, 3, 3]
    cond: np.ndarray          # float64 [n_kept]

    @property
    def n_kept(self) -> int:
        return int(self.kept.size)


def sample_diagonal(n_samples, blk_start, blk_len, blk_band, bands):
    """diag(N^-1) per sample: c_0 of the covering block's band, 1 for samples outside every
    block (stbmm copies uncovered rows unchanged, i.e. a unit diagonal)."""
    diag = np.ones(n_samples, dtype=np.float64)
    for s, L, b in zip(blk_start, blk_len, blk_band):
        diag[int(s):int(s) + int(L)] = float(bands[int(b)][0])
    return diag


def hits_global(pix, n_pix_global):
    """Number of unflagged samples observing each global pixel (MAPMAT local pixel set)."""
    pix = np.asarray(pix)
    ok = pix >= 0
    return np.bincount(pix[ok].astype(np.int64), minlength=n_pix_global).astype(np.int64)


def bj_blocks_global(pix, wq, wu, diag, n_pix_global):
    """B_p = sum over samples of pixel p of diag(N^-1)_s w_s w_s^T with w = (1, cos, sin)
    (block-Jacobi preconditioner, first construction step)."""
    pix = np.asarray(pix)
    ok = pix >= 0
    p = pix[ok].astype(np.int64)
    w = [np.ones(p.size), np.asarray(wq, np.float64)[ok], np.asarray(wu, np.float64)[ok]]
    c = np.asarray(diag, np.float64)[ok]
    B = np.zeros((n_pix_global, 3, 3))
    for a in range(3):
        for b in range(a, 3):
            v = np.bincount(p, weights=c * w[a] * w[b], minlength=n_pix_global)
            B[:, a, b] = v
            B[:, b, a] = v
    return B


def condition_numbers(B):
    """2-norm condition number of each symmetric 3x3 block (inf when not positive definite)."""
    ev = np.linalg.eigvalsh(B)
    lo, hi = ev[:, 0], ev[:, -1]
    with np.errstate(divide="ignore", invalid="ignore"):
        cond = np.where(lo > 0.0, hi / np.where(lo > 0.0, lo, 1.0), np.inf)
    return cond


def build_plan(pix, wq, wu, n_pix_global, blk_start, blk_len, blk_band, bands,
               cond_max=DEFAULT_COND_MAX, min_hits=MIN_HITS):
    """Hits, BJ blocks, excision of ill-conditioned pixels and global->local compaction.

    Follows the BJ construction (accumulate, then invert each block and evaluate its condition
    number, excising pixels above the threshold together with their samples) and the MAPMAT
    global/local pixel indexing (local index = rank of the global id among kept pixels)."""
    pix = np.asarray(pix).astype(np.int64)
    n_s = pix.size
    if np.any(pix < -1) or np.any(pix >= n_pix_global):
        raise ValueError("pixel index out of range")
    bands64 = [np.asarray(b, np.float64) for b in bands]
    diag = sample_diagonal(n_s, blk_start, blk_len, blk_band, bands64)
    h = hits_global(pix, n_pix_global)
    Bg = bj_blocks_global(pix, wq, wu, diag, n_pix_global)
    observed = h > 0
    cond = np.full(n_pix_global, np.inf)
    if np.any(observed):
        cond[observed] = condition_numbers(Bg[observed])
    keep = observed & (h >= min_hits) & (cond <= cond_max)
    kept = np.flatnonzero(keep).astype(np.int64)
    local = np.full(n_pix_global, -1, np.int64)
    local[kept] = np.arange(kept.size)
    lpix = np.where(pix >= 0, local[np.maximum(pix, 0)], -1)
    B = Bg[kept]
    Minv = np.linalg.inv(B) if kept.size else np.zeros((0, 3, 3))
    return OraclePlan(
        n_samples=n_s, n_pix_global=int(n_pix_global), lpix=lpix,
        wq=np.asarray(wq, np.float64), wu=np.asarray(wu, np.float64), kept=kept,
        hits=h[kept], n_excised=int(observed.sum() - kept.size),
        blk_start=np.asarray(blk_start, np.int64), blk_len=np.asarray(blk_len, np.int64),
        blk_band=np.asarray(blk_band, np.int64), bands=bands64, diag=diag, B=B, Minv=Minv,
        cond=cond[kept])


def plan_from_problem(prob, cond_max=DEFAULT_COND_MAX):
    """Convenience wrapper taking any object with the problem's array attributes."""
    return build_plan(prob.pix, prob.wq, prob.wu, prob.n_pix_global, prob.blk_start,
                      prob.blk_len, prob.blk_band, prob.bands, cond_max=cond_max)


# --------------------------------------------------------------------------------------------
# Block-diagonal banded Toeplitz N^-1  (Toeplitz algebra package, Eq. MADCAP)
# --------------------------------------------------------------------------------------------

def noise_weight_direct(x, plan):
    """y = N^-1 x by the definition: y_i = sum_{j in block, |i-j| <= lambda} c_|i-j| x_j inside
    each block (truncated at its edges), y_i = x_i for samples outside every block (stbmm)."""
    x = np.asarray(x, np.float64)
    y = x.copy()
    for s, L, b in zip(plan.blk_start, plan.blk_len, plan.blk_band):
        s, L = int(s), int(L)
        c = plan.bands[int(b)]
        xb = x[s:s + L]
        yb = c[0] * xb
        for k in range(1, min(c.size, L)):
            yb[k:] += c[k] * xb[:-k]
            yb[:-k] += c[k] * xb[k:]
        y[s:s + L] = yb
    return y


def default_fft_size(lam):
    """Smallest power of two >= 4 lambda (at least 8): half of each segment is output."""
    n = 8
    while n < 4 * lam:
        n *= 2
    return n


def noise_weight_fft(x, plan, nfft=None, single=False):
    """y = N^-1 x by the shift-and-overlap algorithm of the Toeplitz package: each block is cut
    into overlapping segments of nfft samples (nfft - 2 lambda outputs each), every segment's
    product is done by embedding the band in an nfft circulant and using real FFTs.  Zero
    padding of lambda samples at both block ends truncates the band there.  ``single=True``
    computes the FFTs in single precision (used only to measure the FP32 precision floor)."""
    x = np.asarray(x, np.float64)
    y = x.copy()
    ftype = np.float32 if single else np.float64
    for s, L, b in zip(plan.blk_start, plan.blk_len, plan.blk_band):
        s, L = int(s), int(L)
        c = plan.bands[int(b)]
        lam = c.size - 1
        if lam == 0:
            y[s:s + L] = c[0] * x[s:s + L]
            continue
        n = nfft or default_fft_size(lam)
        if n <= 2 * lam:
            raise ValueError("nfft must exceed 2 lambda")
        out = n - 2 * lam
        n_seg = -(-L // out)
        h = np.zeros(n)
        h[0] = c[0]
        h[1:lam + 1] = c[1:]
        h[n - lam:] = c[1:][::-1]
        H = sfft.rfft(h.astype(ftype))
        xp = np.zeros(n_seg * out + 2 * lam)
        xp[lam:lam + L] = x[s:s + L]
        idx = np.arange(n_seg)[:, None] * out + np.arange(n)[None, :]
        seg = xp[idx].astype(ftype)
        Y = sfft.irfft(sfft.rfft(seg, axis=1, workers=_threads()) * H[None, :], n, axis=1,
                       workers=_threads())
        y[s:s + L] = Y[:, lam:lam + out].reshape(-1)[:L].astype(np.float64)
    return y


def noise_weight(x, plan, method="auto", single=False):
    if method == "direct":
        return noise_weight_direct(x, plan)
    if method == "fft":
        return noise_weight_fft(x, plan, single=single)
    lam = max((c.size - 1 for c in plan.bands), default=0)
    if single or lam > 64:
        return noise_weight_fft(x, plan, single=single)
    return noise_weight_direct(x, plan)


# --------------------------------------------------------------------------------------------
# Pointing: un-pointing t = P m and pointing m = P^T t  (MAPMAT core operations)
# --------------------------------------------------------------------------------------------

def unpoint(plan, m):
    """t_s = m[p_s, I] + cos2psi_s m[p_s, Q] + sin2psi_s m[p_s, U]; zero at gap samples."""
    m = np.asarray(m, np.float64).reshape(-1, 3)
    ok = plan.lpix >= 0
    lp = np.where(ok, plan.lpix, 0)
    t = m[lp, 0] + plan.wq * m[lp, 1] + plan.wu * m[lp, 2]
    return np.where(ok, t, 0.0)


def point(plan, t):
    """(P^T t)[p] = sum over samples of pixel p of (1, cos2psi, sin2psi) t_s."""
    t = np.asarray(t, np.float64)
    ok = plan.lpix >= 0
    p = plan.lpix[ok]
    tt = t[ok]
    out = np.zeros((plan.n_kept, 3))
    out[:, 0] = np.bincount(p, weights=tt, minlength=plan.n_kept)
    out[:, 1] = np.bincount(p, weights=plan.wq[ok] * tt, minlength=plan.n_kept)
    out[:, 2] = np.bincount(p, weights=plan.wu[ok] * tt, minlength=plan.n_kept)
    return out


def rhs(plan, d, method="auto"):
    """b = P^T N^-1 d, with d zeroed at gap samples (flagged or excised)."""
    d = np.where(plan.lpix >= 0, np.asarray(d, np.float64), 0.0)
    return point(plan, noise_weight(d, plan, method))


def to_fp32(v):
    """Round to the nearest float32 and return as float64 (the rounding of a stored FP32
    time-domain vector)."""
    return np.asarray(v, np.float64).astype(np.float32).astype(np.float64)


def apply_A(plan, x, method="auto", emulate_fp32=False):
    """A x = P^T N^-1 P x applied right to left: un-point, Toeplitz product, point.

    ``emulate_fp32`` models single-precision time-domain storage and arithmetic (a
    precision-floor study, not the method): the un-pointed vector is rounded to float32, the
    Toeplitz product runs with float32 FFTs, and its result is rounded to float32 before the
    float64 pointing sums.  Pointing sums and everything in the pixel domain stay float64."""
    t = unpoint(plan, x)
    if emulate_fp32:
        u = to_fp32(noise_weight(to_fp32(t), plan, "fft", single=True))
    else:
        u = noise_weight(t, plan, method)
    return point(plan, u)


def precond_bj(plan, r):
    """z_p = M_BD r_p = B_p^-1 r_p per kept pixel."""
    r = np.asarray(r, np.float64).reshape(-1, 3)
    return np.einsum("pab,pb->pa", plan.Minv, r)


# --------------------------------------------------------------------------------------------
# PCG (Alg. 1) and the CG-Lanczos spectrum estimate
# --------------------------------------------------------------------------------------------

@dataclasses.dataclass
class PCGResult:
    x: np.ndarray
    iterations: int
    relres: float            # recursive ||r_k|| / ||b||
    true_relres: float       # ||b - A x_k|| / ||b||
    converged: bool
    alphas: list
    betas: list
    history: list            # recursive relative residual after each iteration
    status: str = "ok"


def pcg(plan, b, tol=1e-8, max_iter=10000, x0=None, apply=None, precond=None):
    """Alg. 1: r0 = b - A x0, z0 = M r0, p0 = z0; per step alpha = <r,z>/<Ap,p>, x += alpha p,
    r -= alpha Ap, stop when ||r|| < eps ||b||, z = M r, beta = <r',z'>/<r,z>, p = z + beta p."""
    A = apply or (lambda v: apply_A(plan, v))
    M = precond or (lambda v: precond_bj(plan, v))
    b = np.asarray(b, np.float64).reshape(-1, 3)
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, np.float64).reshape(-1, 3).copy()
    nb = float(np.linalg.norm(b))
    alphas, betas, hist = [], [], []
    if nb == 0.0:
        return PCGResult(np.zeros_like(b), 0, 0.0, 0.0, True, alphas, betas, hist)
    r = b - A(x) if x0 is not None else b.copy()
    if np.linalg.norm(r) < tol * nb:
        return PCGResult(x, 0, float(np.linalg.norm(r) / nb), float(np.linalg.norm(r) / nb),
                         True, alphas, betas, hist)
    z = M(r)
    p = z.copy()
    rz = float(np.sum(r * z))
    status = "no_conv"
    k = 0
    converged = False
    while k < max_iter:
        q = A(p)
        pq = float(np.sum(p * q))
        if not (pq > 0.0) or not (rz > 0.0):
            status = "not_spd"
            break
        alpha = rz / pq
        x = x + alpha * p
        r = r - alpha * q
        k += 1
        alphas.append(alpha)
        rel = float(np.linalg.norm(r) / nb)
        hist.append(rel)
        if rel < tol:
            converged = True
            status = "ok"
            break
        z = M(r)
        rz_new = float(np.sum(r * z))
        beta = rz_new / rz
        betas.append(beta)
        rz = rz_new
        p = z + beta * p
    true_rel = float(np.linalg.norm(b - A(x)) / nb)
    return PCGResult(x, k, hist[-1] if hist else 1.0, true_rel, converged, alphas, betas, hist,
                     status)


def lanczos_extremes(alphas, betas):
    """Extreme eigenvalues of M A estimated from the CG coefficients: the CG recurrences are a
    Lanczos process (Eq. lanczosDecomp) whose tridiagonal has diagonal 1/alpha_0,
    1/alpha_j + beta_{j-1}/alpha_{j-1} and off-diagonal sqrt(beta_{j-1})/alpha_{j-1}."""
    a = np.asarray(alphas, np.float64)
    bt = np.asarray(betas[: max(0, a.size - 1)], np.float64)
    if a.size == 0:
        return np.nan, np.nan
    d = 1.0 / a
    d[1:] += bt / a[:-1]
    e = np.sqrt(bt) / a[:-1]
    ev = sla.eigvalsh_tridiagonal(d, e) if a.size > 1 else d
    return float(ev[0]), float(ev[-1])


# --------------------------------------------------------------------------------------------
# Closed forms and brute force for tiny problems
# --------------------------------------------------------------------------------------------

def binned_map(plan, d):
    """Binned estimator (diagonal, unit weights): m_p = (sum w w^T)^-1 sum w d per kept pixel."""
    d = np.asarray(d, np.float64)
    ok = plan.lpix >= 0
    p = plan.lpix[ok]
    w = [np.ones(p.size), plan.wq[ok], plan.wu[ok]]
    G = np.zeros((plan.n_kept, 3, 3))
    v = np.zeros((plan.n_kept, 3))
    for a in range(3):
        v[:, a] = np.bincount(p, weights=w[a] * d[ok], minlength=plan.n_kept)
        for c in range(3):
            G[:, a, c] = np.bincount(p, weights=w[a] * w[c], minlength=plan.n_kept)
    return np.linalg.solve(G, v[..., None])[..., 0]


def dense_pointing(plan):
    """Dense P: row s holds (1, cos2psi_s, sin2psi_s) in the columns of its pixel."""
    P = np.zeros((plan.n_samples, 3 * plan.n_kept))
    for s in range(plan.n_samples):
        p = int(plan.lpix[s])
        if p >= 0:
            P[s, 3 * p] = 1.0
            P[s, 3 * p + 1] = plan.wq[s]
            P[s, 3 * p + 2] = plan.wu[s]
    return P


def dense_noise_inverse(plan):
    """Dense block-diagonal N^-1 with identity rows/columns outside blocks (brute force)."""
    n = plan.n_samples
    Ninv = np.eye(n)
    for s, L, b in zip(plan.blk_start, plan.blk_len, plan.blk_band):
        s, L = int(s), int(L)
        c = plan.bands[int(b)]
        for i in range(L):
            for j in range(L):
                k = abs(i - j)
                Ninv[s + i, s + j] = c[k] if k < c.size else 0.0
    return Ninv


def dense_A(plan):
    P = dense_pointing(plan)
    return P.T @ dense_noise_inverse(plan) @ P


def solve_dense(plan, b):
    """m* = A^-1 b by Cholesky of the dense system matrix (tiny problems only)."""
    A = dense_A(plan)
    c = sla.cho_factor(A)
    return sla.cho_solve(c, np.asarray(b, np.float64).reshape(-1)).reshape(-1, 3)


# --------------------------------------------------------------------------------------------
# Several right-hand sides sharing P and N^-1
# --------------------------------------------------------------------------------------------

@dataclasses.dataclass
class BlockPCGResult:
    x: np.ndarray            # [k, n_kept, 3]
    iterations: np.ndarray   # per column: iteration at which the column met the stop test
    relres: np.ndarray
    converged: np.ndarray
    block_iterations: int = 0


def block_pcg(plan, B, tol=1e-8, max_iter=10000):
    """Each column solved by Alg. 1 independently (the reference for batched solves)."""
    B = np.asarray(B, np.float64)
    k = B.shape[0]
    X = np.zeros_like(B.reshape(k, -1, 3))
    it = np.zeros(k, np.int64)
    rr = np.zeros(k)
    cv = np.zeros(k, bool)
    for j in range(k):
        res = pcg(plan, B[j], tol=tol, max_iter=max_iter)
        X[j], it[j], rr[j], cv[j] = res.x, res.iterations, res.relres, res.converged
    return BlockPCGResult(X, it, rr, cv, int(it.max()) if k else 0)


def sym_pinv(G, rtol=1e-12):
    """Pseudo-inverse of a symmetric positive semi-definite matrix by its eigen-decomposition,
    dropping directions with eigenvalue below rtol * largest (rank-revealing safeguard)."""
    w, V = np.linalg.eigh(G)
    keep = w > rtol * max(w.max(), 0.0) if w.size else w > 0
    inv = np.zeros_like(w)
    inv[keep] = 1.0 / w[keep]
    return (V * inv) @ V.T


def block_ecg(plan, B, tol=1e-8, max_iter=10000, apply=None, precond=None, rtol=1e-12,
              on_iter=None):
    """Enlarged-CG recurrences (Alg. 2, Orthomin variant) on t stacked right-hand sides.

    R_0 = B (X_0 = 0), Z_1 = M R_0; per iteration with W = A Z_k and G = Z_k^T W:
    P_k = Z_k G^{-1/2}, alpha = P_k^T R, X += P_k alpha, R -= A P_k alpha, then
    Z_{k+1} = (I - P_k P_k^T A) M R.  Folding G^{-1/2} G^{-1/2} = G^{-1} the updates read
    X += Z G^-1 (Z^T R), R -= W G^-1 (Z^T R), Z <- M R - Z G^-1 (W^T M R).  G^-1 is the
    eigen-based pseudo-inverse (rank drop below rtol * largest eigenvalue) -- a safeguard the
    paper's Cholesky square root lacks.  A column stops (its X frozen and it leaves the block)
    when ||R_j|| < eps ||B_j||: the per-column stop test of Alg. 1 applied to stacked systems.
    With t = 1 the recurrences are those of Alg. 1.  ``on_iter(k, X, R)`` (optional) sees the
    stacked iterate and residual after iteration k."""
    A = apply or (lambda v: apply_A(plan, v))
    M = precond or (lambda v: precond_bj(plan, v))
    B = np.asarray(B, np.float64)
    t = B.shape[0]
    shape = B.shape[1:]
    Bf = B.reshape(t, -1)
    X = np.zeros_like(Bf)
    R = Bf.copy()
    nb = np.linalg.norm(Bf, axis=1)
    iters = np.zeros(t, np.int64)
    conv = nb == 0.0
    active = np.flatnonzero(~conv)
    Z = np.stack([M(R[j].reshape(shape)).reshape(-1) for j in active]) if active.size else R[:0]
    k = 0
    while active.size and k < max_iter:
        W = np.stack([A(Z[i].reshape(shape)).reshape(-1) for i in range(Z.shape[0])])
        G = Z @ W.T
        Gi = sym_pinv(G, rtol)
        a1 = Gi @ (Z @ R[active].T)                      # [z, active]
        X[active] += (Z.T @ a1).T
        R[active] -= (W.T @ a1).T
        k += 1
        if on_iter is not None:
            on_iter(k, X.reshape(B.shape), R.reshape(B.shape))
        rel = np.linalg.norm(R[active], axis=1) / nb[active]
        done = rel < tol
        iters[active] = k
        conv[active[done]] = True
        keep = ~done
        if not keep.any():
            active = active[keep]
            break
        MR = np.stack([M(R[j].reshape(shape)).reshape(-1) for j in active[keep]])
        a2 = Gi @ (W @ MR.T)
        Z = MR - (Z.T @ a2).T
        active = active[keep]
    relres = np.where(nb > 0, np.linalg.norm(R, axis=1) / np.where(nb > 0, nb, 1.0), 0.0)
    return BlockPCGResult(X.reshape(B.shape), iters, relres, conv, k)


def _sym_inv_sqrt(G, rtol):
    """G^(-1/2) of a symmetric positive semi-definite matrix by its eigen-decomposition,
    restricted to eigenvalues above rtol * largest (the same rank rule as sym_pinv)."""
    w, V = np.linalg.eigh(0.5 * (G + G.T))
    keep = w > rtol * max(w.max(), 0.0) if w.size else w > 0
    s = np.zeros_like(w)
    s[keep] = 1.0 / np.sqrt(w[keep])
    return (V * s) @ V.T


def block_ecg_literal(plan, B, tol=1e-8, max_iter=10000, apply=None, precond=None,
                      rtol=1e-12, on_iter=None):
    """Alg. 2 (Orthomin) step by step on t stacked right-hand sides, with the search block
    normalised explicitly:

        P_k = Z_k (Z_k^T A Z_k)^(-1/2),   alpha_k = P_k^T R_(k-1),
        X_k = X_(k-1) + P_k alpha_k,      R_k = R_(k-1) - (A P_k) alpha_k,
        Z_(k+1) = (I - P_k P_k^T A) M R_k.

    The inverse square root is taken by eigen-decomposition with the rank rule of sym_pinv (the
    paper uses a Cholesky factor; any square root gives the same X and R, since only
    P_k P_k^T enters them).  As in block_ecg, each column is its own right-hand side and leaves
    the block once ||R_j|| < eps ||B_j||.  A reference for block_ecg's folded recurrences."""
    A = apply or (lambda v: apply_A(plan, v))
    M = precond or (lambda v: precond_bj(plan, v))
    B = np.asarray(B, np.float64)
    t = B.shape[0]
    shape = B.shape[1:]
    Bf = B.reshape(t, -1)
    X = np.zeros_like(Bf)
    R = Bf.copy()
    nb = np.linalg.norm(Bf, axis=1)
    iters = np.zeros(t, np.int64)
    conv = nb == 0.0
    active = np.flatnonzero(~conv)
    # columns of the search block are stored as rows: Zr[i] is column i of Z_k
    Zr = np.stack([M(R[j].reshape(shape)).reshape(-1) for j in active]) if active.size else R[:0]
    k = 0
    while active.size and k < max_iter:
        AZ = np.stack([A(z.reshape(shape)).reshape(-1) for z in Zr])
        S = _sym_inv_sqrt(Zr @ AZ.T, rtol)               # (Z^T A Z)^(-1/2)
        Pr = S @ Zr                                       # rows of P_k = Z S
        APr = S @ AZ                                      # rows of A P_k
        alpha = Pr @ R[active].T                          # P_k^T R, [z, active]
        X[active] += (Pr.T @ alpha).T
        R[active] -= (APr.T @ alpha).T
        k += 1
        if on_iter is not None:
            on_iter(k, X.reshape(B.shape), R.reshape(B.shape))
        rel = np.linalg.norm(R[active], axis=1) / nb[active]
        done = rel < tol
        iters[active] = k
        conv[active[done]] = True
        keep = ~done
        active = active[keep]
        if not active.size:
            break
        MR = np.stack([M(R[j].reshape(shape)).reshape(-1) for j in active])
        Zr = MR - (Pr.T @ (APr @ MR.T)).T                 # (I - P P^T A) M R
    relres = np.where(nb > 0, np.linalg.norm(R, axis=1) / np.where(nb > 0, nb, 1.0), 0.0)
    return BlockPCGResult(X.reshape(B.shape), iters, relres, conv, k)


# --------------------------------------------------------------------------------------------
# Two-level a posteriori preconditioner (Eq. 2lvlDef, Alg. 3)
# --------------------------------------------------------------------------------------------

@dataclasses.dataclass
class LanczosResult:
    alpha: np.ndarray        # [m] diagonal of T_m
    beta: np.ndarray         # [m + 1]: beta[0] = ||r0||, beta[k] couples v_k and v_(k+1)
    V: np.ndarray            # [m, n_kept, 3] Lanczos vectors v_1..v_m
    AV: np.ndarray           # [m, n_kept, 3] the stored products A v_k
    v_next: np.ndarray       # v_(m+1) (zero when the process stopped on beta < eps)
    m: int

    def T(self):
        """The tridiagonal T_m = tridiag(beta_i, alpha_i, beta_(i+1))."""
        m = self.m
        t = np.diag(self.alpha[:m])
        if m > 1:
            off = self.beta[1:m]
            t += np.diag(off, 1) + np.diag(off, -1)
        return t


def lanczos(plan, r0, m, apply=None, eps=None):
    """Alg. 3 on A from the start vector r0 (= b - A x0; r0 = b for x0 = 0): v_1 = r0/||r0||;
    per step w = A v_k - beta_k v_(k-1) (A v_k stored), alpha_k = <w, v_k>, w -= alpha_k v_k,
    beta_(k+1) = ||w||, stop when beta_(k+1) < eps, else v_(k+1) = w / beta_(k+1).  eps defaults
    to machine precision times ||r0||."""
    A = apply or (lambda v: apply_A(plan, v))
    r0 = np.asarray(r0, np.float64).reshape(-1, 3)
    b1 = float(np.linalg.norm(r0))
    if eps is None:
        eps = np.finfo(np.float64).eps * max(b1, 1.0)
    alpha = np.zeros(m)
    beta = np.zeros(m + 1)
    beta[0] = b1
    V = np.zeros((m,) + r0.shape)
    AV = np.zeros((m,) + r0.shape)
    if b1 == 0.0:
        return LanczosResult(alpha[:0], beta[:1], V[:0], AV[:0], np.zeros_like(r0), 0)
    v = r0 / b1
    v_prev = np.zeros_like(r0)
    k_done = m
    v_next = np.zeros_like(r0)
    for k in range(m):
        V[k] = v
        av = A(v)
        AV[k] = av
        w = av - (beta[k] * v_prev if k > 0 else 0.0)
        alpha[k] = float(np.sum(w * v))
        w = w - alpha[k] * v
        beta[k + 1] = float(np.linalg.norm(w))
        if beta[k + 1] < eps:
            k_done = k + 1
            v_next = np.zeros_like(r0)
            break
        v_prev, v = v, w / beta[k + 1]
        v_next = v
    return LanczosResult(alpha[:k_done], beta[:k_done + 1], V[:k_done], AV[:k_done], v_next,
                         k_done)


@dataclasses.dataclass
class Deflation:
    Z: np.ndarray            # [dim, n_kept, 3] deflation vectors
    Zp: np.ndarray           # [dim, n_kept, 3] Z' = A Z
    E: np.ndarray            # [dim, dim] coarse matrix Z^T A Z (= Z^T Z')
    Einv: np.ndarray         # pseudo-inverse of E
    theta: np.ndarray        # Ritz values of T_m


def deflation_from_lanczos(lz, rtol=1e-12):
    """Ritz pairs of T_m give Z = V_m X and Z' = (A V_m) X; the coarse matrix E = Z^T Z' and its
    pseudo-inverse complete the preconditioner (2lvl a posteriori construction)."""
    theta, X = np.linalg.eigh(lz.T())
    m = lz.m
    Vf = lz.V.reshape(m, -1)
    AVf = lz.AV.reshape(m, -1)
    Z = X.T @ Vf                 # row j = sum_i X[i, j] v_i
    Zp = X.T @ AVf
    E = Z @ Zp.T
    Einv = sym_pinv(0.5 * (E + E.T), rtol)
    shape = (m,) + lz.V.shape[1:]
    return Deflation(Z.reshape(shape), Zp.reshape(shape), E, Einv, theta)


def precond_2lvl(plan, defl, r):
    """Eq. 2lvlDef0: M_2lvl r = M_BD r - M_BD Z' E^-1 Z^T r + Z E^-1 Z^T r, applied factor by
    factor from the right."""
    r = np.asarray(r, np.float64).reshape(-1, 3)
    dim = defl.Z.shape[0]
    Zf = defl.Z.reshape(dim, -1)
    Zpf = defl.Zp.reshape(dim, -1)
    c = defl.Einv @ (Zf @ r.reshape(-1))
    return precond_bj(plan, r - (Zpf.T @ c).reshape(-1, 3)) + (Zf.T @ c).reshape(-1, 3)
