"""FP64 reference for template map-making -- TEST INFRASTRUCTURE ONLY.

Plain NumPy in float64, written from the paper (arXiv:2112.03370):

  system     (P^T F_T P) m = P^T F_T d                              Eq. genMapEstimator
  filter     F_T = W^-1 (I - T (T^T W^-1 T)^+ T^T W^-1)             Eq. defFT
  weights    W^-1 diagonal (template map-making of the solvers section): per sample the c_0 of
             its block's band (1 outside blocks), 0 at flagged and excised samples (gaps)
  templates  Legendre polynomials P_k, k < n_poly, on each baseline interval, rescaled to unit
             norm on the interval (Appendix A, Eq. polytemplate); one column of T per (baseline,
             degree), supported on its interval only
  kernel     block-diagonal T^T W^-1 T, one n_poly x n_poly block per baseline, inverted by an
             eigen pseudo-inverse that drops directions below 1e-12 of the largest eigenvalue
             (the paper's SVD with a 1e-12 threshold)
  solver     PCG as Alg. 1 with the block-Jacobi preconditioner (P^T W^-1 P)^-1

Readings where the paper is silent (also listed in the design notes):
  * sample j of a baseline of L samples sits at x_j = (2 j + 1) / L - 1 (the midpoints of L equal
    cells of [-1, 1]); the template of degree k is sqrt((2k + 1) / L) P_k(x_j), so that the
    midpoint rule of the continuous orthonormality gives unit norm;
  * the pseudo-inverse threshold is relative to the largest eigenvalue of each block;
  * samples outside every baseline carry no template: there F_T = W^-1.
"""

from __future__ import annotations

import dataclasses

import numpy as np
from numpy.polynomial import legendre as npleg

from . import mapmaking as mm

__all__ = ["TemplatePlan", "build_template_plan", "template_plan_from_problem",
           "legendre_templates", "sample_weights", "template_kernels", "template_filter",
           "template_apply_A", "template_rhs", "template_pcg"]


@dataclasses.dataclass
class TemplatePlan:
    plan: mm.OraclePlan       # pointing, BJ blocks, excision (weights = c_0 of the bands)
    w: np.ndarray             # float64 [N_s] diagonal W^-1, 0 at gap samples
    base_start: np.ndarray    # int64 [n_base]
    base_len: np.ndarray      # int64 [n_base]
    n_poly: int
    Kinv: np.ndarray          # float64 [n_base, n_poly, n_poly] pseudo-inverse of each block


def legendre_templates(L, n_poly):
    """[L, n_poly] columns sqrt((2k+1)/L) P_k(x_j) at the midpoints x_j = (2j+1)/L - 1."""
    x = (2.0 * np.arange(L) + 1.0) / L - 1.0
    V = npleg.legvander(x, max(n_poly - 1, 0))[:, :n_poly]
    return V * np.sqrt((2.0 * np.arange(n_poly) + 1.0) / L)[None, :]


def sample_weights(plan):
    """Diagonal W^-1: c_0 of the sample's band (1 outside blocks), zero at gap samples."""
    return np.where(plan.lpix >= 0, plan.diag, 0.0)


def template_kernels(w, base_start, base_len, n_poly, rtol=1e-12):
    """Pseudo-inverse of each block T_b^T diag(w_b) T_b of the orthogonalisation kernel."""
    nb = len(base_start)
    Kinv = np.zeros((nb, n_poly, n_poly))
    for i, (s, L) in enumerate(zip(base_start, base_len)):
        T = legendre_templates(int(L), n_poly)
        K = T.T @ (w[int(s):int(s) + int(L), None] * T)
        Kinv[i] = mm.sym_pinv(0.5 * (K + K.T), rtol)
    return Kinv


def build_template_plan(plan, base_start, base_len, n_poly):
    w = sample_weights(plan)
    base_start = np.asarray(base_start, np.int64)
    base_len = np.asarray(base_len, np.int64)
    return TemplatePlan(plan, w, base_start, base_len, int(n_poly),
                        template_kernels(w, base_start, base_len, int(n_poly)))


def template_plan_from_problem(prob, n_poly=None, cond_max=mm.DEFAULT_COND_MAX):
    plan = mm.plan_from_problem(prob, cond_max=cond_max)
    npol = prob.meta["n_poly"] if n_poly is None else n_poly
    return build_template_plan(plan, prob.meta["base_start"], prob.meta["base_len"], npol)


def template_filter(tp, t):
    """F_T t = W^-1 t - W^-1 T K^+ T^T W^-1 t (Eq. defFT), baseline by baseline: project the
    weighted vector on the templates, solve with the kernel block, subtract the fit."""
    u = tp.w * np.asarray(t, np.float64)
    if tp.n_poly == 0:
        return u
    out = u.copy()
    for i, (s, L) in enumerate(zip(tp.base_start, tp.base_len)):
        s, L = int(s), int(L)
        T = legendre_templates(L, tp.n_poly)
        a = T.T @ u[s:s + L]                  # T^T W^-1 t
        c = tp.Kinv[i] @ a                    # K^+ T^T W^-1 t
        out[s:s + L] -= tp.w[s:s + L] * (T @ c)
    return out


def template_apply_A(tp, x):
    """P^T F_T P x, applied right to left (the template map-making product)."""
    return mm.point(tp.plan, template_filter(tp, mm.unpoint(tp.plan, x)))


def template_rhs(tp, d):
    """P^T F_T d with d zeroed at gap samples."""
    d = np.where(tp.plan.lpix >= 0, np.asarray(d, np.float64), 0.0)
    return mm.point(tp.plan, template_filter(tp, d))


def template_pcg(tp, b, tol=1e-8, max_iter=10000):
    """Alg. 1 on the template system with the block-Jacobi preconditioner (P^T W^-1 P)^-1."""
    return mm.pcg(tp.plan, b, tol=tol, max_iter=max_iter, apply=lambda v: template_apply_A(tp, v))
