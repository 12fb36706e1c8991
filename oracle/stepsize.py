"""Step-size selection of Appendix B: Landweber bound and largest singular value.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).
"""
from __future__ import annotations

import numpy as np

from . import freq


def sigma_max2_matrix(a: np.ndarray) -> float:
    """Largest squared singular value of a dense matrix (library SVD)."""
    return float(np.linalg.svd(np.asarray(a), compute_uv=False)[0] ** 2)


def landweber(a, y, alpha: float, iters: int, x0=None):
    """Landweber iteration x <- x + alpha A^T (y - A x) (Appendix B).  Returns the
    final iterate and the history of residual norms ||y - A x||."""
    a = np.asarray(a, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    x = np.zeros(a.shape[1]) if x0 is None else np.array(x0, dtype=np.float64)
    hist = []
    for _ in range(iters):
        res = y - a @ x
        hist.append(float(np.linalg.norm(res)))
        x = x + alpha * (a.T @ res)
    return x, hist


def steepest_descent(a, y, iters: int):
    """Gradient descent with the exact line search alpha_k = ||g||^2 / ||A g||^2."""
    a = np.asarray(a, dtype=np.float64)
    x = np.zeros(a.shape[1])
    for _ in range(iters):
        g = a.T @ (y - a @ x)
        ag = a @ g
        den = float(ag @ ag)
        if den == 0.0:
            break
        x = x + float(g @ g) / den * g
    return x


def sigma_max2_kernel(d: np.ndarray, nf: int) -> tuple:
    """Largest squared singular value of the MDC operator, taken from the kernel:
    max over retained frequencies k of sigma_max(D_k)^2, D_k = [ns x nr] spectrum of
    the down-going wavefield (Appendix B: the operator's singular values are those
    of the frequency-domain kernel).  Returns (max, per-frequency array)."""
    df = np.moveaxis(freq.spectra(d, nf), -1, 0)
    s = np.linalg.svd(df, compute_uv=False)[:, 0] ** 2
    return float(s.max()), s


def power_iteration(apply_normal, shape, iters: int, seed: int = 0) -> float:
    """Matrix-free power iteration on a symmetric positive semi-definite operator
    (e.g. A^T A applied through forward and adjoint passes); returns the Rayleigh
    quotient of the final iterate."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(shape)
    x /= np.linalg.norm(x)
    lam = 0.0
    for _ in range(iters):
        y = apply_normal(x)
        lam = float(np.vdot(x, y).real)
        x = y / np.linalg.norm(y)
    return lam


def stochastic_alpha(sigma2: float, kappa: float = 0.5) -> float:
    """Step size kappa * 2 / sigma_max^2 (Appendix B: 40-60 % of the Landweber limit)."""
    return kappa * 2.0 / sigma2
