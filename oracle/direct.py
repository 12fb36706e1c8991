"""Direct time-domain definition of the multi-dimensional convolution operator.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Layouts (C order, time fastest): d [ns][nr][nt] down-going wavefield,
R [nr][nvs][nt] local reflection response, u [ns][nvs][nt] up-going wavefield.

Conventions (readings taken where the paper is silent on them):
forward DFT X[k] = sum_t x[t] exp(-2 pi i k t / nt) with no normalisation,
inverse with 1/nt; nfft = nt, so products of spectra are circular convolutions;
bins k < nf are retained and the kernel d is band-limited to them (`bandlimit`),
unit quadrature weights in the receiver integral.
"""
from __future__ import annotations

import numpy as np


def dft_matrix(nt: int) -> np.ndarray:
    """W[k, t] = exp(-2 pi i k t / nt), built entry by entry from its definition."""
    k = np.arange(nt)[:, None]
    t = np.arange(nt)[None, :]
    return np.exp(-2j * np.pi * ((k * t) % nt) / nt)


def dft(x: np.ndarray) -> np.ndarray:
    """Brute-force DFT along the last axis (explicit sum, no FFT)."""
    return np.asarray(x, dtype=np.complex128) @ dft_matrix(x.shape[-1]).T


def idft(xf: np.ndarray) -> np.ndarray:
    """Brute-force inverse DFT along the last axis, with the 1/nt factor."""
    nt = xf.shape[-1]
    return (np.asarray(xf, dtype=np.complex128) @ np.conj(dft_matrix(nt)).T) / nt


def retained_bins(nt: int, nf: int) -> np.ndarray:
    """Boolean mask over the nt DFT bins kept by a band limit of nf one-sided bins:
    bin k is kept iff min(k, nt - k) <= nf - 1 (a real signal keeps both k and nt-k)."""
    k = np.arange(nt)
    return np.minimum(k, nt - k) <= nf - 1


def bandlimit(x: np.ndarray, nf: int) -> np.ndarray:
    """Project real traces onto the first nf one-sided frequency bins.

    The frequency-domain form of the operator (the per-frequency matrix product of
    the Theory section, evaluated only for the retained bins) is exactly the time-
    domain operator with a band-limited kernel; this builds that kernel."""
    nt = x.shape[-1]
    keep = retained_bins(nt, nf)
    if keep.all():
        return np.array(x, dtype=np.float64)
    xf = dft(x)
    xf[..., ~keep] = 0.0
    return np.real(idft(xf))


def mdc(d: np.ndarray, r: np.ndarray) -> np.ndarray:
    """Forward MDC, u[s, v, t] = sum_r sum_tau d[s, r, tau] R[r, v, (t - tau) mod nt].

    The discrete, circular form of the MDC integral (Theory section, first
    equation): a sum over receivers x_R of a time convolution, which per
    frequency is the matrix product P-_f = P+_f R_f."""
    d = np.asarray(d, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    ns, nr, nt = d.shape
    nr2, nvs, nt2 = r.shape
    assert nr == nr2 and nt == nt2
    u = np.zeros((ns, nvs, nt))
    for tau in range(nt):
        # np.roll(R, tau)[..., t] == R[..., (t - tau) mod nt]
        u += np.einsum("sr,rvt->svt", d[:, :, tau], np.roll(r, tau, axis=2))
    return u


def mdc_adjoint(d: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Adjoint MDC, g[r, w, t] = sum_s sum_tau d[s, r, tau] V[s, w, (t + tau) mod nt].

    A cross-correlation of the up-going data with the down-going wavefield; the
    operator is real so its adjoint is its transpose."""
    d = np.asarray(d, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    ns, nr, nt = d.shape
    ns2, nvs, nt2 = v.shape
    assert ns == ns2 and nt == nt2
    g = np.zeros((nr, nvs, nt))
    for tau in range(nt):
        # np.roll(V, -tau)[..., t] == V[..., (t + tau) mod nt]
        g += np.einsum("sr,svt->rvt", d[:, :, tau], np.roll(v, -tau, axis=2))
    return g


def batch_loss_grad(d_bl: np.ndarray, r: np.ndarray, u: np.ndarray, idx) -> tuple:
    """Loss and mini-batch gradient over the sources in ``idx``.

    loss = 1/2 sum_{s in idx} || u_s - P+_s R ||^2   (the finite-sum functional)
    grad = - sum_{s in idx} P+_s^T (u_s - P+_s R)    (the mini-batch gradient)
    The gradient is a SUM over the batch, as printed.  Repeated indices count twice.
    ``d_bl`` is the (band-limited) kernel."""
    idx = np.asarray(idx, dtype=np.int64)
    ds = np.asarray(d_bl, dtype=np.float64)[idx]
    e = mdc(ds, r) - np.asarray(u, dtype=np.float64)[idx]
    loss = 0.5 * float(np.sum(e * e))
    return loss, mdc_adjoint(ds, e)
