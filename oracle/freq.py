"""The same operator as oracle.direct, through numpy's FFT and complex128 matmuls.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Used where the direct sums are too slow (the 201- and 301-trace lines and column
samples of the 1600-trace patch); its agreement with oracle.direct is itself a
test.  It follows the three steps of the MDC cost analysis (Appendix A): Fourier
transform along time, one matrix-matrix product per frequency, inverse Fourier
transform; only the first nf one-sided bins are kept, which is the operator with
the band-limited kernel of oracle.direct.bandlimit.
"""
from __future__ import annotations

import numpy as np


def spectra(x: np.ndarray, nf: int) -> np.ndarray:
    """One-sided spectra of real traces along the last axis, bins 0..nf-1 (complex128)."""
    return np.fft.rfft(np.asarray(x, dtype=np.float64), axis=-1)[..., :nf]


def traces(xf: np.ndarray, nt: int) -> np.ndarray:
    """Real traces of length nt from bins 0..nf-1 (higher bins are zero), with 1/nt."""
    full = np.zeros(xf.shape[:-1] + (nt // 2 + 1,), dtype=np.complex128)
    full[..., : xf.shape[-1]] = xf
    return np.fft.irfft(full, n=nt, axis=-1)


def bandlimit(x: np.ndarray, nf: int) -> np.ndarray:
    return traces(spectra(x, nf), x.shape[-1])


def mdc(d: np.ndarray, r: np.ndarray, nf: int) -> np.ndarray:
    """u = P+ R: per retained frequency k, U_k = D_k R_k ([ns x nr] @ [nr x nvs])."""
    nt = d.shape[-1]
    df = np.moveaxis(spectra(d, nf), -1, 0)      # [nf][ns][nr]
    rf = np.moveaxis(spectra(r, nf), -1, 0)      # [nf][nr][nvs]
    uf = np.matmul(df, rf)                       # [nf][ns][nvs]
    return traces(np.moveaxis(uf, 0, -1), nt)


def mdc_adjoint(d: np.ndarray, v: np.ndarray, nf: int) -> np.ndarray:
    """g = P+^H V: per retained frequency k, G_k = D_k^H V_k ([nr x ns] @ [ns x nvs])."""
    nt = d.shape[-1]
    df = np.moveaxis(spectra(d, nf), -1, 0)      # [nf][ns][nr]
    vf = np.moveaxis(spectra(v, nf), -1, 0)      # [nf][ns][nvs]
    gf = np.matmul(np.conj(np.swapaxes(df, 1, 2)), vf)
    return traces(np.moveaxis(gf, 0, -1), nt)


def batch_loss_grad(d: np.ndarray, r: np.ndarray, u: np.ndarray, idx, nf: int) -> tuple:
    """Mini-batch loss (time domain, 1/2 sum of squared residual samples) and summed
    gradient -sum_{s in idx} P+_s^H (u_s - P+_s R).  Passing a slice of virtual-source
    columns of ``r`` and ``u`` gives exactly those columns of the gradient and their
    share of the loss, since columns do not interact without reciprocity."""
    idx = np.asarray(idx, dtype=np.int64)
    ds = np.asarray(d, dtype=np.float64)[idx]
    e = mdc(ds, r, nf) - np.asarray(u, dtype=np.float64)[idx]
    return 0.5 * float(np.sum(e * e)), mdc_adjoint(ds, e, nf)
