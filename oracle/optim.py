"""Preconditioners, update rules, batch schedule and error metric.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).
"""
from __future__ import annotations

import math

import numpy as np


def causal_mask(onset: np.ndarray, nt: int) -> np.ndarray:
    """Causality preconditioner as a 0/1 array [nr][nvs][nt]: sample t of trace
    (r, vs) is kept iff t >= onset[r, vs] (mutes everything before the direct
    arrival; Theory section, preconditioned functional)."""
    t = np.arange(nt)
    return (t[None, None, :] >= np.asarray(onset)[:, :, None]).astype(np.float64)


def apply_mask(x: np.ndarray, onset) -> np.ndarray:
    if onset is None:
        return np.array(x, dtype=np.float64)
    return np.asarray(x, dtype=np.float64) * causal_mask(onset, x.shape[-1])


def reciprocity(z: np.ndarray) -> np.ndarray:
    """Reciprocity preconditioner C_r z = (z + z^T) / 2, with ^T swapping the
    receiver and virtual-source axes (Theory section)."""
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * (z + np.swapaxes(z, 0, 1))


def sgd(r, g, lr, onset=None):
    """Plain stochastic gradient step r <- C_c (r - lr g) (Theory section)."""
    return apply_mask(np.asarray(r, dtype=np.float64) - lr * np.asarray(g, dtype=np.float64), onset)


def adam(r, m, v, g, t, lr, beta1=0.9, beta2=0.999, eps=1e-8, onset=None):
    """Adam (Kingma and Ba) step number t >= 1 with bias correction; the mask is kept
    on the model.  Returns (r, m, v).  Not in the paper: used for the Adam runs."""
    g = np.asarray(g, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    r = np.asarray(r, dtype=np.float64) - lr * mhat / (np.sqrt(vhat) + eps)
    return apply_mask(r, onset), m, v


def nesterov(r, vel, grad_fn, lr, mu, onset=None):
    """Stochastic gradient with Nesterov momentum in the Sutskever et al. form:
    vel <- mu vel - lr grad(r + mu vel);  r <- r + vel.  Returns (r, vel)."""
    vel = mu * np.asarray(vel, dtype=np.float64) - lr * grad_fn(np.asarray(r) + mu * vel)
    vel = apply_mask(vel, onset)
    return apply_mask(np.asarray(r, dtype=np.float64) + vel, onset), vel


def batches(perm, nb: int):
    """Split one epoch's source permutation into ceil(ns / nb) batches of consecutive
    entries (the last one partial), each sorted ascending.  An epoch uses every
    source once (Theory section)."""
    perm = np.asarray(perm)
    n = math.ceil(len(perm) / nb)
    return [np.sort(perm[j * nb:(j + 1) * nb]).astype(np.int32) for j in range(n)]


def rmse(r_true, r_est) -> float:
    """Error metric of the Examples section: the Euclidean norm of the difference of
    the two responses, each divided by its own largest absolute value (read as the
    plain 2-norm; the printed square root of a squared norm cancels)."""
    a = np.asarray(r_true, dtype=np.float64)
    b = np.asarray(r_est, dtype=np.float64)
    return float(np.linalg.norm((a / np.max(np.abs(a)) - b / np.max(np.abs(b))).ravel()))
