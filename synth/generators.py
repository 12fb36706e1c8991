"""Seeded synthetic inputs for stochastic multi-dimensional deconvolution.

This module is shared by the FP64 oracle's tests and by the GPU path's tests and
benchmark.  It only draws random numbers and evaluates closed-form wavelets; it
holds none of the method's arithmetic (no convolution, no Fourier transform, no
gradient).  The up-going data u = P+ R_true is therefore NOT produced here: the
oracle (for tests) or the library's own forward operator (for the benchmark)
computes it from the arrays returned by ``make_problem``.

The paper's datasets (finite-difference modelled OBC, subsalt and Volve data,
Examples section) are not available; these generators stand in for them with
the same shapes and structure: co-located sources / receivers / virtual sources
on a line (2D) or a square patch (3D), Ricker wavelets, hyperbolic moveout, and
periodic "free-surface-multiple-like" trains of down-going events.

Random streams: ``np.random.SeedSequence(seed).spawn(5)`` gives, in order,
[down-going events, reflection events, noise, batch permutations, model draws].
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field

import numpy as np

V_MASK = 2500.0  # largest velocity of the reflection events (m/s)


@dataclass(frozen=True)
class Workload:
    name: str
    ns: int
    nr: int
    nvs: int
    nt: int
    dt: float
    nf: int
    dx: float
    grid: str            # "line" or "patch"
    grid_nx: int         # patch side (only for grid == "patch")
    f0: float            # Ricker peak frequency (Hz)
    d_kind: str          # "random" or "periodic"
    d_events: int
    d_t0: tuple          # (lo, hi) of t0 (random) or t1 (periodic) in s
    d_period: tuple      # (lo, hi) of the period T (periodic only)
    r_events: int
    r_tau: tuple         # (lo, hi) zero-offset time of the reflections
    snr_db: float | None
    nb: int
    optimizer: str       # "sgd" or "adam"
    epochs: int
    mask: bool
    seed: int
    nb_sweep: tuple = field(default_factory=tuple)
    vs_first: int = 0    # receiver position of the first virtual source

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


WORKLOADS = {
    # Tiny 2D MDD, 32 sources / receivers / virtual sources on a 10 m line.
    "tiny2d": Workload("tiny2d", 32, 32, 32, 128, 0.004, 65, 10.0, "line", 0, 20.0,
                       "random", 4, (0.05, 0.3), (0.0, 0.0), 3, (0.05, 0.3),
                       None, 8, "sgd", 10, False, 0),
    # 2D line, 201 x 201 x 201 at 10 m, 1024 samples.
    "line2d": Workload("line2d", 201, 201, 201, 1024, 0.004, 257, 10.0, "line", 0, 15.0,
                       "periodic", 8, (0.05, 0.3), (0.2, 0.3), 5, (0.1, 0.8),
                       20.0, 16, "adam", 50, True, 0),
    # Differentiation-form checks, 301 x 301 x 301, batch sizes {8, 32, 64}.
    "diff301": Workload("diff301", 301, 301, 301, 1024, 0.004, 257, 10.0, "line", 0, 15.0,
                        "periodic", 8, (0.05, 0.3), (0.2, 0.3), 5, (0.1, 0.8),
                        20.0, 64, "adam", 1, False, 1, (8, 32, 64)),
    # 3D patch, 1600 points on a 40 x 40 grid at 25 m, 512 samples, 200 bins.
    "patch3d": Workload("patch3d", 1600, 1600, 1600, 512, 0.004, 200, 25.0, "patch", 40, 12.0,
                        "periodic", 10, (0.05, 0.2), (0.1, 0.15), 5, (0.05, 0.5),
                        None, 64, "adam", 20, True, 0),
    # Single virtual source in the middle of the 2D line (receiver 100), batches of 32.
    "line2d_vs1": Workload("line2d_vs1", 201, 201, 1, 1024, 0.004, 257, 10.0, "line", 0, 15.0,
                           "periodic", 8, (0.05, 0.3), (0.2, 0.3), 5, (0.1, 0.8),
                           20.0, 32, "nsgd", 20, True, 0, vs_first=100),
    # Single virtual source in the middle of the 3D patch (grid point (20, 20)).
    "patch3d_vs1": Workload("patch3d_vs1", 1600, 1600, 1, 512, 0.004, 200, 25.0, "patch", 40,
                            12.0, "periodic", 10, (0.05, 0.2), (0.1, 0.15), 5, (0.05, 0.5),
                            None, 64, "adam", 20, True, 0, vs_first=820),
}


def streams(seed: int):
    """The five independent generators [d events, r events, noise, batches, model]."""
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(5)]


def positions(n: int, wl: Workload) -> np.ndarray:
    """(n, 2) coordinates in metres: a line x_i = i*dx, or a square patch."""
    i = np.arange(n)
    if wl.grid == "line":
        return np.stack([i * wl.dx, np.zeros(n)], axis=1)
    nx = wl.grid_nx
    return np.stack([(i % nx) * wl.dx, (i // nx) * wl.dx], axis=1)


def ricker(tau, f0: float, xp=np):
    """Zero-phase Ricker wavelet (1 - 2 pi^2 f0^2 tau^2) exp(-pi^2 f0^2 tau^2)."""
    a = (math.pi * f0) ** 2 * tau * tau
    return (1.0 - 2.0 * a) * xp.exp(-a)


def _signed_amplitudes(rng, n):
    return rng.choice([-1.0, 1.0], size=n) * rng.uniform(0.5, 1.0, size=n)


def vs_positions(wl: Workload, nvs=None) -> np.ndarray:
    """Virtual-source coordinates: receiver positions vs_first .. vs_first + nvs - 1."""
    nvs = nvs or wl.nvs
    return positions(wl.vs_first + nvs, wl)[wl.vs_first:]


def down_events(wl: Workload, rng=None) -> dict:
    """Event parameters of the down-going wavefield: t0 (s), v (m/s), a."""
    rng = rng or streams(wl.seed)[0]
    n = wl.d_events
    if wl.d_kind == "random":
        v = rng.uniform(1500.0, 2500.0, size=n)
        t0 = rng.uniform(*wl.d_t0, size=n)
        a = _signed_amplitudes(rng, n)
    else:  # periodic train, free-surface-multiple-like: t0_k = t1 + k*T, a_k = (-0.6)^k
        t1 = rng.uniform(*wl.d_t0)
        period = rng.uniform(*wl.d_period)
        v = np.full(n, rng.uniform(1500.0, 2500.0))
        t0 = t1 + period * np.arange(n)
        a = (-0.6) ** np.arange(n)
    return {"t0": t0, "v": v, "a": a}


def reflection_events(wl: Workload, rng=None) -> dict:
    """Event parameters of the true local reflection response."""
    rng = rng or streams(wl.seed)[1]
    n = wl.r_events
    if wl.d_kind == "random":  # tiny case: same distributions as the down-going events
        tau = rng.uniform(*wl.d_t0, size=n)
    else:
        tau = rng.uniform(*wl.r_tau, size=n)
    w = rng.uniform(1500.0, 2500.0, size=n)
    a = _signed_amplitudes(rng, n)
    return {"t0": tau, "v": w, "a": a}


def event_cube(src: np.ndarray, rec: np.ndarray, nt: int, dt: float, f0: float,
               ev: dict, rows=None, xp=np, device=None, dtype=None):
    """Sum of hyperbolic Ricker events, out[i, j, t] for source row i, receiver j.

    arrival(i, j) = sqrt(t0^2 + |src_i - rec_j|^2 / v^2).  ``rows`` selects a
    subset of source rows.  ``xp`` may be numpy or torch (then ``device``)."""
    if rows is not None:
        src = src[np.asarray(rows)]
    h2 = ((src[:, None, :] - rec[None, :, :]) ** 2).sum(-1)
    if xp is np:
        t = np.arange(nt) * dt
        out = np.zeros((src.shape[0], rec.shape[0], nt), dtype=dtype or np.float64)
        for t0, v, a in zip(ev["t0"], ev["v"], ev["a"]):
            arr = np.sqrt(t0 * t0 + h2 / (v * v))
            out += a * ricker(t[None, None, :] - arr[:, :, None], f0)
        return out
    import torch
    dtype = dtype or torch.float64
    h2t = torch.as_tensor(h2, device=device, dtype=torch.float64)
    t = torch.arange(nt, device=device, dtype=torch.float64) * dt
    out = torch.zeros((src.shape[0], rec.shape[0], nt), device=device, dtype=dtype)
    for t0, v, a in zip(ev["t0"], ev["v"], ev["a"]):
        arr = torch.sqrt(float(t0) ** 2 + h2t / float(v) ** 2)
        out += (float(a) * ricker(t[None, None, :] - arr[:, :, None], f0, xp=torch)).to(dtype)
    return out


def onsets(wl: Workload, nr=None, nvs=None) -> np.ndarray:
    """Causality mask onset (samples) per (receiver, virtual source), int32.

    A sample t of trace (r, vs) is kept iff t >= onset[r, vs]; the onset is the
    direct-arrival time |x_r - x_vs| / V_MASK minus 1.5 Ricker periods."""
    nr = nr or wl.nr
    nvs = nvs or wl.nvs
    xr, xv = positions(nr, wl), vs_positions(wl, nvs)
    h = np.sqrt(((xr[:, None, :] - xv[None, :, :]) ** 2).sum(-1))
    on = np.ceil((h / V_MASK - 1.5 / wl.f0) / wl.dt)
    return np.maximum(on, 0).astype(np.int32)


def make_problem(wl: Workload, with_noise: bool = True) -> dict:
    """FP64 host arrays: d [ns][nr][nt], r_true [nr][nvs][nt], noise [ns][nvs][nt]
    (standard normal, unscaled), onset [nr][nvs] and the event parameters."""
    g = streams(wl.seed)
    xs, xr, xv = positions(wl.ns, wl), positions(wl.nr, wl), vs_positions(wl)
    dev, rev = down_events(wl, g[0]), reflection_events(wl, g[1])
    out = {
        "d": event_cube(xs, xr, wl.nt, wl.dt, wl.f0, dev),
        "r_true": event_cube(xr, xv, wl.nt, wl.dt, wl.f0, rev),
        "onset": onsets(wl),
        "d_events": dev,
        "r_events": rev,
    }
    if with_noise and wl.snr_db is not None:
        out["noise"] = g[2].standard_normal((wl.ns, wl.nvs, wl.nt))
    return out


def scale_noise(u: np.ndarray, noise: np.ndarray, snr_db: float) -> np.ndarray:
    """Noise scaled so that 10 log10(sum u^2 / sum n^2) = snr_db over the cube."""
    eu = float(np.sum(np.asarray(u, dtype=np.float64) ** 2))
    en = float(np.sum(np.asarray(noise, dtype=np.float64) ** 2))
    return noise * math.sqrt(eu / (en * 10.0 ** (snr_db / 10.0)))


def epoch_permutations(wl: Workload, n_epochs: int, ns: int | None = None, rng=None):
    """The random source permutations drawn at the start of each epoch."""
    rng = rng or streams(wl.seed)[3]
    ns = ns or wl.ns
    return [rng.permutation(ns) for _ in range(n_epochs)]


def model_draw(wl: Workload, shape, rng=None) -> np.ndarray:
    """Standard-normal model / probe arrays (derivative checks start from these)."""
    rng = rng or streams(wl.seed)[4]
    return rng.standard_normal(shape)


def random_arrays(seed: int, *shapes, dtype=np.float64):
    """Independent standard-normal arrays (one child stream per shape) for
    derivative checks and parity cases that need no physical structure."""
    kids = np.random.SeedSequence(seed).spawn(len(shapes))
    return [np.random.default_rng(k).standard_normal(s).astype(dtype) for k, s in zip(kids, shapes)]


def random_batch(ns: int, nb: int, seed: int, replace: bool = False) -> np.ndarray:
    """A sorted batch of nb source indices drawn from range(ns) (int32)."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(ns, size=nb, replace=replace or nb > ns)).astype(np.int32)


def random_onsets(nr: int, nvs: int, nt: int, seed: int) -> np.ndarray:
    """Mask onsets drawn uniformly from [0, nt/2) per trace (int32), for mask tests
    that need no geometry."""
    return np.random.default_rng(seed).integers(0, nt // 2, size=(nr, nvs)).astype(np.int32)


def data_events(wl: Workload, n: int = 6, rng=None) -> dict:
    """Hyperbolic events standing in for up-going data where it is not produced by
    the operator (column-sampled checks at sizes the oracle cannot model whole)."""
    rng = rng or streams(wl.seed)[4]
    return {"t0": rng.uniform(0.1, 0.9, size=n), "v": rng.uniform(1500.0, 2500.0, size=n),
            "a": _signed_amplitudes(rng, n)}


def cube_on_device(src, rec, wl: Workload, ev: dict, device, rows_per_chunk: int = 0):
    """event_cube evaluated on a torch device in row chunks, returned as float32."""
    import torch
    n = src.shape[0]
    out = torch.empty((n, rec.shape[0], wl.nt), dtype=torch.float32, device=device)
    step = rows_per_chunk or max(1, (1 << 26) // (rec.shape[0] * wl.nt))
    for s0 in range(0, n, step):
        rows = np.arange(s0, min(n, s0 + step))
        out[s0:s0 + len(rows)] = event_cube(src, rec, wl.nt, wl.dt, wl.f0, ev, rows=rows,
                                            xp=torch, device=device, dtype=torch.float32)
    return out
