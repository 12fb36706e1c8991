"""Shared set-up for the GPU parity tests (not collected by pytest)."""
import numpy as np
import torch

import synth


def dev():
    return torch.device("cuda", 0)


def T(x, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(x)).to(device=dev(), dtype=dtype)


def H(t):
    return t.detach().cpu().numpy().astype(np.float64)


def relerr(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def f32(x):
    """The float32 values the GPU sees, as float64 for the oracle."""
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def random_case(ns, nr, nvs, nt, seed):
    d, u, r = synth.random_arrays(seed, (ns, nr, nt), (ns, nvs, nt), (nr, nvs, nt))
    return f32(d), f32(u), f32(r)


def make_plan(d, u=None, onset=None, nb_max=8, precision="fp32", store_rf=False, nf=None):
    from paper_2202_04486_amd.plan import Plan
    ns, nr, nt = d.shape
    nvs = u.shape[1] if u is not None else None
    if nvs is None:
        raise ValueError("u is needed to size the plan")
    plan = Plan(ns, nr, nvs, nt, nf, nb_max, precision=precision, store_rf=store_rf)
    plan.mdd_set_kernel(T(d))
    plan.mdd_set_data(T(u))
    if onset is not None:
        plan.mdd_set_mask(T(onset, torch.int32))
    return plan


def batch(ns, nb, seed, dup=False):
    return synth.random_batch(ns, nb, seed, replace=dup)
