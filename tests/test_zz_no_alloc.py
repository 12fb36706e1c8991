"""mdd_stoch_grad_noalloc: the gradient on the library's static workspace, against the
same gradient through a plan on a caller workspace (mdd_stoch_grad), and against the
FP64 oracle, on two calls in a row with the second one smaller."""
import ctypes

import numpy as np
import pytest
import torch

from gpu_helpers import H, T, batch, random_case, relerr
from oracle import freq, optim

import synth

pytestmark = pytest.mark.gpu

# (ns, nr, nvs, nt, nf, nb, mask): the second case of each pair is the smaller one
CASES = [
    [(70, 64, 40, 256, 100, 40, True), (24, 17, 9, 128, 65, 6, False)],
    [(48, 40, 33, 128, 50, 20, True), (20, 9, 5, 128, 40, 3, True)],
]


def _noalloc(lib, prec, nf, d, u, onset, R, idx):
    from paper_2202_04486_amd import native
    ns, nr, nt = d.shape
    nvs = u.shape[1]
    dims = native.make_dims(ns, nr, nvs, nt, nf, len(idx), precision=prec)
    G = torch.full_like(R, float("nan"))
    loss = torch.full((1,), float("nan"), dtype=torch.float64, device=R.device)
    gn = torch.full_like(loss, float("nan"))
    st = lib.mdd_stoch_grad_noalloc(
        ctypes.byref(dims), ctypes.c_void_p(d.data_ptr()), ctypes.c_void_p(u.data_ptr()),
        ctypes.c_void_p(onset.data_ptr()) if onset is not None else None,
        ctypes.c_void_p(R.data_ptr()), ctypes.c_void_p(idx.data_ptr()), len(idx),
        ctypes.c_void_p(G.data_ptr()), ctypes.c_void_p(loss.data_ptr()),
        ctypes.c_void_p(gn.data_ptr()), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    native.check("mdd_stoch_grad_noalloc", st)
    return G, loss, gn


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("pair", range(len(CASES)))
def test_noalloc_gradient_equals_plan_gradient(prec, pair):
    from paper_2202_04486_amd import native
    from paper_2202_04486_amd.plan import Plan
    lib = native.load()
    for j, (ns, nr, nvs, nt, nf, nb, mask) in enumerate(CASES[pair]):
        print(f"noalloc {prec} pair {pair} call {j}: ns={ns} nr={nr} nvs={nvs} nt={nt} nf={nf} "
              f"nb={nb} mask={mask}", flush=True)
        assert native.workspace_bytes(native.make_dims(ns, nr, nvs, nt, nf, nb)) <= \
            native.NOALLOC_WORKSPACE_BYTES
        d, u, r = random_case(ns, nr, nvs, nt, seed=100 + 10 * pair + j)
        on = synth.random_onsets(nr, nvs, nt, seed=7 + j) if mask else None
        idx = batch(ns, nb, seed=200 + j, dup=True)
        dt, ut, rt = T(d), T(u), T(r)
        it = T(idx, torch.int32)
        ot = T(on, torch.int32) if mask else None
        plan = Plan(ns, nr, nvs, nt, nf, nb, precision=prec)
        plan.mdd_set_kernel(dt)
        plan.mdd_set_data(ut)
        if mask:
            plan.mdd_set_mask(ot)
        G0, l0, g0 = plan.mdd_stoch_grad(rt, it)
        G1, l1, g1 = _noalloc(lib, prec, nf, dt, ut, ot, rt, it)
        torch.cuda.synchronize()
        # the same kernels on the same inputs: bitwise the plan's results
        assert torch.equal(G1, G0)
        assert torch.equal(l1, l0) and torch.equal(g1, g0)
        lo, go = freq.batch_loss_grad(d, r, u, idx, nf)
        if mask:
            go = optim.apply_mask(go, on)
        tol = 1e-5 if prec == "fp32" else 1e-3
        assert relerr(H(G1), go) <= tol
        assert abs(l1.item() - lo) <= tol * abs(lo)
        plan.close()
