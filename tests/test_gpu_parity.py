"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Shapes are ragged on purpose: column counts that are not multiples of the
16-column blocks, receiver counts beyond one 64-receiver chunk, batches of 1,
duplicates, and both band limits (nf < nt/2+1 and the full nf = nt/2+1 with the
Nyquist bin).  Float32 tolerance: relative 2-norm error <= 1e-5.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import freq, optim

from gpu_helpers import H, T, batch, f32, make_plan, random_case, relerr

pytestmark = pytest.mark.gpu

TOL = 1e-5

# (ns, nr, nvs, nt, nf, nb)
CASES = [
    (21, 19, 37, 128, 65, 5),
    (21, 19, 37, 128, 30, 16),
    (40, 33, 18, 256, 129, 17),
    (20, 70, 17, 1024, 257, 12),
    (24, 17, 16, 1024, 513, 1),
    (70, 50, 45, 512, 200, 33),
    (130, 90, 20, 512, 257, 64),
]


def case_id(c):
    return "ns{}_nr{}_nvs{}_nt{}_nf{}_nb{}".format(*c)


@pytest.mark.parametrize("case", CASES, ids=case_id)
def test_forward_adjoint(case):
    ns, nr, nvs, nt, nf, nb = case
    d, u, r = random_case(ns, nr, nvs, nt, seed=ns + nt)
    plan = make_plan(d, u, nb_max=nb, nf=nf)
    idx = batch(ns, nb, seed=1)
    ug = plan.mdc_forward(T(r), T(idx, torch.int32))
    uo = freq.mdc(d[idx], r, nf)
    assert relerr(H(ug), uo) <= TOL
    v = u[idx]
    gg = plan.mdc_adjoint(T(v), T(idx, torch.int32))
    go = freq.mdc_adjoint(d[idx], v, nf)
    assert relerr(H(gg), go) <= TOL
    # adjoint pairing on the GPU results themselves
    lhs, rhs = float(np.sum(H(ug) * v)), float(np.sum(r * H(gg)))
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


@pytest.mark.parametrize("case", CASES, ids=case_id)
@pytest.mark.parametrize("masked", [False, True])
def test_stoch_grad(case, masked):
    ns, nr, nvs, nt, nf, nb = case
    d, u, r = random_case(ns, nr, nvs, nt, seed=3 * ns + nt)
    onset = None
    if masked:
        onset = synth.random_onsets(nr, nvs, nt, seed=5)
    plan = make_plan(d, u, onset=onset, nb_max=nb, nf=nf)
    idx = batch(ns, nb, seed=2, dup=True)
    G, loss, gn = plan.mdd_stoch_grad(T(r), T(idx, torch.int32))
    lo, go = freq.batch_loss_grad(d, r, u, idx, nf)
    go = optim.apply_mask(go, onset)
    assert relerr(H(G), go) <= TOL
    assert abs(loss.item() - lo) <= TOL * lo
    assert abs(gn.item() - float(np.sum(go * go))) <= 2 * TOL * float(np.sum(go * go))
    if masked:
        t = np.arange(nt)
        assert np.all(H(G)[t[None, None, :] < onset[:, :, None]] == 0.0)


def test_bad_index_is_a_zero_source():
    ns, nr, nvs, nt, nf = 12, 10, 9, 128, 65
    d, u, r = random_case(ns, nr, nvs, nt, seed=11)
    plan = make_plan(d, u, nb_max=4, nf=nf)
    idx = np.array([1, 5, ns + 3, -2], dtype=np.int32)
    G, loss, _ = plan.mdd_stoch_grad(T(r), T(idx, torch.int32))
    lo, go = freq.batch_loss_grad(d, r, u, [1, 5], nf)
    assert relerr(H(G), go) <= TOL
    assert abs(loss.item() - lo) <= TOL * lo


def test_batch_larger_than_plan_is_rejected():
    from paper_2202_04486_amd import MddError
    d, u, r = random_case(10, 8, 8, 128, seed=12)
    plan = make_plan(d, u, nb_max=2, nf=65)
    with pytest.raises((MddError, ValueError)):
        plan.mdd_stoch_grad(T(r), T(np.arange(3, dtype=np.int32), torch.int32))


def test_deterministic_bitwise():
    d, u, r = random_case(40, 33, 18, 256, seed=13)
    plan = make_plan(d, u, nb_max=17, nf=100)
    idx = T(batch(40, 17, seed=3), torch.int32)
    g1, l1, n1 = plan.mdd_stoch_grad(T(r), idx)
    g1, l1, n1 = g1.clone(), l1.clone(), n1.clone()
    g2, l2, n2 = plan.mdd_stoch_grad(T(r), idx)
    assert torch.equal(g1, g2) and torch.equal(l1, l2) and torch.equal(n1, n2)


@pytest.mark.parametrize("opt", ["sgd", "adam", "nsgd"])
@pytest.mark.parametrize("store_rf", [False, True])
def test_steps_match_oracle(opt, store_rf):
    ns, nr, nvs, nt, nf, nb = 37, 29, 22, 256, 100, 9
    d, u, r0 = random_case(ns, nr, nvs, nt, seed=17)
    onset = synth.onsets(synth.WORKLOADS["tiny2d"].replace(dt=0.002), nr, nvs)
    plan = make_plan(d, u, onset=onset, nb_max=nb, nf=nf, store_rf=store_rf)
    R = T(r0)
    s0 = torch.zeros_like(R)
    s1 = torch.zeros_like(R)
    ro = r0.copy()
    m = np.zeros_like(ro)
    v = np.zeros_like(ro)
    lr = {"sgd": 2e-4, "adam": 1e-2, "nsgd": 1e-4}[opt]
    perm = synth.epoch_permutations(synth.WORKLOADS["tiny2d"], 1, ns=ns)[0]
    for t, b in enumerate(optim.batches(perm, nb)[:3], start=1):
        loss, _ = plan.mdd_step(R, T(b, torch.int32), opt=opt, lr=lr, s0=s0, s1=s1, t=t, mu=0.9)

        def grad(x, b=b):
            return optim.apply_mask(freq.batch_loss_grad(d, x, u, b, nf)[1], onset)
        lo = freq.batch_loss_grad(d, ro + (0.9 * m if opt == "nsgd" else 0.0), u, b, nf)[0]
        assert abs(loss.item() - lo) <= TOL * lo
        if opt == "sgd":
            ro = optim.sgd(ro, grad(ro), lr, onset)
        elif opt == "adam":
            ro, m, v = optim.adam(ro, m, v, grad(ro), t, lr, onset=onset)
        else:
            ro, m = optim.nesterov(ro, m, grad, lr, 0.9, onset)
    assert relerr(H(R) - r0, ro - r0) <= 1e-4
    if opt != "sgd":
        assert relerr(H(s0), m) <= 1e-4


def test_store_rf_equals_recomputed():
    ns, nr, nvs, nt, nf, nb = 30, 20, 33, 512, 150, 8
    d, u, r0 = random_case(ns, nr, nvs, nt, seed=19)
    outs = []
    for store in (False, True):
        plan = make_plan(d, u, nb_max=nb, nf=nf, store_rf=store)
        R, m, v = T(r0), torch.zeros(nr, nvs, nt, device="cuda"), torch.zeros(nr, nvs, nt, device="cuda")
        for t in range(1, 4):
            plan.mdd_step(R, T(batch(ns, nb, seed=t), torch.int32), opt="adam", lr=1e-2, s0=m, s1=v, t=t)
        outs.append(H(R))
    assert relerr(outs[1], outs[0]) <= 1e-6


@pytest.mark.parametrize("prec,tol", [("bf16x3", 1e-3), ("fp16x3", 1e-3)])
def test_split_precision_gradient(prec, tol):
    ns, nr, nvs, nt, nf, nb = 64, 70, 40, 1024, 257, 16
    wl = synth.WORKLOADS["line2d"].replace(ns=ns, nr=nr, nvs=nvs)
    p = synth.make_problem(wl, with_noise=False)
    d = f32(p["d"])
    r = f32(p["r_true"])
    u = f32(synth.random_arrays(23, (ns, nvs, nt))[0])
    idx = batch(ns, nb, seed=5)
    lo, go = freq.batch_loss_grad(d, r, u, idx, nf)
    plan = make_plan(d, u, nb_max=nb, nf=nf, precision=prec)
    G, loss, _ = plan.mdd_stoch_grad(T(r), T(idx, torch.int32))
    e = relerr(H(G), go)
    assert e <= tol, e
    assert abs(loss.item() - lo) <= tol * lo
    plan1 = make_plan(d, u, nb_max=nb, nf=nf, precision="bf16")
    G1, _, _ = plan1.mdd_stoch_grad(T(r), T(idx, torch.int32))
    assert relerr(H(G1), go) > e       # the single-product form is the less accurate one


def test_sigma_max_matches_svd():
    from oracle import stepsize
    wl = synth.WORKLOADS["tiny2d"]
    p = synth.make_problem(wl)
    d = f32(p["d"])
    u = f32(synth.random_arrays(29, (wl.ns, wl.nvs, wl.nt))[0])
    plan = make_plan(d, u, nb_max=8, nf=wl.nf)
    lam = H(plan.mdd_sigma_max2(iters=300))
    s2, per_k = stepsize.sigma_max2_kernel(d, wl.nf)
    assert abs(lam.max() - s2) <= 1e-4 * s2
    assert np.all(lam <= per_k * (1 + 1e-5) + 1e-9 * s2)


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-6), ("bf16x3", 1e-4)])
def test_zero_gradient_at_the_true_model(prec, tol):
    """Noise-free data u = P+ R_true (made by the oracle): every batch's loss and gradient
    vanish at R_true, up to the arithmetic's rounding, relative to their values at 0."""
    wl = synth.WORKLOADS["tiny2d"]
    p = synth.make_problem(wl)
    d = f32(p["d"])
    r_true = f32(p["r_true"])
    u = f32(freq.mdc(d, r_true, wl.nf))
    plan = make_plan(d, u, nb_max=wl.nb, nf=wl.nf, precision=prec)
    for b in optim.batches(synth.epoch_permutations(wl, 1)[0], wl.nb):
        it = T(b, torch.int32)
        g0, l0, _ = plan.mdd_stoch_grad(torch.zeros(wl.nr, wl.nvs, wl.nt, device="cuda"), it)
        g0, l0 = H(g0), l0.item()
        g1, l1, _ = plan.mdd_stoch_grad(T(r_true), it)
        assert np.linalg.norm(H(g1)) <= tol * np.linalg.norm(g0)
        assert l1.item() <= tol * tol * l0
