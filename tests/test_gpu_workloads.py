"""The named workloads at their full sizes, in the configuration the benchmark
times: the tiny 2D case over its whole 10-epoch SGD run, and the 201-trace 2D
line (Adam, batches of 16, mask, stored model spectra) over its first steps."""
import numpy as np
import pytest
import torch

import synth
from oracle import freq, optim, stepsize

from gpu_helpers import H, T, f32, make_plan, relerr

pytestmark = pytest.mark.gpu


def test_tiny2d_sgd_trajectory():
    wl = synth.WORKLOADS["tiny2d"]
    p = synth.make_problem(wl)
    d = f32(p["d"])
    u = f32(freq.mdc(d, f32(p["r_true"]), wl.nf))           # noise-free
    s2, _ = stepsize.sigma_max2_kernel(d, wl.nf)
    lr = 1.0 / s2
    plan = make_plan(d, u, nb_max=wl.nb, nf=wl.nf)
    R = torch.zeros(wl.nr, wl.nvs, wl.nt, device="cuda")
    ro = np.zeros((wl.nr, wl.nvs, wl.nt))
    losses = []
    for perm in synth.epoch_permutations(wl, wl.epochs):
        for b in optim.batches(perm, wl.nb):
            loss, _ = plan.mdd_step(R, T(b, torch.int32), opt="sgd", lr=lr)
            lo, g = freq.batch_loss_grad(d, ro, u, b, wl.nf)
            assert abs(loss.item() - lo) <= 1e-5 * lo
            losses.append(lo)
            ro = optim.sgd(ro, g, lr)
        assert relerr(H(R), ro) <= 1e-5
    assert losses[-1] < 0.2 * losses[0]                     # it is converging


@pytest.fixture(scope="module")
def line2d():
    wl = synth.WORKLOADS["line2d"]
    p = synth.make_problem(wl)
    d = f32(p["d"])
    u_clean = freq.mdc(d, f32(p["r_true"]), wl.nf)
    u = f32(u_clean + synth.scale_noise(u_clean, p["noise"], wl.snr_db))
    return wl, d, u, p["onset"]


def test_line2d_gradient_full_size(line2d):
    wl, d, u, onset = line2d
    plan = make_plan(d, u, onset=onset, nb_max=wl.nb, nf=wl.nf)
    b = optim.batches(synth.epoch_permutations(wl, 1)[0], wl.nb)[0]
    r = f32(synth.model_draw(wl, (wl.nr, wl.nvs, wl.nt)))
    G, loss, gn = plan.mdd_stoch_grad(T(r), T(b, torch.int32))
    lo, go = freq.batch_loss_grad(d, r, u, b, wl.nf)
    go = optim.apply_mask(go, onset)
    assert relerr(H(G), go) <= 1e-5
    assert abs(loss.item() - lo) <= 1e-5 * lo
    assert abs(gn.item() - np.sum(go * go)) <= 2e-5 * np.sum(go * go)


def _adam_run(line2d, eps, steps=4, lr=1e-2):
    wl, d, u, onset = line2d
    plan = make_plan(d, u, onset=onset, nb_max=wl.nb, nf=wl.nf, store_rf=True)
    R = torch.zeros(wl.nr, wl.nvs, wl.nt, device="cuda")
    m, v = torch.zeros_like(R), torch.zeros_like(R)
    ro = np.zeros((wl.nr, wl.nvs, wl.nt))
    mo, vo = np.zeros_like(ro), np.zeros_like(ro)
    bs = optim.batches(synth.epoch_permutations(wl, 1)[0], wl.nb)
    for t, b in enumerate(bs[:steps], start=1):
        loss, _ = plan.mdd_step(R, T(b, torch.int32), opt="adam", lr=lr, s0=m, s1=v, t=t, eps=eps)
        lo, g = freq.batch_loss_grad(d, ro, u, b, wl.nf)
        assert abs(loss.item() - lo) <= 1e-5 * lo
        ro, mo, vo = optim.adam(ro, mo, vo, optim.apply_mask(g, onset), t, lr, eps=eps, onset=onset)
    assert relerr(H(m), mo) <= 1e-5
    assert relerr(H(v), vo) <= 1e-5
    return np.abs(H(R) - ro), ro


def test_line2d_adam_update_every_entry(line2d):
    """Adam as the benchmark runs it (eps = 1e-8), one step at a time from the GPU's own
    state: the gradient the step uses (mdd_stoch_grad at the GPU's model, the same
    kernels) against the oracle's at that model, and the updated model and moments
    against the oracle's Adam applied to that gradient from that state, on every entry.
    This separates the update's arithmetic from the amplification of the gradient's
    rounding that a whole trajectory shows (next test)."""
    wl, d, u, onset = line2d
    lr, eps = 1e-2, 1e-8
    plan = make_plan(d, u, onset=onset, nb_max=wl.nb, nf=wl.nf, store_rf=True)
    R = torch.zeros(wl.nr, wl.nvs, wl.nt, device="cuda")
    m, v = torch.zeros_like(R), torch.zeros_like(R)
    bs = optim.batches(synth.epoch_permutations(wl, 1)[0], wl.nb)
    for t, b in enumerate(bs[:4], start=1):
        it = T(b, torch.int32)
        r0, m0, v0 = H(R), H(m), H(v)
        g, _, _ = plan.mdd_stoch_grad(R, it)
        g = H(g)
        _, go = freq.batch_loss_grad(d, r0, u, b, wl.nf)
        assert relerr(g, optim.apply_mask(go, onset)) <= 1e-5
        plan.mdd_step(R, it, opt="adam", lr=lr, s0=m, s1=v, t=t, eps=eps)
        r1, m1, v1 = optim.adam(r0, m0, v0, g, t, lr, eps=eps, onset=onset)
        assert np.abs(H(R) - r1).max() <= 1e-5 * lr, t       # every entry, at step t
        assert relerr(H(m), m1) <= 1e-6 and relerr(H(v), v1) <= 1e-6


def test_line2d_adam_steps_full_size(line2d):
    """Adam as the benchmark runs it (eps = 1e-8) over four steps against the oracle's own
    trajectory.  The moments are smooth in g and match tightly.  The model moves by
    lr * m_hat / (sqrt(v_hat) + eps) per entry, a map close to the sign of m_hat: the
    float32 gradient's rounding (about 2e-7 of the largest entry per entry) changes the
    step of an entry whose gradient is that close to zero by up to lr, and the operator
    spreads each such change into the next steps' gradients.  The update itself matches
    on every entry (previous test); here most entries agree far below the step size and
    none differs by more than the steps can move it."""
    lr, steps = 1e-2, 4
    diff, _ = _adam_run(line2d, 1e-8, steps=steps, lr=lr)
    assert np.median(diff) <= 1e-5 * lr
    assert np.mean(diff > 1e-2 * lr) <= 1e-2
    assert diff.max() <= 2 * steps * lr


def test_line2d_adam_smooth_eps_full_size(line2d):
    """With eps at 1 % of the gradient's rms the update is Lipschitz in g, and every
    entry of the model must follow the oracle."""
    lr = 1e-2
    diff, ro = _adam_run(line2d, 16.0, lr=lr)
    assert np.linalg.norm(diff) <= 1e-4 * np.linalg.norm(ro)
    assert diff.max() <= 1e-2 * lr


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16x3", 1e-3), ("fp16x3", 1e-3)])
def test_line2d_error_per_epoch(line2d, prec, tol):
    """The precision form over its own Adam run: at the end of each of two epochs the
    gradient on the next epoch's first batch, at the form's current model, against the
    oracle's gradient at that same model."""
    wl, d, u, onset = line2d
    plan = make_plan(d, u, onset=onset, nb_max=wl.nb, nf=wl.nf, precision=prec, store_rf=True)
    R = torch.zeros(wl.nr, wl.nvs, wl.nt, device="cuda")
    m, v = torch.zeros_like(R), torch.zeros_like(R)
    perms = synth.epoch_permutations(wl, 3)
    t = 0
    for e in range(2):
        for b in optim.batches(perms[e], wl.nb):
            t += 1
            plan.mdd_step(R, T(b, torch.int32), opt="adam", lr=1e-2, s0=m, s1=v, t=t)
        b0 = optim.batches(perms[e + 1], wl.nb)[0]
        g, _, _ = plan.mdd_stoch_grad(R, T(b0, torch.int32))
        _, go = freq.batch_loss_grad(d, H(R), u, b0, wl.nf)
        assert relerr(H(g), optim.apply_mask(go, onset)) <= tol, e
