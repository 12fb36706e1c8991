"""Edge cases of the GPU path: split-precision operators, a single virtual source,
mask removal, stored-spectra invalidation, rejected optimiser parameters."""
import numpy as np
import pytest
import torch

import synth
from oracle import freq, optim

from gpu_helpers import H, T, batch, f32, make_plan, random_case, relerr

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,tol", [("bf16x3", 1e-3), ("fp16x3", 1e-3), ("fp32", 1e-5)])
@pytest.mark.parametrize("nb", [7, 30, 64])
def test_operators_all_precisions(prec, tol, nb):
    ns, nr, nvs, nt, nf = 70, 90, 45, 512, 200
    d, u, r = random_case(ns, nr, nvs, nt, seed=nb + 31)
    plan = make_plan(d, u, nb_max=nb, nf=nf, precision=prec)
    idx = batch(ns, nb, seed=nb)
    ug = plan.mdc_forward(T(r), T(idx, torch.int32))
    assert relerr(H(ug), freq.mdc(d[idx], r, nf)) <= tol
    gg = plan.mdc_adjoint(T(u[idx]), T(idx, torch.int32))
    assert relerr(H(gg), freq.mdc_adjoint(d[idx], u[idx], nf)) <= tol
    G, loss, _ = plan.mdd_stoch_grad(T(r), T(idx, torch.int32))
    lo, go = freq.batch_loss_grad(d, r, u, idx, nf)
    assert relerr(H(G), go) <= tol
    assert abs(loss.item() - lo) <= tol * lo


def test_single_virtual_source():
    """One virtual source (matrix-vector products per frequency)."""
    ns, nr, nvs, nt, nf = 40, 37, 1, 1024, 257
    d, u, r = random_case(ns, nr, nvs, nt, seed=41)
    plan = make_plan(d, u, nb_max=16, nf=nf)
    idx = batch(ns, 16, seed=3)
    G, loss, _ = plan.mdd_stoch_grad(T(r), T(idx, torch.int32))
    lo, go = freq.batch_loss_grad(d, r, u, idx, nf)
    assert relerr(H(G), go) <= 1e-5
    assert abs(loss.item() - lo) <= 1e-5 * lo


def test_mask_can_be_removed():
    ns, nr, nvs, nt, nf = 20, 18, 19, 256, 100
    d, u, r = random_case(ns, nr, nvs, nt, seed=43)
    onset = synth.random_onsets(nr, nvs, nt, seed=2)
    plan = make_plan(d, u, onset=onset, nb_max=8, nf=nf)
    idx = batch(ns, 8, seed=4)
    G1, _, _ = plan.mdd_stoch_grad(T(r), T(idx, torch.int32))
    _, go = freq.batch_loss_grad(d, r, u, idx, nf)
    assert relerr(H(G1), optim.apply_mask(go, onset)) <= 1e-5
    plan.mdd_set_mask(None)
    G2, _, _ = plan.mdd_stoch_grad(T(r), T(idx, torch.int32))
    assert relerr(H(G2), go) <= 1e-5


def test_invalidate_after_external_change():
    """With stored spectra, changing R outside mdd_step needs the invalidation call;
    after it the step equals one on a fresh plan."""
    ns, nr, nvs, nt, nf, nb = 24, 20, 21, 256, 129, 8
    d, u, r0 = random_case(ns, nr, nvs, nt, seed=47)
    idx = T(batch(ns, nb, seed=5), torch.int32)
    plan = make_plan(d, u, nb_max=nb, nf=nf, store_rf=True)
    R = T(r0)
    plan.mdd_step(R, idx, opt="sgd", lr=1e-4)
    R.copy_(T(r0 * 0.5))                    # changed behind the library's back
    plan.mdd_invalidate_model_spectra()
    plan.mdd_step(R, idx, opt="sgd", lr=1e-4)
    fresh = make_plan(d, u, nb_max=nb, nf=nf)
    R2 = T(r0 * 0.5)
    fresh.mdd_step(R2, idx, opt="sgd", lr=1e-4)
    assert relerr(H(R), H(R2)) <= 1e-6


@pytest.mark.parametrize("kw", [dict(opt="adam", beta1=1.0), dict(opt="adam", eps=0.0),
                                dict(opt="adam", t=0), dict(opt="nsgd", mu=1.5),
                                dict(opt="sgd", lr=-1.0), dict(opt="adam", s1=None)])
def test_bad_optimiser_parameters_rejected(kw):
    from paper_2202_04486_amd import MddError
    ns, nr, nvs, nt, nf = 10, 8, 8, 128, 65
    d, u, r0 = random_case(ns, nr, nvs, nt, seed=53)
    plan = make_plan(d, u, nb_max=4, nf=nf)
    R = T(r0)
    st = {"s0": torch.zeros_like(R), "s1": torch.zeros_like(R)}
    st.update({k: v for k, v in kw.items() if k in ("s0", "s1")})
    args = {k: v for k, v in kw.items() if k not in ("s0", "s1")}
    before = R.clone()
    with pytest.raises(MddError):
        plan.mdd_step(R, T(np.arange(4, dtype=np.int32), torch.int32), s0=st["s0"], s1=st["s1"], **args)
    torch.cuda.synchronize()
    assert torch.equal(R, before)           # nothing was enqueued


@pytest.mark.parametrize("prec", ["bf16x3", "fp16x3"])
@pytest.mark.parametrize("nb", [17, 32, 33, 63])
def test_split_batches_with_bad_and_repeated_indices(prec, nb):
    """Split-precision products at the batch-size boundaries of their tilings (17..32 and
    33..64 rows), receivers not a multiple of the 64-receiver chunk, columns not a multiple
    of the column group, a repeated index (counted twice) and two rejected indices (zero
    wavefields), with the causality mask."""
    ns, nr, nvs, nt, nf = 80, 131, 70, 256, 100
    d, u, r = random_case(ns, nr, nvs, nt, seed=nb + 61)
    onset = synth.onsets(synth.WORKLOADS["tiny2d"].replace(dt=0.002), nr, nvs)
    plan = make_plan(d, u, onset=onset, nb_max=nb, nf=nf, precision=prec)
    good = batch(ns, nb - 3, seed=nb)
    idx = np.concatenate([good, [good[0], -1, ns]]).astype(np.int32)
    G, loss, gn = plan.mdd_stoch_grad(T(r), T(idx, torch.int32))
    used = np.concatenate([good, [good[0]]])
    lo, go = freq.batch_loss_grad(d, r, u, used, nf)
    go = optim.apply_mask(go, onset)
    assert relerr(H(G), go) <= 1e-3
    assert abs(loss.item() - lo) <= 1e-3 * lo
    assert abs(gn.item() - float(np.sum(go * go))) <= 2e-3 * float(np.sum(go * go))
    G2, loss2, gn2 = plan.mdd_stoch_grad(T(r), T(idx, torch.int32))
    assert torch.equal(G, G2) and torch.equal(loss, loss2) and torch.equal(gn, gn2)


@pytest.mark.parametrize("prec", ["bf16x3", "fp16x3"])
@pytest.mark.parametrize("nb,nr", [(1, 33), (9, 256), (16, 201), (16, 257)])
def test_split_small_batches(prec, nb, nr):
    """Split-precision fused products at batches of at most 16: the persistent kernel up to
    256 receivers (and the tiled kernel beyond), with a rejected index, the mask and
    columns that do not fill the last 16-column block."""
    ns, nvs, nt, nf = 40, 37, 256, 100
    d, u, r = random_case(ns, nr, nvs, nt, seed=nb + nr)
    onset = synth.onsets(synth.WORKLOADS["tiny2d"].replace(dt=0.002), nr, nvs)
    plan = make_plan(d, u, onset=onset, nb_max=nb, nf=nf, precision=prec)
    good = batch(ns, nb, seed=nb)
    idx = good.copy()
    if nb > 1:
        idx[-1] = ns + 1          # rejected: a source with zero wavefields
        good = good[:-1]
    G, loss, gn = plan.mdd_stoch_grad(T(r), T(idx.astype(np.int32), torch.int32))
    lo, go = freq.batch_loss_grad(d, r, u, good, nf)
    go = optim.apply_mask(go, onset)
    assert relerr(H(G), go) <= 1e-3
    assert abs(loss.item() - lo) <= 1e-3 * lo
    G2, loss2, _ = plan.mdd_stoch_grad(T(r), T(idx.astype(np.int32), torch.int32))
    assert torch.equal(G, G2) and torch.equal(loss, loss2)


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16x3", 1e-3), ("fp16x3", 1e-3)])
@pytest.mark.parametrize("nr,nvs", [(1, 1), (5, 3), (17, 65)])
def test_large_batch_small_operators(prec, tol, nr, nvs):
    """Batches of 33..64 (the warp-specialised fused kernels) on one or a few receivers and
    virtual sources: a single partial receiver chunk and column groups mostly out of range."""
    ns, nt, nf, nb = 48, 128, 65, 40
    d, u, r = random_case(ns, nr, nvs, nt, seed=nr * 7 + nvs)
    plan = make_plan(d, u, nb_max=nb, nf=nf, precision=prec)
    idx = batch(ns, nb, seed=nr)
    G, loss, _ = plan.mdd_stoch_grad(T(r), T(idx, torch.int32))
    lo, go = freq.batch_loss_grad(d, r, u, idx, nf)
    assert relerr(H(G), go) <= tol
    assert abs(loss.item() - lo) <= tol * lo


def test_check_batch_host_through_the_binding():
    """Plan.mdd_check_batch_host accepts a valid device batch and rejects an index
    outside [0, ns) or an oversize batch, which the device path would take as a
    zero source or refuse."""
    from paper_2202_04486_amd import MddError
    d, u, r = random_case(12, 8, 8, 128, seed=3)
    plan = make_plan(d, u, nb_max=4, nf=65)
    plan.mdd_check_batch_host(T(np.array([0, 11, 11]), torch.int32))
    for bad in ([0, 12], [-1], [0, 1, 2, 3, 4]):
        with pytest.raises(MddError):
            plan.mdd_check_batch_host(T(np.array(bad), torch.int32))


def test_steps_replay_from_a_captured_hip_graph():
    """mdd_step enqueues only kernels on the caller's stream, so torch's graph capture
    records it.  Three captured Adam steps, replayed three times from the same
    starting state with eager library work between the replays, give the eager
    result bitwise every time."""
    ns, nr, nvs, nt, nf, nb = 30, 20, 17, 256, 100, 8
    d, u, r0 = random_case(ns, nr, nvs, nt, seed=51)
    plan = make_plan(d, u, nb_max=nb, nf=nf, store_rf=True)
    R = T(r0)
    m, v = torch.zeros_like(R), torch.zeros_like(R)
    idx = [T(batch(ns, nb, seed=s), torch.int32) for s in range(3)]
    loss = torch.zeros(3, dtype=torch.float64, device=R.device)

    def steps():
        for j in range(3):
            plan.mdd_step(R, idx[j], opt="adam", lr=1e-2, s0=m, s1=v, t=j + 1,
                          loss_out=loss[j:j + 1])

    def reset():
        R.copy_(T(r0))
        m.zero_()
        v.zero_()
        loss.zero_()
        plan.mdd_invalidate_model_spectra()

    reset()
    steps()
    torch.cuda.synchronize()
    want = (R.clone(), m.clone(), v.clone(), loss.clone())
    reset()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        steps()
    for rep in range(3):
        reset()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = (R, m, v, loss)
        assert all(torch.equal(a, b) for a, b in zip(got, want)), rep
        plan.mdd_invalidate_model_spectra()
        plan.mdd_stoch_grad(T(r0), idx[rep])          # eager work between replays
        torch.cuda.synchronize()


@pytest.mark.parametrize("nb", [33, 47, 64])
def test_fp32_operators_large_batches(nb):
    """The forward and adjoint operators alone at 33..64 batch rows in fp32 (the
    warp-specialised kernel's forward and adjoint kinds): receivers not a multiple of the
    64-receiver chunk, columns not a multiple of the 64-column group, a repeated index and
    two rejected ones (zero rows of the forward output, no adjoint contribution)."""
    ns, nr, nvs, nt, nf = 80, 131, 70, 256, 100
    d, u, r = random_case(ns, nr, nvs, nt, seed=nb + 71)
    plan = make_plan(d, u, nb_max=nb, nf=nf)
    good = batch(ns, nb - 3, seed=nb)
    idx = np.concatenate([good, [good[0], -1, ns]]).astype(np.int32)
    ok = (idx >= 0) & (idx < ns)
    ug = plan.mdc_forward(T(r), T(idx, torch.int32))
    want = np.zeros((nb, nvs, nt))
    want[ok] = freq.mdc(d[idx[ok]], r, nf)
    assert relerr(H(ug), want) <= 1e-5
    v = synth.random_arrays(nb, (nb, nvs, nt))[0]
    gg = plan.mdc_adjoint(T(v), T(idx, torch.int32))
    assert relerr(H(gg), freq.mdc_adjoint(d[idx[ok]], f32(v)[ok], nf)) <= 1e-5


@pytest.mark.parametrize("nb,nr", [(9, 257), (16, 300), (24, 300), (32, 131)])
def test_fp32_tiled_products(nb, nr):
    """The tiled fp32 kernel (three real products per complex multiply-add) where the
    persistent one does not apply: batches of at most 16 over more than 224 receivers, and
    17..32 rows over several receiver chunks.  Fused with the mask and a rejected index,
    then the forward and adjoint operators alone."""
    ns, nvs, nt, nf = 40, 37, 256, 100
    d, u, r = random_case(ns, nr, nvs, nt, seed=nb + nr + 5)
    onset = synth.onsets(synth.WORKLOADS["tiny2d"].replace(dt=0.002), nr, nvs)
    plan = make_plan(d, u, onset=onset, nb_max=nb, nf=nf)
    good = batch(ns, nb, seed=nb)
    idx = good.copy()
    idx[-1] = ns + 1              # rejected: a source with zero wavefields
    good = good[:-1]
    G, loss, _ = plan.mdd_stoch_grad(T(r), T(idx.astype(np.int32), torch.int32))
    lo, go = freq.batch_loss_grad(d, r, u, good, nf)
    assert relerr(H(G), optim.apply_mask(go, onset)) <= 1e-5
    assert abs(loss.item() - lo) <= 1e-5 * lo
    ops = make_plan(d, u, nb_max=nb, nf=nf)
    it = T(good.astype(np.int32), torch.int32)
    assert relerr(H(ops.mdc_forward(T(r), it)), freq.mdc(d[good], r, nf)) <= 1e-5
    assert relerr(H(ops.mdc_adjoint(T(u[good]), it)), freq.mdc_adjoint(d[good], u[good], nf)) <= 1e-5


@pytest.mark.parametrize("nb,nr", [(9, 257), (24, 300), (47, 131), (64, 90)])
def test_fp32_cgemm_form(nb, nr):
    """The comparison precision MDD_PREC_FP32_CGEMM (four real products per complex one in
    every kernel) through the tiled kernels (batches of 9 over 257 receivers, 24 rows) and
    the warp-specialised ones (47 and 64 rows): the fused gradient and the two operators
    alone against the oracle."""
    ns, nvs, nt, nf = 70, 45, 256, 100
    d, u, r = random_case(ns, nr, nvs, nt, seed=nb * 3 + nr)
    idx = batch(ns, nb, seed=nb)
    it = T(idx, torch.int32)
    plan = make_plan(d, u, nb_max=nb, nf=nf, precision="fp32_cgemm")
    G, loss, _ = plan.mdd_stoch_grad(T(r), it)
    lo, go = freq.batch_loss_grad(d, r, u, idx, nf)
    assert relerr(H(G), go) <= 1e-5
    assert abs(loss.item() - lo) <= 1e-5 * lo
    assert relerr(H(plan.mdc_forward(T(r), it)), freq.mdc(d[idx], r, nf)) <= 1e-5
    assert relerr(H(plan.mdc_adjoint(T(u[idx]), it)), freq.mdc_adjoint(d[idx], u[idx], nf)) <= 1e-5
