"""Kernel rows staged per batch (MDD_FLAG_STREAM_KERNEL, for a kernel that does not fit
in device memory): every product kernel takes D row b of the staged batch instead of row
idx[b] of the resident spectra.  The staged rows go through the same transform as the
resident ones, so every result equals the resident plan's bitwise (fp16x3 takes its
scale from the staged rows only, so it is compared with the oracle), and the streaming
helper that copies rows from pinned host memory one batch ahead gives the same
trajectory as the resident plan."""
import numpy as np
import pytest
import torch

import synth
from oracle import freq, optim

from gpu_helpers import H, T, batch, make_plan, random_case, relerr

pytestmark = pytest.mark.gpu


def streamed_plan(d, u, nb_max, nf, precision="fp32", store_rf=False, onset=None):
    from paper_2202_04486_amd.plan import Plan
    ns, nr, nt = d.shape
    plan = Plan(ns, nr, u.shape[1], nt, nf, nb_max, precision=precision, store_rf=store_rf,
                stream_kernel=True)
    plan.mdd_set_data(T(u))
    if onset is not None:
        plan.mdd_set_mask(T(onset, torch.int32))
    return plan


# (nvs, nb, precision): the persistent fp32 and split kernels (nb <= 16), the tiled ones
# (17..32), the warp-specialised ones (33..64), and the matrix-vector kernel (nvs = 1).
CASES = [(20, 9, "fp32"), (20, 16, "bf16x3"), (37, 30, "fp32"), (37, 30, "bf16x3"),
         (40, 64, "fp32"), (40, 50, "bf16x3"), (1, 40, "fp32"), (1, 8, "fp32")]


@pytest.mark.parametrize("nvs,nb,prec", CASES, ids=[f"nvs{a}-nb{b}-{c}" for a, b, c in CASES])
def test_staged_equals_resident(nvs, nb, prec):
    ns, nr, nt, nf = 70, 53, 256, 100
    d, u, r = random_case(ns, nr, nvs, nt, seed=nb + nvs)
    res = make_plan(d, u, nb_max=nb, nf=nf, precision=prec)
    st = streamed_plan(d, u, nb, nf, precision=prec)
    idx = batch(ns, nb, seed=nb)
    idx[nb // 2] = idx[0]                                    # a repeated source
    it = T(idx, torch.int32)
    st.mdd_stage_kernel(T(d[idx]))
    for name, args in (("mdd_stoch_grad", (T(r), it)), ("mdc_forward", (T(r), it)),
                       ("mdc_adjoint", (T(u[idx]), it))):
        a = getattr(res, name)(*args)
        b = getattr(st, name)(*args)
        for x, y in zip(a if isinstance(a, tuple) else (a,), b if isinstance(b, tuple) else (b,)):
            assert torch.equal(x, y), name
    G, loss, _ = st.mdd_stoch_grad(T(r), it)
    lo, go = freq.batch_loss_grad(d, r, u, idx, nf)
    tol = 1e-5 if prec == "fp32" else 1e-3
    assert relerr(H(G), go) <= tol
    assert abs(loss.item() - lo) <= tol * lo


def test_staged_fp16x3_against_oracle():
    ns, nr, nvs, nt, nf, nb = 60, 45, 33, 256, 100, 40
    d, u, r = random_case(ns, nr, nvs, nt, seed=5)
    st = streamed_plan(d, u, nb, nf, precision="fp16x3")
    idx = batch(ns, nb, seed=1)
    st.mdd_stage_kernel(T(d[idx]))
    G, loss, _ = st.mdd_stoch_grad(T(r), T(idx, torch.int32))
    lo, go = freq.batch_loss_grad(d, r, u, idx, nf)
    assert relerr(H(G), go) <= 1e-3
    assert abs(loss.item() - lo) <= 1e-3 * lo


def test_bad_index_with_staged_rows():
    """An index outside [0, ns) is a zero source whatever its staged row holds."""
    ns, nr, nvs, nt, nf, nb = 30, 21, 18, 128, 65, 6
    d, u, r = random_case(ns, nr, nvs, nt, seed=7)
    st = streamed_plan(d, u, nb, nf)
    idx = np.array([3, ns + 1, 7, -1, 12, 3], dtype=np.int32)
    rows = np.stack([d[i] if 0 <= i < ns else np.full(d.shape[1:], 1e3) for i in idx])
    st.mdd_stage_kernel(T(rows))
    G, loss, _ = st.mdd_stoch_grad(T(r), T(idx, torch.int32))
    lo, go = freq.batch_loss_grad(d, r, u, [3, 7, 12, 3], nf)
    assert relerr(H(G), go) <= 1e-5
    assert abs(loss.item() - lo) <= 1e-5 * lo


def test_staged_plan_state_errors():
    from paper_2202_04486_amd import MddError
    ns, nr, nvs, nt, nf, nb = 20, 16, 16, 128, 65, 8
    d, u, r = random_case(ns, nr, nvs, nt, seed=9)
    st = streamed_plan(d, u, nb, nf)
    idx = T(batch(ns, nb, seed=2), torch.int32)
    with pytest.raises(MddError):                 # nothing staged yet
        st.mdd_stoch_grad(T(r), idx)
    with pytest.raises(MddError):                 # the kernel is not resident on this plan
        st.mdd_set_kernel(T(d))
    with pytest.raises(MddError):
        st.mdd_sigma_max2(iters=5)
    st.mdd_stage_kernel(T(d[:5]))
    with pytest.raises(MddError):                 # the batch is not the staged length
        st.mdd_stoch_grad(T(r), idx)
    with pytest.raises(MddError):                 # more rows than nb_max
        st.mdd_stage_kernel(T(np.concatenate([d[:5], d[:5]])))


@pytest.mark.parametrize("opt,store_rf", [("adam", True), ("nsgd", False)])
def test_streamed_epoch_from_pinned_host_memory(opt, store_rf):
    """One epoch and a half of steps with the rows copied from pinned host memory one batch
    ahead on a side stream: bitwise the resident plan's trajectory."""
    from paper_2202_04486_amd.solver import StreamedKernel
    wl = synth.WORKLOADS["tiny2d"]
    ns, nr, nvs, nt, nf, nb = 45, 40, 33, 256, 100, 16
    d, u, _ = random_case(ns, nr, nvs, nt, seed=13)
    onset = synth.onsets(wl.replace(dt=0.002), nr, nvs)
    res = make_plan(d, u, onset=onset, nb_max=nb, nf=nf, store_rf=store_rf)
    st = streamed_plan(d, u, nb, nf, store_rf=store_rf, onset=onset)
    ks = StreamedKernel(st, torch.from_numpy(np.ascontiguousarray(d, dtype=np.float32)))
    perms = synth.epoch_permutations(wl, 2, ns=ns)
    bs = optim.batches(perms[0], nb) + optim.batches(perms[1], nb)[:2]
    lr = 1e-2 if opt == "adam" else 1e-4
    states = []
    for plan, streamed in ((res, False), (st, True)):
        R = torch.zeros(nr, nvs, nt, device="cuda")
        m, v = torch.zeros_like(R), torch.zeros_like(R)
        losses = torch.zeros(len(bs), dtype=torch.float64, device="cuda")
        if streamed:
            ks.prefetch(bs[0])
        for j, b in enumerate(bs):
            if streamed:
                ks.stage()
                if j + 1 < len(bs):
                    ks.prefetch(bs[j + 1])
            plan.mdd_step(R, T(b, torch.int32), opt=opt, lr=lr, s0=m, s1=v, t=j + 1, mu=0.9,
                          loss_out=losses[j:j + 1])
        torch.cuda.synchronize()
        states.append((R, m, v, losses))
    for x, y in zip(*states):
        assert torch.equal(x, y)


@pytest.mark.parametrize("nb", [9, 64])
def test_staged_reciprocity_operators_equal_resident(nb):
    """mdc_forward_rec / mdc_adjoint_rec (C_r on spectra, nr == nvs) with the kernel rows
    staged per batch: bitwise the resident plan's results."""
    ns, n, nt, nf = 70, 40, 256, 100
    d, u, r = random_case(ns, n, n, nt, seed=nb + 3)
    res = make_plan(d, u, nb_max=nb, nf=nf)
    st = streamed_plan(d, u, nb, nf)
    idx = batch(ns, nb, seed=nb + 1)
    it = T(idx, torch.int32)
    st.mdd_stage_kernel(T(d[idx]))
    assert torch.equal(res.mdc_forward_rec(T(r), it), st.mdc_forward_rec(T(r), it))
    assert torch.equal(res.mdc_adjoint_rec(T(u[idx]), it), st.mdc_adjoint_rec(T(u[idx]), it))


def streamed_data_plan(nb_max, nf, ns, nr, nvs, nt, precision="fp32", store_rf=False, onset=None):
    from paper_2202_04486_amd.plan import Plan
    plan = Plan(ns, nr, nvs, nt, nf, nb_max, precision=precision, store_rf=store_rf,
                stream_kernel=True, stream_data=True)
    if onset is not None:
        plan.mdd_set_mask(T(onset, torch.int32))
    return plan


@pytest.mark.parametrize("nvs,nb,prec", CASES, ids=[f"nvs{a}-nb{b}-{c}" for a, b, c in CASES])
def test_staged_data_equals_resident(nvs, nb, prec):
    """MDD_FLAG_STREAM_DATA: the data rows and their out-of-band energies staged per batch
    beside the kernel rows give bitwise the resident plan's gradient, loss and step."""
    ns, nr, nt, nf = 70, 53, 256, 100
    d, u, r = random_case(ns, nr, nvs, nt, seed=nb + nvs + 1)
    res = make_plan(d, u, nb_max=nb, nf=nf, precision=prec)
    st = streamed_data_plan(nb, nf, ns, nr, nvs, nt, precision=prec)
    idx = batch(ns, nb, seed=nb + 2)
    idx[nb // 2] = idx[0]                                    # a repeated source
    it = T(idx, torch.int32)
    st.mdd_stage_kernel(T(d[idx]))
    st.mdd_stage_data(T(u[idx]))
    a = res.mdd_stoch_grad(T(r), it)
    b = st.mdd_stoch_grad(T(r), it)
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    Ra, Rb = T(r), T(r)
    la = res.mdd_step(Ra, it, opt="sgd", lr=1e-4)[0]
    lb = st.mdd_step(Rb, it, opt="sgd", lr=1e-4)[0]
    assert torch.equal(Ra, Rb) and torch.equal(la, lb)
    lo, go = freq.batch_loss_grad(d, r, u, idx, nf)
    tol = 1e-5 if prec == "fp32" else 1e-3
    assert relerr(H(b[0]), go) <= tol
    assert abs(b[1].item() - lo) <= tol * lo


def test_staged_data_state_errors():
    from paper_2202_04486_amd import MddError
    ns, nr, nvs, nt, nf, nb = 20, 16, 16, 128, 65, 8
    d, u, r = random_case(ns, nr, nvs, nt, seed=19)
    st = streamed_data_plan(nb, nf, ns, nr, nvs, nt)
    idx = batch(ns, nb, seed=3)
    it = T(idx, torch.int32)
    with pytest.raises(MddError):                 # the data are not resident on this plan
        st.mdd_set_data(T(u))
    st.mdd_stage_kernel(T(d[idx]))
    with pytest.raises(MddError):                 # no data rows staged yet
        st.mdd_stoch_grad(T(r), it)
    st.mdd_stage_data(T(u[idx[:5]]))
    with pytest.raises(MddError):                 # the data rows are not the batch's length
        st.mdd_stoch_grad(T(r), it)
    st.mdd_stage_data(T(u[idx]))
    G, loss, _ = st.mdd_stoch_grad(T(r), it)
    lo, go = freq.batch_loss_grad(d, r, u, idx, nf)
    assert relerr(H(G), go) <= 1e-5
    other = streamed_plan(d, u, nb, nf)            # kernel rows only: no data rows to stage
    with pytest.raises(MddError):
        other.mdd_stage_data(T(u[idx]))


def test_out_of_core_beyond_4096_sources():
    """8192 sources, more than a resident plan takes: the kernel and the data stay in
    pinned host memory and only each batch's rows reach the device.  Batches drawn over
    the whole index range; each gradient and loss against the oracle on the batch's rows,
    then Adam steps streamed one batch ahead against the oracle's trajectory."""
    from paper_2202_04486_amd.solver import StreamedKernel
    ns, nr, nvs, nt, nf, nb = 8192, 64, 64, 256, 100, 64
    print(f"out of core: ns={ns} nr={nr} nvs={nvs} nt={nt} nf={nf} nb={nb}", flush=True)
    d, u = synth.random_arrays(31, (ns, nr, nt), (ns, nvs, nt), dtype=np.float32)
    r = synth.random_arrays(32, (nr, nvs, nt))[0]
    r = r.astype(np.float32).astype(np.float64)
    onset = synth.random_onsets(nr, nvs, nt, seed=33)
    st = streamed_data_plan(nb, nf, ns, nr, nvs, nt, store_rf=True, onset=onset)
    ks = StreamedKernel(st, torch.from_numpy(d), torch.from_numpy(u))
    perm = np.random.default_rng(34).permutation(ns)
    bs = [np.sort(perm[j * nb:(j + 1) * nb]).astype(np.int32) for j in range(4)]
    bs.append(np.sort(np.concatenate([perm[-nb // 2:], [0, ns - 1]] +
                                     [perm[:nb // 2 - 2]])).astype(np.int32))
    assert min(b.min() for b in bs) == 0 and max(b.max() for b in bs) == ns - 1
    d64 = lambda b: d[b].astype(np.float64)               # noqa: E731
    u64 = lambda b: u[b].astype(np.float64)               # noqa: E731
    for b in bs:                                          # gradients at a fixed model
        ks.prefetch(b)
        ks.stage()
        G, loss, _ = st.mdd_stoch_grad(T(r), T(b, torch.int32))
        lo, go = freq.batch_loss_grad(d64(b), r, u64(b), np.arange(nb), nf)
        go = optim.apply_mask(go, onset)
        assert relerr(H(G), go) <= 1e-5
        assert abs(loss.item() - lo) <= 1e-5 * lo
    st.mdd_invalidate_model_spectra()
    R = torch.zeros(nr, nvs, nt, device="cuda")
    m, v = torch.zeros_like(R), torch.zeros_like(R)
    ro = np.zeros((nr, nvs, nt))
    mo, vo = np.zeros_like(ro), np.zeros_like(ro)
    _, g0 = freq.batch_loss_grad(d64(bs[0]), ro, u64(bs[0]), np.arange(nb), nf)
    eps = 1e-2 * float(np.sqrt(np.mean(optim.apply_mask(g0, onset) ** 2)))
    ks.prefetch(bs[0])
    for t, b in enumerate(bs, start=1):
        ks.stage()
        if t < len(bs):
            ks.prefetch(bs[t])
        st.mdd_step(R, T(b, torch.int32), opt="adam", lr=1e-2, s0=m, s1=v, t=t, eps=eps)
        _, g = freq.batch_loss_grad(d64(b), ro, u64(b), np.arange(nb), nf)
        ro, mo, vo = optim.adam(ro, mo, vo, optim.apply_mask(g, onset), t, 1e-2, eps=eps,
                                onset=onset)
    torch.cuda.synchronize()
    assert relerr(H(m), mo) <= 1e-5
    assert relerr(H(v), vo) <= 1e-5
    diff = np.abs(H(R) - ro)
    assert np.linalg.norm(diff) <= 1e-4 * np.linalg.norm(ro)
    assert diff.max() <= 1e-2 * 1e-2
