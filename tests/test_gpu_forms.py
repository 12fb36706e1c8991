"""The two forms beside the plain FP32 step, at their workloads' full sizes.

Differentiation form (301 x 301 x 301, nt 1024, nf 257, batches of 8 / 32 / 64,
reciprocity (z + z^T)/2 in-graph, random models of seed 1): adjoint
dot-product test, exact central differences of the quadratic loss, and the
gradient against the FP64 oracle.

Precision form at the 1600-trace 3D patch (40 x 40 grid at 25 m, nt 512,
nf 200, batch 64, mask): the mini-batch gradient of the FP32 and the
BF16 / FP16 split forms on sampled virtual-source columns, against the oracle
on the same columns (without reciprocity the columns are independent).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import freq, optim

from gpu_helpers import H, T, f32, relerr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def diff301():
    from paper_2202_04486_amd.plan import Plan
    wl = synth.WORKLOADS["diff301"]
    p = synth.make_problem(wl)
    d = f32(p["d"])
    u_clean = freq.mdc(d, f32(p["r_true"]), wl.nf)
    u = f32(u_clean + synth.scale_noise(u_clean, p["noise"], wl.snr_db))
    plan = Plan(wl.ns, wl.nr, wl.nvs, wl.nt, wl.nf, 64)
    plan.mdd_set_kernel(T(d))
    plan.mdd_set_data(T(u))
    z, v, y = synth.random_arrays(1, (wl.nr, wl.nvs, wl.nt), (wl.nr, wl.nvs, wl.nt),
                                  (64, wl.nvs, wl.nt))
    return wl, d, u, plan, f32(z), f32(v), f32(y)


@pytest.mark.parametrize("nb", [8, 32, 64])
def test_autograd_gradient_with_reciprocity(diff301, nb):
    from paper_2202_04486_amd.autograd import mdc, reciprocity
    wl, d, u, plan, z0, _, _ = diff301
    idx = optim.batches(synth.epoch_permutations(wl, 1)[0], nb)[0]
    it = T(idx, torch.int32)
    z = T(z0).requires_grad_(True)
    ub = T(u[idx])
    pred = mdc(reciprocity(z), it, plan)
    loss = 0.5 * ((pred - ub).double() ** 2).sum()
    loss.backward()
    r = optim.reciprocity(z0)
    lo, go = freq.batch_loss_grad(d, r, u, idx, wl.nf)
    go = optim.reciprocity(go)                  # C_r is self-adjoint
    assert abs(loss.item() - lo) <= 1e-5 * lo
    assert relerr(H(z.grad), go) <= 1e-5


@pytest.mark.parametrize("nb", [8, 64])
def test_autograd_dot_product(diff301, nb):
    from paper_2202_04486_amd.autograd import mdc
    wl, _, _, plan, x0, _, y0 = diff301
    idx = T(optim.batches(synth.epoch_permutations(wl, 1)[0], nb)[0], torch.int32)
    x = T(x0).requires_grad_(True)
    y = T(y0[:nb])
    ax = mdc(x, idx, plan)
    (ax * y).sum().backward()                   # x.grad = A^T y
    lhs = float((H(ax) * y0[:nb]).sum())
    rhs = float((x0 * H(x.grad)).sum())
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


def test_autograd_central_difference(diff301):
    """For the quadratic loss the central difference equals <grad, V> for any step h.
    V is the oracle's gradient direction (scaled to |z|), so the difference is large
    compared with the float32 rounding of the loss."""
    from paper_2202_04486_amd.autograd import mdc, reciprocity
    wl, d, u, plan, z0, _, _ = diff301
    b = optim.batches(synth.epoch_permutations(wl, 1)[0], 32)[0]
    idx = T(b, torch.int32)
    ub = T(u[b])

    def loss_of(zz):
        return 0.5 * ((mdc(reciprocity(zz), idx, plan) - ub).double() ** 2).sum()

    _, go = freq.batch_loss_grad(d, optim.reciprocity(z0), u, b, wl.nf)
    v0 = optim.reciprocity(go)
    v0 = f32(v0 * (np.linalg.norm(z0) / np.linalg.norm(v0)))
    z = T(z0).requires_grad_(True)
    loss_of(z).backward()
    g = H(z.grad)
    ip = float(np.sum(g * v0))
    for h in (1e-2, 1.0):
        with torch.no_grad():
            lp = loss_of(T(z0 + h * v0)).item()
            lm = loss_of(T(z0 - h * v0)).item()
        fd = (lp - lm) / (2 * h)
        assert abs(fd - ip) <= 1e-4 * abs(ip), (h, fd, ip)


@pytest.fixture(scope="module")
def patch3d():
    wl = synth.WORKLOADS["patch3d"]
    dev = torch.device("cuda", 0)
    xs = synth.positions(wl.ns, wl)
    d = synth.cube_on_device(xs, xs, wl, synth.down_events(wl), dev)
    r = synth.cube_on_device(xs, xs, wl, synth.reflection_events(wl), dev)
    u = synth.cube_on_device(xs, xs, wl, synth.data_events(wl), dev)
    onset = synth.onsets(wl)
    idx = optim.batches(synth.epoch_permutations(wl, 1)[0], wl.nb)[0]
    cols = np.array([0, 15, 16, 37, 799, 1203, 1584, 1599])
    d_b = H(d[torch.from_numpy(idx.astype(np.int64)).to(dev)])
    u_b = H(u[torch.from_numpy(idx.astype(np.int64)).to(dev)][:, cols, :])
    r_c = H(r[:, cols, :])
    _, go = freq.batch_loss_grad(d_b, r_c, u_b, np.arange(wl.nb), wl.nf)
    go = optim.apply_mask(go, onset[:, cols])
    return wl, d, r, u, onset, idx, cols, go


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("fp32_cgemm", 1e-5), ("bf16x3", 1e-3),
                                      ("fp16x3", 1e-3)])
def test_patch3d_gradient_sampled_columns(patch3d, prec, tol):
    from paper_2202_04486_amd.plan import Plan
    wl, d, r, u, onset, idx, cols, go = patch3d
    plan = Plan(wl.ns, wl.nr, wl.nvs, wl.nt, wl.nf, wl.nb, precision=prec)
    plan.mdd_set_kernel(d)
    plan.mdd_set_data(u)
    plan.mdd_set_mask(T(onset, torch.int32))
    G, loss, gn = plan.mdd_stoch_grad(r, T(idx, torch.int32))
    gs = H(G[:, torch.from_numpy(cols).to(G.device), :])
    e = relerr(gs, go)
    print(f"patch3d {prec}: sampled-column gradient rel err {e:.3e}")
    assert e <= tol
    assert np.isfinite(loss.item()) and np.isfinite(gn.item())
    del G
    plan.close()
    torch.cuda.empty_cache()


def test_patch3d_adam_epoch_sampled_columns(patch3d):
    """One whole epoch (25 steps of 64 sources) of fp32 Adam with the mask and stored
    spectra on the full 1600-trace patch, against the oracle's trajectory of 8 sampled
    virtual-source columns (without reciprocity the columns do not interact, so the
    oracle follows them exactly on the same batches).  eps is 1 % of the oracle's first
    gradient rms, so the update is Lipschitz in g and every entry must follow."""
    from paper_2202_04486_amd.plan import Plan
    wl, d, r, u, onset, idx, cols, go0 = patch3d
    dev = d.device
    eps = 1e-2 * float(np.sqrt(np.mean(go0 ** 2)))
    lr = 1e-2
    plan = Plan(wl.ns, wl.nr, wl.nvs, wl.nt, wl.nf, wl.nb, store_rf=True)
    plan.mdd_set_kernel(d)
    plan.mdd_set_data(u)
    plan.mdd_set_mask(T(onset, torch.int32))
    R = torch.zeros(wl.nr, wl.nvs, wl.nt, device=dev)
    m, v = torch.zeros_like(R), torch.zeros_like(R)
    oc = onset[:, cols]
    ro = np.zeros((wl.nr, len(cols), wl.nt))
    mo, vo = np.zeros_like(ro), np.zeros_like(ro)
    ct = torch.from_numpy(cols).to(dev)
    for t, b in enumerate(optim.batches(synth.epoch_permutations(wl, 1)[0], wl.nb), start=1):
        plan.mdd_step(R, T(b, torch.int32), opt="adam", lr=lr, s0=m, s1=v, t=t, eps=eps)
        bt = torch.from_numpy(b.astype(np.int64)).to(dev)
        _, g = freq.batch_loss_grad(H(d[bt]), ro, H(u[bt][:, ct, :]), np.arange(len(b)), wl.nf)
        ro, mo, vo = optim.adam(ro, mo, vo, optim.apply_mask(g, oc), t, lr, eps=eps, onset=oc)
    assert relerr(H(m[:, ct, :]), mo) <= 1e-5
    assert relerr(H(v[:, ct, :]), vo) <= 1e-5
    diff = np.abs(H(R[:, ct, :]) - ro)
    assert np.linalg.norm(diff) <= 1e-4 * np.linalg.norm(ro)
    assert diff.max() <= 1e-2 * lr
    plan.close()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("n,nt", [(1, 128), (2, 1024), (7, 256), (37, 512), (300, 128),
                                  (301, 1024)])
def test_reciprocity_kernel(n, nt):
    """mdd_reciprocity: bit-exact against (z + z^T) * 0.5 in float32 (one addition and an
    exact halving), out of place and in place, and within rounding of the FP64 oracle."""
    import ctypes
    from paper_2202_04486_amd import native
    z0 = np.random.default_rng(n).standard_normal((n, n, nt)).astype(np.float32)
    want = (z0 + z0.transpose(1, 0, 2)) * np.float32(0.5)      # float32 arithmetic
    assert want.dtype == np.float32
    z = T(z0)
    out = torch.full_like(z, float("nan"))
    lib = native.load()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    native.check("mdd_reciprocity", lib.mdd_reciprocity(ctypes.c_void_p(z.data_ptr()),
                                                        ctypes.c_void_p(out.data_ptr()), n, nt, s))
    torch.cuda.synchronize()
    assert np.array_equal(H(out).astype(np.float32), want)
    assert np.array_equal(H(z).astype(np.float32), z0)
    native.check("mdd_reciprocity", lib.mdd_reciprocity(ctypes.c_void_p(z.data_ptr()),
                                                        ctypes.c_void_p(z.data_ptr()), n, nt, s))
    torch.cuda.synchronize()
    assert np.array_equal(H(z).astype(np.float32), want)
    assert relerr(H(out), optim.reciprocity(z0.astype(np.float64))) <= 1e-7


def test_reciprocity_kernel_rejects_bad_arguments():
    import ctypes
    from paper_2202_04486_amd import native
    lib = native.load()
    z = torch.zeros(4, 4, 128, device="cuda")
    p = ctypes.c_void_p(z.data_ptr())
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    codes = [lib.mdd_reciprocity(None, p, 4, 128, s),
             lib.mdd_reciprocity(ctypes.c_void_p(z.data_ptr() + 4), p, 4, 128, s),
             lib.mdd_reciprocity(p, p, 0, 128, s),
             lib.mdd_reciprocity(p, p, 4097, 128, s),
             lib.mdd_reciprocity(p, p, 4, 200, s)]
    assert codes == [native.MDD_EINVAL] * 2 + [native.MDD_ESHAPE] * 3


@pytest.mark.parametrize("nb", [8, 32, 64])
def test_mdc_rec_gradient_full_size(diff301, nb):
    """The fused operator mdc_rec (C_r applied to spectra inside the library) at 301 traces:
    the loss and the gradient through autograd against the oracle's gradient through C_r."""
    from paper_2202_04486_amd.autograd import mdc_rec
    wl, d, u, plan, z0, _, _ = diff301
    idx = optim.batches(synth.epoch_permutations(wl, 1)[0], nb)[0]
    it = T(idx, torch.int32)
    z = T(z0).requires_grad_(True)
    loss = 0.5 * ((mdc_rec(z, it, plan) - T(u[idx])).double() ** 2).sum()
    loss.backward()
    lo, go = freq.batch_loss_grad(d, optim.reciprocity(z0), u, idx, wl.nf)
    assert abs(loss.item() - lo) <= 1e-5 * lo
    assert relerr(H(z.grad), optim.reciprocity(go)) <= 1e-5


def test_mdc_rec_dot_product(diff301):
    """<P C_r z, y> = <z, C_r P^H y> for the fused pair, in float64 sums of float32 results."""
    wl, d, u, plan, z0, v0, y0 = diff301
    idx = optim.batches(synth.epoch_permutations(wl, 1)[0], 64)[0]
    it = T(idx, torch.int32)
    a = H(plan.mdc_forward_rec(T(z0), it))
    b = H(plan.mdc_adjoint_rec(T(y0), it))
    lhs, rhs = float(np.sum(a * y0)), float(np.sum(z0 * b))
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


@pytest.mark.parametrize("n,nt,nf,nb", [(1, 128, 65, 3), (17, 256, 100, 5), (37, 256, 129, 40)])
def test_mdc_rec_operators_ragged(n, nt, nf, nb):
    """mdc_forward_rec and mdc_adjoint_rec at trace counts that leave the last 16-column
    block partial (and a single trace, where C_r is the identity), against the oracle and
    against the separate reciprocity kernel plus the plain operators."""
    from gpu_helpers import batch, make_plan, random_case
    from paper_2202_04486_amd.autograd import _reciprocity
    ns = max(nb + 3, 12)
    d, u, r = random_case(ns, n, n, nt, seed=n + nb)
    plan = make_plan(d, u, nb_max=nb, nf=nf)
    idx = batch(ns, nb, seed=n)
    it = T(idx, torch.int32)
    fwd = plan.mdc_forward_rec(T(r), it)
    assert relerr(H(fwd), freq.mdc(d[idx], optim.reciprocity(r), nf)) <= 1e-5
    assert relerr(H(fwd), H(plan.mdc_forward(_reciprocity(T(r)), it))) <= 1e-6
    adj = plan.mdc_adjoint_rec(T(u[idx]), it)
    assert relerr(H(adj), optim.reciprocity(freq.mdc_adjoint(d[idx], u[idx], nf))) <= 1e-5
    assert relerr(H(adj), H(_reciprocity(plan.mdc_adjoint(T(u[idx]), it)))) <= 1e-6


def test_mdc_rec_needs_square_models():
    from gpu_helpers import make_plan, random_case
    from paper_2202_04486_amd import MddError
    d, u, r = random_case(10, 12, 9, 128, seed=3)
    plan = make_plan(d, u, nb_max=4, nf=65)
    it = T(np.arange(4, dtype=np.int32), torch.int32)
    with pytest.raises(MddError):
        plan.mdc_forward_rec(T(r), it)
    with pytest.raises(MddError):
        plan.mdc_adjoint_rec(T(u[:4]), it)


def test_patch3d_fp32_gradient_after_250_steps():
    """The 3D patch's geometry with 1600 receivers (so the products sum over 1600
    receivers), 256 sources and 32 virtual sources, noise-free data u = P+ R_true made by
    the oracle, and 250 steps of fp32 Adam (batches of 64, eps 1e-8, the bench's setting,
    mask on), as many as ten epochs of the full patch.  The model fits
    the data and the gradient shrinks to a few per cent of its size at R = 0, while the
    rounding of D_b R_k - U_b stays at the data's scale.  The gradient at that model must
    still match the oracle to 1e-5: the products' compensated two-level sum keeps that
    rounding small enough (one float32 accumulator over the 1600 receivers did not)."""
    from paper_2202_04486_amd.plan import Plan
    wl = synth.WORKLOADS["patch3d"].replace(ns=256, nvs=32, vs_first=784)
    dev = torch.device("cuda", 0)
    xs, xr = synth.positions(wl.ns, wl), synth.positions(wl.nr, wl)
    xv = synth.vs_positions(wl)
    d = synth.cube_on_device(xs, xr, wl, synth.down_events(wl), dev)
    r_true = synth.cube_on_device(xr, xv, wl, synth.reflection_events(wl), dev)
    onset = synth.onsets(wl)
    d64 = H(d)
    u = f32(freq.mdc(d64, H(r_true), wl.nf))
    del r_true
    plan = Plan(wl.ns, wl.nr, wl.nvs, wl.nt, wl.nf, wl.nb, store_rf=True)
    plan.mdd_set_kernel(d)
    plan.mdd_set_data(T(u))
    plan.mdd_set_mask(T(onset, torch.int32))
    R = torch.zeros(wl.nr, wl.nvs, wl.nt, device=dev)
    m, v = torch.zeros_like(R), torch.zeros_like(R)
    perms = synth.epoch_permutations(wl, 64)
    t = 0
    for e in range(63):
        for b in optim.batches(perms[e], wl.nb):
            t += 1
            plan.mdd_step(R, T(b, torch.int32), opt="adam", lr=1e-2, s0=m, s1=v, t=t)
    b0 = optim.batches(perms[63], wl.nb)[0]
    G, _, _ = plan.mdd_stoch_grad(R, T(b0, torch.int32))
    _, go = freq.batch_loss_grad(d64, H(R), u, b0, wl.nf)
    go = optim.apply_mask(go, onset)
    _, g0 = freq.batch_loss_grad(d64, np.zeros_like(go), u, b0, wl.nf)
    g0 = optim.apply_mask(g0, onset)
    e = relerr(H(G), go)
    ratio = np.linalg.norm(go) / np.linalg.norm(g0)
    print(f"patch3d fp32, 256 sources, 32 virtual sources, after {t} steps: gradient {ratio:.3f} of its size "
          f"at R = 0, rel err {e:.3e}, err over the gradient at R = 0 {e * ratio:.2e}")
    assert ratio < 0.05                                 # the model has fitted the data
    assert e <= 1e-5
    plan.close()
    torch.cuda.empty_cache()
