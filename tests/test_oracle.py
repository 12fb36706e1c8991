"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a library
routine (numpy FFT, scipy circulant, numpy pinv / SVD), a closed form, an
invariant of the finite-sum functional, or a value printed in the paper
(fixtures under tests/golden/, each with its citation).  Shapes are deliberately
non-square (ns != nr != nvs) so a transposed operand or swapped axis fails.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg

import synth
from oracle import direct, freq, optim, stepsize

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


# ---------------------------------------------------------------- P1: conventions

@pytest.mark.parametrize("nt", [8, 15, 32])
def test_dft_matches_numpy_fft(nt):
    x = rand((3, nt), 1)
    np.testing.assert_allclose(direct.dft(x), np.fft.fft(x, axis=-1), rtol=0, atol=1e-12)
    np.testing.assert_allclose(direct.idft(direct.dft(x)).real, x, atol=1e-13)


def _mdc_by_circulant(d, r):
    """Forward operator assembled from scipy circulant blocks: block (s, r) applied to a
    trace is circular convolution with d[s, r, :] (library routine, independent code)."""
    ns, nr, nt = d.shape
    nvs = r.shape[1]
    u = np.zeros((ns, nvs, nt))
    for s in range(ns):
        for ir in range(nr):
            c = scipy.linalg.circulant(d[s, ir])   # c[i, j] = d[(i - j) mod nt]
            u[s] += (c @ r[ir].T).T
    return u


def test_mdc_is_sum_of_circular_convolutions():
    d, r = rand((3, 4, 16), 2), rand((4, 5, 16), 3)
    np.testing.assert_allclose(direct.mdc(d, r), _mdc_by_circulant(d, r), rtol=0, atol=1e-12)


def test_mdc_convolution_theorem_bruteforce():
    """Per frequency the operator is the matrix product P-_f = P+_f R_f (Theory section)."""
    d, r = rand((3, 4, 16), 4), rand((4, 5, 16), 5)
    df, rf = direct.dft(d), direct.dft(r)
    uf = np.einsum("srk,rvk->svk", df, rf)
    np.testing.assert_allclose(direct.mdc(d, r), direct.idft(uf).real, atol=1e-12)


def test_adjoint_is_transpose_of_assembled_operator():
    d, v = rand((3, 4, 12), 6), rand((3, 5, 12), 7)
    ns, nr, nt = d.shape
    g = np.zeros((nr, 5, nt))
    for s in range(ns):
        for ir in range(nr):
            c = scipy.linalg.circulant(d[s, ir])
            g[ir] += (c.T @ v[s].T).T
    np.testing.assert_allclose(direct.mdc_adjoint(d, v), g, atol=1e-12)


@pytest.mark.parametrize("nt,nf", [(16, 9), (16, 5), (16, 1), (32, 7)])
def test_bandlimit_projection(nt, nf):
    x = rand((2, 3, nt), 8)
    xb = direct.bandlimit(x, nf)
    keep = direct.retained_bins(nt, nf)
    xf = np.fft.fft(xb, axis=-1)
    if (~keep).any():
        assert np.abs(xf[..., ~keep]).max() < 1e-12                  # nothing out of band
    np.testing.assert_allclose(np.fft.fft(x, axis=-1)[..., keep], xf[..., keep], atol=1e-12)
    np.testing.assert_allclose(direct.bandlimit(xb, nf), xb, atol=1e-12)  # idempotent
    np.testing.assert_allclose(freq.bandlimit(x, nf), xb, atol=1e-12)
    if nf == nt // 2 + 1:
        np.testing.assert_allclose(xb, x, atol=1e-12)


@pytest.mark.parametrize("nf", [9, 6])
def test_freq_oracle_matches_direct(nf):
    nt = 16
    d, r, v = rand((3, 4, nt), 9), rand((4, 5, nt), 10), rand((3, 5, nt), 11)
    dbl = direct.bandlimit(d, nf)
    np.testing.assert_allclose(freq.mdc(d, r, nf), direct.mdc(dbl, r), atol=1e-12)
    np.testing.assert_allclose(freq.mdc_adjoint(d, v, nf), direct.mdc_adjoint(dbl, v), atol=1e-12)
    u = rand((3, 5, nt), 12)
    idx = [0, 2, 2]
    l1, g1 = freq.batch_loss_grad(d, r, u, idx, nf)
    l2, g2 = direct.batch_loss_grad(dbl, r, u, idx)
    assert abs(l1 - l2) <= 1e-12 * abs(l2)
    np.testing.assert_allclose(g1, g2, atol=1e-11)


# ---------------------------------------------------------------- P2: adjoint pairing

@pytest.mark.parametrize("impl", ["direct", "freq"])
def test_dot_product_identity(impl):
    nt, nf = 32, 12
    d, x, y = rand((5, 3, nt), 13), rand((3, 4, nt), 14), rand((5, 4, nt), 15)
    if impl == "direct":
        ax, aty = direct.mdc(d, x), direct.mdc_adjoint(d, y)
    else:
        ax, aty = freq.mdc(d, x, nf), freq.mdc_adjoint(d, y, nf)
    lhs, rhs = float(np.sum(ax * y)), float(np.sum(x * aty))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


# ---------------------------------------------------------------- P3: finite sum

def test_finite_sum_identity():
    """The batch gradients of a partition of the sources add up to the full gradient,
    and the full gradient is ns times the mean of the single-source gradients."""
    nt, nf, ns = 16, 9, 7
    d, r, u = rand((ns, 3, nt), 16), rand((3, 4, nt), 17), rand((ns, 4, nt), 18)
    dbl = direct.bandlimit(d, nf)
    lf, gf = direct.batch_loss_grad(dbl, r, u, np.arange(ns))
    parts = optim.batches(np.random.default_rng(0).permutation(ns), 3)
    res = [direct.batch_loss_grad(dbl, r, u, b) for b in parts]
    np.testing.assert_allclose(sum(g for _, g in res), gf, atol=1e-11)
    assert abs(sum(l for l, _ in res) - lf) <= 1e-12 * lf
    singles = [direct.batch_loss_grad(dbl, r, u, [s])[1] for s in range(ns)]
    np.testing.assert_allclose(ns * np.mean(singles, axis=0), gf, atol=1e-11)


def test_duplicate_indices_count_twice():
    nt = 16
    d, r, u = rand((4, 3, nt), 19), rand((3, 2, nt), 20), rand((4, 2, nt), 21)
    l1, g1 = direct.batch_loss_grad(d, r, u, [1, 1])
    l2, g2 = direct.batch_loss_grad(d, r, u, [1])
    np.testing.assert_allclose(g1, 2 * g2, atol=1e-12)
    assert abs(l1 - 2 * l2) < 1e-12 * l1


# ---------------------------------------------------------------- P4: zero gradient at truth

def test_zero_gradient_at_truth_tiny_workload():
    wl = synth.WORKLOADS["tiny2d"]
    p = synth.make_problem(wl)
    dbl = direct.bandlimit(p["d"], wl.nf)
    u = direct.mdc(dbl, p["r_true"])
    _, g0 = direct.batch_loss_grad(dbl, np.zeros_like(p["r_true"]), u, np.arange(8))
    for b in optim.batches(synth.epoch_permutations(wl, 1)[0], wl.nb):
        loss, g = direct.batch_loss_grad(dbl, p["r_true"], u, b)
        assert loss <= 1e-20 * float(np.sum(u * u))
        assert np.linalg.norm(g) <= 1e-12 * np.linalg.norm(g0)


# ---------------------------------------------------------------- P5: recovery

def test_exact_recovery_well_conditioned():
    """Kernel = identity spike plus weak events, so every D_k is invertible: Landweber
    from zero with alpha = 1/sigma_max^2 recovers R_true (no nullspace)."""
    ns = nr = 6
    nvs, nt = 3, 16
    d = 0.015 * rand((ns, nr, nt), 22)
    d[np.arange(ns), np.arange(nr), 0] += 1.0
    assert np.linalg.svd(np.moveaxis(np.fft.fft(d, axis=-1), -1, 0), compute_uv=False).min() > 0.5
    r_true = rand((nr, nvs, nt), 23)
    u = direct.mdc(d, r_true)
    s2, _ = stepsize.sigma_max2_kernel(d, nt // 2 + 1)
    r = np.zeros_like(r_true)
    for _ in range(300):
        _, g = direct.batch_loss_grad(d, r, u, np.arange(ns))
        r = optim.sgd(r, g, 1.0 / s2)
    assert np.abs(r - r_true).max() < 1e-10


def test_full_gradient_limit_is_min_norm_solution():
    """With fewer sources than receivers (rank-deficient D_k) gradient descent from zero
    converges to the minimum-norm solution R_k = pinv(D_k) U_k, not to R_true."""
    ns, nr, nvs, nt, nf = 3, 5, 2, 8, 5
    d, r_true = rand((ns, nr, nt), 24), rand((nr, nvs, nt), 25)
    u = freq.mdc(d, r_true, nf)
    s2, _ = stepsize.sigma_max2_kernel(d, nf)
    r = np.zeros_like(r_true)
    for _ in range(4000):
        _, g = freq.batch_loss_grad(d, r, u, np.arange(ns), nf)
        r = optim.sgd(r, g, 1.0 / s2)
    df = np.moveaxis(freq.spectra(d, nf), -1, 0)
    uf = np.moveaxis(freq.spectra(u, nf), -1, 0)
    rf = np.matmul(np.linalg.pinv(df), uf)                 # [nf][nr][nvs]
    r_mn = freq.traces(np.moveaxis(rf, 0, -1), nt)
    np.testing.assert_allclose(r, r_mn, atol=1e-8)
    assert np.abs(r - r_true).max() > 1e-2                  # the nullspace is real


# ---------------------------------------------------------------- P6: Landweber example

def test_landweber_example_from_paper():
    gx = golden("landweber_example.json")
    a = np.array(gx["A"], dtype=np.float64)
    x = np.array(gx["x"], dtype=np.float64)
    s2 = stepsize.sigma_max2_matrix(a)
    assert abs(s2 - (67 + math.sqrt(1525)) / 2) < 1e-12    # closed form of A^T A
    assert round(s2) == gx["sigma2_printed"]
    y = a @ x
    xc, hc = stepsize.landweber(a, y, gx["alpha_factor_converges"] / s2, 400)
    np.testing.assert_allclose(xc, x, atol=1e-8)
    _, hd = stepsize.landweber(a, y, gx["alpha_factor_diverges"] / s2, 400)
    assert hd[-1] > 1e3 * hd[0]
    assert abs(100 * (gx["alpha_factor_diverges"] / 2 - 1) - gx["percent_above_limit"]) < 1e-9
    np.testing.assert_allclose(stepsize.steepest_descent(a, y, 50), x, atol=1e-10)


# ---------------------------------------------------------------- P7: sigma_max

def test_operator_sigma_equals_kernel_sigma():
    """Matrix-free power iteration on A^T A of the time-domain operator gives the largest
    per-frequency squared singular value of the kernel (Appendix B)."""
    ns, nr, nvs, nt, nf = 4, 3, 2, 16, 7
    d = rand((ns, nr, nt), 26)
    dbl = direct.bandlimit(d, nf)
    lam = stepsize.power_iteration(lambda x: direct.mdc_adjoint(dbl, direct.mdc(dbl, x)),
                                   (nr, nvs, nt), 400)
    s2, per_k = stepsize.sigma_max2_kernel(d, nf)
    assert abs(lam - s2) <= 1e-9 * s2
    assert per_k.shape == (nf,)


# ---------------------------------------------------------------- P8: schedule

def test_steps_per_epoch_from_paper():
    gx = golden("schedule_obc.json")
    perm = np.random.default_rng(0).permutation(gx["ns"])
    bs = optim.batches(perm, gx["nb"])
    assert len(bs) == gx["steps_per_epoch"] == gx["ns"] // gx["nb"] + 1
    assert sorted(np.concatenate(bs).tolist()) == list(range(gx["ns"]))
    assert len(bs[-1]) == 9
    assert all(np.all(np.diff(b) > 0) for b in bs)


@pytest.mark.parametrize("ns,nb,steps,last", [(201, 16, 13, 9), (1600, 64, 25, 64),
                                               (301, 8, 38, 5), (301, 32, 10, 13),
                                               (301, 64, 5, 45), (32, 8, 4, 8)])
def test_batch_counts(ns, nb, steps, last):
    bs = optim.batches(np.arange(ns)[::-1], nb)
    assert len(bs) == steps and len(bs[-1]) == last


# ---------------------------------------------------------------- P9: Parseval loss

@pytest.mark.parametrize("nt,nf", [(16, 9), (16, 4), (32, 17)])
def test_loss_in_frequency_domain(nt, nf):
    """The time-domain loss equals the Hermitian-weighted in-band sum of squared residual
    spectra over 2 nt plus the out-of-band energy of the data (Parseval)."""
    d, r, u = rand((4, 3, nt), 27), rand((3, 2, nt), 28), rand((4, 2, nt), 29)
    idx = [0, 3]
    loss, _ = freq.batch_loss_grad(d, r, u, idx, nf)
    df = np.fft.rfft(d[idx], axis=-1)[..., :nf]
    rf = np.fft.rfft(r, axis=-1)[..., :nf]
    uf = np.fft.rfft(u[idx], axis=-1)
    res = np.einsum("srk,rvk->svk", df, rf) - uf[..., :nf]
    w = np.full(nt // 2 + 1, 2.0)
    w[0] = 1.0
    w[nt // 2] = 1.0
    inband = np.sum(w[:nf] * np.abs(res) ** 2) / (2 * nt)
    oob = np.sum(w[nf:] * np.abs(uf[..., nf:]) ** 2) / (2 * nt)
    assert abs(loss - (inband + oob)) <= 1e-12 * loss


# ---------------------------------------------------------------- P10: finite differences

def test_central_difference_is_exact_for_quadratic_loss():
    nt, nf = 16, 9
    d, r, u, v = rand((4, 3, nt), 30), rand((3, 2, nt), 31), rand((4, 2, nt), 32), rand((3, 2, nt), 33)
    idx = [1, 2, 3]
    _, g = freq.batch_loss_grad(d, r, u, idx, nf)
    for h in (1e-3, 1.0, 10.0):
        lp, _ = freq.batch_loss_grad(d, r + h * v, u, idx, nf)
        lm, _ = freq.batch_loss_grad(d, r - h * v, u, idx, nf)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - float(np.sum(g * v))) <= 1e-9 * max(abs(fd), 1.0) * max(1.0, h * h)


# ---------------------------------------------------------------- P11 / P12: preconditioners

def test_causal_mask_algebra():
    wl = synth.WORKLOADS["tiny2d"].replace(mask=True)
    on = synth.onsets(wl)
    x = rand((wl.nr, wl.nvs, wl.nt), 34)
    mx = optim.apply_mask(x, on)
    np.testing.assert_array_equal(optim.apply_mask(mx, on), mx)
    t = np.arange(wl.nt)
    assert np.all(mx[t[None, None, :] < on[:, :, None]] == 0.0)
    assert np.array_equal(on, on.T)                          # onset symmetric in (r, vs)
    np.testing.assert_allclose(optim.reciprocity(optim.apply_mask(x, on)),
                               optim.apply_mask(optim.reciprocity(x), on), atol=0)


def test_mask_passes_true_response():
    wl = synth.WORKLOADS["line2d"].replace(ns=8, nr=40, nvs=40)
    p = synth.make_problem(wl, with_noise=False)
    r = p["r_true"]
    leak = np.abs(r - optim.apply_mask(r, p["onset"])).max()
    assert leak < 1e-6 * np.abs(r).max()


@pytest.mark.parametrize("name", ["line2d_vs1", "patch3d_vs1"])
def test_single_virtual_source_workloads(name):
    """The one virtual source sits at the middle receiver position, its column of the
    multi-source workload: same onsets, same true response, and the mask passes it."""
    wl = synth.WORKLOADS[name]
    full = synth.WORKLOADS[name.replace("_vs1", "")]
    assert wl.nvs == 1 and synth.vs_positions(full).shape[0] == full.nvs
    np.testing.assert_array_equal(synth.vs_positions(wl)[0], synth.positions(full.nr, full)[wl.vs_first])
    np.testing.assert_array_equal(synth.onsets(wl)[:, 0], synth.onsets(full)[:, wl.vs_first])
    p = synth.make_problem(wl.replace(ns=4, nt=256), with_noise=False)
    xr = synth.positions(full.nr, full)
    col = synth.event_cube(xr, xr[[wl.vs_first]], 256, wl.dt, wl.f0, p["r_events"])
    np.testing.assert_array_equal(p["r_true"], col)
    leak = np.abs(p["r_true"] - optim.apply_mask(p["r_true"], p["onset"])).max()
    assert leak < 1e-6 * np.abs(p["r_true"]).max()


def test_reciprocity_self_adjoint_idempotent():
    z, w = rand((5, 5, 8), 35), rand((5, 5, 8), 36)
    cz = optim.reciprocity(z)
    np.testing.assert_allclose(optim.reciprocity(cz), cz, atol=1e-15)
    assert abs(np.sum(cz * w) - np.sum(z * optim.reciprocity(w))) < 1e-12
    np.testing.assert_allclose(cz, np.swapaxes(cz, 0, 1), atol=0)


def test_reciprocity_commutes_with_the_trace_transform():
    """C_r acts on each time sample alone, so it can be applied to the retained spectra of
    the model (or of the adjoint's output) instead of the traces: on every bin,
    rfft(C_r z) = (Z + Z^T) / 2 with Z = rfft(z), so every retained band sees the same model."""
    z = rand((7, 7, 16), 37)
    Z = np.fft.rfft(z, axis=-1)
    np.testing.assert_allclose(np.fft.rfft(optim.reciprocity(z), axis=-1),
                               0.5 * (Z + np.swapaxes(Z, 0, 1)), atol=1e-13)


# ---------------------------------------------------------------- updates

def test_adam_constant_gradient_closed_form():
    """With bias correction and a constant gradient, every Adam step moves each entry
    by exactly lr * g / (|g| + eps) (m_hat = g, v_hat = g^2)."""
    g = np.array([0.5, -2.0, 1e-3])
    r = np.array([1.0, 2.0, 3.0])
    m = np.zeros(3)
    v = np.zeros(3)
    lr, eps = 0.01, 1e-8
    for t in range(1, 6):
        r_new, m, v = optim.adam(r, m, v, g, t, lr, eps=eps)
        np.testing.assert_allclose(r - r_new, lr * g / (np.abs(g) + eps), rtol=1e-12)
        r = r_new


def test_sgd_and_mask():
    r = np.ones((1, 1, 4))
    g = np.array([[[1.0, 2.0, 3.0, 4.0]]])
    on = np.array([[2]], dtype=np.int32)
    np.testing.assert_allclose(optim.sgd(r, g, 0.5, on), [[[0.0, 0.0, -0.5, -1.0]]])


# Nesterov momentum (Theory section: the N-SGD iteration, after Sutskever et al.).  The
# pins below fix the look-ahead point, the order of the two updates and the masking,
# each against something other than oracle.optim.nesterov itself.

def test_nesterov_without_momentum_is_sgd():
    """mu = 0: the velocity is -lr g(r) and the step is the SGD step, every step."""
    r = rand((3, 2, 8), 60)
    vel = np.zeros_like(r)
    tgt = rand((3, 2, 8), 61)
    on = np.array([[0, 3], [5, 1], [8, 2]], dtype=np.int32)
    r = optim.apply_mask(r, on)
    r_sgd = r.copy()
    for _ in range(4):
        r, vel = optim.nesterov(r, vel, lambda x: x - tgt, 0.3, 0.0, onset=on)
        r_sgd = optim.sgd(r_sgd, r_sgd - tgt, 0.3, onset=on)
        np.testing.assert_allclose(r, r_sgd, rtol=0, atol=1e-15)


# f(x) = a x^2 / 2 with a = 2, lr = 0.1, mu = 0.5, x0 = 1, v0 = 0, unrolled by hand:
#   v1 = -lr a x0 = -0.2,                    x1 = 0.8
#   v2 = mu v1 - lr a (x1 + mu v1) = -0.24,  x2 = 0.56
#   v3 = mu v2 - lr a (x2 + mu v2) = -0.208, x3 = 0.352
_NESTEROV_1D = [(0.8, -0.2), (0.56, -0.24), (0.352, -0.208)]


def _nesterov_1d(step):
    x, v = np.array([1.0]), np.array([0.0])
    out = []
    for _ in range(3):
        x, v = step(x, v)
        out.append((float(x[0]), float(v[0])))
    return out


def test_nesterov_hand_unrolled_scalar_quadratic():
    got = _nesterov_1d(lambda x, v: optim.nesterov(x, v, lambda y: 2.0 * y, 0.1, 0.5))
    np.testing.assert_allclose(got, _NESTEROV_1D, rtol=0, atol=1e-15)


def test_nesterov_three_term_recurrence_on_landweber_system():
    """On the quadratic 1/2 ||A x - y||^2 of the Landweber example (Appendix B), each
    eigen-direction of A^T A with eigenvalue lam follows the scalar three-term
    recurrence e_{t+1} = (1 + mu)(1 - lr lam) e_t - mu (1 - lr lam) e_{t-1} (e = error
    along that direction), with e_1 = (1 - lr lam) e_0 from v0 = 0.  The eigen-pairs
    come from numpy's eigh, the recurrence is propagated per direction, and the iterates
    must meet x = [1, 1]."""
    gx = golden("landweber_example.json")
    a = np.array(gx["A"], dtype=np.float64)
    x_true = np.array(gx["x"], dtype=np.float64)
    y = a @ x_true
    lam, q = np.linalg.eigh(a.T @ a)
    lr, mu = 1.0 / lam.max(), 0.9
    x = np.zeros(2)
    vel = np.zeros(2)
    e_prev = q.T @ (x - x_true)
    e_cur = (1.0 - lr * lam) * e_prev
    for t in range(60):
        x, vel = optim.nesterov(x, vel, lambda z: a.T @ (a @ z - y), lr, mu)
        np.testing.assert_allclose(q.T @ (x - x_true), e_cur, rtol=0, atol=1e-12)
        e_prev, e_cur = e_cur, (1 + mu) * (1 - lr * lam) * e_cur - mu * (1 - lr * lam) * e_prev
    for _ in range(400):
        x, vel = optim.nesterov(x, vel, lambda z: a.T @ (a @ z - y), lr, mu)
    np.testing.assert_allclose(x, x_true, atol=1e-10)


def test_nesterov_look_ahead_reparametrisation():
    """In the look-ahead variable phi = r + mu vel the same iteration reads
    phi <- phi + mu^2 vel - (1 + mu) lr g(phi), vel <- mu vel - lr g(phi): the gradient is
    evaluated at phi, the point the next step starts from."""
    c = rand((4, 6), 62)
    h = c.T @ c + 0.1 * np.eye(6)
    b = rand(6, 63)

    def grad(z):
        return h @ z - b

    lr, mu = 0.05, 0.8
    r = rand(6, 64)
    vel = rand(6, 65)
    phi = r + mu * vel
    vphi = vel.copy()
    for _ in range(10):
        r, vel = optim.nesterov(r, vel, grad, lr, mu)
        g = grad(phi)
        phi = phi + mu * mu * vphi - (1 + mu) * lr * g
        vphi = mu * vphi - lr * g
        np.testing.assert_allclose(r + mu * vel, phi, rtol=0, atol=1e-12)
        np.testing.assert_allclose(vel, vphi, rtol=0, atol=1e-12)


def test_nesterov_keeps_muted_samples_zero():
    """Causality preconditioner: model and velocity stay zero before each trace's onset,
    even with a gradient that is nonzero there."""
    on = np.array([[2, 0], [7, 4]], dtype=np.int32)
    r = optim.apply_mask(rand((2, 2, 8), 66), on)
    vel = np.zeros_like(r)
    keep = optim.causal_mask(on, 8)
    for _ in range(5):
        r, vel = optim.nesterov(r, vel, lambda z: z + 1.0, 0.2, 0.9, onset=on)
        assert np.all(r[keep == 0] == 0.0) and np.all(vel[keep == 0] == 0.0)
        assert np.all(r[keep == 1] != 0.0)


def test_nesterov_pins_catch_planted_look_ahead_mistake():
    """The gradient taken at r instead of r + mu vel (heavy-ball momentum) must fail the
    hand-unrolled pin; so must the velocity update applied after the model update."""
    def heavy_ball(x, v):
        v = 0.5 * v - 0.1 * 2.0 * x
        return x + v, v

    def late_velocity(x, v):
        x = x + v
        return x, 0.5 * v - 0.1 * 2.0 * (x + 0.5 * v)

    for wrong in (heavy_ball, late_velocity):
        got = _nesterov_1d(wrong)
        assert np.abs(np.array(got) - np.array(_NESTEROV_1D)).max() > 1e-3


def test_rmse_properties():
    a = rand((3, 4, 5), 37)
    assert optim.rmse(a, a) == 0.0
    assert optim.rmse(a, 3.7 * a) < 1e-15
    assert abs(optim.rmse(a, -a) - 2 * np.linalg.norm(a / np.abs(a).max())) < 1e-12


def test_stochastic_alpha_within_paper_range():
    gx = golden("stochastic_stepsize.json")
    a = stepsize.stochastic_alpha(53.0)
    assert gx["fraction_low"] <= a / (2 / 53.0) <= gx["fraction_high"]


# ---------------------------------------------------------------- planted mistakes

def test_pins_catch_planted_mistakes():
    """A wrong time index (correlation instead of convolution) in the oracle's forward
    operator must fail the circulant pin; a dropped conjugate / wrong roll in the adjoint
    must fail the dot-product pin."""
    d, r = rand((3, 4, 16), 38), rand((4, 5, 16), 39)

    def bad_mdc(dd, rr):
        u = np.zeros((dd.shape[0], rr.shape[1], dd.shape[2]))
        for tau in range(dd.shape[2]):
            u += np.einsum("sr,rvt->svt", dd[:, :, tau], np.roll(rr, -tau, axis=2))
        return u

    assert np.abs(bad_mdc(d, r) - _mdc_by_circulant(d, r)).max() > 1e-3
    y = rand((3, 5, 16), 40)
    x = rand((4, 5, 16), 41)
    lhs = float(np.sum(direct.mdc(d, x) * y))
    wrong = np.zeros_like(x)
    for tau in range(16):  # adjoint with the roll direction flipped
        wrong += np.einsum("sr,svt->rvt", d[:, :, tau], np.roll(y, tau, axis=2))
    assert abs(lhs - float(np.sum(x * wrong))) > 1e-3 * abs(lhs)
