#!/usr/bin/env python3
"""Stochastic-MDD benchmark on one MI355X: gradient evaluations per second.

A step is one `mdd_step` (model spectra [stored by the previous step], the
fused per-frequency products with residual and loss, inverse transforms with
mask, gradient norm and Adam update, float64 reductions) on one batch of
sources.  The default workload is the synthetic 3D patch: 1600 sources /
receivers / virtual sources on a 40 x 40 grid at 25 m, 512 samples at 4 ms,
200 retained bins, Ricker 12 Hz, 10 periodic down-going events, 5 reflections,
batches of 64, Adam, causality mask.  The FP32 form gives `value`; the bf16
and fp16 split forms (and the single-pass bf16 diagnostic, and the float32
form with four real products per complex one) are timed on the same data and
reported beside it with their gradient error against the FP64 oracle on
sampled virtual-source columns.  `--workload line2d` runs the 201-trace 2D
line (1024 samples, 257 bins, batches of 16, 20 dB noise) instead;
`line2d_vs1` and `patch3d_vs1` invert for one virtual source in the middle of
the line (batches of 32, Nesterov momentum) or of the patch (batches of 64,
Adam), where the products are matrix-vector products; `diff301` times the
differentiation form (a gradient through torch.autograd at 301 traces for
batches of 8, 32 and 64, and the reciprocity kernel).  One full-gradient
iteration (every source, SGD) is timed beside the stochastic epoch.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
                    [--workload patch3d|line2d|line2d_vs1|patch3d_vs1|diff301]

Prints one JSON line.  Inputs are resident in HBM before timing starts.  `value` is
timed over K steps with no instrumentation; the per-kernel durations behind the
roofline come from HIP events on the plan's stream over K further steps.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "stochastic MDD grad evals/s + % MFMA roofline, BF16-split vs FP32 at stated err"
WORKLOAD_TEXT = {
    "line2d": "line2d: ns=nr=nvs=201 (10 m line), nt=1024 (4 ms), nf=257, batch 16, Adam, "
              "causality mask, 20 dB noise, stored model spectra",
    "patch3d": "patch3d: ns=nr=nvs=1600 (40x40 grid at 25 m), nt=512 (4 ms), nf=200, batch 64, "
               "Adam, causality mask, noise-free, stored model spectra",
    "line2d_vs1": "line2d_vs1: ns=nr=201 (10 m line), one virtual source at receiver 100, "
                  "nt=1024 (4 ms), nf=257, batch 32, Nesterov momentum 0.9 at the kernel-derived "
                  "step, causality mask, 20 dB noise, stored model spectra",
    "patch3d_vs1": "patch3d_vs1: ns=nr=1600 (40x40 grid at 25 m), one virtual source at grid "
                   "point (20, 20), nt=512 (4 ms), nf=200, batch 64, Adam, causality mask, "
                   "noise-free, stored model spectra",
}
DEFAULT_EPOCHS = {"line2d": 10, "patch3d": 1, "line2d_vs1": 50, "patch3d_vs1": 10}
AUTOGRAD_TEXT = ("diff301: differentiation form, ns=nr=nvs=301 (10 m line), nt=1024, nf=257, "
                 "loss 1/2 ||P_b C_r z - u_b||^2 through torch.autograd (mdc_forward_rec / "
                 "mdc_adjoint_rec: C_r on the spectra inside the operators), random N(0,1) "
                 "model, batches 8 / 32 / 64")
# Model-sized float32 arrays each update reads and writes (R and the optimiser state).
STATE_ARRAYS = {"adam": 3, "nsgd": 2, "sgd": 1}
HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"fp32": 157.3, "fp32_cgemm": 157.3, "bf16x3": 2516.6, "fp16x3": 2516.6,
                    "bf16": 2516.6}
TRAFFIC_FILE = {w: os.path.join(ROOT, "profiles", f"traffic_{w}.md")
                for w in list(WORKLOAD_TEXT) + ["diff301"]}
CSRC = os.path.join(ROOT, "paper_2202_04486_amd", "csrc")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_inputs(wl, dev):
    """d, R_true on the GPU from the closed-form events; noise from the seeded host stream."""
    import torch

    import synth
    g = synth.streams(wl.seed)
    xs, xr, xv = synth.positions(wl.ns, wl), synth.positions(wl.nr, wl), synth.vs_positions(wl)
    d = synth.cube_on_device(xs, xr, wl, synth.down_events(wl, g[0]), dev)
    r_true = synth.cube_on_device(xr, xv, wl, synth.reflection_events(wl, g[1]), dev)
    noise = None
    if wl.snr_db is not None:
        noise = torch.from_numpy(g[2].standard_normal((wl.ns, wl.nvs, wl.nt), dtype=np.float32)).to(dev)
    return d, r_true, noise, synth.onsets(wl)


def up_going(plan, r_true, noise, wl, dev):
    """u = P+ R_true with the library's forward operator, plus noise at the stated SNR."""
    import torch
    u = torch.empty((wl.ns, wl.nvs, wl.nt), dtype=torch.float32, device=dev)
    nb = plan.nb_max
    for s0 in range(0, wl.ns, nb):
        idx = torch.arange(s0, min(wl.ns, s0 + nb), dtype=torch.int32, device=dev)
        plan.mdc_forward(r_true, idx, out=u[s0:s0 + idx.numel()])
    if noise is not None:
        eu = float((u.double() ** 2).sum())
        en = float((noise.double() ** 2).sum())
        u += noise * math.sqrt(eu / (en * 10.0 ** (wl.snr_db / 10.0)))
    return u


def step_tables(wl, nb, n_steps, dev):
    """The batch sequence of as many epochs as needed, on the device."""
    import torch

    import synth
    from paper_2202_04486_amd.solver import epoch_index_table
    spe = math.ceil(wl.ns / nb)
    perms = synth.epoch_permutations(wl, math.ceil(n_steps / spe) + 1)
    tabs, lens = [], []
    for p in perms:
        t, ln = epoch_index_table(p, nb)
        tabs.append(t)
        lens.append(ln)
    return torch.from_numpy(np.concatenate(tabs)).to(dev), np.concatenate(lens), spe


def time_full_gradient(wl, d, u, onset_t, dev, iters, warmup=2):
    """Milliseconds per full-gradient iteration (every source, SGD update, stored spectra):
    the baseline a stochastic epoch is compared with (one pass over the data each)."""
    import torch

    from paper_2202_04486_amd.plan import Plan
    plan = Plan(wl.ns, wl.nr, wl.nvs, wl.nt, wl.nf, wl.nb, store_rf=True, device=dev,
                full_grad=True)
    plan.mdd_set_kernel(d)
    plan.mdd_set_data(u)
    plan.mdd_set_mask(onset_t)
    R = torch.zeros((wl.nr, wl.nvs, wl.nt), dtype=torch.float32, device=dev)
    loss = torch.zeros(warmup + iters, dtype=torch.float64, device=dev)
    for j in range(warmup):
        plan.mdd_full_step(R, opt="sgd", lr=1e-6, loss_out=loss[j:j + 1])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in range(warmup, warmup + iters):
        plan.mdd_full_step(R, opt="sgd", lr=1e-6, loss_out=loss[j:j + 1])
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / iters
    del plan
    torch.cuda.empty_cache()
    return ms


def run_form(form, wl, d, u, onset_t, idx_tab, lens, warmup, steps, dev, lr=1e-2, store_rf=True):
    """Adam at lr, or Nesterov momentum (mu 0.9) at half the kernel-derived step
    2 / sigma_max^2 (Appendix B), as the workload states."""
    import torch

    from paper_2202_04486_amd.plan import Plan
    plan = Plan(wl.ns, wl.nr, wl.nvs, wl.nt, wl.nf, wl.nb, precision=form, store_rf=store_rf,
                device=dev)
    plan.mdd_set_kernel(d)
    plan.mdd_set_data(u)
    plan.mdd_set_mask(onset_t)
    opt = wl.optimizer
    if opt == "nsgd":
        lr = 0.5 * 2.0 / float(plan.mdd_sigma_max2(iters=100).max().item())
    R = torch.zeros((wl.nr, wl.nvs, wl.nt), dtype=torch.float32, device=dev)
    m, v = torch.zeros_like(R), torch.zeros_like(R)
    loss = torch.zeros(warmup + 3 * steps, dtype=torch.float64, device=dev)
    gn = torch.zeros_like(loss)

    def step(j):
        plan.mdd_step(R, idx_tab[j, :lens[j]], opt=opt, lr=lr, s0=m, s1=v, t=j + 1, mu=0.9,
                      loss_out=loss[j:j + 1], gnorm2_out=gn[j:j + 1])

    for j in range(warmup):
        step(j)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in range(warmup, warmup + steps):
        step(j)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # Per-kernel durations: HIP events around every launch, over the next `steps` steps.
    # They are taken apart from the throughput above because each event record on the
    # stream adds a few microseconds between kernels.
    plan.profile_enable(True, capacity=8 * steps + 64)
    torch.cuda.synchronize()
    for j in range(warmup + steps, warmup + 2 * steps):
        step(j)
    torch.cuda.synchronize()
    prof = plan.profile_read()
    plan.profile_enable(False)
    # Distribution of single-step times: one event pair per step over K more steps.
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    ev[0].record()
    for i, j in enumerate(range(warmup + 2 * steps, warmup + 3 * steps)):
        step(j)
        ev[i + 1].record()
    torch.cuda.synchronize()
    per_step = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    losses = loss.cpu().numpy()
    return plan, R, elapsed, prof, losses, per_step


def time_streamed_kernel(wl, d, u, onset_t, idx_tab, lens, warmup, steps, dev):
    """Adam steps (fp32, stored spectra) with the kernel in pinned host memory: each
    batch's rows are copied to the device one batch ahead on a side stream and staged
    on the plan (MDD_FLAG_STREAM_KERNEL).  Returns ms per step and the host-to-device
    bytes per step."""
    import torch

    from paper_2202_04486_amd.plan import Plan
    from paper_2202_04486_amd.solver import StreamedKernel
    d_host = torch.empty(tuple(d.shape), dtype=torch.float32, pin_memory=True)
    d_host.copy_(d)
    plan = Plan(wl.ns, wl.nr, wl.nvs, wl.nt, wl.nf, wl.nb, store_rf=True, device=dev,
                stream_kernel=True)
    plan.mdd_set_data(u)
    plan.mdd_set_mask(onset_t)
    ks = StreamedKernel(plan, d_host)
    tab = idx_tab.cpu().numpy()
    bs = [tab[j, :lens[j]] for j in range(warmup + steps)]
    R = torch.zeros((wl.nr, wl.nvs, wl.nt), dtype=torch.float32, device=dev)
    m, v = torch.zeros_like(R), torch.zeros_like(R)

    def run(j0, j1):
        ks.prefetch(bs[j0])
        for j in range(j0, j1):
            ks.stage()
            if j + 1 < j1:
                ks.prefetch(bs[j + 1])
            plan.mdd_step(R, idx_tab[j, :lens[j]], opt="adam", lr=1e-2, s0=m, s1=v, t=j + 1)

    run(0, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(warmup, warmup + steps)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    h2d = float(np.mean([len(b) for b in bs[warmup:]])) * wl.nr * wl.nt * 4.0
    del plan, ks, d_host
    torch.cuda.empty_cache()
    return ms, h2d


def source_hash(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def stored_traffic(workload, key):
    """HBM bytes per launch of kernel `key` ("update", "gemm_fp32", "gemm_bf16x3", ...) from
    the committed counter summary of the workload, or None if it is missing or the kernel's
    source file changed since the counters were taken."""
    path = TRAFFIC_FILE.get(workload)
    if not path or not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.strip().startswith("- "):
            k, _, v = line.strip()[2:].partition(":")
            vals[k.strip()] = v.strip().strip("`")
    src = vals.get(f"{key}_source")
    if not src or vals.get(f"{key}_source_sha256") != source_hash(os.path.join(CSRC, src)):
        return None
    try:
        return float(vals[f"{key}_hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


# Virtual-source columns on which the oracle checks the GPU gradient.  Without the
# reciprocity preconditioner the columns of the gradient do not interact (each column of
# the per-frequency product depends only on the same column of the model and the data),
# so the oracle evaluated on a few columns gives exactly those columns of the gradient.
ERROR_COLUMNS = {"line2d": None, "patch3d": (0, 15, 16, 37, 799, 1203, 1584, 1599),
                 "line2d_vs1": None, "patch3d_vs1": None}   # None: every column
EPOCH_COLUMNS = {"line2d": (0, 16, 100, 200), "patch3d": (37, 1203),
                 "line2d_vs1": None, "patch3d_vs1": None}


def relerr(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def column_list(cols, nvs):
    return np.arange(nvs) if cols is None else np.asarray(cols, dtype=np.int64)


def oracle_gradient_columns(wl, d, u, onset, R_cols_host, idx, cols, reps=1):
    """The FP64 oracle's masked gradient of batch `idx` on virtual-source columns `cols`
    (model columns given on the host, float64), with the data columns repeated `reps`
    times along the column axis (several models' columns checked in one oracle call)."""
    import torch

    from oracle import freq, optim
    it = torch.as_tensor(np.asarray(idx, dtype=np.int64), device=d.device)
    ct = torch.as_tensor(cols, device=d.device)
    d_b = d.index_select(0, it).double().cpu().numpy()
    u_b = u.index_select(0, it).index_select(1, ct).double().cpu().numpy()
    on = onset[:, cols]
    if reps > 1:
        u_b = np.concatenate([u_b] * reps, axis=1)
        on = np.concatenate([on] * reps, axis=1)
    _, g = freq.batch_loss_grad(d_b, R_cols_host, u_b, np.arange(len(idx)), wl.nf)
    return optim.apply_mask(g, on)


def gradient_errors(wl, d, u, onset, R, grads, idx, cols):
    """Each form's gradient (batch idx, model R) against the oracle on columns `cols`."""
    import torch
    ct = torch.as_tensor(cols, device=R.device)
    go = oracle_gradient_columns(wl, d, u, onset, R.index_select(1, ct).double().cpu().numpy(),
                                 idx, cols)
    return {f: relerr(g.index_select(1, ct).double().cpu().numpy(), go) for f, g in grads.items()}


def error_per_epoch(wl, d, u, onset_t, onset, forms, epochs, cols, dev, lr=1e-2):
    """Each form's gradient error against the FP64 oracle at the end of each epoch of
    its own Adam run (untimed): the gradient on the next epoch's first batch at the
    form's current model, against the oracle's gradient at that same model, on the
    virtual-source columns `cols`.  The forms' model columns of one epoch are checked
    in one oracle call."""
    import torch

    import synth
    from paper_2202_04486_amd.plan import Plan
    from paper_2202_04486_amd.solver import batches
    perms = synth.epoch_permutations(wl, epochs + 1)
    ct = torch.as_tensor(cols, device=dev)
    snaps = {}
    for form in forms:
        log(f"error per epoch: {epochs} epochs of {form}")
        plan = Plan(wl.ns, wl.nr, wl.nvs, wl.nt, wl.nf, wl.nb, precision=form, store_rf=True,
                    device=dev)
        plan.mdd_set_kernel(d)
        plan.mdd_set_data(u)
        plan.mdd_set_mask(onset_t)
        R = torch.zeros((wl.nr, wl.nvs, wl.nt), dtype=torch.float32, device=dev)
        m, v = torch.zeros_like(R), torch.zeros_like(R)
        t, snaps[form] = 0, []
        for e in range(epochs):
            for b in batches(perms[e], wl.nb):
                t += 1
                plan.mdd_step(R, torch.as_tensor(b, dtype=torch.int32, device=dev), opt="adam",
                              lr=lr, s0=m, s1=v, t=t)
            b0 = np.sort(perms[e + 1][:wl.nb])
            g, _, _ = plan.mdd_stoch_grad(R, torch.as_tensor(b0, dtype=torch.int32, device=dev))
            snaps[form].append((R.index_select(1, ct).cpu().numpy(),
                                g.index_select(1, ct).cpu().numpy()))
            del g
        del plan, R, m, v
        torch.cuda.empty_cache()
    out = {f: [] for f in forms}
    scaled = {f: [] for f in forms}
    ratio = []
    k = len(cols)
    for e in range(epochs):
        b0 = np.sort(perms[e + 1][:wl.nb])
        # the forms' model columns, then zero columns: the gradient at R = 0 is -P_b^H u_b,
        # the data's own scale on this batch
        r_stack = np.concatenate([snaps[f][e][0] for f in forms] +
                                 [np.zeros_like(snaps[forms[0]][e][0])], axis=1).astype(np.float64)
        go = oracle_gradient_columns(wl, d, u, onset, r_stack, b0, cols, reps=len(forms) + 1)
        g0 = np.linalg.norm(go[:, len(forms) * k:])
        for i, f in enumerate(forms):
            gi = go[:, i * k:(i + 1) * k]
            err = np.linalg.norm(snaps[f][e][1] - gi)
            out[f].append(float(err / np.linalg.norm(gi)))
            scaled[f].append(float(err / g0))
        ratio.append(float(np.linalg.norm(go[:, :k]) / g0))
        if (e + 1) % 5 == 0 or e + 1 == epochs:
            log(f"error per epoch: oracle at epoch {e + 1} of {epochs}")
    return out, scaled, ratio


def host_cpu():
    """The host CPU as the kernel reports it: model name, vendor, family / model /
    stepping, and the logical CPUs this process may run on."""
    info = {}
    try:
        for line in open("/proc/cpuinfo"):
            k, _, v = line.partition(":")
            k = k.strip()
            if k in ("model name", "vendor_id", "cpu family", "model", "stepping") and k not in info:
                info[k] = v.strip()
    except OSError:
        pass
    name = info.get("model name", "")
    fam = " ".join(f"{k} {info[k]}" for k in ("cpu family", "model", "stepping") if k in info)
    desc = f"{name} ({info.get('vendor_id', '?')}, {fam})" if fam else name
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    return desc, ncpu


def oracle_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        return os.cpu_count() or 1


def cpu_baseline(wl, d, u, onset, budget_s=20.0):
    """The FP64 oracle, as it stands, timed on the host cores on a bounded sample
    of the same workload: Adam steps (oracle.freq gradient + oracle.optim.adam) on the
    first batches of the first epoch, at full size."""
    from oracle import freq, optim
    import synth
    cores = oracle_threads()
    d64 = d.double().cpu().numpy()
    u64 = u.double().cpu().numpy()
    bs = optim.batches(synth.epoch_permutations(wl, 1)[0], wl.nb)

    def run(limit):
        r = np.zeros((wl.nr, wl.nvs, wl.nt))
        m = np.zeros_like(r)
        v = np.zeros_like(r)
        n = 0
        t0 = time.perf_counter()
        while n < len(bs) and (time.perf_counter() - t0) < limit:
            _, g = freq.batch_loss_grad(d64, r, u64, bs[n], wl.nf)
            r, m, v = optim.adam(r, m, v, optim.apply_mask(g, onset), n + 1, 1e-2, onset=onset)
            n += 1
        return n, time.perf_counter() - t0

    n, el = run(budget_s)
    one = None
    try:  # the same sample on one core (BLAS and FFT threads limited to 1)
        from threadpoolctl import threadpool_limits
        with threadpool_limits(1):
            n1, el1 = run(budget_s)
        one = n1 / el1
    except ImportError:
        pass
    model, ncpu = host_cpu()
    return {"value": n / el, "unit": "grad evals/s", "cores": int(cores), "kind": "oracle",
            "one_core_value": one, "cpu_model": model, "host_logical_cpus": ncpu,
            "sample": f"{n} Adam steps (batches of {wl.nb}) of the first epoch of the "
                      f"{wl.ns}-trace line at full size, oracle.freq gradient + "
                      f"oracle.optim.adam in float64, {el:.1f} s"}


def cpu_baseline_columns(wl, d, u, onset, budget_s=20.0, ks=(8, 32), steps_per_k=2):
    """The FP64 oracle timed on the host cores on virtual-source columns of the full
    workload: Adam steps (oracle.freq gradient + oracle.optim.adam) of the first epoch's
    batches with the model restricted to k columns, for two column counts.  Without the
    reciprocity preconditioner the columns do not interact, so a step's cost is the
    batch's kernel transform (shared) plus a per-column part: the time per step is
    fitted as a + b k and evaluated at k = nvs, which gives the rate of a full step."""
    import torch

    import synth
    from oracle import freq, optim
    cores = oracle_threads()
    bs = optim.batches(synth.epoch_permutations(wl, 1)[0], wl.nb)[:steps_per_k]
    per_step = {}
    for k in ks:
        cols = np.unique(np.linspace(0, wl.nvs - 1, k).round().astype(np.int64))
        ct = torch.as_tensor(cols, device=d.device)
        host = []
        for b in bs:   # the batch's rows, on the host, outside the timed region
            it = torch.as_tensor(b.astype(np.int64), device=d.device)
            host.append((d.index_select(0, it).double().cpu().numpy(),
                         u.index_select(0, it).index_select(1, ct).double().cpu().numpy()))
        on = onset[:, cols]
        r = np.zeros((wl.nr, len(cols), wl.nt))
        m = np.zeros_like(r)
        v = np.zeros_like(r)
        t0 = time.perf_counter()
        for n, (d_b, u_b) in enumerate(host):
            _, g = freq.batch_loss_grad(d_b, r, u_b, np.arange(d_b.shape[0]), wl.nf)
            r, m, v = optim.adam(r, m, v, optim.apply_mask(g, on), n + 1, 1e-2, onset=on)
        per_step[len(cols)] = (time.perf_counter() - t0) / len(host)
        log(f"oracle on {len(cols)} columns: {per_step[len(cols)]:.2f} s per step")
        del host
        if sum(per_step.values()) * steps_per_k > budget_s:
            break
    (k1, t1), (k2, t2) = sorted(per_step.items())[0], sorted(per_step.items())[-1]
    slope = (t2 - t1) / (k2 - k1) if k2 > k1 else t1 / k1
    full = max(t1 - slope * k1, 0.0) + slope * wl.nvs
    model, ncpu = host_cpu()
    return {"value": 1.0 / full, "unit": "grad evals/s", "cores": int(cores), "kind": "oracle",
            "one_core_value": None, "cpu_model": model, "host_logical_cpus": ncpu,
            "seconds_per_step_measured": {str(k): t for k, t in per_step.items()},
            "seconds_per_full_step": full,
            "sample": f"{steps_per_k} Adam steps (first batches of {wl.nb} sources of the first "
                      f"epoch, full {wl.ns}-source kernel and {wl.nr} receivers) with the model "
                      f"restricted to {k1} and to {k2} of the {wl.nvs} virtual-source columns, "
                      "oracle.freq gradient + oracle.optim.adam in float64; the seconds per "
                      "step, fitted as a + b * columns (the columns do not interact without "
                      f"reciprocity; a is the batch's shared kernel transform), evaluated at "
                      f"{wl.nvs} columns give value"}


def practical_hbm_gbs(dev, mib=1024, reps=5, launches=10):
    """The streaming rate a plain elementwise kernel reaches on this device, in GB/s:
    torch's in-place multiply of a `mib` MiB float32 buffer (each launch reads it and
    writes it once), best of `reps` runs of `launches` launches.  Larger than the caches,
    so it measures HBM."""
    import torch
    a = torch.ones(mib * (1 << 20) // 4, dtype=torch.float32, device=dev)
    for _ in range(3):
        a.mul_(1.0)
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(launches):
            a.mul_(1.0)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / launches
        best = ms if best is None else min(best, ms)
    nbytes = 2.0 * a.numel() * 4
    del a
    return nbytes / (best * 1e-3) / 1e9


PRACTICAL_HOW = ("torch in-place multiply of a 1 GiB float32 buffer (read and written once per "
                 "launch), best of 5 x 10 launches, measured in this run")


def add_practical(roof, practical, ms):
    """The practical streaming rate beside the published peak, and the kernel's fraction of
    it by algorithmic bytes and, where the counters are current, by measured traffic."""
    roof["practical_peak"] = {"value": practical, "unit": "GB/s", "how": PRACTICAL_HOW}
    roof["frac_of_practical"] = roof["achieved"] / practical
    tr = roof.get("traffic")
    if tr:
        roof["traffic_gbs"] = tr / (ms * 1e-3) / 1e9
        roof["traffic_frac_of_practical"] = roof["traffic_gbs"] / practical


CALIBRATION_VARIANTS = {0: "the update kernel's grid and 8-byte per-lane accesses",
                        1: "the same grid with 16-byte per-lane accesses",
                        2: "flat streams over the arrays (two launches)"}


def best_launch_ms(call, reps=5, launches=4):
    """Best over `reps` runs of the milliseconds per launch of `launches` back-to-back calls,
    after two untimed calls."""
    import torch
    for _ in range(2):
        call()
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(launches):
            call()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / launches
        best = ms if best is None else min(best, ms)
    return best


def spectra_stream_floor(wl, dev):
    """Milliseconds per launch of the model spectra [nr][nvb][nf][16] complex read and
    written in place as one flat stream (mdd_calibrate_update, variant 3): the bytes the
    per-frequency products read as R_k and write as G, with no arithmetic."""
    import ctypes

    import torch

    from paper_2202_04486_amd import native
    lib = native.load()
    nvb = -(-wl.nvs // 16)
    S = torch.zeros((wl.nr, nvb, wl.nf, 16, 2), dtype=torch.float32, device=dev)
    one = torch.zeros(4, dtype=torch.float32, device=dev)   # the state arrays are not touched
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    ptrs = [ctypes.c_void_p(t.data_ptr()) for t in (one, one, one, S)]

    def call():
        native.check("mdd_calibrate_update",
                     lib.mdd_calibrate_update(*ptrs, wl.nr, wl.nvs, wl.nt, wl.nf, 3, st))
    ms = best_launch_ms(call)
    del S
    torch.cuda.empty_cache()
    return ms, 2 * 8.0 * wl.nr * nvb * 16 * wl.nf


def kernel_rows_floor(wl, dev, idx):
    """Milliseconds per launch of mdd_calibrate_rows: the batch's kernel rows (rows idx of
    D_k at every frequency, synthetic values) read with the one-virtual-source products'
    grid and none of their arithmetic, reductions or barriers."""
    import ctypes

    import torch

    from paper_2202_04486_amd import native
    lib = native.load()
    nrp = -(-wl.nr // 16) * 16
    nb = int(idx.numel())
    D = torch.zeros((wl.nf, wl.ns, nrp, 2), dtype=torch.float32, device=dev)
    out = torch.zeros((wl.nf, -(-nb // 8), nrp // 2, 4), dtype=torch.float32, device=dev)
    ix = idx.to(device=dev, dtype=torch.int32).contiguous()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def call():
        native.check("mdd_calibrate_rows",
                     lib.mdd_calibrate_rows(ctypes.c_void_p(D.data_ptr()), ctypes.c_void_p(ix.data_ptr()),
                                            ctypes.c_void_p(out.data_ptr()), nb, wl.nf, wl.ns, wl.nr, 0, st))
    ms = best_launch_ms(call)
    del D, out
    torch.cuda.empty_cache()
    return ms, 8.0 * nb * nrp * wl.nf


def update_traffic_floor(wl, dev, reps=5, launches=4):
    """Milliseconds per launch of each variant of mdd_calibrate_update at this workload's
    model size: the Adam update's HBM bytes (model and both moments in place, the
    spectra in place) without its transforms.  The best variant is the floor the
    memory system sets for the update kernel."""
    import ctypes

    import torch

    from paper_2202_04486_amd import native
    lib = native.load()
    nvb = -(-wl.nvs // 16)
    R = torch.zeros((wl.nr, wl.nvs, wl.nt), dtype=torch.float32, device=dev)
    M, V = torch.zeros_like(R), torch.zeros_like(R)
    S = torch.zeros((wl.nr, nvb, wl.nf, 16, 2), dtype=torch.float32, device=dev)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    ptrs = [ctypes.c_void_p(t.data_ptr()) for t in (R, M, V, S)]
    out = {}
    for var in CALIBRATION_VARIANTS:
        def call():
            native.check("mdd_calibrate_update",
                         lib.mdd_calibrate_update(*ptrs, wl.nr, wl.nvs, wl.nt, wl.nf, var, st))
        out[var] = best_launch_ms(call, reps, launches)
    del R, M, V, S
    torch.cuda.empty_cache()
    return out


def fp32_mfma_share(nb, nr, fused=True):
    """Executed MFMA flops of the float32 products over the algorithmic 8 flops per complex
    multiply-add: the persistent fused kernel (at most 16 batch rows, at most 224
    receivers) issues four real 16x16x4 products per complex one, the tiled and
    warp-specialised kernels three."""
    return 1.0 if fused and nb <= 16 and nr <= 224 else 0.75


def copy_calibration(mib, dev):
    """A plain device copy of `mib` MiB, whose HBM counters scale the kernels' counters."""
    import torch
    if not mib:
        return
    src = torch.ones(mib * (1 << 20) // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def bench_autograd(args, dev):
    """Differentiation form: one gradient of 1/2 ||P_b C_r z - u_b||^2 with respect to z
    through torch.autograd.  The operator P_b C_r is mdc_rec (C_r applied to the spectra
    inside mdc_forward_rec, and C_r P_b^H in mdc_adjoint_rec for the backward).  Timed per
    batch size; kernel times from the plan's HIP events over separate evaluations; at the
    largest batch also mdc(reciprocity(z)), C_r as its own kernel on the traces, which is
    timed on its own as well."""
    import torch

    import synth
    from paper_2202_04486_amd.autograd import _reciprocity, mdc, mdc_rec, reciprocity
    from paper_2202_04486_amd.plan import Plan
    wl = synth.WORKLOADS["diff301"]
    log("generating inputs")
    d, r_true, noise, _ = make_inputs(wl, dev)
    plan = Plan(wl.ns, wl.nr, wl.nvs, wl.nt, wl.nf, max(wl.nb_sweep), device=dev)
    plan.mdd_set_kernel(d)
    u = up_going(plan, r_true, noise, wl, dev)
    del r_true, noise
    gen = torch.Generator(device=dev)
    gen.manual_seed(wl.seed)
    z = torch.randn((wl.nr, wl.nvs, wl.nt), generator=gen, device=dev).requires_grad_(True)
    copy_calibration(args.copy_calibration_mib, dev)
    K = args.steps or 20
    W = args.warmup if args.warmup is not None else 3
    by_batch = {}
    for nb in wl.nb_sweep:
        idx_tab, lens, _ = step_tables(wl, nb, W + 2 * K, dev)

        def ev(j, fused=True):
            idx = idx_tab[j, :lens[j]]
            pred = mdc_rec(z, idx, plan) if fused else mdc(reciprocity(z), idx, plan)
            loss = 0.5 * ((pred - u.index_select(0, idx.long())) ** 2).sum()
            return torch.autograd.grad(loss, z)[0]

        for j in range(W):
            ev(j)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for j in range(W, W + K):
            ev(j)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        plan.profile_enable(True, capacity=16 * K + 64)
        for j in range(W + K, W + 2 * K):
            ev(j)
        torch.cuda.synchronize()
        prof = plan.profile_read()
        plan.profile_enable(False)
        gemm_ms = prof["gemm"][0] / K          # forward and adjoint product launches per evaluation
        flops = 16.0 * nb * wl.nr * wl.nvs * wl.nf
        by_batch[nb] = {"value": K / el, "ms_per_eval": 1e3 * el / K,
                        "kernel_ms_per_eval": {k: v[0] / K for k, v in prof.items() if v[1]},
                        "products_tflops": flops / (gemm_ms * 1e-3) / 1e12,
                        "products_mfma_frac": flops / (gemm_ms * 1e-3) / 1e12 / MFMA_PEAK_TFLOPS["fp32"]}
        if nb == max(wl.nb_sweep):   # the same evaluations with C_r as a kernel on the traces
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for j in range(W, W + K):
                ev(j, fused=False)
            torch.cuda.synchronize()
            by_batch[nb]["unfused_ms_per_eval"] = 1e3 * (time.perf_counter() - t0) / K
            by_batch[nb]["unfused_note"] = "mdc(reciprocity(z)): mdd_reciprocity on the traces"
    # the reciprocity kernel alone: z read once, the result written once
    zz = z.detach()
    for _ in range(3):
        _reciprocity(zz)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        _reciprocity(zz)
    e1.record()
    torch.cuda.synchronize()
    rec_ms = e0.elapsed_time(e1) / 20
    rec_bytes = 8.0 * wl.nr * wl.nvs * wl.nt
    rec = {"ms": rec_ms, "algorithmic_bytes": rec_bytes,
           "traffic": stored_traffic("diff301", "reciprocity"),
           "achieved": rec_bytes / (rec_ms * 1e-3) / 1e9, "unit": "GB/s", "peak": HBM_PEAK_GBS,
           "frac": rec_bytes / (rec_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    add_practical(rec, practical_hbm_gbs(dev), rec_ms)
    # C_r on the spectra alone (the model spectra of one mdc_forward_rec), by the plan's events
    plan.profile_enable(True, capacity=64)
    idx_last = idx_tab[0, :lens[0]]
    for _ in range(10):
        plan.mdc_forward_rec(zz, idx_last)
    srec = plan.profile_read()["reciprocity"]
    plan.profile_enable(False)
    srec_ms = srec[0] / max(srec[1], 1)
    srec_bytes = 2 * 8.0 * wl.nr * wl.nvs * wl.nf
    rec["spectral"] = {"ms": srec_ms, "algorithmic_bytes": srec_bytes,
                       "traffic": stored_traffic("diff301", "spec_reciprocity"),
                       "achieved": srec_bytes / (srec_ms * 1e-3) / 1e9, "unit": "GB/s",
                       "frac": srec_bytes / (srec_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                       "note": "C_r on the nr x nvs x nf retained spectra, read and written once"}
    top = by_batch[max(wl.nb_sweep)]
    out = {
        "metric": METRIC, "value": top["value"], "unit": "grad evals/s", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": top["ms_per_eval"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": AUTOGRAD_TEXT, "global_batch": max(wl.nb_sweep), "seq_len": wl.nt,
                   "parallelism": "none (1 GPU)"},
        "workload": "diff301",
        "roofline": {"kernel": "products (forward and adjoint launches) at the largest batch",
                     "bound": "mfma", "achieved": top["products_tflops"],
                     "peak": MFMA_PEAK_TFLOPS["fp32"], "unit": "TFLOP/s",
                     "frac": top["products_mfma_frac"],
                     "traffic": stored_traffic("diff301", "products"),
                     "traffic_unit": "HBM bytes per evaluation (counters, both launches)",
                     "algorithmic_flops": 16.0 * max(wl.nb_sweep) * wl.nr * wl.nvs * wl.nf,
                     "executed_mfma_flops": 16.0 * max(wl.nb_sweep) * wl.nr * wl.nvs * wl.nf *
                     fp32_mfma_share(max(wl.nb_sweep), wl.nr, fused=False)},
        "reciprocity": rec,
        "by_batch": by_batch,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 1 epoch of patch3d, 10 epochs of line2d)")
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="patch3d", choices=list(WORKLOAD_TEXT) + ["diff301"],
                    help="patch3d (default: the 1600-trace 3D patch), the 201-trace 2D line, "
                         "either with a single virtual source, or the differentiation form")
    ap.add_argument("--forms", default=None,
                    help="precision forms to time (default: fp32,bf16x3,fp16x3 and bf16, the "
                         "single-pass diagnostic; at the 3D patch also fp32_cgemm, the float32 "
                         "products with four real products per complex one)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--stream-kernel", action="store_true",
                    help="also time the steps with the kernel streamed from pinned host memory")
    ap.add_argument("--no-full-gradient", action="store_true",
                    help="skip timing the full-gradient iteration (every source per update)")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--error-epochs", type=int, default=None,
                    help="epochs of each form's untimed run whose ends are checked against the "
                         "oracle on sampled columns (with the CPU-baseline leg; default: the "
                         "workload's run length, 20 epochs at the 3D patch, 50 at the 2D line)")
    ap.add_argument("--no-store-rf", action="store_true",
                    help="recompute the model spectra at each step instead of storing them")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one plain device copy of this size first (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    if args.workload == "diff301":
        bench_autograd(args, torch.device("cuda", 0))
        return
    wl = synth.WORKLOADS[args.workload]
    spe0 = math.ceil(wl.ns / wl.nb)
    if args.steps is None:
        args.steps = DEFAULT_EPOCHS[args.workload] * spe0
    if args.warmup is None:
        args.warmup = spe0 if wl.grid == "line" else 5
    if args.workload not in ("line2d", "patch3d"):
        args.no_cpu_baseline = True
    if args.error_epochs is None:
        args.error_epochs = wl.epochs
    dev = torch.device("cuda", 0)
    log("generating inputs")
    d, r_true, noise, onset = make_inputs(wl, dev)
    onset_t = torch.from_numpy(onset).to(dev)
    from paper_2202_04486_amd.plan import Plan
    p0 = Plan(wl.ns, wl.nr, wl.nvs, wl.nt, wl.nf, wl.nb, device=dev)
    p0.mdd_set_kernel(d)
    u = up_going(p0, r_true, noise, wl, dev)
    del p0, r_true, noise
    torch.cuda.empty_cache()
    idx_tab, lens, spe = step_tables(wl, wl.nb, args.warmup + 3 * args.steps, dev)
    torch.cuda.synchronize()
    copy_calibration(args.copy_calibration_mib, dev)

    if args.forms is None:
        args.forms = ("fp32,fp32_cgemm,bf16x3,fp16x3,bf16" if args.workload == "patch3d" else
                      "fp32,bf16x3,fp16x3,bf16" if args.workload == "line2d" else "fp32,bf16x3,fp16x3")
    forms = [f for f in args.forms.split(",") if f]
    if "fp32" not in forms:
        forms.insert(0, "fp32")
    vs1 = wl.nvs == 1
    if vs1:
        forms = ["fp32"]  # one virtual source: every precision setting runs the float32 kernel
    res, grads = {}, {}
    idx0 = idx_tab[0, :lens[0]]
    R_eval = None
    for form in forms:
        log(f"timing {form}")
        plan, R, el, prof, losses, per_step = run_form(form, wl, d, u, onset_t, idx_tab, lens,
                                             args.warmup, args.steps, dev,
                                             store_rf=not args.no_store_rf)
        if R_eval is None:
            R_eval = R.clone()
        g, _, _ = plan.mdd_stoch_grad(R_eval, idx0)
        grads[form] = g
        res[form] = {"elapsed": el, "prof": prof, "loss_first": float(losses[0]),
                     "loss_last": float(losses[-1]), "per_step": per_step}
        del plan
        torch.cuda.synchronize()

    K = args.steps
    fp = res["fp32"]
    value = K / fp["elapsed"]
    ms_step = 1e3 * fp["elapsed"] / K
    Mt = wl.nr * wl.nvs * wl.nt
    nb = wl.nb

    def per_launch(prof, name):
        ms, cnt = prof[name]
        return (ms / cnt) if cnt else 0.0

    cls_ms = {k: per_launch(fp["prof"], k) for k in fp["prof"]}
    dominant = max(cls_ms, key=lambda k: cls_ms[k] * fp["prof"][k][1])
    upd_ms = cls_ms["update"]
    upd_bytes = 8.0 * STATE_ARRAYS[wl.optimizer] * Mt   # R and its state, read and written
    traffic = stored_traffic(args.workload, "update")
    gemm_flops = 16.0 * nb * wl.nr * wl.nvs * wl.nf
    # One virtual source: D_b read once, U_b, the model spectra in and the gradient out.
    gemv_bytes = 8.0 * nb * wl.nr * wl.nf + 8.0 * nb * wl.nf + 2 * 8.0 * wl.nr * wl.nf
    if dominant == "gemm" and vs1:
        gm_ms = roof_ms = cls_ms["gemm"]
        roofline = {"kernel": "gemv (one pass over D_b: forward product + residual + loss + "
                              "adjoint product)", "bound": "hbm",
                    "achieved": gemv_bytes / (gm_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "traffic": stored_traffic(args.workload, "gemv"),
                    "traffic_unit": "HBM bytes per launch (counters)",
                    "algorithmic_bytes": gemv_bytes}
    elif dominant == "gemm":
        gm_ms = roof_ms = cls_ms["gemm"]
        roofline = {"kernel": "gemm (forward product + residual + loss + adjoint product)",
                    "bound": "mfma", "achieved": gemm_flops / (gm_ms * 1e-3) / 1e12,
                    "peak": MFMA_PEAK_TFLOPS["fp32"], "unit": "TFLOP/s",
                    "traffic": stored_traffic(args.workload, "gemm_fp32"),
                    "traffic_unit": "HBM bytes per launch (counters)",
                    "algorithmic_flops": gemm_flops,
                    "executed_mfma_flops": gemm_flops * fp32_mfma_share(nb, wl.nr)}
    else:
        roof_ms = upd_ms
        roofline = {"kernel": f"update (inverse FFT + mask + {wl.optimizer} + model FFT)",
                    "bound": "hbm",
                    "achieved": upd_bytes / (upd_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "traffic": traffic,
                    "traffic_unit": "HBM bytes per launch (counters)",
                    "algorithmic_bytes": upd_bytes}
    roofline["frac"] = roofline["achieved"] / roofline["peak"]
    if roofline["bound"] == "hbm":
        add_practical(roofline, practical_hbm_gbs(dev), roof_ms)
    if dominant == "gemm" and vs1:
        # The floor of the products' access pattern: the batch's kernel rows read with the
        # same grid and no arithmetic (mdd_calibrate_rows).
        log("timing the kernel-row stream of the matrix-vector products")
        rows_ms, rows_bytes = kernel_rows_floor(wl, dev, idx_tab[0, :lens[0]])
        roofline["elementwise_peak"] = roofline.pop("practical_peak")
        roofline.pop("frac_of_practical", None)
        roofline.pop("traffic_frac_of_practical", None)
        roofline["practical_peak"] = {
            "value": rows_bytes / (rows_ms * 1e-3) / 1e9, "unit": "GB/s",
            "how": "mdd_calibrate_rows: the batch's kernel rows (D_b at every frequency) read "
                   "with the matrix-vector kernel's grid and none of its arithmetic, reductions "
                   "or barriers, one partial per group written; the kernel's time includes the "
                   "launch that adds the group partials",
            "floor_ms": rows_ms, "bytes_per_launch": rows_bytes}
        roofline["frac_of_practical"] = rows_ms / roof_ms
        roofline["frac_ceiling_at_practical"] = gemv_bytes / (rows_ms * 1e-3) / 1e9 / HBM_PEAK_GBS
    if dominant == "update" and wl.optimizer == "adam" and not vs1:
        # The floor of the update kernel's own traffic: its bytes moved by a kernel with
        # the same accesses and no arithmetic (mdd_calibrate_update), best of three layouts.
        log("timing the update's traffic without its transforms")
        floor = update_traffic_floor(wl, dev)
        best = min(floor, key=floor.get)
        nvb = -(-wl.nvs // 16)
        counted = upd_bytes + 2 * 8.0 * wl.nr * nvb * 16 * wl.nf   # + spectra in and out
        roofline["elementwise_peak"] = roofline.pop("practical_peak")
        roofline.pop("frac_of_practical", None)
        roofline.pop("traffic_frac_of_practical", None)
        roofline["practical_peak"] = {
            "value": counted / (floor[best] * 1e-3) / 1e9, "unit": "GB/s",
            "how": "mdd_calibrate_update: the update launch's bytes (model and Adam moments read "
                   "and written in place, the gradient spectra read and the next model's "
                   "spectra written in place) without the transforms; best of "
                   f"{len(floor)} layouts: {CALIBRATION_VARIANTS[best]}",
            "floor_ms": floor[best],
            "variants_ms": {CALIBRATION_VARIANTS[k]: v for k, v in floor.items()},
            "bytes_per_launch": counted}
        roofline["frac_of_practical"] = floor[best] / roof_ms
        roofline["frac_ceiling_at_practical"] = upd_bytes / (floor[best] * 1e-3) / 1e9 / HBM_PEAK_GBS

    products_floor = None
    if not vs1:
        # The products move R_k in, G out, D_b and U_b: the spectra part streamed flat with
        # no arithmetic, scaled to all of the products' bytes, is the floor of their traffic.
        log("timing the spectra stream")
        st_ms, st_bytes = spectra_stream_floor(wl, dev)
        nvb = -(-wl.nvs // 16)
        pr_bytes = st_bytes + 8.0 * nb * wl.nr * wl.nf + 8.0 * nb * nvb * 16 * wl.nf
        products_floor = {"spectra_stream_ms": st_ms, "spectra_bytes": st_bytes,
                          "spectra_gbs": st_bytes / (st_ms * 1e-3) / 1e9,
                          "products_bytes": pr_bytes, "floor_ms": st_ms * pr_bytes / st_bytes,
                          "how": "mdd_calibrate_update variant 3: the model spectra read and "
                                 "written in place as one flat stream; floor_ms scales it to "
                                 "the products' bytes (R_k in, G out, D_b and U_b in)"}

    def gemm_roof(form):
        ms = per_launch(res[form]["prof"], "gemm")
        if vs1:
            tr = stored_traffic(args.workload, "gemv")
            return {"ms": ms, "bound": "hbm", "algorithmic_bytes": gemv_bytes,
                    "achieved_gbs": gemv_bytes / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                    "frac": gemv_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                    "useful_tflops": gemm_flops / (ms * 1e-3) / 1e12,
                    "traffic": tr, "hbm_gbs": (tr / (ms * 1e-3) / 1e9) if tr else None}
        # The work counted against the dtype's peak: the method's complex products for
        # float32; for the split forms each of the three hi/lo products is required work.
        split = form in ("bf16x3", "fp16x3")
        counted = gemm_flops * (3 if split else 1)
        hw = gemm_flops * (3 if split else 1 if form == "fp32_cgemm" else
                           fp32_mfma_share(nb, wl.nr))                 # what the MFMA units execute
        tr = stored_traffic(args.workload, f"gemm_{form}")
        hbm = {}
        if products_floor:
            hbm = {"hbm_bytes_frac": products_floor["products_bytes"] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                   "frac_of_traffic_floor": products_floor["floor_ms"] / ms}
        return {"ms": ms, "useful_tflops": gemm_flops / (ms * 1e-3) / 1e12, **hbm,
                "counted_tflops": counted / (ms * 1e-3) / 1e12, "peak": MFMA_PEAK_TFLOPS[form],
                "frac": counted / (ms * 1e-3) / 1e12 / MFMA_PEAK_TFLOPS[form],
                "mfma_tflops": hw / (ms * 1e-3) / 1e12,
                "mfma_frac": hw / (ms * 1e-3) / 1e12 / MFMA_PEAK_TFLOPS[form],
                "traffic": tr, "hbm_gbs": (tr / (ms * 1e-3) / 1e9) if tr else None}

    alg_bytes = upd_bytes + (1 if vs1 else 2) * 8.0 * nb * wl.nr * wl.nf + 8.0 * nb * wl.nvs * wl.nf
    out = {
        "metric": METRIC, "value": value, "unit": "grad evals/s", "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[args.workload],
                   "global_batch": nb, "seq_len": wl.nt, "parallelism": "none (1 GPU)"},
        "epoch_ms": ms_step * spe,
        "steps_per_epoch": spe,
        "kernel_ms": cls_ms,
        "kernel_ms_source": "HIP events on the plan's stream around every launch, over K steps "
                            "run right after the K timed ones (the event records add a few us "
                            "between kernels, so value is timed without them)",
        "dominant_kernel": dominant,
        "workload": args.workload,
        "roofline": roofline,
        "method_roofline_frac": (alg_bytes / HBM_PEAK_GBS / 1e9) / (ms_step * 1e-3),
        "gemm_roofline": {f: gemm_roof(f) for f in forms},
        "products_traffic_floor": products_floor,
        "step_ms_quantiles": {q: float(np.percentile(fp["per_step"], v))
                              for q, v in (("p10", 10), ("median", 50), ("p90", 90))},
        "step_ms_quantiles_source": "one HIP event pair per step over K further steps",
        "forms": {f: {"value": K / res[f]["elapsed"], "ms_per_step": 1e3 * res[f]["elapsed"] / K,
                      "speedup_vs_fp32": fp["elapsed"] / res[f]["elapsed"],
                      "gemm_speedup_vs_fp32": per_launch(fp["prof"], "gemm") /
                      max(per_launch(res[f]["prof"], "gemm"), 1e-12)} for f in forms},
    }
    if "bf16" in res:
        out["forms"]["bf16"]["note"] = ("single bf16 product per complex one (no lo halves): a "
                                        "diagnostic, expected to miss the 1e-3 bound")
    if "fp32_cgemm" in res:   # the precision forms against the plain complex-GEMM float32 form
        cg = res["fp32_cgemm"]
        for f in forms:
            out["forms"][f]["speedup_vs_fp32_cgemm"] = cg["elapsed"] / res[f]["elapsed"]
            out["forms"][f]["gemm_speedup_vs_fp32_cgemm"] = (
                per_launch(cg["prof"], "gemm") / max(per_launch(res[f]["prof"], "gemm"), 1e-12))
    if not args.no_full_gradient:
        log("timing full-gradient iterations")
        it_ms = time_full_gradient(wl, d, u, onset_t, dev, iters=5 if args.workload == "line2d" else 2)
        out["full_gradient"] = {"iteration_ms": it_ms, "stochastic_epoch_ms": ms_step * spe,
                                "epoch_over_iteration": ms_step * spe / it_ms,
                                "note": "one full-gradient SGD (Landweber) iteration over all "
                                        f"{wl.ns} sources in batches of {wl.nb}, fp32"}
    if args.stream_kernel:
        log("timing steps with the kernel streamed from host memory")
        s_ms, h2d = time_streamed_kernel(wl, d, u, onset_t, idx_tab, lens, args.warmup, K, dev)
        out["streamed_kernel"] = {
            "ms_per_step": s_ms, "value": 1e3 / s_ms, "unit": "grad evals/s",
            "resident_ms_per_step": ms_step, "h2d_bytes_per_step": h2d,
            "h2d_gbs_needed": h2d / (s_ms * 1e-3) / 1e9,
            "note": "fp32 Adam steps; the batch's kernel rows copied from pinned host memory "
                    "one batch ahead on a side stream, then transformed on the device"}
    if "bf16x3" in res:   # the precision form against the shipped float32 form
        pf = out["forms"]["bf16x3"]
        out["precision_form"] = {
            "form": "bf16x3", "value": pf["value"], "unit": "grad evals/s",
            "speedup_vs_fp32": pf["speedup_vs_fp32"],
            "products_speedup_vs_fp32": pf["gemm_speedup_vs_fp32"],
            "speedup_vs_fp32_cgemm": pf.get("speedup_vs_fp32_cgemm"),
            "products_speedup_vs_fp32_cgemm": pf.get("gemm_speedup_vs_fp32_cgemm"),
            "target": ">= 2x the plain fp32 form at gradient rel. err <= 1e-3",
            "note": "fp32 is the float32 form the library ships (three real products per complex "
                    "multiply-add in the tiled and warp-specialised kernels); fp32_cgemm (four) is "
                    "a secondary comparison.  The update kernel (inverse transform, mask, Adam, "
                    "next model's transform) is the same in every form and HBM-bound, so the "
                    "whole-step ratio stays far below the products' ratio under Adam"}
    if not args.no_cpu_baseline:
        log("timing the oracle on the host")
        if args.workload == "patch3d":
            out["cpu_baseline"] = cpu_baseline_columns(wl, d, u, onset, args.cpu_budget)
        else:
            out["cpu_baseline"] = cpu_baseline(wl, d, u, onset, args.cpu_budget)
        cols = column_list(ERROR_COLUMNS[args.workload], wl.nvs)
        log(f"gradient error against the oracle on {len(cols)} columns")
        errs = gradient_errors(wl, d, u, onset, R_eval, grads, idx0.cpu().numpy(), cols)
        for f in forms:
            out["forms"][f]["grad_rel_err_vs_fp64_oracle"] = errs[f]
        out["grad_error_columns"] = ("all" if ERROR_COLUMNS[args.workload] is None else
                                     [int(c) for c in cols])
        out["grad_error_note"] = ("gradient of the first batch at the fp32 form's model after the "
                                  "timed steps, every form at that same model, against the FP64 "
                                  "oracle on these virtual-source columns (relative 2-norm)")
        if args.error_epochs > 0:
            ecols = column_list(EPOCH_COLUMNS[args.workload], wl.nvs)
            eforms = [f for f in forms if f != "fp32_cgemm"]
            per_epoch, scaled, ratio = error_per_epoch(wl, d, u, onset_t, onset, eforms,
                                                       args.error_epochs, ecols, dev)
            for f in eforms:
                out["forms"][f]["grad_rel_err_per_epoch"] = per_epoch[f]
                out["forms"][f]["grad_err_over_zero_model_grad_per_epoch"] = scaled[f]
                out["forms"][f]["grad_rel_err_max_over_epochs"] = max(per_epoch[f])
                out["forms"][f]["grad_rel_err_bound"] = (1e-5 if f.startswith("fp32") else
                                                         None if f == "bf16" else 1e-3)
            out["grad_error_per_epoch_columns"] = ("all" if EPOCH_COLUMNS[args.workload] is None
                                                   else [int(c) for c in ecols])
            out["grad_norm_over_zero_model_grad_per_epoch"] = ratio
            out["grad_error_per_epoch_note"] = (
                f"each form's own Adam run (lr 1e-2) over {args.error_epochs} epochs; at the end "
                "of each epoch its gradient on the next epoch's first batch at its current model, "
                "against the FP64 oracle at that model on these virtual-source columns.  "
                "grad_err_over_zero_model_grad divides the same error by the norm of the batch's "
                "gradient at R = 0 (P_b^H u_b, the data's scale), and "
                "grad_norm_over_zero_model_grad is the fp32 model's gradient norm on that scale: "
                "as the model fits the data the gradient shrinks while the rounding error of "
                "forming D_b R_k - U_b stays at the data's scale, so the relative error grows "
                "by the inverse of that ratio")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
