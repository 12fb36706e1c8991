"""Host side of stochastic MDD: the batch schedule and the epoch loop.

An epoch visits every source once: the epoch's random source permutation is
cut into ceil(ns / nb) consecutive batches (the last one partial), each sorted
(Theory section: sources grouped in batches, an epoch uses all of them;
Examples: floor(201/32)+1 = 7 steps).  Each step is one `mdd_step` of the
library; the whole epoch's batch indices go to the device in one copy and the
per-step losses stay on the device until the epoch ends (one host sync per
epoch).  The step size can be set from the largest singular value of the
kernel (Appendix B): alpha = kappa * 2 / sigma_max^2, kappa = 0.4..0.6.

FullGradientMDD is the full-gradient baseline (every source per iteration, e.g. the
Landweber iteration) on the same kernels.

StreamedKernel keeps the kernel d in pinned host memory for plans made with
stream_kernel=True (a kernel larger than the device memory, Examples: 3D): each
batch's rows are copied to the device on a side stream one batch ahead and
staged on the plan (mdd_stage_kernel) just before the step that uses them.

Checkpoint / resume: `state_dict` captures the model, optimiser state, step
counter, epoch / batch cursor and the permutation in use, so an interrupted
epoch resumes on exactly the same batches.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from .plan import Plan


class Diverged(RuntimeError):
    """The loss became non-finite or grew by more than `blowup` over its first value."""


def check_divergence(losses, loss0: float, blowup: float = 1e6) -> None:
    """Raise Diverged if any loss is non-finite or exceeds blowup * loss0 (the
    step size is above the stable range, e.g. beyond the Landweber limit)."""
    losses = np.asarray(losses, dtype=np.float64)
    if losses.size == 0:
        return
    if not np.all(np.isfinite(losses)) or float(np.max(losses)) > blowup * loss0:
        raise Diverged(f"loss {float(np.max(losses)):.3e} vs first {loss0:.3e}")


def batches(perm, nb: int):
    """ceil(ns / nb) consecutive slices of the permutation, each sorted (int32)."""
    perm = np.asarray(perm)
    n = math.ceil(len(perm) / nb)
    return [np.sort(perm[j * nb:(j + 1) * nb]).astype(np.int32) for j in range(n)]


def epoch_index_table(perm, nb: int):
    """All batches of one epoch as an int32 [n_batches, nb] table (rows padded) plus
    the length of each row."""
    bs = batches(perm, nb)
    tab = np.zeros((len(bs), nb), dtype=np.int32)
    lens = np.array([len(b) for b in bs], dtype=np.int64)
    for j, b in enumerate(bs):
        tab[j, :len(b)] = b
    return tab, lens


class StochasticMDD:
    """Stochastic gradient solver over a `Plan` whose kernel and data are set."""

    def __init__(self, plan: Plan, optimizer: str = "adam", lr: float = 1e-2, nb: int | None = None,
                 beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, mu: float = 0.9,
                 R0: torch.Tensor | None = None, blowup: float = 1e6):
        self.plan = plan
        self.opt = optimizer
        self.lr = float(lr)
        self.nb = nb or plan.nb_max
        self.beta1, self.beta2, self.eps, self.mu = beta1, beta2, eps, mu
        shape = (plan.nr, plan.nvs, plan.nt)
        dev = plan.device
        self.R = R0.clone() if R0 is not None else torch.zeros(shape, dtype=torch.float32, device=dev)
        self.s0 = torch.zeros(shape, dtype=torch.float32, device=dev) if optimizer != "sgd" else None
        self.s1 = torch.zeros(shape, dtype=torch.float32, device=dev) if optimizer == "adam" else None
        self.t = 0
        self.epoch = 0
        self.cursor = 0
        self.perm = None
        self.blowup = blowup
        self.loss0 = None
        self.history = []

    def step_size_from_kernel(self, kappa: float = 0.5, iters: int = 100) -> float:
        lam = self.plan.mdd_sigma_max2(iters=iters)
        s2 = float(lam.max().item())
        self.lr = kappa * 2.0 / s2
        return self.lr

    def run_epoch(self, perm, max_steps: int | None = None):
        """Run (the rest of) one epoch over `perm`; returns the per-step losses."""
        if self.perm is None or self.cursor == 0:
            self.perm = np.asarray(perm)
        tab, lens = epoch_index_table(self.perm, self.nb)
        dev = self.plan.device
        idx = torch.from_numpy(tab).to(dev)
        losses = torch.zeros(len(lens), dtype=torch.float64, device=dev)
        gnorm = torch.zeros(len(lens), dtype=torch.float64, device=dev)
        stop = len(lens) if max_steps is None else min(len(lens), self.cursor + max_steps)
        first = self.cursor
        for j in range(self.cursor, stop):
            self.t += 1
            self.plan.mdd_step(self.R, idx[j, :lens[j]], opt=self.opt, lr=self.lr, s0=self.s0,
                               s1=self.s1, t=self.t, beta1=self.beta1, beta2=self.beta2,
                               eps=self.eps, mu=self.mu, loss_out=losses[j:j + 1],
                               gnorm2_out=gnorm[j:j + 1])
        self.cursor = stop
        out = losses[first:stop].cpu().numpy()
        if self.cursor == len(lens):
            self.cursor = 0
            self.epoch += 1
            self.perm = None
        self._check(out)
        self.history.extend(out.tolist())
        return out

    def _check(self, losses):
        if len(losses) == 0:
            return
        if self.loss0 is None:
            self.loss0 = float(losses[0])
        check_divergence(losses, self.loss0, self.blowup)

    def state_dict(self):
        st = {"R": self.R.cpu().numpy(), "t": self.t, "epoch": self.epoch, "cursor": self.cursor,
              "perm": np.asarray(self.perm if self.perm is not None else [], dtype=np.int64),
              "lr": self.lr}
        if self.s0 is not None:
            st["s0"] = self.s0.cpu().numpy()
        if self.s1 is not None:
            st["s1"] = self.s1.cpu().numpy()
        return st

    def load_state_dict(self, st):
        dev = self.plan.device
        self.R.copy_(torch.from_numpy(np.asarray(st["R"])).to(dev))
        if self.s0 is not None:
            self.s0.copy_(torch.from_numpy(np.asarray(st["s0"])).to(dev))
        if self.s1 is not None:
            self.s1.copy_(torch.from_numpy(np.asarray(st["s1"])).to(dev))
        self.t = int(st["t"])
        self.epoch = int(st["epoch"])
        self.cursor = int(st["cursor"])
        perm = np.asarray(st["perm"])
        self.perm = perm if perm.size else None
        self.lr = float(st["lr"])
        self.plan.mdd_invalidate_model_spectra()

    def save(self, path):
        np.savez(path, **self.state_dict())

    def load(self, path):
        with np.load(path, allow_pickle=False) as z:
            self.load_state_dict({k: z[k] for k in z.files})


class FullGradientMDD:
    """Full-gradient baseline the paper compares stochastic epochs with: every iteration
    uses all sources (Theory section, the finite-sum functional; Appendix A, one full
    iteration against one epoch).  With optimizer 'sgd' and lr = kappa * 2 / sigma_max^2
    this is the Landweber iteration (Appendix B).  Needs a plan made with full_grad=True."""

    def __init__(self, plan: Plan, optimizer: str = "sgd", lr: float | None = None,
                 kappa: float = 0.5, mu: float = 0.9, R0: torch.Tensor | None = None,
                 blowup: float = 1e6):
        self.plan = plan
        self.opt = optimizer
        self.mu = mu
        shape = (plan.nr, plan.nvs, plan.nt)
        dev = plan.device
        self.R = R0.clone() if R0 is not None else torch.zeros(shape, dtype=torch.float32, device=dev)
        self.s0 = torch.zeros(shape, dtype=torch.float32, device=dev) if optimizer != "sgd" else None
        self.s1 = torch.zeros(shape, dtype=torch.float32, device=dev) if optimizer == "adam" else None
        if lr is None:
            lam = plan.mdd_sigma_max2(iters=100)
            lr = kappa * 2.0 / float(lam.max().item())
        self.lr = float(lr)
        self.t = 0
        self.blowup = blowup
        self.loss0 = None
        self.history = []

    def run(self, iters: int):
        """`iters` full iterations; returns their losses (taken before each update)."""
        dev = self.plan.device
        losses = torch.zeros(iters, dtype=torch.float64, device=dev)
        for i in range(iters):
            self.t += 1
            self.plan.mdd_full_step(self.R, opt=self.opt, lr=self.lr, s0=self.s0, s1=self.s1,
                                    t=self.t, mu=self.mu, loss_out=losses[i:i + 1])
        out = losses.cpu().numpy()
        if len(out):
            if self.loss0 is None:
                self.loss0 = float(out[0])
            check_divergence(out, self.loss0, self.blowup)
        self.history.extend(out.tolist())
        return out


class StreamedKernel:
    """The kernel d [ns][nr][nt] float32 (and, for a plan made with stream_data=True, the
    up-going data u [ns][nvs][nt]) in pinned host memory, streamed a batch at a time to a
    plan made with stream_kernel=True.

    prefetch(idx) starts copying the rows idx[b] into one of two device buffers on a
    side stream (default priority); stage() makes the caller's current stream wait for
    that copy and stages the rows on the plan, so the next mdd_step / mdd_stoch_grad on
    this batch reads them.  A buffer is refilled only after the stream that staged it
    has passed the staging (an event), so the copy of batch j + 1 overlaps step j."""

    def __init__(self, plan: Plan, d_host: torch.Tensor, u_host: torch.Tensor | None = None):
        if not plan.stream_kernel:
            raise ValueError("StreamedKernel needs a plan made with stream_kernel=True")
        if plan.stream_data and u_host is None:
            raise ValueError("a plan made with stream_data=True needs u_host")
        if u_host is not None and not plan.stream_data:
            raise ValueError("u_host needs a plan made with stream_data=True")
        self.plan = plan
        self.d = self._pinned(d_host, (plan.ns, plan.nr, plan.nt), "d_host")
        self.u = None if u_host is None else self._pinned(u_host, (plan.ns, plan.nvs, plan.nt),
                                                          "u_host")
        dev = plan.device
        self.buf = [torch.empty((plan.nb_max, plan.nr, plan.nt), dtype=torch.float32, device=dev)
                    for _ in range(2)]
        self.ubuf = None if self.u is None else [
            torch.empty((plan.nb_max, plan.nvs, plan.nt), dtype=torch.float32, device=dev)
            for _ in range(2)]
        self.copy_stream = torch.cuda.Stream(dev)
        self.ready = [torch.cuda.Event() for _ in range(2)]
        self.free = [torch.cuda.Event() for _ in range(2)]
        self.nb = [0, 0]
        self.fill = 0      # buffer the next prefetch writes
        self.use = 0       # buffer the next stage reads

    @staticmethod
    def _pinned(x: torch.Tensor, shape, name) -> torch.Tensor:
        if tuple(x.shape) != shape or x.dtype != torch.float32 or x.is_cuda:
            raise ValueError(f"{name} must be a float32 host tensor of shape {shape}")
        if not x.is_pinned():
            pinned = torch.empty(shape, dtype=torch.float32, pin_memory=True)
            pinned.copy_(x)
            x = pinned
        return x.contiguous()

    def prefetch(self, idx) -> None:
        idx = np.asarray(idx, dtype=np.int64).ravel()
        if not 1 <= idx.size <= self.plan.nb_max:
            raise ValueError(f"a batch has 1..{self.plan.nb_max} entries")
        slot = self.fill
        s = self.copy_stream
        s.wait_event(self.free[slot])
        with torch.cuda.stream(s):
            for b, src in enumerate(idx):
                if 0 <= src < self.plan.ns:   # other entries are zero sources: row unused
                    self.buf[slot][b].copy_(self.d[src], non_blocking=True)
                    if self.u is not None:
                        self.ubuf[slot][b].copy_(self.u[src], non_blocking=True)
            self.ready[slot].record(s)
        self.nb[slot] = int(idx.size)
        self.fill ^= 1

    def stage(self) -> None:
        slot = self.use
        cur = torch.cuda.current_stream(self.plan.device)
        cur.wait_event(self.ready[slot])
        self.plan.mdd_stage_kernel(self.buf[slot][:self.nb[slot]])
        if self.u is not None:
            self.plan.mdd_stage_data(self.ubuf[slot][:self.nb[slot]])
        self.free[slot].record(cur)
        self.use ^= 1
