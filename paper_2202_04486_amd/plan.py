"""Torch-facing binding of the C ABI: one `Plan` per problem size.

Every method only checks shapes / dtypes / devices and passes raw device
pointers and the current HIP stream to libmdd.so; all arithmetic runs in the
library's HIP kernels.  PyTorch provides device memory and streams.
"""
from __future__ import annotations

import ctypes

import torch

from . import native
from .native import MddError, Opt, check, load, make_dims, workspace_bytes

__all__ = ["Plan", "MddError"]


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _need(t, name, shape, dtype, device):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device != device:
        raise ValueError(f"{name} must be on {device}, got {t.device}")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


class Plan:
    """Sizes, workspace and stream of one stochastic-MDD problem on one GPU.

    ns sources, nr receivers, nvs virtual sources, nt time samples, nf retained
    one-sided frequency bins, nb_max the largest batch; precision one of
    'fp32', 'bf16x3', 'fp16x3', 'bf16' (single pass, diagnostic) and 'fp32_cgemm'
    (float32 with four real products per complex one, for comparison)."""

    def __init__(self, ns, nr, nvs, nt, nf, nb_max, precision="fp32", store_rf=False,
                 device=None, full_grad=False, stream_kernel=False, stream_data=False):
        self.lib = load()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        if self.device.type != "cuda":
            raise ValueError("Plan needs a GPU device")
        self.ns, self.nr, self.nvs, self.nt, self.nf, self.nb_max = ns, nr, nvs, nt, nf, nb_max
        self.precision = precision
        self.dims = make_dims(ns, nr, nvs, nt, nf, nb_max, precision,
                              (native.FLAG_STORE_RF if store_rf else 0) |
                              (native.FLAG_FULL_GRAD if full_grad else 0) |
                              (native.FLAG_STREAM_KERNEL if stream_kernel else 0) |
                              (native.FLAG_STREAM_DATA if stream_data else 0))
        self.stream_kernel = stream_kernel
        self.stream_data = stream_data
        nbytes = workspace_bytes(self.dims)
        if nbytes == 0:
            raise MddError("mdd_workspace_bytes", native.MDD_ESHAPE)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        self._ws_ptr = ctypes.c_void_p(self.workspace.data_ptr() + off)
        self._ws_bytes = nbytes
        self._plan = ctypes.c_void_p()
        stream = torch.cuda.current_stream(self.device).cuda_stream
        check("mdd_plan_create", self.lib.mdd_plan_create(
            ctypes.byref(self.dims), self._ws_ptr, nbytes, ctypes.c_void_p(stream),
            ctypes.byref(self._plan)))
        self._keep = []

    # ---------------------------------------------------------------- helpers
    def _sync_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        check("mdd_plan_set_stream", self.lib.mdd_plan_set_stream(self._plan, ctypes.c_void_p(s)))

    def _idx(self, idx):
        _need(idx, "idx", None, torch.int32, self.device)
        if idx.dim() != 1 or not 1 <= idx.numel() <= self.nb_max:
            raise ValueError(f"idx must be 1-D with 1..{self.nb_max} entries")
        return idx.numel()

    def _call(self, name, *args):
        self._sync_stream()
        check(name, getattr(self.lib, name)(self._plan, *args), self._plan)

    def close(self):
        if self._plan:
            self.lib.mdd_plan_destroy(self._plan)
            self._plan = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- setup
    def mdd_set_kernel(self, d):
        _need(d, "d", (self.ns, self.nr, self.nt), torch.float32, self.device)
        self._call("mdd_set_kernel", _ptr(d))

    def mdd_stage_kernel(self, d_rows):
        """Kernel rows of the next batch (stream_kernel=True): d_rows [nb][nr][nt], row b
        the source that the next call's idx[b] names."""
        _need(d_rows, "d_rows", None, torch.float32, self.device)
        if d_rows.dim() != 3 or d_rows.shape[1:] != (self.nr, self.nt) or not d_rows.is_contiguous():
            raise ValueError(f"d_rows must be contiguous [nb][{self.nr}][{self.nt}]")
        self._call("mdd_stage_kernel", _ptr(d_rows), int(d_rows.shape[0]))

    def mdd_stage_data(self, u_rows):
        """Data rows of the next batch (stream_data=True): u_rows [nb][nvs][nt], row b
        the source that the next call's idx[b] names."""
        _need(u_rows, "u_rows", None, torch.float32, self.device)
        if u_rows.dim() != 3 or u_rows.shape[1:] != (self.nvs, self.nt) or not u_rows.is_contiguous():
            raise ValueError(f"u_rows must be contiguous [nb][{self.nvs}][{self.nt}]")
        self._call("mdd_stage_data", _ptr(u_rows), int(u_rows.shape[0]))

    def mdd_set_data(self, u):
        _need(u, "u", (self.ns, self.nvs, self.nt), torch.float32, self.device)
        self._call("mdd_set_data", _ptr(u))

    def mdd_set_mask(self, onset):
        if onset is None:
            self._call("mdd_set_mask", ctypes.c_void_p(0))
            return
        _need(onset, "onset", (self.nr, self.nvs), torch.int32, self.device)
        self._call("mdd_set_mask", _ptr(onset))

    # ---------------------------------------------------------------- operator
    def mdc_forward(self, R, idx, out=None, entry="mdc_forward"):
        _need(R, "R", (self.nr, self.nvs, self.nt), torch.float32, self.device)
        nb = self._idx(idx)
        if out is None:
            out = torch.empty((nb, self.nvs, self.nt), dtype=torch.float32, device=self.device)
        _need(out, "U_out", (nb, self.nvs, self.nt), torch.float32, self.device)
        self._call(entry, _ptr(R), _ptr(idx), nb, _ptr(out))
        return out

    def mdc_adjoint(self, V, idx, out=None, entry="mdc_adjoint"):
        nb = self._idx(idx)
        _need(V, "V", (nb, self.nvs, self.nt), torch.float32, self.device)
        if out is None:
            out = torch.empty((self.nr, self.nvs, self.nt), dtype=torch.float32, device=self.device)
        _need(out, "G_out", (self.nr, self.nvs, self.nt), torch.float32, self.device)
        self._call(entry, _ptr(V), _ptr(idx), nb, _ptr(out))
        return out

    def mdc_forward_rec(self, R, idx, out=None):
        """mdc_forward of C_r R (nr == nvs), with C_r applied to the spectra of R."""
        return self.mdc_forward(R, idx, out, entry="mdc_forward_rec")

    def mdc_adjoint_rec(self, V, idx, out=None):
        """C_r of mdc_adjoint(V) (nr == nvs), with C_r applied to the adjoint's spectra."""
        return self.mdc_adjoint(V, idx, out, entry="mdc_adjoint_rec")

    def _scalar(self, t, name):
        if t is None:
            t = torch.empty(1, dtype=torch.float64, device=self.device)
        _need(t, name, None, torch.float64, self.device)
        if t.numel() < 1:
            raise ValueError(f"{name} needs at least one element")
        return t

    def mdd_stoch_grad(self, R, idx, G_out=None, loss_out=None, gnorm2_out=None):
        """Summed mini-batch gradient (masked), float64 loss and ||G||^2 (device)."""
        _need(R, "R", (self.nr, self.nvs, self.nt), torch.float32, self.device)
        nb = self._idx(idx)
        if G_out is None:
            G_out = torch.empty_like(R)
        _need(G_out, "G_out", (self.nr, self.nvs, self.nt), torch.float32, self.device)
        loss_out = self._scalar(loss_out, "loss_out")
        gnorm2_out = self._scalar(gnorm2_out, "gnorm2_out")
        self._call("mdd_stoch_grad", _ptr(R), _ptr(idx), nb, _ptr(G_out), _ptr(loss_out),
                   _ptr(gnorm2_out))
        return G_out, loss_out, gnorm2_out

    def mdd_step(self, R, idx, opt="adam", lr=1e-2, s0=None, s1=None, t=1, beta1=0.9,
                 beta2=0.999, eps=1e-8, mu=0.9, loss_out=None, gnorm2_out=None):
        """One in-place optimiser step on R (and s0 / s1); returns (loss, gnorm2) tensors."""
        _need(R, "R", (self.nr, self.nvs, self.nt), torch.float32, self.device)
        nb = self._idx(idx)
        kind = native.OPT[opt]
        for name, st in (("s0", s0), ("s1", s1)):
            if st is not None:
                _need(st, name, (self.nr, self.nvs, self.nt), torch.float32, self.device)
        o = Opt(kind, 0, float(lr), float(beta1), float(beta2), float(eps), float(mu), int(t))
        loss_out = self._scalar(loss_out, "loss_out")
        gnorm2_out = self._scalar(gnorm2_out, "gnorm2_out")
        self._call("mdd_step", _ptr(R), _ptr(s0), _ptr(s1), ctypes.byref(o), _ptr(idx), nb,
                   _ptr(loss_out), _ptr(gnorm2_out))
        return loss_out, gnorm2_out

    def mdd_full_grad(self, R, G_out=None, loss_out=None, gnorm2_out=None):
        """Gradient of the whole finite-sum functional (every source; needs full_grad=True)."""
        _need(R, "R", (self.nr, self.nvs, self.nt), torch.float32, self.device)
        if G_out is None:
            G_out = torch.empty_like(R)
        _need(G_out, "G_out", (self.nr, self.nvs, self.nt), torch.float32, self.device)
        loss_out = self._scalar(loss_out, "loss_out")
        gnorm2_out = self._scalar(gnorm2_out, "gnorm2_out")
        self._call("mdd_full_grad", _ptr(R), _ptr(G_out), _ptr(loss_out), _ptr(gnorm2_out))
        return G_out, loss_out, gnorm2_out

    def mdd_full_step(self, R, opt="sgd", lr=1e-2, s0=None, s1=None, t=1, beta1=0.9,
                      beta2=0.999, eps=1e-8, mu=0.9, loss_out=None, gnorm2_out=None):
        """One in-place full-gradient iteration (SGD: Landweber); returns (loss, gnorm2)."""
        _need(R, "R", (self.nr, self.nvs, self.nt), torch.float32, self.device)
        for name, st in (("s0", s0), ("s1", s1)):
            if st is not None:
                _need(st, name, (self.nr, self.nvs, self.nt), torch.float32, self.device)
        o = Opt(native.OPT[opt], 0, float(lr), float(beta1), float(beta2), float(eps), float(mu),
                int(t))
        loss_out = self._scalar(loss_out, "loss_out")
        gnorm2_out = self._scalar(gnorm2_out, "gnorm2_out")
        self._call("mdd_full_step", _ptr(R), _ptr(s0), _ptr(s1), ctypes.byref(o),
                   _ptr(loss_out), _ptr(gnorm2_out))
        return loss_out, gnorm2_out

    def mdd_check_batch_host(self, idx):
        """Raise MddError if the batch has the wrong size or an index outside [0, ns)
        (the device entry points treat such an index as a zero source).  Host only."""
        host = (idx.detach().cpu() if isinstance(idx, torch.Tensor) else torch.as_tensor(idx))
        host = host.to(torch.int32).contiguous()
        check("mdd_check_batch_host", self.lib.mdd_check_batch_host(
            ctypes.c_void_p(host.data_ptr()), host.numel(), self.ns, self.nb_max))

    def mdd_invalidate_model_spectra(self):
        self._call("mdd_invalidate_model_spectra")

    def mdd_sigma_max2(self, iters=50, out=None):
        """Per-frequency largest squared singular value of the kernel (device float64 [nf])."""
        if out is None:
            out = torch.empty(self.nf, dtype=torch.float64, device=self.device)
        _need(out, "lam_out", (self.nf,), torch.float64, self.device)
        self._call("mdd_sigma_max2", int(iters), _ptr(out))
        return out

    # ---------------------------------------------------------------- timing
    def profile_enable(self, enable=True, capacity=4096):
        self._call("mdd_profile_enable", 1 if enable else 0, int(capacity))

    def profile_read(self):
        ms = (ctypes.c_double * len(native.KC_NAMES))()
        cnt = (ctypes.c_int64 * len(native.KC_NAMES))()
        self._call("mdd_profile_read", ms, cnt)
        return {n: (ms[i], cnt[i]) for i, n in enumerate(native.KC_NAMES)}
