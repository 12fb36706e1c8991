// Host layer of the C ABI declared in include/mdd.h: argument validation
// (always before any HIP call), the workspace layout, and the sequence of
// kernel launches for each entry point on the plan's stream.
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <new>
#include <vector>

#include "mdd_internal.h"

using namespace mdd;

namespace {

constexpr int MAX_EXTENT = 4096;  // ns, nr, nvs: the power iteration keeps vectors in LDS
// ns of a plan with MDD_FLAG_STREAM_KERNEL: such a plan runs no power iteration and
// keeps no per-source kernel spectra (and, with MDD_FLAG_STREAM_DATA, no per-source data).
constexpr int MAX_STREAM_NS = 1 << 20;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

bool valid_nt(int nt) { return nt == 128 || nt == 256 || nt == 512 || nt == 1024; }

struct Layout {
  size_t tw, df, uf, oob, oobp, onset, f, bsp, lossp, gnp, dmx, red2, f2, sidx, lossb, gvp, total;
};

Layout make_layout(const mdd_dims& d) {
  const size_t nrp = round16(d.nr), nvsp = round16(d.nvs), nvb = nblocks(d.nvs);
  const size_t c8 = sizeof(float2);
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align256(bytes);
    return at;
  };
  L.tw = take(c8 * 2 * d.nt);  // twiddle tables (at most 2 nt entries)
  // kernel spectra: every source, or (MDD_FLAG_STREAM_KERNEL) the staged batch rows
  const size_t drows = (d.flags & MDD_FLAG_STREAM_KERNEL) ? d.nb_max : d.ns;
  L.df = take(c8 * d.nf * drows * nrp);
  // data spectra and out-of-band energies: every source, or (MDD_FLAG_STREAM_DATA) the
  // staged batch rows
  const size_t urows = (d.flags & MDD_FLAG_STREAM_DATA) ? d.nb_max : d.ns;
  L.uf = take(c8 * d.nf * urows * nvsp);
  L.oob = take(sizeof(double) * urows);
  L.oobp = take(sizeof(double) * urows * nvb);
  L.onset = take(sizeof(int32_t) * d.nr * d.nvs);
  L.f = take(c8 * d.nr * nvb * d.nf * CB);
  L.bsp = take(c8 * d.nb_max * nvb * d.nf * CB);
  // nvs = 1: the matrix-vector products write one loss partial per row group.
  const size_t ngv = d.nvs == 1 ? gemv_groups(d.nb_max, d.nf) : 0;
  L.lossp = take(sizeof(double) * d.nf * (ngv > nvb ? ngv : nvb));
  // gradient / update modes: one partial per workgroup, trace_update_split(nt) per block
  L.gnp = take(sizeof(double) * d.nr * nvb * trace_update_split(d.nt));
  L.dmx = take(sizeof(float) * d.nf);               // per-frequency max |D| (fp16 scaling)
  L.red2 = take(sizeof(double) * 512);              // two-level reduction stage
  const bool full = (d.flags & MDD_FLAG_FULL_GRAD) != 0;  // full gradient: G buffer, sources, losses
  L.f2 = take(full ? c8 * d.nr * nvb * d.nf * CB : 0);
  L.sidx = take(full ? sizeof(int32_t) * d.ns : 0);
  L.lossb = take(full ? sizeof(double) * ((d.ns + d.nb_max - 1) / d.nb_max) : 0);
  L.gvp = take(ngv > 1 ? sizeof(float4) * d.nf * ngv * (nrp / 2) : 0);  // row-group partials
  L.total = o;
  return L;
}

mdd_status check_dims(const mdd_dims* d) {
  if (!d) return MDD_EINVAL;
  if (d->ns < 1 || d->nr < 1 || d->nvs < 1 || d->nb_max < 1 || d->nf < 1) return MDD_ESHAPE;
  const int ns_max = (d->flags & MDD_FLAG_STREAM_KERNEL) ? MAX_STREAM_NS : MAX_EXTENT;
  if (d->ns > ns_max || d->nr > MAX_EXTENT || d->nvs > MAX_EXTENT) return MDD_ESHAPE;
  if (!valid_nt(d->nt)) return MDD_ESHAPE;
  if (d->nf > d->nt / 2 + 1) return MDD_ESHAPE;
  if (d->nb_max > d->ns || d->nb_max > NB_LIMIT) return MDD_ESHAPE;
  if (d->precision < MDD_PREC_FP32 || d->precision > MDD_PREC_FP32_CGEMM) return MDD_EUNSUPPORTED;
  if (d->flags & ~(MDD_FLAG_STORE_RF | MDD_FLAG_FULL_GRAD | MDD_FLAG_STREAM_KERNEL |
                   MDD_FLAG_STREAM_DATA))
    return MDD_EINVAL;
  // staged data rows come with staged kernel rows
  if ((d->flags & MDD_FLAG_STREAM_DATA) && !(d->flags & MDD_FLAG_STREAM_KERNEL)) return MDD_EINVAL;
  // the full gradient visits every source: it needs the resident kernel spectra
  if ((d->flags & MDD_FLAG_FULL_GRAD) && (d->flags & MDD_FLAG_STREAM_KERNEL)) return MDD_EINVAL;
  return MDD_OK;
}

// Column groups of one frequency in the product kernels (must match launch_gemm).
int gemm_ncg(int nb, int nvb) {
  const int tnb = nb <= 16 ? 1 : (nb <= 32 ? 2 : 4);
  return (nvb + tnb - 1) / tnb;
}

}  // namespace

struct mdd_plan {
  mdd_dims d{};
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  Layout L{};
  int nrp = 0, nvsp = 0, nvb = 0;
  bool kernel_set = false, data_set = false, mask_set = false;
  // MDD_FLAG_STORE_RF: the model whose next evaluation point's spectra F holds.
  const float* spec_model = nullptr;
  const float* spec_vel = nullptr;
  double spec_mu = 0.0;
  // MDD_FLAG_FULL_GRAD: the two spectra buffers swap roles when a full step stores the
  // next model's spectra where the gradient was accumulated.
  bool fswap = false;
  int32_t last_hip = 0;
  bool prof = false;
  int cap = 0, nrec = 0;
  std::vector<hipEvent_t> ev;
  std::vector<int> cls;

  template <class T>
  T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
  float2* tw() const { return at<float2>(L.tw); }
  float2* Df() const { return at<float2>(L.df); }
  float2* Uf() const { return at<float2>(L.uf); }
  double* oob() const { return at<double>(L.oob); }
  double* oobp() const { return at<double>(L.oobp); }
  int32_t* onset() const { return at<int32_t>(L.onset); }
  float2* F() const { return at<float2>(fswap ? L.f2 : L.f); }
  float2* F2() const { return at<float2>(fswap ? L.f : L.f2); }
  float2* Bsp() const { return at<float2>(L.bsp); }
  double* lossp() const { return at<double>(L.lossp); }
  double* gnp() const { return at<double>(L.gnp); }
  float* dmx() const { return at<float>(L.dmx); }
  double* red2() const { return at<double>(L.red2); }
  int32_t* sidx() const { return at<int32_t>(L.sidx); }
  double* lossb() const { return at<double>(L.lossb); }
  float4* gvp() const { return at<float4>(L.gvp); }
  bool full() const { return (d.flags & MDD_FLAG_FULL_GRAD) != 0; }
  // MDD_FLAG_STREAM_KERNEL: Df holds the rows of the last staged batch (staged_nb rows).
  bool streamed() const { return (d.flags & MDD_FLAG_STREAM_KERNEL) != 0; }
  int staged_nb = 0;
  // MDD_FLAG_STREAM_DATA: Uf and oob hold the rows of the last staged batch.
  bool streamed_data() const { return (d.flags & MDD_FLAG_STREAM_DATA) != 0; }
  int staged_u_nb = 0;
  // A call on a batch of nb entries: with staged kernel (and data) rows, the batch must
  // be the staged one (same length; entry b uses staged row b).
  mdd_status batch_ok(int nb) const {
    if (nb < 1 || nb > d.nb_max) return MDD_ESHAPE;
    if (streamed() && staged_nb == 0) return MDD_ESTATE;
    if (streamed() && nb != staged_nb) return MDD_ESHAPE;
    return MDD_OK;
  }
  // The same for the operators that read the data rows (gradient, step).
  mdd_status data_batch_ok(int nb) const {
    if (streamed_data() && staged_u_nb == 0) return MDD_ESTATE;
    if (streamed_data() && nb != staged_u_nb) return MDD_ESHAPE;
    return MDD_OK;
  }
  // One virtual source: the time arrays [rows][1][nt] are handled as one row of `rows`
  // columns, so spectra blocks hold 16 receivers (or batch rows), and the products are
  // matrix-vector products.
  bool vs1() const { return d.nvs == 1; }
  // Float64 partials of ||g||^2 written by the gradient / update kernels.
  int n_gn() const { return (vs1() ? nblocks(d.nr) : d.nr * nvb) * trace_update_split(d.nt); }
  // Float64 loss partials written by one fused product launch over a batch of nb.
  int n_loss(int nb) const { return d.nf * (vs1() ? gemv_groups(nb, d.nf) : gemm_ncg(nb, nvb)); }

  template <class Fn>
  mdd_status run(int kclass, Fn&& fn) {
    const bool rec = prof && nrec < cap;
    if (rec) {
      const hipError_t e = hipEventRecord(ev[2 * nrec], stream);
      if (e != hipSuccess) return fail(e);
    }
    const hipError_t err = fn();
    if (err != hipSuccess) return fail(err);
    if (rec) {
      const hipError_t e = hipEventRecord(ev[2 * nrec + 1], stream);
      if (e != hipSuccess) return fail(e);
      cls[nrec] = kclass;
      ++nrec;
    }
    return MDD_OK;
  }
  mdd_status fail(hipError_t e) {
    last_hip = (int32_t)e;
    return MDD_EHIP;
  }

  // Trace-kernel geometry of a [rows][nvs][nt] time array against blocked spectra.
  TraceArgs blocked(float2* spec, int rows) const {
    TraceArgs a{};
    a.nt = d.nt;
    a.nf = d.nf;
    a.rows = vs1() ? 1 : rows;
    a.ncols = vs1() ? rows : d.nvs;
    a.ncb = vs1() ? nblocks(rows) : nvb;
    a.spec = spec;
    a.s_row = (long long)a.ncb * d.nf * CB;
    a.s_cb = (long long)d.nf * CB;
    a.s_k = CB;
    a.tw = tw();
    return a;
  }

  GemmArgs gemm(const int32_t* idx, int nb) const {
    GemmArgs g{};
    g.Df = Df();
    g.Uf = Uf();
    g.F = F();
    g.Bsp = Bsp();
    g.idx = idx;
    g.loss_part = lossp();
    g.dmax = d.precision == MDD_PREC_FP16X3 ? dmx() : nullptr;
    g.ns = d.ns;
    g.nr = d.nr;
    g.nrp = nrp;
    g.nvs = d.nvs;
    g.nvsp = nvsp;
    g.nvb = nvb;
    g.nf = d.nf;
    g.nt = d.nt;
    g.nb = nb;
    g.dns = streamed() ? d.nb_max : d.ns;
    g.dpos = streamed() ? 1 : 0;
    g.uns = streamed_data() ? d.nb_max : d.ns;
    g.upos = streamed_data() ? 1 : 0;
    if (vs1()) {
      g.P = gemv_groups(nb, d.nf);
      g.gpart = gvp();
    }
    return g;
  }

  // Per-frequency products of one batch (any kind) on the plan's stream.
  mdd_status products(int kind, const GemmArgs& g) {
    return run(MDD_KC_GEMM, [&] {
      return vs1() ? launch_gemv(kind, g, stream) : launch_gemm(kind, d.precision, g, stream);
    });
  }

  mdd_status model_fft(const float* R, const float* vel, double mu) {
    TraceArgs a = blocked(F(), d.nr);
    a.x_in = R;
    a.x_in2 = vel;
    a.mu2 = (float)mu;
    return run(MDD_KC_FFT_MODEL, [&] { return launch_trace(TM_RFFT, a, stream); });
  }

  mdd_status reduce(const int32_t* idx, int nb, bool with_loss, double* loss_out,
                    double* gnorm2_out) {
    if (!loss_out && !gnorm2_out) return MDD_OK;
    ReduceArgs r{};
    r.loss_part = lossp();
    r.n_loss = with_loss ? n_loss(nb) : 0;
    r.loss_scale = 1.0 / (2.0 * d.nt);
    r.oob = with_loss ? oob() : nullptr;
    r.idx = idx;
    r.nb = nb;
    r.ns = d.ns;
    r.oob_pos = streamed_data() ? 1 : 0;
    r.gn_part = gnp();
    r.n_gn = gnorm2_out ? n_gn() : 0;
    r.loss_out = loss_out;
    r.gnorm2_out = gnorm2_out;
    r.stage = red2();
    return run(MDD_KC_REDUCE, [&] { return launch_reduce(r, stream); });
  }

  // Full gradient, products part: every source in order, batches of nb_max, the
  // adjoint products summed into F2; batch j's loss into lossb[j].  F keeps R_k.
  mdd_status full_products() {
    const int nsub = (d.ns + d.nb_max - 1) / d.nb_max;
    for (int j = 0; j < nsub; ++j) {
      const int nb = d.ns - j * d.nb_max < d.nb_max ? d.ns - j * d.nb_max : d.nb_max;
      const int32_t* idx = sidx() + (size_t)j * d.nb_max;
      GemmArgs g = gemm(idx, nb);
      g.Gout = F2();
      g.gacc = j > 0 ? 1 : 0;
      mdd_status st = products(GK_FUSED, g);
      if (st != MDD_OK) return st;
      st = reduce(idx, nb, true, lossb() + j, nullptr);
      if (st != MDD_OK) return st;
    }
    return MDD_OK;
  }

  // Full gradient, final sums: the batches' losses in order and ||g||^2.
  mdd_status full_reduce(double* loss_out, double* gnorm2_out) {
    if (!loss_out && !gnorm2_out) return MDD_OK;
    ReduceArgs r{};
    r.loss_part = lossb();
    r.n_loss = (d.ns + d.nb_max - 1) / d.nb_max;
    r.loss_scale = 1.0;
    r.oob = nullptr;
    r.idx = nullptr;
    r.nb = 0;
    r.ns = d.ns;
    r.gn_part = gnp();
    r.n_gn = n_gn();
    r.loss_out = loss_out;
    r.gnorm2_out = gnorm2_out;
    r.stage = red2();
    return run(MDD_KC_REDUCE, [&] { return launch_reduce(r, stream); });
  }
};

// Optimiser fields of the update kernel from mdd_opt; validates them.
mdd_status update_args(const mdd_opt& o, float* s0, float* s1, TraceArgs& a, int& mode) {
  switch (o.kind) {
    case MDD_OPT_SGD: mode = TM_SGD; break;
    case MDD_OPT_ADAM:
      if (!s0 || !s1) return MDD_EINVAL;
      if (!(o.beta1 >= 0.0 && o.beta1 < 1.0) || !(o.beta2 >= 0.0 && o.beta2 < 1.0)) return MDD_EINVAL;
      if (!(o.eps > 0.0) || o.t < 1) return MDD_EINVAL;
      mode = TM_ADAM;
      break;
    case MDD_OPT_NSGD:
      if (!s0) return MDD_EINVAL;
      if (!(o.mu >= 0.0 && o.mu < 1.0)) return MDD_EINVAL;
      mode = TM_NSGD;
      break;
    default: return MDD_EINVAL;
  }
  if (!(o.lr > 0.0) || !std::isfinite(o.lr)) return MDD_EINVAL;
  a.st0 = s0;
  a.st1 = s1;
  a.lr = (float)o.lr;
  a.beta1 = (float)o.beta1;
  a.beta2 = (float)o.beta2;
  a.eps = (float)o.eps;
  a.mu = (float)o.mu;
  a.omb1 = (float)(1.0 - o.beta1);
  a.omb2 = (float)(1.0 - o.beta2);
  if (mode == TM_ADAM) {
    a.inv_bc1 = (float)(1.0 / (1.0 - std::pow(o.beta1, (double)o.t)));
    a.inv_bc2 = (float)(1.0 / (1.0 - std::pow(o.beta2, (double)o.t)));
  }
  return MDD_OK;
}

#define MDD_TRY(x)                 \
  do {                             \
    const mdd_status s_ = (x);     \
    if (s_ != MDD_OK) return s_;   \
  } while (0)

extern "C" {

size_t mdd_workspace_bytes(const mdd_dims* dims) {
  if (check_dims(dims) != MDD_OK) return 0;
  return make_layout(*dims).total;
}

}  // extern "C"

// Lays a plan out in a workspace of at least make_layout(*dims).total bytes and
// enqueues its tables (dims already checked).
static hipError_t init_plan(mdd_plan* p, const mdd_dims* dims, const Layout& L, void* workspace,
                            void* stream) {
  p->d = *dims;
  p->stream = reinterpret_cast<hipStream_t>(stream);
  p->ws = reinterpret_cast<char*>(workspace);
  p->L = L;
  p->nrp = round16(dims->nr);
  p->nvsp = round16(dims->nvs);
  p->nvb = nblocks(dims->nvs);
  hipError_t e = launch_twiddles(p->tw(), dims->nt, p->stream);
  if (e == hipSuccess && p->full()) e = launch_iota(p->sidx(), dims->ns, p->stream);
  return e;
}

extern "C" {

mdd_status mdd_plan_create(const mdd_dims* dims, void* workspace, size_t ws_bytes, void* stream,
                           mdd_plan** out) {
  if (!out) return MDD_EINVAL;
  *out = nullptr;
  MDD_TRY(check_dims(dims));
  const Layout L = make_layout(*dims);
  if (!workspace || ws_bytes < L.total || (reinterpret_cast<uintptr_t>(workspace) & 255))
    return MDD_ENOMEM;
  mdd_plan* p = new (std::nothrow) mdd_plan();
  if (!p) return MDD_ENOMEM;
  if (init_plan(p, dims, L, workspace, stream) != hipSuccess) {
    delete p;
    return MDD_EHIP;
  }
  *out = p;
  return MDD_OK;
}

mdd_status mdd_plan_destroy(mdd_plan* plan) {
  if (!plan) return MDD_EINVAL;
  for (hipEvent_t e : plan->ev) (void)hipEventDestroy(e);
  delete plan;
  return MDD_OK;
}

mdd_status mdd_plan_set_stream(mdd_plan* plan, void* stream) {
  if (!plan) return MDD_EINVAL;
  plan->stream = reinterpret_cast<hipStream_t>(stream);
  return MDD_OK;
}

mdd_status mdd_set_kernel(mdd_plan* p, const float* d) {
  if (!p || !d) return MDD_EINVAL;
  if (p->streamed()) return MDD_ESTATE;  // such a plan takes batch rows (mdd_stage_kernel)
  TraceArgs a{};
  a.nt = p->d.nt;
  a.nf = p->d.nf;
  a.rows = p->d.ns;
  a.ncols = p->d.nr;
  a.ncb = nblocks(p->d.nr);
  a.x_in = d;
  a.spec = p->Df();
  a.s_row = p->nrp;
  a.s_cb = CB;
  a.s_k = (long long)p->d.ns * p->nrp;
  a.tw = p->tw();
  MDD_TRY(p->run(MDD_KC_DATA_FFT, [&] { return launch_trace(TM_RFFT, a, p->stream); }));
  if (p->d.precision == MDD_PREC_FP16X3)
    MDD_TRY(p->run(MDD_KC_DATA_FFT, [&] {
      return launch_freq_absmax(p->Df(), p->d.nf, (long long)p->d.ns * p->nrp,
                                (long long)p->d.ns * p->nrp, p->dmx(), p->stream);
    }));
  p->kernel_set = true;
  return MDD_OK;
}

mdd_status mdd_stage_kernel(mdd_plan* p, const float* d_rows, int32_t nb) {
  if (!p || !d_rows) return MDD_EINVAL;
  if (!p->streamed()) return MDD_ESTATE;
  if (nb < 1 || nb > p->d.nb_max) return MDD_ESHAPE;
  TraceArgs a{};
  a.nt = p->d.nt;
  a.nf = p->d.nf;
  a.rows = nb;
  a.ncols = p->d.nr;
  a.ncb = nblocks(p->d.nr);
  a.x_in = d_rows;
  a.spec = p->Df();
  a.s_row = p->nrp;
  a.s_cb = CB;
  a.s_k = (long long)p->d.nb_max * p->nrp;
  a.tw = p->tw();
  MDD_TRY(p->run(MDD_KC_DATA_FFT, [&] { return launch_trace(TM_RFFT, a, p->stream); }));
  if (p->d.precision == MDD_PREC_FP16X3)
    MDD_TRY(p->run(MDD_KC_DATA_FFT, [&] {
      return launch_freq_absmax(p->Df(), p->d.nf, (long long)nb * p->nrp,
                                (long long)p->d.nb_max * p->nrp, p->dmx(), p->stream);
    }));
  p->staged_nb = nb;
  p->kernel_set = true;
  return MDD_OK;
}

// Data spectra and out-of-band energies of `rows` sources u [rows][nvs][nt], into data
// spectra with `urows` rows per frequency.
static mdd_status data_spectra(mdd_plan* p, const float* u, int rows, int urows) {
  TraceArgs a{};
  a.nt = p->d.nt;
  a.nf = p->d.nf;
  a.rows = rows;
  a.ncols = p->d.nvs;
  a.ncb = p->nvb;
  a.x_in = u;
  a.spec = p->Uf();
  a.s_row = p->nvsp;
  a.s_cb = CB;
  a.s_k = (long long)urows * p->nvsp;
  a.part = p->oobp();
  a.tw = p->tw();
  MDD_TRY(p->run(MDD_KC_DATA_FFT, [&] { return launch_trace(TM_RFFT, a, p->stream); }));
  return p->run(MDD_KC_REDUCE, [&] {
    return launch_row_sum(p->oobp(), rows, p->nvb, 1.0 / (2.0 * p->d.nt), p->oob(), p->stream);
  });
}

mdd_status mdd_stage_data(mdd_plan* p, const float* u_rows, int32_t nb) {
  if (!p || !u_rows) return MDD_EINVAL;
  if (!p->streamed_data()) return MDD_ESTATE;
  if (nb < 1 || nb > p->d.nb_max) return MDD_ESHAPE;
  MDD_TRY(data_spectra(p, u_rows, nb, p->d.nb_max));
  p->staged_u_nb = nb;
  p->data_set = true;
  return MDD_OK;
}

mdd_status mdd_set_data(mdd_plan* p, const float* u) {
  if (!p || !u) return MDD_EINVAL;
  if (p->streamed_data()) return MDD_ESTATE;  // such a plan takes batch rows (mdd_stage_data)
  MDD_TRY(data_spectra(p, u, p->d.ns, p->d.ns));
  p->data_set = true;
  return MDD_OK;
}

mdd_status mdd_set_mask(mdd_plan* p, const int32_t* onset) {
  if (!p) return MDD_EINVAL;
  if (!onset) {
    p->mask_set = false;
    return MDD_OK;
  }
  const hipError_t e = hipMemcpyAsync(p->onset(), onset, sizeof(int32_t) * p->d.nr * p->d.nvs,
                                      hipMemcpyDeviceToDevice, p->stream);
  if (e != hipSuccess) return p->fail(e);
  p->mask_set = true;
  return MDD_OK;
}

mdd_status mdc_forward(mdd_plan* p, const float* R, const int32_t* idx, int32_t nb, float* U_out) {
  if (!p || !R || !idx || !U_out) return MDD_EINVAL;
  MDD_TRY(p->batch_ok(nb));
  if (!p->kernel_set) return MDD_ESTATE;
  p->spec_model = nullptr;
  MDD_TRY(p->model_fft(R, nullptr, 0.0));
  const GemmArgs g = p->gemm(idx, nb);
  MDD_TRY(p->products(GK_FWD, g));
  TraceArgs a = p->blocked(p->Bsp(), nb);
  a.x_out = U_out;
  return p->run(MDD_KC_DATA_FFT, [&] { return launch_trace(TM_IRFFT, a, p->stream); });
}

mdd_status mdc_adjoint(mdd_plan* p, const float* V, const int32_t* idx, int32_t nb, float* G_out) {
  if (!p || !V || !idx || !G_out) return MDD_EINVAL;
  MDD_TRY(p->batch_ok(nb));
  if (!p->kernel_set) return MDD_ESTATE;
  p->spec_model = nullptr;
  TraceArgs a = p->blocked(p->Bsp(), nb);
  a.x_in = V;
  MDD_TRY(p->run(MDD_KC_DATA_FFT, [&] { return launch_trace(TM_RFFT, a, p->stream); }));
  const GemmArgs g = p->gemm(idx, nb);
  MDD_TRY(p->products(GK_ADJ, g));
  TraceArgs b = p->blocked(p->F(), p->d.nr);
  b.x_out = G_out;
  return p->run(MDD_KC_UPDATE, [&] { return launch_trace(TM_IRFFT, b, p->stream); });
}

// C_r on the plan's model / gradient spectra (nr = nvs; identity for a single trace).
static mdd_status spec_reciprocity(mdd_plan* p) {
  if (p->d.nr == 1) return MDD_OK;
  const TraceArgs a = p->blocked(p->F(), p->d.nr);
  return p->run(MDD_KC_RECIPROCITY, [&] {
    return launch_spec_reciprocity(p->F(), p->d.nr, p->d.nf, a.s_row, a.s_cb, p->stream);
  });
}

mdd_status mdc_forward_rec(mdd_plan* p, const float* R, const int32_t* idx, int32_t nb,
                           float* U_out) {
  if (!p || !R || !idx || !U_out) return MDD_EINVAL;
  if (p->d.nr != p->d.nvs) return MDD_ESHAPE;
  MDD_TRY(p->batch_ok(nb));
  if (!p->kernel_set) return MDD_ESTATE;
  p->spec_model = nullptr;
  MDD_TRY(p->model_fft(R, nullptr, 0.0));
  MDD_TRY(spec_reciprocity(p));
  const GemmArgs g = p->gemm(idx, nb);
  MDD_TRY(p->products(GK_FWD, g));
  TraceArgs a = p->blocked(p->Bsp(), nb);
  a.x_out = U_out;
  return p->run(MDD_KC_DATA_FFT, [&] { return launch_trace(TM_IRFFT, a, p->stream); });
}

mdd_status mdc_adjoint_rec(mdd_plan* p, const float* V, const int32_t* idx, int32_t nb,
                           float* G_out) {
  if (!p || !V || !idx || !G_out) return MDD_EINVAL;
  if (p->d.nr != p->d.nvs) return MDD_ESHAPE;
  MDD_TRY(p->batch_ok(nb));
  if (!p->kernel_set) return MDD_ESTATE;
  p->spec_model = nullptr;
  TraceArgs a = p->blocked(p->Bsp(), nb);
  a.x_in = V;
  MDD_TRY(p->run(MDD_KC_DATA_FFT, [&] { return launch_trace(TM_RFFT, a, p->stream); }));
  const GemmArgs g = p->gemm(idx, nb);
  MDD_TRY(p->products(GK_ADJ, g));
  MDD_TRY(spec_reciprocity(p));
  TraceArgs b = p->blocked(p->F(), p->d.nr);
  b.x_out = G_out;
  return p->run(MDD_KC_UPDATE, [&] { return launch_trace(TM_IRFFT, b, p->stream); });
}

mdd_status mdd_stoch_grad(mdd_plan* p, const float* R, const int32_t* idx, int32_t nb,
                          float* G_out, double* loss_out, double* gnorm2_out) {
  if (!p || !R || !idx || !G_out) return MDD_EINVAL;
  MDD_TRY(p->batch_ok(nb));
  if (!p->kernel_set || !p->data_set) return MDD_ESTATE;
  MDD_TRY(p->data_batch_ok(nb));
  p->spec_model = nullptr;
  MDD_TRY(p->model_fft(R, nullptr, 0.0));
  const GemmArgs g = p->gemm(idx, nb);
  MDD_TRY(p->products(GK_FUSED, g));
  TraceArgs a = p->blocked(p->F(), p->d.nr);
  a.x_out = G_out;
  a.onset = p->mask_set ? p->onset() : nullptr;
  a.part = p->gnp();
  MDD_TRY(p->run(MDD_KC_UPDATE, [&] { return launch_trace(TM_GRAD, a, p->stream); }));
  return p->reduce(idx, nb, true, loss_out, gnorm2_out);
}

mdd_status mdd_step(mdd_plan* p, float* R, float* s0, float* s1, const mdd_opt* opt,
                    const int32_t* idx, int32_t nb, double* loss_out, double* gnorm2_out) {
  if (!p || !R || !opt || !idx) return MDD_EINVAL;
  MDD_TRY(p->batch_ok(nb));
  if (!p->kernel_set || !p->data_set) return MDD_ESTATE;
  MDD_TRY(p->data_batch_ok(nb));
  TraceArgs a = p->blocked(p->F(), p->d.nr);
  int mode = 0;
  MDD_TRY(update_args(*opt, s0, s1, a, mode));
  const bool store = (p->d.flags & MDD_FLAG_STORE_RF) != 0;
  const float* vel = mode == TM_NSGD ? s0 : nullptr;
  const double mu = mode == TM_NSGD ? opt->mu : 0.0;
  const bool have = store && p->spec_model == R && p->spec_vel == vel && p->spec_mu == mu;
  p->spec_model = nullptr;
  if (!have) MDD_TRY(p->model_fft(R, vel, mu));
  const GemmArgs g = p->gemm(idx, nb);
  MDD_TRY(p->products(GK_FUSED, g));
  a.model = R;
  a.store_spec = store ? 1 : 0;
  a.onset = p->mask_set ? p->onset() : nullptr;
  a.part = p->gnp();
  MDD_TRY(p->run(MDD_KC_UPDATE, [&] { return launch_trace(mode, a, p->stream); }));
  if (store) {
    p->spec_model = R;
    p->spec_vel = vel;
    p->spec_mu = mu;
  }
  return p->reduce(idx, nb, true, loss_out, gnorm2_out);
}

mdd_status mdd_stoch_grad_noalloc(const mdd_dims* dims, const float* d, const float* u,
                                  const int32_t* onset, const float* R, const int32_t* idx,
                                  int32_t nb, float* G_out, double* loss_out, double* gnorm2_out,
                                  void* stream) {
  if (!dims || !d || !u || !R || !idx || !G_out) return MDD_EINVAL;
  MDD_TRY(check_dims(dims));
  if (dims->flags & (MDD_FLAG_STREAM_KERNEL | MDD_FLAG_FULL_GRAD)) return MDD_EINVAL;
  if (nb < 1 || nb > dims->nb_max) return MDD_ESHAPE;
  const Layout L = make_layout(*dims);
  if (L.total > static_workspace_bytes()) return MDD_ELIMIT;
  const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return MDD_EHIP;
  if (s) {  // the stream must belong to the current device, whose workspace is used
    int sdev = -1;
    if (hipStreamGetDevice(s, &sdev) != hipSuccess) return MDD_EHIP;
    if (sdev != dev) return MDD_EINVAL;
  }
  void* ws = nullptr;
  if (static_workspace(dev, &ws) != hipSuccess) return MDD_EHIP;
  mdd_plan p;  // host object on the stack; its event lists stay empty
  if (init_plan(&p, dims, L, ws, stream) != hipSuccess) return MDD_EHIP;
  MDD_TRY(mdd_set_kernel(&p, d));
  MDD_TRY(mdd_set_data(&p, u));
  MDD_TRY(mdd_set_mask(&p, onset));
  return mdd_stoch_grad(&p, R, idx, nb, G_out, loss_out, gnorm2_out);
}

mdd_status mdd_full_grad(mdd_plan* p, const float* R, float* G_out, double* loss_out,
                         double* gnorm2_out) {
  if (!p || !R || !G_out) return MDD_EINVAL;
  if (!p->kernel_set || !p->data_set || !p->full()) return MDD_ESTATE;
  p->spec_model = nullptr;
  MDD_TRY(p->model_fft(R, nullptr, 0.0));
  MDD_TRY(p->full_products());
  TraceArgs a = p->blocked(p->F2(), p->d.nr);
  a.x_out = G_out;
  a.onset = p->mask_set ? p->onset() : nullptr;
  a.part = p->gnp();
  MDD_TRY(p->run(MDD_KC_UPDATE, [&] { return launch_trace(TM_GRAD, a, p->stream); }));
  if (p->d.flags & MDD_FLAG_STORE_RF) {  // F still holds the spectra of R
    p->spec_model = R;
    p->spec_vel = nullptr;
    p->spec_mu = 0.0;
  }
  return p->full_reduce(loss_out, gnorm2_out);
}

mdd_status mdd_full_step(mdd_plan* p, float* R, float* s0, float* s1, const mdd_opt* opt,
                         double* loss_out, double* gnorm2_out) {
  if (!p || !R || !opt) return MDD_EINVAL;
  if (!p->kernel_set || !p->data_set || !p->full()) return MDD_ESTATE;
  TraceArgs a = p->blocked(p->F2(), p->d.nr);  // the update reads the summed gradient
  int mode = 0;
  MDD_TRY(update_args(*opt, s0, s1, a, mode));
  const bool store = (p->d.flags & MDD_FLAG_STORE_RF) != 0;
  const float* vel = mode == TM_NSGD ? s0 : nullptr;
  const double mu = mode == TM_NSGD ? opt->mu : 0.0;
  const bool have = store && p->spec_model == R && p->spec_vel == vel && p->spec_mu == mu;
  p->spec_model = nullptr;
  if (!have) MDD_TRY(p->model_fft(R, vel, mu));
  MDD_TRY(p->full_products());
  a.model = R;
  a.store_spec = store ? 1 : 0;
  a.onset = p->mask_set ? p->onset() : nullptr;
  a.part = p->gnp();
  MDD_TRY(p->run(MDD_KC_UPDATE, [&] { return launch_trace(mode, a, p->stream); }));
  if (store) {  // the next point's spectra are where the gradient was: swap the buffers
    p->fswap = !p->fswap;
    p->spec_model = R;
    p->spec_vel = vel;
    p->spec_mu = mu;
  }
  return p->full_reduce(loss_out, gnorm2_out);
}

mdd_status mdd_reciprocity(const float* z, float* out, int32_t n, int32_t nt, void* stream) {
  if (!z || !out) return MDD_EINVAL;
  if ((reinterpret_cast<uintptr_t>(z) | reinterpret_cast<uintptr_t>(out)) & 15) return MDD_EINVAL;
  if (n < 1 || n > MAX_EXTENT || !valid_nt(nt)) return MDD_ESHAPE;
  return launch_reciprocity(z, out, n, nt, reinterpret_cast<hipStream_t>(stream)) == hipSuccess
             ? MDD_OK
             : MDD_EHIP;
}

mdd_status mdd_calibrate_update(float* R, float* s0, float* s1, float* spec, int32_t rows,
                                int32_t ncols, int32_t nt, int32_t nf, int32_t variant,
                                void* stream) {
  if (!R || !s0 || !s1 || !spec) return MDD_EINVAL;
  if ((reinterpret_cast<uintptr_t>(R) | reinterpret_cast<uintptr_t>(s0) |
       reinterpret_cast<uintptr_t>(s1) | reinterpret_cast<uintptr_t>(spec)) & 15)
    return MDD_EINVAL;
  if (variant < 0 || variant > 3) return MDD_EINVAL;
  if (rows < 1 || rows > MAX_EXTENT || ncols < 1 || ncols > MAX_EXTENT || !valid_nt(nt))
    return MDD_ESHAPE;
  if (nf < 1 || nf > nt / 2 + 1) return MDD_ESHAPE;
  return launch_calibrate_update(R, s0, s1, reinterpret_cast<float2*>(spec), rows, ncols, nt, nf,
                                 variant, reinterpret_cast<hipStream_t>(stream)) == hipSuccess
             ? MDD_OK
             : MDD_EHIP;
}

mdd_status mdd_calibrate_rows(const float* D, const int32_t* idx, float* out, int32_t nb,
                              int32_t nf, int32_t ns, int32_t nr, int32_t groups, void* stream) {
  if (!D || !idx || !out) return MDD_EINVAL;
  if ((reinterpret_cast<uintptr_t>(D) | reinterpret_cast<uintptr_t>(out)) & 15) return MDD_EINVAL;
  if (nb < 1 || nb > NB_LIMIT || ns < 1 || ns > MAX_STREAM_NS || nr < 1 || nr > MAX_EXTENT ||
      nf < 1 || nf > MAX_EXTENT / 2 + 1)
    return MDD_ESHAPE;
  if (groups == 0) groups = gemv_groups(nb, nf);
  if (groups < 1 || groups > nb) return MDD_ESHAPE;
  return launch_calibrate_rows(reinterpret_cast<const float2*>(D), idx, reinterpret_cast<float2*>(out),
                               nb, nf, ns, static_cast<int>(round16(nr)), groups,
                               reinterpret_cast<hipStream_t>(stream)) == hipSuccess
             ? MDD_OK
             : MDD_EHIP;
}

mdd_status mdd_check_batch_host(const int32_t* idx_host, int32_t nb, int32_t ns, int32_t nb_max) {
  if (!idx_host) return MDD_EINVAL;
  if (nb < 1 || nb > nb_max) return MDD_ESHAPE;
  for (int32_t b = 0; b < nb; ++b)
    if (idx_host[b] < 0 || idx_host[b] >= ns) return MDD_EINVAL;
  return MDD_OK;
}

mdd_status mdd_invalidate_model_spectra(mdd_plan* p) {
  if (!p) return MDD_EINVAL;
  p->spec_model = nullptr;
  return MDD_OK;
}

mdd_status mdd_sigma_max2(mdd_plan* p, int32_t iters, double* lam_out) {
  if (!p || !lam_out) return MDD_EINVAL;
  if (iters < 1) return MDD_EINVAL;
  if (!p->kernel_set || p->streamed()) return MDD_ESTATE;  // needs every source's D_k
  return p->run(MDD_KC_REDUCE, [&] {
    return launch_sigma(p->Df(), p->d.nf, p->d.ns, p->d.nr, p->nrp, iters, lam_out, p->stream);
  });
}

mdd_status mdd_profile_enable(mdd_plan* p, int32_t enable, int32_t capacity) {
  if (!p) return MDD_EINVAL;
  if (!enable) {
    p->prof = false;
    return MDD_OK;
  }
  if (capacity < 1) return MDD_EINVAL;
  if ((int)p->ev.size() < 2 * capacity) {
    const size_t have = p->ev.size();
    p->ev.resize(2 * (size_t)capacity, nullptr);
    for (size_t i = have; i < p->ev.size(); ++i) {
      const hipError_t e = hipEventCreate(&p->ev[i]);
      if (e != hipSuccess) {
        p->ev.resize(i);
        return p->fail(e);
      }
    }
  }
  p->cls.assign(capacity, 0);
  p->cap = capacity;
  p->nrec = 0;
  p->prof = true;
  return MDD_OK;
}

mdd_status mdd_profile_read(mdd_plan* p, double* ms_host, int64_t* count_host) {
  if (!p || !ms_host || !count_host) return MDD_EINVAL;
  for (int c = 0; c < MDD_KC_COUNT; ++c) {
    ms_host[c] = 0.0;
    count_host[c] = 0;
  }
  hipError_t e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return p->fail(e);
  for (int i = 0; i < p->nrec; ++i) {
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, p->ev[2 * i], p->ev[2 * i + 1]);
    if (e != hipSuccess) return p->fail(e);
    ms_host[p->cls[i]] += ms;
    count_host[p->cls[i]] += 1;
  }
  p->nrec = 0;
  return MDD_OK;
}

const char* mdd_status_string(mdd_status s) {
  switch (s) {
    case MDD_OK: return "ok";
    case MDD_EINVAL: return "invalid argument";
    case MDD_ESHAPE: return "inconsistent sizes";
    case MDD_ENOMEM: return "workspace missing, misaligned or too small";
    case MDD_EHIP: return "HIP runtime error";
    case MDD_EUNSUPPORTED: return "unsupported precision or optimiser";
    case MDD_ESTATE: return "kernel or data not set";
    case MDD_ELIMIT: return "sizes need more than the library's static workspace";
    default: return "unknown status";
  }
}

int32_t mdd_plan_last_hip_error(const mdd_plan* p) { return p ? p->last_hip : 0; }

}  // extern "C"
