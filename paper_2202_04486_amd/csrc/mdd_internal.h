// Internal declarations shared by the host layer (api.cpp) and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "mdd.h"

namespace mdd {

// Frequency-domain traces are stored in blocks of CB consecutive columns
// (virtual sources, or receivers for the kernel); a block of one row holds
// [nf][CB] complex values, 128 bytes per frequency.
constexpr int CB = 16;
constexpr int NB_LIMIT = 64;  // largest batch: D_b rows and residuals live in LDS

enum TraceMode : int {
  TM_RFFT = 0,        // time -> spectra (+ optional out-of-band energy)
  TM_IRFFT = 1,       // spectra -> time
  TM_GRAD = 2,        // spectra -> time, mask, ||g||^2
  TM_SGD = 3,         // spectra -> gradient -> SGD update of the model
  TM_ADAM = 4,        // ... Adam update
  TM_NSGD = 5,        // ... Nesterov-momentum update
};

struct ReduceArgs {
  const double* loss_part;
  int n_loss;
  double loss_scale;      // 1 / (2 nt)
  const double* oob;      // [ns] per-source out-of-band energy (already / (2 nt))
  const int32_t* idx;
  int nb, ns;
  int oob_pos;            // 1: oob[b] for batch entry b (staged data), else oob[idx[b]]
  const double* gn_part;
  int n_gn;
  double* loss_out;
  double* gnorm2_out;
  double* stage;          // [2 * 256] for the two-level sum of long partial arrays
};

// Partial arrays longer than this are summed in two levels (fixed order either way).
constexpr int RED_TWO_LEVEL = 32768;

// One launch of the trace kernel: a grid of tiles, tile (row, cb) holding the
// traces (row, cb*CB + c), c < CB, of a [rows][ncols][nt] time-domain array.
// Spectral element (row, cb, k, c) lives at spec[row*s_row + cb*s_cb + k*s_k + c].
struct TraceArgs {
  int nt, nf, rows, ncols, ncb;
  const float* x_in;      // TM_RFFT input
  const float* x_in2;     // TM_RFFT: optional second input, transformed is x_in + mu2 * x_in2
  float mu2;
  float* x_out;           // TM_IRFFT / TM_GRAD output
  float2* spec;
  long long s_row, s_cb, s_k;
  float* model;           // update modes: R (in place)
  float* st0;             // first optimiser state (Adam m / Nesterov velocity)
  float* st1;             // second optimiser state (Adam v)
  float lr, beta1, beta2, eps, mu, inv_bc1, inv_bc2;
  float omb1, omb2;       // 1 - beta1, 1 - beta2 rounded once from double
  int store_spec;         // update modes: write spectra of the next evaluation point
  const int32_t* onset;   // [rows][ncols] or NULL
  double* part;           // per-tile float64 partial: out-of-band energy or ||g||^2
  const float2* tw;       // exp(-2 pi i m / nt), m < nt
};

enum GemmKind : int {
  GK_FUSED = 0,   // Res = D_b R_k - U_b (loss partials); G_k = D_b^H Res, written over R_k
  GK_FWD = 1,     // P_k = D_b R_k -> batch spectra
  GK_ADJ = 2,     // G_k = D_b^H V_k, V from batch spectra
};

struct GemmArgs {
  const float2* Df;       // [nf][ns][nrp]
  const float2* Uf;       // [nf][ns][nvsp]
  float2* F;              // [nr][nvb][nf][CB]   model / gradient spectra
  float2* Bsp;            // [nb][nvb][nf][CB]   batch spectra
  const int32_t* idx;
  double* loss_part;      // [gridDim.x * gridDim.y]
  const float* dmax;      // [nf] largest |Re|, |Im| of D_k (fp16 split forms; else NULL)
  float2* Gout;           // adjoint product destination (same layout as F); NULL: over R_k in F
  int gacc;               // 1: add the adjoint product to Gout instead of writing it
  int ns, nr, nrp, nvs, nvsp, nvb, nf, nt, nb;
  // Rows of D per frequency in Df (ns, or nb_max for staged batch rows) and where batch
  // entry b finds its row: 0 = row idx[b] (resident spectra), 1 = row b (staged).
  int dns, dpos;
  // The same for the rows of U_k (uns rows per frequency; upos 1 = staged row b).
  int uns, upos;
  // Single virtual source (launch_gemv): row groups per frequency and their adjoint
  // partials [nf][P][nrp / 2] (receiver pairs).
  int P;
  float4* gpart;
};

hipError_t launch_twiddles(float2* tw, int nt, hipStream_t s);
hipError_t launch_trace(int mode, const TraceArgs& a, hipStream_t s);
// Workgroups per 16-column block in the gradient / update modes at this nt; each
// writes one float64 partial, so those launches write rows * ncb * split partials.
int trace_update_split(int nt);
hipError_t launch_gemm(int kind, int precision, const GemmArgs& a, hipStream_t s);
// bf16x3 / fp16x3 products (gemm_split.hip): 16 < nb <= NB_LIMIT, or the fused kind
// at nb <= 16 over at most SPLIT_PIPE_KC receivers (persistent kernel).
constexpr int SPLIT_PIPE_KC = 256;
hipError_t launch_gemm_split(int kind, int precision, const GemmArgs& a, hipStream_t s);
// nvs = 1 products (gemv_kernels.hip): every kind, every precision, in float32; spectra
// in the one-row layout.  a.P = gemv_groups(nb, nf) row groups per frequency; with P > 1
// the adjoint kinds take a second launch that adds the group partials.
int gemv_groups(int nb, int nf);
hipError_t launch_gemv(int kind, const GemmArgs& a, hipStream_t s);
hipError_t launch_reduce(const ReduceArgs& a, hipStream_t s);
hipError_t launch_row_sum(const double* part, int rows, int cols, double scale, double* out,
                          hipStream_t s);
hipError_t launch_iota(int32_t* out, int n, hipStream_t s);
hipError_t launch_reciprocity(const float* z, float* out, int n, int nt, hipStream_t s);
hipError_t launch_spec_reciprocity(float2* X, int n, int nf, long long s_row, long long s_cb,
                                   hipStream_t s);
hipError_t launch_freq_absmax(const float2* Df, int nf, long long count, long long stride,
                              float* out, hipStream_t s);
hipError_t launch_sigma(const float2* Df, int nf, int ns, int nr, int nrp, int iters,
                        double* lam_out, hipStream_t s);

// Measurement aid (calibrate.hip): the update kernel's HBM traffic without its transforms.
hipError_t launch_calibrate_update(float* R, float* M, float* V, float2* spec, int rows,
                                   int ncols, int nt, int nf, int variant, hipStream_t s);
// Measurement aid (calibrate.hip): the batch's kernel rows [nf][ns][nrp] read with the
// matrix-vector kernel's grid and no arithmetic; out holds nf * groups * nrp / 2 float4.
hipError_t launch_calibrate_rows(const float2* D, const int32_t* idx, float2* out, int nb, int nf,
                                 int ns, int nrp, int groups, hipStream_t s);

// The library's static workspace (noalloc.hip): its size, and its address on `device`,
// which must be the current device (looked up once per device, then cached).
size_t static_workspace_bytes();
hipError_t static_workspace(int device, void** out);

// Blocks of ncols columns.
inline int nblocks(int ncols) { return (ncols + CB - 1) / CB; }
inline int round16(int n) { return nblocks(n) * CB; }

}  // namespace mdd
