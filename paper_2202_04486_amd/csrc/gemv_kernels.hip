// Products for a single virtual source (nvs = 1): at each retained frequency the
// operator's matrix-matrix product reduces to a matrix-vector product (cost analysis,
// Appendix A), so D_b is the only large operand and the work is bound by its bytes.
//
//   k_gemv<GK_FUSED>  res_i = D_{b,k}[i, :] . r_k - U_{b,k}[i]  (float64 loss partials),
//                     g_k += conj(D_{b,k}[i, :]) res_i  over the rows i of the workgroup
//   k_gemv<GK_FWD>    P_k[i] = D_{b,k}[i, :] . r_k  -> batch spectra
//   k_gemv<GK_ADJ>    g_k = sum_i conj(D_{b,k}[i, :]) V_k[i], V from batch spectra
//
// One pass over D_b: each row of D_{b,k} is loaded once into registers, reduced to
// res_i across the workgroup and, still in registers, multiplied into the adjoint sum.
// The rows of one frequency are split into P groups (one workgroup each) so that the
// grid covers the chip; with P > 1 the group partials of g_k go to a scratch buffer and
// k_gemv_sum adds them in group order (a second launch: a device-scope fence per
// workgroup, needed for a last-group-sums scheme, writes back the whole L2 on this
// chip and costs more than the launch).
//
// Layout at nvs = 1 (the trace kernels see one row of nr columns): model and gradient
// spectra hold receiver j at frequency k at ((j / 16) * nf + k) * 16 + j % 16; batch
// spectra hold batch row i at ((i / 16) * nf + k) * 16 + i % 16.  Arithmetic is float32
// on the vector units for every precision setting: the product is bound by D_b's bytes.
#include "device_common.h"
#include "mdd_internal.h"

namespace mdd {
namespace {

constexpr int GV_THREADS = 256;
constexpr int GV_GR = 2;  // rows reduced per workgroup barrier

__device__ __forceinline__ float2 wave_sum2(float2 v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    v.x += __shfl_xor(v.x, off, 64);
    v.y += __shfl_xor(v.y, off, 64);
  }
  return v;
}

// g += conj(d) * s for the two complex values of d.
__device__ __forceinline__ void cmac_conj(float4& g, float4 d, float2 s) {
  g.x += d.x * s.x + d.y * s.y;
  g.y += d.x * s.y - d.y * s.x;
  g.z += d.z * s.x + d.w * s.y;
  g.w += d.z * s.y - d.w * s.x;
}

// Adjoint product for receivers 2q, 2q + 1 at frequency k: written over R_k in F (Gout
// NULL), or into Gout, or added to Gout (gacc), in the one-row spectra layout.
__device__ __forceinline__ void store_pair(const GemmArgs& a, int k, int q, float4 v) {
  const int c = 2 * q;
  float4* dst = reinterpret_cast<float4*>(a.Gout ? a.Gout : a.F) +
                ((((long long)(c >> 4) * a.nf + k) * CB + (c & 15)) >> 1);
  if (a.gacc) {
    const float4 o = *dst;
    v.x += o.x;
    v.y += o.y;
    v.z += o.z;
    v.w += o.w;
  }
  *dst = v;
}

template <int KIND, int MQ>
__global__ __launch_bounds__(GV_THREADS) void k_gemv(GemmArgs a) {
  __shared__ float2 s_red[2][GV_GR][GV_THREADS / 64];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // The P groups of one frequency run on one XCD (dispatch is round-robin over the 8).
  const int total = a.nf * a.P;
  const int bid = blockIdx.x;
  const int full = (total / 8) * 8;
  const int logical = bid < full ? (bid % 8) * (total / 8) + bid / 8 : bid;
  const int k = logical / a.P, p = logical % a.P;
  const int rpg = (a.nb + a.P - 1) / a.P;
  const int i0 = p * rpg;
  const int i1 = min(a.nb, i0 + rpg);
  const int npair = a.nrp / 2;  // receiver pairs (2q, 2q + 1), zero-padded to nrp
  const double wk = (k == 0 || 2 * k == a.nt) ? 1.0 : 2.0;

  const float4* D4 = reinterpret_cast<const float4*>(a.Df);
  // Spectra element (column c, frequency k) of the one-row layout, c even -> float4 index.
  auto spec4 = [&](int c) -> long long { return (((long long)(c >> 4) * a.nf + k) * CB + (c & 15)) >> 1; };
  auto spec2 = [&](int c) -> long long { return ((long long)(c >> 4) * a.nf + k) * CB + (c & 15); };

  // Model spectra r_k: pairs q = tid + 256 m (zero beyond the padded receivers).
  float4 rv[MQ];
  float4 gv[MQ];
#pragma unroll
  for (int m = 0; m < MQ; ++m) {
    const int q = tid + GV_THREADS * m;
    gv[m] = make_float4(0.f, 0.f, 0.f, 0.f);
    rv[m] = make_float4(0.f, 0.f, 0.f, 0.f);
    if constexpr (KIND != GK_ADJ) {
      const int qc = q < npair ? q : npair - 1;
      const float4 v = reinterpret_cast<const float4*>(a.F)[spec4(2 * qc)];
      rv[m] = q < npair ? v : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }

  double lpart = 0.0;
  int par = 0;
#pragma unroll 1
  for (int i = i0; i < i1; i += GV_GR, par ^= 1) {
    int src[GV_GR];
    float4 dv[GV_GR][MQ];
#pragma unroll
    for (int r = 0; r < GV_GR; ++r) {
      const int ii = i + r;
      int s = ii < i1 ? a.idx[ii] : -1;
      if (s < 0 || s >= a.ns) s = -1;
      src[r] = s;
      const long long row = ((long long)k * a.dns + (s < 0 ? 0 : drow_of(a, ii, s))) * (a.nrp / 2);
#pragma unroll
      for (int m = 0; m < MQ; ++m) {
        const int q = tid + GV_THREADS * m;
        dv[r][m] = D4[row + (q < npair ? q : npair - 1)];
      }
    }
    float2 res[GV_GR];
    if constexpr (KIND == GK_ADJ) {
#pragma unroll
      for (int r = 0; r < GV_GR; ++r) {
        const int ii = i + r;
        const float2 v = a.Bsp[spec2(ii < i1 ? ii : i)];
        res[r] = src[r] >= 0 ? v : make_float2(0.f, 0.f);
      }
    } else {
#pragma unroll
      for (int r = 0; r < GV_GR; ++r) {
        float2 acc = make_float2(0.f, 0.f);
#pragma unroll
        for (int m = 0; m < MQ; ++m) {
          const float4 d = dv[r][m], x = rv[m];
          acc.x += d.x * x.x - d.y * x.y;
          acc.y += d.x * x.y + d.y * x.x;
          acc.x += d.z * x.z - d.w * x.w;
          acc.y += d.z * x.w + d.w * x.z;
        }
        acc = wave_sum2(acc);
        if (lane == 0) s_red[par][r][wave] = acc;
      }
      __syncthreads();  // the other buffer (par ^ 1) is free again after this barrier
#pragma unroll
      for (int r = 0; r < GV_GR; ++r) {
        float2 z = s_red[par][r][0];
#pragma unroll
        for (int w = 1; w < GV_THREADS / 64; ++w) z = cadd(z, s_red[par][r][w]);
        const int ii = i + r;
        if constexpr (KIND == GK_FUSED) {
          if (src[r] >= 0) {
            z = csub(z, a.Uf[urow_off(a, k, ii, src[r])]);
            lpart += wk * ((double)z.x * z.x + (double)z.y * z.y);
          } else {
            z = make_float2(0.f, 0.f);
          }
        } else {
          if (tid == 0 && ii < i1) a.Bsp[spec2(ii)] = src[r] >= 0 ? z : make_float2(0.f, 0.f);
        }
        res[r] = z;
      }
    }
    if constexpr (KIND != GK_FWD) {
#pragma unroll
      for (int r = 0; r < GV_GR; ++r)
#pragma unroll
        for (int m = 0; m < MQ; ++m) cmac_conj(gv[m], dv[r][m], res[r]);
    }
  }

  if constexpr (KIND == GK_FUSED) {
    if (tid == 0) a.loss_part[logical] = lpart;
  }
  if constexpr (KIND == GK_FWD) return;

  // Adjoint product of this group's rows -> G (P == 1) or the group partial.
#pragma unroll
  for (int m = 0; m < MQ; ++m) {
    const int q = tid + GV_THREADS * m;
    if (q >= npair) continue;
    if (a.P == 1)
      store_pair(a, k, q, gv[m]);
    else
      a.gpart[((long long)k * a.P + p) * npair + q] = gv[m];
  }
}

// G_k for receiver pairs q: the P group partials added in group order.
__global__ __launch_bounds__(GV_THREADS) void k_gemv_sum(GemmArgs a) {
  const int npair = a.nrp / 2;
  const int nqb = (npair + GV_THREADS - 1) / GV_THREADS;
  const int k = blockIdx.x / nqb;
  const int q = (blockIdx.x % nqb) * GV_THREADS + threadIdx.x;
  if (q >= npair) return;
  const float4* part = a.gpart + (long long)k * a.P * npair + q;
  float4 s = part[0];
  for (int g = 1; g < a.P; ++g) {
    const float4 v = part[(long long)g * npair];
    s.x += v.x;
    s.y += v.y;
    s.z += v.z;
    s.w += v.w;
  }
  store_pair(a, k, q, s);
}

template <int KIND, int MQ>
hipError_t launch_kind(const GemmArgs& a, hipStream_t s) {
  hipLaunchKernelGGL((k_gemv<KIND, MQ>), dim3(a.nf * a.P), dim3(GV_THREADS), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || KIND == GK_FWD || a.P == 1) return e;
  const int nqb = (a.nrp / 2 + GV_THREADS - 1) / GV_THREADS;
  hipLaunchKernelGGL(k_gemv_sum, dim3(a.nf * nqb), dim3(GV_THREADS), 0, s, a);
  return hipGetLastError();
}

template <int MQ>
hipError_t launch_mq(int kind, const GemmArgs& a, hipStream_t s) {
  switch (kind) {
    case GK_FUSED: return launch_kind<GK_FUSED, MQ>(a, s);
    case GK_FWD: return launch_kind<GK_FWD, MQ>(a, s);
    case GK_ADJ: return launch_kind<GK_ADJ, MQ>(a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int gemv_groups(int nb, int nf) {
  const int most = (nb + 7) / 8;                 // at least 8 rows per group
  int want = (3 * 256 + nf - 1) / nf;            // about three workgroups per CU,
  if (want < 4) want = 4;                        // and at least four groups
  return want < most ? want : most;
}

hipError_t launch_gemv(int kind, const GemmArgs& a, hipStream_t s) {
  if (a.nb < 1 || a.nb > NB_LIMIT || a.nvs != 1 || a.P < 1) return hipErrorInvalidValue;
  if (a.P > 1 && !a.gpart) return hipErrorInvalidValue;
  const int pairs = a.nrp / 2;
  if (pairs <= 1 * GV_THREADS) return launch_mq<1>(kind, a, s);
  if (pairs <= 2 * GV_THREADS) return launch_mq<2>(kind, a, s);
  if (pairs <= 4 * GV_THREADS) return launch_mq<4>(kind, a, s);
  if (pairs <= 8 * GV_THREADS) return launch_mq<8>(kind, a, s);
  return hipErrorInvalidValue;
}

}  // namespace mdd
