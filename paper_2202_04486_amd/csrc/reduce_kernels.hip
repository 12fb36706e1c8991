// Float64 reductions (loss, gradient norm, out-of-band data energy), the
// per-frequency power iteration for the largest singular value of the kernel, and
// the small helpers: the reciprocity average (z + z^T) / 2, per-frequency maxima of
// D_k, the list of every source.  Every sum runs in a fixed order (no atomics), so
// results are bitwise reproducible run to run.
#include "device_common.h"
#include "mdd_internal.h"

namespace mdd {
namespace {

constexpr int RED_THREADS = 1024;

// loss = scale * sum(loss partials) + sum_b oob[idx[b]] (oob[b] for staged data);
// gnorm2 = sum(gnorm partials).
// The per-source constants are gathered by one thread each (no serial chain of
// dependent loads) and added in batch order.
__global__ __launch_bounds__(RED_THREADS) void k_reduce(ReduceArgs a) {
  __shared__ double red[RED_THREADS / 64];
  __shared__ double s_oob[NB_LIMIT];
  if (threadIdx.x < a.nb) {
    double o = 0.0;
    if (a.oob) {
      const int s = a.idx[threadIdx.x];
      if (s >= 0 && s < a.ns) o = a.oob[a.oob_pos ? threadIdx.x : s];
    }
    s_oob[threadIdx.x] = o;
  }
  const double l = block_fixed_sum<RED_THREADS>(a.loss_part, a.n_loss, red);
  const double g = block_fixed_sum<RED_THREADS>(a.gn_part, a.n_gn, red);
  if (threadIdx.x == 0) {
    double o = 0.0;
    for (int b = 0; b < a.nb; ++b) o += s_oob[b];
    if (a.loss_out) a.loss_out[0] = l * a.loss_scale + o;
    if (a.gnorm2_out) a.gnorm2_out[0] = g;
  }
}

// First level of a two-level sum for long partial arrays: block j of row y adds
// slice j of array y (y = 0: loss partials, 1: gradient-norm partials) in a fixed
// order.  The second level is k_reduce over the 2 * RED_SLICES results.
constexpr int RED_SLICES = 256;
__global__ __launch_bounds__(256) void k_presum(const double* loss_part, int n_loss, const double* gn_part,
                                                int n_gn, double* stage) {
  __shared__ double red[4];
  const double* p = blockIdx.y == 0 ? loss_part : gn_part;
  const int n = blockIdx.y == 0 ? n_loss : n_gn;
  const int per = (n + RED_SLICES - 1) / RED_SLICES;
  const int lo = min(n, (int)blockIdx.x * per), hi = min(n, lo + per);
  const double v = block_fixed_sum<256>(p + lo, hi - lo, red);
  if (threadIdx.x == 0) stage[blockIdx.y * RED_SLICES + blockIdx.x] = v;
}

__global__ void k_row_sum(const double* part, int rows, int cols, double scale, double* out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < rows) {
    double s = 0.0;
    for (int c = 0; c < cols; ++c) s += part[(size_t)r * cols + c];
    out[r] = s * scale;
  }
}

// Power iteration on D_k^H D_k (all ns sources) for one frequency per
// workgroup.  Returns the Rayleigh quotient ||D_k v||^2 of the final unit v.
__global__ __launch_bounds__(256) void k_sigma(const float2* Df, int ns, int nr, int nrp, int iters,
                                               double* lam_out) {
  extern __shared__ double smem_d[];
  double* vr = smem_d;            // [nr] real / imag of v (then of z)
  double* vi = vr + nr;
  double* yr = vi + nr;           // [ns]
  double* yi = yr + ns;
  __shared__ double red[4];
  __shared__ double bc;
  const int k = blockIdx.x;
  const float2* D = Df + (size_t)k * ns * nrp;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  double n2 = 0.0;
  for (int r = tid; r < nr; r += 256) {  // deterministic, non-degenerate start
    vr[r] = 1.0 + 0.25 * (double)((r * 37) % 11);
    vi[r] = 0.1 * (double)((r * 17) % 7);
    n2 += vr[r] * vr[r] + vi[r] * vi[r];
  }
  n2 = block_sum256(n2, red);
  if (tid == 0) bc = 1.0 / sqrt(n2);
  __syncthreads();
  for (int r = tid; r < nr; r += 256) {
    vr[r] *= bc;
    vi[r] *= bc;
  }
  __syncthreads();

  double lam = 0.0;
  for (int it = 0; it < iters; ++it) {
    double ynorm = 0.0;
    for (int s = wave; s < ns; s += 4) {  // y = D v
      double ar = 0.0, ai = 0.0;
      for (int r = lane; r < nr; r += 64) {
        const float2 d = D[(size_t)s * nrp + r];
        ar += (double)d.x * vr[r] - (double)d.y * vi[r];
        ai += (double)d.x * vi[r] + (double)d.y * vr[r];
      }
      ar = wave_sum(ar);
      ai = wave_sum(ai);
      if (lane == 0) {
        yr[s] = ar;
        yi[s] = ai;
        ynorm += ar * ar + ai * ai;
      }
    }
    ynorm = block_sum256(ynorm, red);
    if (tid == 0) bc = ynorm;
    __syncthreads();
    lam = bc;
    double z2 = 0.0;
    for (int r = tid; r < nr; r += 256) {  // z = D^H y, written over v
      double zr = 0.0, zi = 0.0;
      for (int s = 0; s < ns; ++s) {
        const float2 d = D[(size_t)s * nrp + r];
        zr += (double)d.x * yr[s] + (double)d.y * yi[s];
        zi += (double)d.x * yi[s] - (double)d.y * yr[s];
      }
      vr[r] = zr;
      vi[r] = zi;
      z2 += zr * zr + zi * zi;
    }
    z2 = block_sum256(z2, red);
    if (tid == 0) bc = z2 > 0.0 ? 1.0 / sqrt(z2) : 0.0;
    __syncthreads();
    for (int r = tid; r < nr; r += 256) {
      vr[r] *= bc;
      vi[r] *= bc;
    }
    __syncthreads();
  }
  if (tid == 0) lam_out[k] = lam;
}

// Largest |Re| or |Im| of D_k over all sources and receivers, per frequency (the
// fp16 split forms scale D_{b,k} by a power of two derived from it).  One
// workgroup per frequency; a maximum does not depend on the order.
// Largest |Re|, |Im| of the first `count` entries of each frequency's block (blocks
// `stride` entries apart).
__global__ __launch_bounds__(256) void k_freq_absmax(const float2* Df, long long count,
                                                     long long stride, float* out) {
  const float2* x = Df + (long long)blockIdx.x * stride;
  const long long per_freq = count;
  float m = 0.f;
  for (long long i = threadIdx.x; i < per_freq; i += 256) m = fmaxf(m, fmaxf(fabsf(x[i].x), fabsf(x[i].y)));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  __shared__ float s_m[4];
  if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = fmaxf(fmaxf(s_m[0], s_m[1]), fmaxf(s_m[2], s_m[3]));
}

// C_r z = (z + z^T) / 2 over the first two axes of [n][n][nt]: the workgroup of
// pair (r, vs), r <= vs, reads both traces and writes the average to both, so the
// call may run in place.
__global__ __launch_bounds__(256) void k_reciprocity(const float* z, float* out, int n, int nt) {
  const int vs = blockIdx.x, r = blockIdx.y;
  if (vs < r) return;
  const long long ta = ((long long)r * n + vs) * nt, tb = ((long long)vs * n + r) * nt;
  for (int i = threadIdx.x * 4; i < nt; i += 256 * 4) {
    const float4 a = *reinterpret_cast<const float4*>(z + ta + i);
    const float4 b = *reinterpret_cast<const float4*>(z + tb + i);
    const float4 m = make_float4((a.x + b.x) * 0.5f, (a.y + b.y) * 0.5f, (a.z + b.z) * 0.5f,
                                 (a.w + b.w) * 0.5f);
    *reinterpret_cast<float4*>(out + ta + i) = m;
    *reinterpret_cast<float4*>(out + tb + i) = m;
  }
}

// C_r on blocked spectra (nr = nvs = n): X(r, vs, k) <- (X(r, vs, k) + X(vs, r, k)) / 2 for
// every retained bin k, which equals the spectra of C_r applied to the traces (the time
// transform acts on each trace alone).  Element (r, vs, k) sits at
// r * s_row + (vs / 16) * s_cb + k * 16 + vs % 16.  Workgroup (pair, k) takes the 16 x 16
// tiles (I, J) and (J, I), I <= J, of bin k: both are read, transposed through LDS, and
// the average is written to both (a diagonal tile is its own mirror).  Receivers and
// columns at or beyond n are left alone.
__global__ __launch_bounds__(256) void k_spec_reciprocity(float2* X, int n, long long s_row,
                                                          long long s_cb, int ntile) {
  __shared__ float2 s_b[16][17];
  int p = blockIdx.x, I = 0;
  while (p >= ntile - I) {  // pair index -> (I, J), I <= J, row-major over the triangle
    p -= ntile - I;
    ++I;
  }
  const int J = I + p;
  const int k = blockIdx.y;
  const int i = threadIdx.x >> 4, j = threadIdx.x & 15;
  const int ra = I * 16 + i, ca = J * 16 + j;  // element of tile (I, J)
  const int rb = J * 16 + i, cb = I * 16 + j;  // element of tile (J, I)
  const bool oka = ra < n && ca < n, okb = rb < n && cb < n;
  float2* pa = X + (oka ? ra : 0) * s_row + (long long)J * s_cb + (long long)k * 16 + j;
  float2* pb = X + (okb ? rb : 0) * s_row + (long long)I * s_cb + (long long)k * 16 + j;
  const float2 a = oka ? *pa : make_float2(0.f, 0.f);
  const float2 b = okb ? *pb : make_float2(0.f, 0.f);
  s_b[i][j] = b;
  __syncthreads();
  // mirror of (ra, ca) = (I*16 + i, J*16 + j) is (J*16 + j, I*16 + i): element (j, i) of tile (J, I)
  const float2 m = s_b[j][i];
  const float2 v = make_float2((a.x + m.x) * 0.5f, (a.y + m.y) * 0.5f);
  __syncthreads();
  s_b[j][i] = v;  // the same value, as seen from tile (J, I)
  __syncthreads();
  if (oka) *pa = v;
  if (okb && I != J) *pb = s_b[i][j];
}

// out[i] = i: the list of every source, batched in order by the full gradient.
__global__ void k_iota(int32_t* out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = i;
}

}  // namespace

hipError_t launch_reduce(const ReduceArgs& a, hipStream_t s) {
  if (a.stage && (a.n_loss > RED_TWO_LEVEL || a.n_gn > RED_TWO_LEVEL)) {
    hipLaunchKernelGGL(k_presum, dim3(RED_SLICES, 2), dim3(256), 0, s, a.loss_part, a.n_loss,
                       a.gn_part, a.n_gn, a.stage);
    ReduceArgs b = a;
    b.loss_part = a.stage;
    b.n_loss = a.n_loss > 0 ? RED_SLICES : 0;
    b.gn_part = a.stage + RED_SLICES;
    b.n_gn = a.n_gn > 0 ? RED_SLICES : 0;
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(RED_THREADS), 0, s, b);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(RED_THREADS), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_reciprocity(const float* z, float* out, int n, int nt, hipStream_t s) {
  hipLaunchKernelGGL(k_reciprocity, dim3(n, n), dim3(256), 0, s, z, out, n, nt);
  return hipGetLastError();
}

hipError_t launch_spec_reciprocity(float2* X, int n, int nf, long long s_row, long long s_cb,
                                   hipStream_t s) {
  const int ntile = (n + 15) / 16;
  const int npair = ntile * (ntile + 1) / 2;
  if (n < 1 || nf < 1 || nf > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_spec_reciprocity, dim3(npair, nf), dim3(256), 0, s, X, n, s_row, s_cb, ntile);
  return hipGetLastError();
}

hipError_t launch_iota(int32_t* out, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_iota, dim3((n + 255) / 256), dim3(256), 0, s, out, n);
  return hipGetLastError();
}

hipError_t launch_freq_absmax(const float2* Df, int nf, long long count, long long stride,
                              float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_freq_absmax, dim3(nf), dim3(256), 0, s, Df, count, stride, out);
  return hipGetLastError();
}

hipError_t launch_row_sum(const double* part, int rows, int cols, double scale, double* out,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_row_sum, dim3((rows + 255) / 256), dim3(256), 0, s, part, rows, cols, scale,
                     out);
  return hipGetLastError();
}

hipError_t launch_sigma(const float2* Df, int nf, int ns, int nr, int nrp, int iters,
                        double* lam_out, hipStream_t s) {
  const size_t sm = sizeof(double) * 2 * ((size_t)nr + ns);
  if (sm > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sigma),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
  hipLaunchKernelGGL(k_sigma, dim3(nf), dim3(256), sm, s, Df, ns, nr, nrp, iters, lam_out);
  return hipGetLastError();
}

}  // namespace mdd
