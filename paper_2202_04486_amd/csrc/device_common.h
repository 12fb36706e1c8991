// Device helpers shared by the HIP kernels of the library.
#pragma once

#include <hip/hip_runtime.h>

namespace mdd {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Orders LDS traffic of one wavefront: every lane's earlier LDS writes are
// visible to every lane's later LDS reads (a wavefront executes in lockstep;
// the fences stop the compiler from moving accesses across this point).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Deterministic block sum of one double per thread (blockDim.x == 256);
// `red` is LDS of at least 4 doubles.  The result is valid in thread 0.
// Adjoint-product output at element `off` of the spectra layout: written over R_k
// in F (Gout NULL), or into Gout, or added to Gout (gacc: a sum over batches).
template <class GemmArgsT>
__device__ __forceinline__ void store_g(const GemmArgsT& a, long long off, float2 v) {
  float2* p = (a.Gout ? a.Gout : a.F) + off;
  if (a.gacc) v = cadd(v, *p);
  *p = v;
}

// Streaming (non-temporal) accesses for data a launch touches once, R_k read and G
// written by the product kernels, so that they do not evict the kernel rows D_b, which
// every column group of a frequency reads again.
typedef float stream_f4 __attribute__((ext_vector_type(4)));
typedef float stream_f2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float4 stream_load4(const float2* p) {
  const stream_f4 v = __builtin_nontemporal_load(reinterpret_cast<const stream_f4*>(p));
  return make_float4(v[0], v[1], v[2], v[3]);
}
// store_g for the plain case (written over R_k in F) as a streaming store.
template <class GemmArgsT>
__device__ __forceinline__ void store_g_stream(const GemmArgsT& a, long long off, float2 v) {
  if (a.gacc || a.Gout) {
    store_g(a, off, v);
  } else {
    __builtin_nontemporal_store(stream_f2{v.x, v.y}, reinterpret_cast<stream_f2*>(a.F + off));
  }
}

// Row of D_k for batch entry b whose source s is valid: s in the resident spectra,
// b in spectra staged for the batch.
template <class GemmArgsT>
__device__ __forceinline__ int drow_of(const GemmArgsT& a, int b, int s) {
  return a.dpos ? b : s;
}

// Offset of row (k, .) of U_k for batch entry b with source s: row s of the resident
// data spectra, or row b of data spectra staged for the batch.  Callers pass b < nb.
template <class GemmArgsT>
__device__ __forceinline__ long long urow_off(const GemmArgsT& a, int k, int b, int s) {
  return ((long long)k * a.uns + (a.upos ? b : s)) * a.nvsp;
}

__device__ __forceinline__ double block_sum256(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) s = ((red[0] + red[1]) + red[2]) + red[3];
  return s;
}

// Sum of n doubles by one workgroup of NTH threads in a fixed order (four
// independent loads per thread per round, then a fixed tree): bitwise
// reproducible.  `red` is LDS of NTH / 64 doubles; the result is in thread 0.
template <int NTH>
__device__ __forceinline__ double block_fixed_sum(const double* p, int n, double* red) {
  double acc = 0.0;
  int i = threadIdx.x;
  for (; i + 3 * NTH < n; i += 4 * NTH) {
    const double x0 = p[i], x1 = p[i + NTH], x2 = p[i + 2 * NTH], x3 = p[i + 3 * NTH];
    acc += (x0 + x1) + (x2 + x3);
  }
  for (; i < n; i += NTH) acc += p[i];
  acc = wave_sum(acc);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = acc;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < NTH / 64; ++w) s += red[w];
  return s;
}

}  // namespace mdd
