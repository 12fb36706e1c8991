// Measurement aid: the HBM traffic of the update kernel without its arithmetic.
//
// The Adam update kernel (inverse transform of the gradient spectra, mask, update,
// transform of the next model) reads and writes the model and both moments in place
// and reads and writes one block of spectra in place.  k_cal_update moves exactly
// those bytes with the same grid, the same workgroup -> (tile, half-block) mapping,
// the same spectra staging through LDS and, in its first variant, the same per-lane
// accesses (lane j of a trace owns float2 elements j + L r), but with a trivial
// update in place of the transforms.  Its time is therefore a floor for the update
// kernel's time on this device, set by the memory system alone.  Two other layouts
// of the same bytes are measured beside it: 16 bytes per lane, and flat streams over
// whole arrays (the fastest form a plain elementwise kernel takes here).
//
// The products for one virtual source are bound by one pass over the batch's kernel
// rows.  k_cal_rows reads exactly those rows (the rows idx[b] of every frequency) with
// the grid of the matrix-vector kernel (nf x groups workgroups, a frequency's groups on
// one XCD, a thread's receiver pairs tid + 256 m), but with no reduction, residual or
// barrier between rows, and writes the same group partials; its time is the floor of
// that access pattern.
#include "device_common.h"
#include "mdd_internal.h"

namespace mdd {
namespace {

typedef float cal2 __attribute__((ext_vector_type(2)));
typedef float cal4 __attribute__((ext_vector_type(4)));

// Grid geometry of the update kernel at NT: 64-lane waves, L = NT / 16 lanes per
// trace; half of a 16-column block per workgroup for NT >= 512.
template <int NT>
struct CalCfg {
  static constexpr int L = NT / 16;
  static constexpr int TPW = 64 / L;
  static constexpr int SPLIT = NT >= 512 ? 2 : 1;
  static constexpr int CW = CB / SPLIT;
  static constexpr int NWAVES = NT == 1024 ? 8 / SPLIT : CW / TPW;
  static constexpr int ITERS = CW / (NWAVES * TPW);
  static constexpr int THREADS = 64 * NWAVES;
  static constexpr int SPS = CW + 1;
  static_assert(ITERS * NWAVES * TPW == CW, "tile");
};

struct CalArgs {
  float *R, *M, *V;
  float2* spec;
  int rows, ncols, ncb, nf;
};

template <int W>
__device__ __forceinline__ void cal_load(const float* p, float* o) {
  if constexpr (W == 2) {
    const cal2 v = __builtin_nontemporal_load(reinterpret_cast<const cal2*>(p));
    o[0] = v.x;
    o[1] = v.y;
  } else {
    const cal4 v = __builtin_nontemporal_load(reinterpret_cast<const cal4*>(p));
    o[0] = v.x;
    o[1] = v.y;
    o[2] = v.z;
    o[3] = v.w;
  }
}

template <int W>
__device__ __forceinline__ void cal_store(float* p, const float* o) {
  if constexpr (W == 2) {
    const cal2 v = {o[0], o[1]};
    __builtin_nontemporal_store(v, reinterpret_cast<cal2*>(p));
  } else {
    const cal4 v = {o[0], o[1], o[2], o[3]};
    __builtin_nontemporal_store(v, reinterpret_cast<cal4*>(p));
  }
}

// W floats per lane access: 2 (the update kernel's layout) or 4.
template <int NT, int W>
__global__ __launch_bounds__(CalCfg<NT>::THREADS) void k_cal_update(CalArgs a) {
  using C = CalCfg<NT>;
  constexpr int L = C::L, TPW = C::TPW, NW = C::NWAVES, CW = C::CW, SPS = C::SPS;
  constexpr int PER = NT / (L * W);  // accesses per lane and array
  extern __shared__ float2 s_spec[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int p = lane / L, j = lane % L;
  int tile = blockIdx.x, half = 0;
  if constexpr (C::SPLIT > 1) {  // the update kernel's mapping: both halves on one XCD
    const int g = blockIdx.x / (8 * C::SPLIT), w = blockIdx.x % (8 * C::SPLIT);
    const int m = min(8, a.rows * a.ncb - 8 * g);
    tile = 8 * g + w % m;
    half = w / m;
  }
  const int row = tile / a.ncb, cb = tile % a.ncb, nf = a.nf;
  float2* gspec = a.spec + ((long long)row * a.ncb + cb) * nf * CB + half * CW;
  for (int i = tid; i < nf * (CW / 2); i += C::THREADS) {
    const int k = i / (CW / 2), c2 = 2 * (i % (CW / 2));
    const float4 z = *reinterpret_cast<const float4*>(gspec + k * CB + c2);
    s_spec[k * SPS + c2] = make_float2(z.x, z.y);
    s_spec[k * SPS + c2 + 1] = make_float2(z.z, z.w);
  }
  __syncthreads();
#pragma unroll 1
  for (int it = 0; it < C::ITERS; ++it) {
    const int c = it * NW * TPW + wave * TPW + p;
    const int col = cb * CB + half * CW + c;
    if (col < a.ncols) {
      const long long base = ((long long)row * a.ncols + col) * NT;
      const float g0 = s_spec[(j % nf) * SPS + c].x;
      float r[PER][W], m[PER][W], v[PER][W];
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const long long o = base + (long long)(j + L * q) * W;
        cal_load<W>(a.R + o, r[q]);
        cal_load<W>(a.M + o, m[q]);
        cal_load<W>(a.V + o, v[q]);
      }
#pragma unroll
      for (int q = 0; q < PER; ++q)
#pragma unroll
        for (int e = 0; e < W; ++e) {
          const float g = g0 + 0.5f * r[q][e];
          m[q][e] = 0.9f * m[q][e] + 0.1f * g;
          v[q][e] = 0.999f * v[q][e] + 0.001f * g * g;
          r[q][e] -= 1e-3f * m[q][e] * __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(v[q][e]) + 1e-8f);
        }
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const long long o = base + (long long)(j + L * q) * W;
        cal_store<W>(a.R + o, r[q]);
        cal_store<W>(a.M + o, m[q]);
        cal_store<W>(a.V + o, v[q]);
      }
    }
  }
  __syncthreads();
  for (int i = tid; i < nf * (CW / 2); i += C::THREADS) {
    const int k = i / (CW / 2), c2 = 2 * (i % (CW / 2));
    const float2 z0 = s_spec[k * SPS + c2], z1 = s_spec[k * SPS + c2 + 1];
    *reinterpret_cast<float4*>(gspec + k * CB + c2) =
        make_float4(0.5f * z0.x, z0.y, z1.x, z1.y);
  }
}

// Flat streams: each thread two float2 of each state array (the best in-place layout
// of a plain elementwise kernel here), then the spectra as float4, two per thread.
__global__ __launch_bounds__(256) void k_cal_flat_state(float* R, float* M, float* V,
                                                        long long n2) {
  const long long i0 = (long long)blockIdx.x * 512 + threadIdx.x;
  cal2 r[2], m[2], v[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const long long i = i0 + 256LL * u;
    if (i < n2) {
      r[u] = __builtin_nontemporal_load(reinterpret_cast<const cal2*>(R) + i);
      m[u] = __builtin_nontemporal_load(reinterpret_cast<const cal2*>(M) + i);
      v[u] = __builtin_nontemporal_load(reinterpret_cast<const cal2*>(V) + i);
    }
  }
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const long long i = i0 + 256LL * u;
    if (i < n2) {
      m[u] = 0.9f * m[u] + 0.1f * r[u];
      v[u] = 0.999f * v[u] + 0.001f * r[u] * r[u];
      r[u] = r[u] - 1e-3f * m[u];
      __builtin_nontemporal_store(r[u], reinterpret_cast<cal2*>(R) + i);
      __builtin_nontemporal_store(m[u], reinterpret_cast<cal2*>(M) + i);
      __builtin_nontemporal_store(v[u], reinterpret_cast<cal2*>(V) + i);
    }
  }
}

__global__ __launch_bounds__(256) void k_cal_flat_spec(float* S, long long n4) {
  const long long i0 = (long long)blockIdx.x * 512 + threadIdx.x;
  cal4 x[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const long long i = i0 + 256LL * u;
    if (i < n4) x[u] = __builtin_nontemporal_load(reinterpret_cast<const cal4*>(S) + i);
  }
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const long long i = i0 + 256LL * u;
    if (i < n4) {
      x[u].x *= 0.5f;
      __builtin_nontemporal_store(x[u], reinterpret_cast<cal4*>(S) + i);
    }
  }
}

// Rows idx[b] of D_k for the batch entries of group p of frequency k (group size
// ceil(nb / groups)), each thread summing its receiver pairs over the rows, four rows
// in flight; then one partial per (k, p, pair).
template <int MQ>
__global__ __launch_bounds__(256) void k_cal_rows(const float4* __restrict__ D, const int* idx,
                                                  float4* out, int nb, int nf, int ns, int npair,
                                                  int groups) {
  const int total = nf * groups, bid = blockIdx.x, full = (total / 8) * 8;
  const int logical = bid < full ? (bid % 8) * (total / 8) + bid / 8 : bid;
  const int k = logical / groups, p = logical % groups;
  const int rpg = (nb + groups - 1) / groups;
  const int i0 = p * rpg, i1 = min(nb, i0 + rpg);
  const int tid = threadIdx.x;
  cal4 acc[MQ];
#pragma unroll
  for (int m = 0; m < MQ; ++m) acc[m] = cal4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
  for (int i = i0; i < i1; ++i) {
    int sidx = idx[i];
    if (sidx < 0 || sidx >= ns) sidx = 0;
    const float4* row = D + ((long long)k * ns + sidx) * npair;
#pragma unroll
    for (int m = 0; m < MQ; ++m) {
      const int q = tid + 256 * m;
      const float4 v = row[q < npair ? q : npair - 1];
      acc[m] += cal4{v.x, v.y, v.z, v.w};
    }
  }
#pragma unroll
  for (int m = 0; m < MQ; ++m) {
    const int q = tid + 256 * m;
    if (q < npair) {
      const cal4 v = acc[m];
      out[((long long)k * groups + p) * npair + q] = make_float4(v.x, v.y, v.z, v.w);
    }
  }
}

template <int NT, int W>
hipError_t launch_cal(const CalArgs& a, hipStream_t s) {
  using C = CalCfg<NT>;
  const size_t sm = sizeof(float2) * (size_t)a.nf * C::SPS;
  if (sm > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_cal_update<NT, W>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
  hipLaunchKernelGGL((k_cal_update<NT, W>), dim3(a.rows * a.ncb * C::SPLIT), dim3(C::THREADS),
                     sm, s, a);
  return hipGetLastError();
}

template <int NT>
hipError_t launch_cal_nt(int variant, const CalArgs& a, hipStream_t s) {
  return variant == 0 ? launch_cal<NT, 2>(a, s) : launch_cal<NT, 4>(a, s);
}

}  // namespace

hipError_t launch_calibrate_update(float* R, float* M, float* V, float2* spec, int rows,
                                   int ncols, int nt, int nf, int variant, hipStream_t s) {
  CalArgs a{R, M, V, spec, rows, ncols, nblocks(ncols), nf};
  if (variant == 3) {  // the spectra alone, as a flat stream
    const long long n4 = (long long)rows * a.ncb * nf * CB / 2;
    hipLaunchKernelGGL(k_cal_flat_spec, dim3((unsigned)((n4 + 511) / 512)), dim3(256), 0, s,
                       reinterpret_cast<float*>(spec), n4);
    return hipGetLastError();
  }
  if (variant == 2) {
    const long long n2 = (long long)rows * ncols * nt / 2;
    const long long n4 = (long long)rows * a.ncb * nf * CB / 2;
    hipLaunchKernelGGL(k_cal_flat_state, dim3((unsigned)((n2 + 511) / 512)), dim3(256), 0, s, R, M,
                       V, n2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cal_flat_spec, dim3((unsigned)((n4 + 511) / 512)), dim3(256), 0, s,
                       reinterpret_cast<float*>(spec), n4);
    return hipGetLastError();
  }
  switch (nt) {
    case 128: return launch_cal_nt<128>(variant, a, s);
    case 256: return launch_cal_nt<256>(variant, a, s);
    case 512: return launch_cal_nt<512>(variant, a, s);
    case 1024: return launch_cal_nt<1024>(variant, a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_calibrate_rows(const float2* D, const int32_t* idx, float2* out, int nb, int nf,
                                 int ns, int nrp, int groups, hipStream_t s) {
  const int npair = nrp / 2;
  const dim3 grid(nf * groups), block(256);
  const float4* D4 = reinterpret_cast<const float4*>(D);
  float4* o4 = reinterpret_cast<float4*>(out);
  if (npair <= 256) hipLaunchKernelGGL(k_cal_rows<1>, grid, block, 0, s, D4, idx, o4, nb, nf, ns, npair, groups);
  else if (npair <= 512) hipLaunchKernelGGL(k_cal_rows<2>, grid, block, 0, s, D4, idx, o4, nb, nf, ns, npair, groups);
  else if (npair <= 1024) hipLaunchKernelGGL(k_cal_rows<4>, grid, block, 0, s, D4, idx, o4, nb, nf, ns, npair, groups);
  else if (npair <= 2048) hipLaunchKernelGGL(k_cal_rows<8>, grid, block, 0, s, D4, idx, o4, nb, nf, ns, npair, groups);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace mdd
