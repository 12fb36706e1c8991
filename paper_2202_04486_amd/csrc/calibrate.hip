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

}  // namespace mdd
