// Split-precision (bf16x3, fp16x3) per-frequency products:
//   k_gemm_spipe     fused kind, nb <= 16: persistent, like the fp32 k_gemm_pipe;
//   k_gemm_split     tiled, every kind, 16 < nb <= 64 (the fused kind up to 32);
//   k_gemm_split_ws  fused kind, 33 <= nb <= 64: warp-specialised.
//
// Same operation as the float32 kernels (Theory section, matrix form of the
// MDC operator per frequency): the forward product D_{b,k} R_k with the
// residual, float64 loss partials and the adjoint D_{b,k}^H Res_k written over
// R_k; or the forward / adjoint product alone.  Every complex operand is split
// into hi + lo halves of bf16 or fp16 and the three significant products
// hi*hi + hi*lo + lo*hi are accumulated in float32 on
// v_mfma_f32_16x16x32_{bf16,f16}.
//
// The split happens once per element, while staging into LDS, into four
// planes (re hi, re lo, im hi, im lo) laid out so that each MFMA operand is a
// single 16-byte LDS read: D_{b,k} as [b][r] for the forward product, its
// conjugate as [r][b] for the adjoint (the two are never live together, so
// they share LDS), and the residual as [column][b].  R_k, the right operand of
// the forward product, goes from HBM to registers and is split there by the
// one wave that uses it.  fp16 carries power-of-two scales so that the low halves
// stay normal: one per frequency for D_{b,k} (from its largest |D|, found when the
// kernel is set), one per receiver chunk of R_k and one per residual block.
#include <type_traits>

#include "device_common.h"
#include "mdd_internal.h"

namespace mdd {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 halfx2 __attribute__((ext_vector_type(2)));

template <int PREC>
struct SplitT {
  static constexpr bool F16 = PREC == MDD_PREC_FP16X3;
  using E = std::conditional_t<F16, _Float16, __bf16>;
  using V = std::conditional_t<F16, halfx8, bf16x8>;
  using V2 = std::conditional_t<F16, halfx2, bf16x2>;
  static __device__ __forceinline__ floatx4 mma(V a, V b, floatx4 c) {
    if constexpr (F16) return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    else return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ void split(float x, E& hi, E& lo) {
    hi = (E)x;
    lo = (E)(x - (float)hi);
  }
};

// Two values split at once (one packed conversion for the two hi halves and one for
// the two lo halves), bf16 only.
typedef float floatx2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void split2_bf16(float x0, float x1, bf16x2& hi, bf16x2& lo) {
  const floatx2 x = {x0, x1};
  hi = __builtin_convertvector(x, bf16x2);
  lo = __builtin_convertvector(x - __builtin_convertvector(hi, floatx2), bf16x2);
}

// The 16x16x16 shape (four k values per lane), for products over at most 16
// batch rows.
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 halfx4 __attribute__((ext_vector_type(4)));
typedef short shortx4 __attribute__((ext_vector_type(4)));

template <int PREC>
struct SplitK16 {
  static constexpr bool F16 = PREC == MDD_PREC_FP16X3;
  using V = std::conditional_t<F16, halfx4, bf16x4>;
  static __device__ __forceinline__ floatx4 mma(V a, V b, floatx4 c) {
    if constexpr (F16) return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
    else
      return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(shortx4, a),
                                                       __builtin_bit_cast(shortx4, b), c, 0, 0, 0);
  }
};

// acc += A * B, complex operands given as (re hi, re lo, im hi, im lo); T
// supplies the MFMA shape.
template <typename T, typename V>
__device__ __forceinline__ void cmma3(const V& arh, const V& arl, const V& aih, const V& ail,
                                      const V& brh, const V& brl, const V& bih, const V& bil,
                                      floatx4& re, floatx4& im) {
  const V naih = -aih, nail = -ail;
  re = T::mma(arh, brh, re);
  re = T::mma(arh, brl, re);
  re = T::mma(arl, brh, re);
  re = T::mma(naih, bih, re);
  re = T::mma(naih, bil, re);
  re = T::mma(nail, bih, re);
  im = T::mma(arh, bih, im);
  im = T::mma(arh, bil, im);
  im = T::mma(arl, bih, im);
  im = T::mma(aih, brh, im);
  im = T::mma(aih, brl, im);
  im = T::mma(ail, brh, im);
}

// acc += A * B with the imaginary part of A given negated (nai = -Im A, which the
// operand staging supplies at no cost): Re += ar br + nai bi and Im += ar bi, while the
// remaining imaginary term nai br goes into u, subtracted once at the end
// (Im = im - u).  No operand is negated per product.
template <typename T, typename V>
__device__ __forceinline__ void cmma3n(const V& arh, const V& arl, const V& naih, const V& nail,
                                       const V& brh, const V& brl, const V& bih, const V& bil,
                                       floatx4& re, floatx4& im, floatx4& u) {
  re = T::mma(arh, brh, re);
  re = T::mma(arh, brl, re);
  re = T::mma(arl, brh, re);
  re = T::mma(naih, bih, re);
  re = T::mma(naih, bil, re);
  re = T::mma(nail, bih, re);
  im = T::mma(arh, bih, im);
  im = T::mma(arh, bil, im);
  im = T::mma(arl, bih, im);
  u = T::mma(naih, brh, u);
  u = T::mma(naih, brl, u);
  u = T::mma(nail, brh, u);
}

// Power-of-two scale bringing max |x| to [2^13, 2^14), and its inverse; the
// exponent is clamped so that both stay finite.
__device__ __forceinline__ float2 pow2_scale_pair(float amax) {
  if (!(amax > 0.f) || !(amax < 3.0e38f)) return make_float2(1.f, 1.f);
  int e;
  frexpf(amax, &e);  // amax = m 2^e, m in [0.5, 1)
  const int sh = min(max(14 - e, -120), 120);
  return make_float2(ldexpf(1.f, sh), ldexpf(1.f, -sh));
}

template <int NBT, int TNB>
struct SCfg {
  static constexpr int MB = NBT * 16;        // batch rows (32 or 64)
  static constexpr int NW = TNB * 16;        // columns per workgroup
  static constexpr int TPWV = NBT * TNB / 4; // forward 16x16 tiles per wave, one column tile
  static constexpr int MT_STEP = 4 / TNB;    // row-tile stride between a wave's tiles
  static constexpr int KCMAX = 64;         // receiver chunk
  static constexpr int KSW = KCMAX / 32;     // forward k-steps per chunk
  // Plane row pitches: 16 elements (32 bytes) of padding make the rows of one MFMA
  // operand read (16 rows, 16-byte pieces four lanes apart) fall in disjoint LDS banks;
  // with 8 elements of padding half of the read cycles were bank conflicts.
  static constexpr int RP = KCMAX + 16;      // forward D plane row pitch (elements)
  static constexpr int BP = MB + 16;         // adjoint D / residual plane row pitch
  static constexpr int DF = 4 * MB * RP;     // elements
  static constexpr int DA = 4 * KCMAX * BP;
  static constexpr int DSZ = DF > DA ? DF : DA;
  static constexpr int RS = 4 * NW * BP;
  static constexpr int FPT = MB * (KCMAX / 2) / 256;      // forward: float4 D loads per thread
  static constexpr int APT = (MB / 2) * KCMAX / 256;       // adjoint: (b, b+1) pairs per thread
  static constexpr size_t SMEM = 2 * ((size_t)DSZ + RS);
  static_assert(NBT * TNB >= 4 && 4 % TNB == 0, "one column tile per wave");
  static_assert(FPT * 256 == MB * (KCMAX / 2) && APT * 256 == (MB / 2) * KCMAX, "staging");
};

template <int PREC, int NBT, int TNB, int KIND>
__global__ __launch_bounds__(256) void k_gemm_split(GemmArgs a) {
  using C = SCfg<NBT, TNB>;
  using T = SplitT<PREC>;
  using E = typename T::E;
  using V = typename T::V;
  using V2 = typename T::V2;
  constexpr int MB = C::MB, NW = C::NW, KCMAX = C::KCMAX;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  E* s_dpl = reinterpret_cast<E*>(smem_raw);  // D planes (forward or adjoint layout)
  E* s_rpl = s_dpl + C::DSZ;                   // residual planes [4][NW][BP]
  __shared__ int s_idx[MB];
  __shared__ long long s_drow[MB];
  __shared__ double s_red[4];
  __shared__ float s_max[4];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  const int ncg = (a.nvb + TNB - 1) / TNB;
  const int total = a.nf * ncg;
  const int bid = blockIdx.x;
  const int full = (total / 8) * 8;
  // consecutive items (same frequency, neighbouring columns) on one XCD
  const int logical = bid < full ? (bid % 8) * (total / 8) + bid / 8 : bid;
  const int k = logical / ncg, cg = logical % ncg;
  const int blk0 = cg * TNB;
  const long long rowstride = (long long)a.nvb * a.nf * CB;
  const int nt_w = wave % TNB;  // forward: this wave's column tile
  const int mt0 = wave / TNB;   // forward: first row tile

  for (int b = tid; b < MB; b += 256) {
    int s = -1;
    if (b < a.nb) {
      s = a.idx[b];
      if (s < 0 || s >= a.ns) s = -1;
    }
    s_idx[b] = s;
    s_drow[b] = s >= 0 ? ((long long)k * a.dns + drow_of(a, b, s)) * a.nrp : -1;
  }
  __syncthreads();

  auto block_max = [&](float m) -> float {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    __syncthreads();
    if (lane == 0) s_max[wave] = m;
    __syncthreads();
    return fmaxf(fmaxf(s_max[0], s_max[1]), fmaxf(s_max[2], s_max[3]));
  };
  auto amax4 = [](float4 v) { return fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))); };
  // D_{b,k}[r .. r+1] (zero beyond nr and for rejected indices)
  auto d_pair = [&](int b, int r) -> float4 {
    const long long off = s_drow[b];
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (off >= 0 && r < a.nr) {
      v = *reinterpret_cast<const float4*>(a.Df + off + r);
      if (r + 1 >= a.nr) v.z = v.w = 0.f;
    }
    return v;
  };
  auto dfw = [&](int p, int b, int r) -> E* { return s_dpl + (p * MB + b) * C::RP + r; };
  auto dad = [&](int p, int r, int b) -> E* { return s_dpl + (p * KCMAX + r) * C::BP + b; };
  auto rsp = [&](int p, int col, int b) -> E* { return s_rpl + (p * NW + col) * C::BP + b; };
  auto put2 = [&](E* dhi, float x0, float x1, E* dlo) {
    E h0, l0, h1, l1;
    T::split(x0, h0, l0);
    T::split(x1, h1, l1);
    V2 hv, lv;
    hv[0] = h0;
    hv[1] = h1;
    lv[0] = l0;
    lv[1] = l1;
    *reinterpret_cast<V2*>(dhi) = hv;
    *reinterpret_cast<V2*>(dlo) = lv;
  };
  auto put1 = [&](E* dhi, E* dlo, float x) {
    E h, l;
    T::split(x, h, l);
    *dhi = h;
    *dlo = l;
  };

  float ss = 1.f, iss = 1.f;  // residual / batch-spectra scale (fp16) and its inverse

  // ------------------------------------------------------------ forward
  if constexpr (KIND != GK_ADJ) {
    floatx4 acc_re[C::TPWV], acc_im[C::TPWV];
#pragma unroll
    for (int t = 0; t < C::TPWV; ++t) {
      acc_re[t] = floatx4{0.f, 0.f, 0.f, 0.f};
      acc_im[t] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
    const int ncol = blk0 + nt_w;
    const float2* fb = a.F + (long long)(lq * 8) * rowstride + ((long long)ncol * a.nf + k) * CB + lr;
    // R_k rows r0 + q*32 + lq*8 + e of this wave's column tile (zero beyond nr)
    auto load_r = [&](float2 (&v)[C::KSW][8], int r0) {
#pragma unroll
      for (int q = 0; q < C::KSW; ++q)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          v[q][e] = make_float2(0.f, 0.f);
          if (r0 + q * 32 + lq * 8 + e < a.nr && ncol < a.nvb)
            v[q][e] = fb[(long long)(r0 + q * 32 + e) * rowstride];
        }
    };
    auto load_dfwd = [&](float4 (&v)[C::FPT], int r0) {
#pragma unroll
      for (int q = 0; q < C::FPT; ++q) {
        const int i = tid + 256 * q;
        v[q] = d_pair(i / (KCMAX / 2), r0 + 2 * (i % (KCMAX / 2)));
      }
    };
    // Software pipeline: the next chunk's R_k fragments (from HBM) are in
    // flight while the current chunk's products run; D rows come from L2 at
    // the top of each chunk (prefetching them too costs the registers of a
    // second wave per SIMD, which loses more than it gains).
    float2 bnx[C::KSW][8];
    float4 dv[C::FPT];
    load_r(bnx, 0);
#pragma unroll 1
    for (int r0 = 0; r0 < a.nr; r0 += KCMAX) {
      const int len = min(KCMAX, a.nr - r0);
      load_dfwd(dv, r0);
      float2 bfr[C::KSW][8];
#pragma unroll
      for (int q = 0; q < C::KSW; ++q)
#pragma unroll
        for (int e = 0; e < 8; ++e) bfr[q][e] = bnx[q][e];
      float2 sd = make_float2(1.f, 1.f), sr = make_float2(1.f, 1.f);
      if constexpr (T::F16) {
        float bm = 0.f;
#pragma unroll
        for (int q = 0; q < C::KSW; ++q)
#pragma unroll
          for (int e = 0; e < 8; ++e) bm = fmaxf(bm, fmaxf(fabsf(bfr[q][e].x), fabsf(bfr[q][e].y)));
        sd = pow2_scale_pair(a.dmax[k]);
        sr = pow2_scale_pair(block_max(bm));
      }
      __syncthreads();  // the previous chunk's planes are no longer read
#pragma unroll
      for (int q = 0; q < C::FPT; ++q) {
        const int i = tid + 256 * q;
        const int b = i / (KCMAX / 2), rr = 2 * (i % (KCMAX / 2));
        put2(dfw(0, b, rr), dv[q].x * sd.x, dv[q].z * sd.x, dfw(1, b, rr));
        put2(dfw(2, b, rr), dv[q].y * sd.x, dv[q].w * sd.x, dfw(3, b, rr));
      }
      __syncthreads();
      if (r0 + KCMAX < a.nr) {
        load_r(bnx, r0 + KCMAX);
      }
      floatx4 cre[C::TPWV], cim[C::TPWV];
#pragma unroll
      for (int t = 0; t < C::TPWV; ++t) {
        if constexpr (T::F16) {
          cre[t] = floatx4{0.f, 0.f, 0.f, 0.f};
          cim[t] = floatx4{0.f, 0.f, 0.f, 0.f};
        } else {  // bf16 carries no scale: accumulate in place
          cre[t] = acc_re[t];
          cim[t] = acc_im[t];
        }
      }
#pragma unroll
      for (int q = 0; q < C::KSW; ++q) {
        if (q * 32 < len) {
          V brh, brl, bih, bil;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            E h, l;
            T::split(bfr[q][e].x * sr.x, h, l);
            brh[e] = h;
            brl[e] = l;
            T::split(bfr[q][e].y * sr.x, h, l);
            bih[e] = h;
            bil[e] = l;
          }
#pragma unroll
          for (int t = 0; t < C::TPWV; ++t) {
            const int row = (mt0 + t * C::MT_STEP) * 16 + lr;
            const int col = q * 32 + lq * 8;
            const V arh = *reinterpret_cast<const V*>(dfw(0, row, col));
            const V arl = *reinterpret_cast<const V*>(dfw(1, row, col));
            const V aih = *reinterpret_cast<const V*>(dfw(2, row, col));
            const V ail = *reinterpret_cast<const V*>(dfw(3, row, col));
            cmma3<T>(arh, arl, aih, ail, brh, brl, bih, bil, cre[t], cim[t]);
          }
        }
      }
#pragma unroll
      for (int t = 0; t < C::TPWV; ++t) {
        if constexpr (T::F16) {
          acc_re[t] += (cre[t] * sd.y) * sr.y;
          acc_im[t] += (cim[t] * sd.y) * sr.y;
        } else {
          acc_re[t] = cre[t];
          acc_im[t] = cim[t];
        }
      }
    }

    // Residual (GK_FUSED) or predicted batch spectra (GK_FWD).
    double lpart = 0.0;
    float rm = 0.f;
    float2 zr[C::TPWV][4];
#pragma unroll
    for (int t = 0; t < C::TPWV; ++t) {
      const int mt = mt0 + t * C::MT_STEP;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = mt * 16 + lq * 4 + e, col = nt_w * 16 + lr;
        const int vs = blk0 * CB + col;
        const bool ok = row < a.nb && vs < a.nvs && s_idx[row] >= 0;
        float2 z = make_float2(acc_re[t][e], acc_im[t][e]);
        if constexpr (KIND == GK_FUSED) {
          if (ok) {
            z = csub(z, a.Uf[urow_off(a, k, row, s_idx[row]) + vs]);
            lpart += (k == 0 || 2 * k == a.nt ? 1.0 : 2.0) * ((double)z.x * z.x + (double)z.y * z.y);
          } else {
            z = make_float2(0.f, 0.f);
          }
          zr[t][e] = z;
          rm = fmaxf(rm, fmaxf(fabsf(z.x), fabsf(z.y)));
        } else {
          if (row < a.nb && blk0 + nt_w < a.nvb)
            a.Bsp[(((size_t)row * a.nvb + blk0 + nt_w) * a.nf + k) * CB + lr] =
                ok ? z : make_float2(0.f, 0.f);
        }
      }
    }
    if constexpr (KIND == GK_FWD) return;
    const double tot = block_sum256(lpart, s_red);
    if (tid == 0) a.loss_part[logical] = tot;
    if constexpr (T::F16) {
      const float2 sc = pow2_scale_pair(block_max(rm));
      ss = sc.x;
      iss = sc.y;
    }
#pragma unroll
    for (int t = 0; t < C::TPWV; ++t) {
      const int mt = mt0 + t * C::MT_STEP;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = mt * 16 + lq * 4 + e, col = nt_w * 16 + lr;
        put1(rsp(0, col, row), rsp(1, col, row), zr[t][e].x * ss);
        put1(rsp(2, col, row), rsp(3, col, row), zr[t][e].y * ss);
      }
    }
  } else {
    // Adjoint alone: the batch spectra V_k are the right operand.
    auto bsp = [&](int i) -> float2 {
      const int row = i / NW, col = i % NW;
      const int blk = blk0 + col / 16;
      if (row < a.nb && blk < a.nvb && s_idx[row] >= 0)
        return a.Bsp[(((size_t)row * a.nvb + blk) * a.nf + k) * CB + (col & 15)];
      return make_float2(0.f, 0.f);
    };
    if constexpr (T::F16) {
      float m = 0.f;
      for (int i = tid; i < MB * NW; i += 256) {
        const float2 z = bsp(i);
        m = fmaxf(m, fmaxf(fabsf(z.x), fabsf(z.y)));
      }
      const float2 sc = pow2_scale_pair(block_max(m));
      ss = sc.x;
      iss = sc.y;
    }
    for (int i = tid; i < MB * NW; i += 256) {
      const float2 z = bsp(i);
      const int row = i / NW, col = i % NW;
      put1(rsp(0, col, row), rsp(1, col, row), z.x * ss);
      put1(rsp(2, col, row), rsp(3, col, row), z.y * ss);
    }
  }

  // ------------------------------------------------------------ adjoint
  // G_k[r][c] = sum_b conj(D[b][r]) Res[b][c]; each wave owns row tiles
  // wave, wave + 4, ... of the chunk and all TNB column tiles.  D is staged
  // as (b, b+1) pairs of one receiver per lane, four lanes per receiver, so
  // that a wave's LDS stores fall in distinct banks; the next chunk's D rows
  // are in flight during the current chunk's products.
  float2 dj[C::APT][2];
  auto load_dadj = [&](int r0) {
#pragma unroll
    for (int q = 0; q < C::APT; ++q) {
      const int u = tid + 256 * q;
      const int r = r0 + ((u >> 2) % KCMAX), b = 2 * ((u & 3) + 4 * (u / (4 * KCMAX)));
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const long long off = s_drow[b + h];
        dj[q][h] = (off >= 0 && r < a.nr) ? a.Df[off + r] : make_float2(0.f, 0.f);
      }
    }
  };
  load_dadj(0);
#pragma unroll 1
  for (int r0 = 0; r0 < a.nr; r0 += KCMAX) {
    const int len = min(KCMAX, a.nr - r0);
    float2 sd = make_float2(1.f, 1.f);
    if constexpr (T::F16) sd = pow2_scale_pair(a.dmax[k]);
    __syncthreads();  // residual planes complete; previous D planes no longer read
#pragma unroll
    for (int q = 0; q < C::APT; ++q) {
      const int u = tid + 256 * q;
      const int rr = (u >> 2) % KCMAX, b = 2 * ((u & 3) + 4 * (u / (4 * KCMAX)));
      put2(dad(0, rr, b), dj[q][0].x * sd.x, dj[q][1].x * sd.x, dad(1, rr, b));
      put2(dad(2, rr, b), -dj[q][0].y * sd.x, -dj[q][1].y * sd.x, dad(3, rr, b));  // conj
    }
    __syncthreads();
    if (r0 + KCMAX < a.nr) load_dadj(r0 + KCMAX);
    for (int mt = wave; mt * 16 < len; mt += 4) {
      V arh[MB / 32], arl[MB / 32], aih[MB / 32], ail[MB / 32];
#pragma unroll
      for (int kk = 0; kk < MB / 32; ++kk) {
        const int r = mt * 16 + lr, b = kk * 32 + lq * 8;
        arh[kk] = *reinterpret_cast<const V*>(dad(0, r, b));
        arl[kk] = *reinterpret_cast<const V*>(dad(1, r, b));
        aih[kk] = *reinterpret_cast<const V*>(dad(2, r, b));
        ail[kk] = *reinterpret_cast<const V*>(dad(3, r, b));
      }
#pragma unroll
      for (int nt = 0; nt < TNB; ++nt) {
        floatx4 re = floatx4{0.f, 0.f, 0.f, 0.f}, im = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < MB / 32; ++kk) {
          const int b = kk * 32 + lq * 8, col = nt * 16 + lr;
          const V brh = *reinterpret_cast<const V*>(rsp(0, col, b));
          const V brl = *reinterpret_cast<const V*>(rsp(1, col, b));
          const V bih = *reinterpret_cast<const V*>(rsp(2, col, b));
          const V bil = *reinterpret_cast<const V*>(rsp(3, col, b));
          cmma3<T>(arh[kk], arl[kk], aih[kk], ail[kk], brh, brl, bih, bil, re, im);
        }
        if constexpr (T::F16) {
          re = (re * sd.y) * iss;
          im = (im * sd.y) * iss;
        }
        const int blk = blk0 + nt;
        if (blk < a.nvb) {
          const int rb = r0 + mt * 16 + lq * 4;
          float2* fw = a.F + rb * rowstride + ((long long)blk * a.nf + k) * CB + lr;
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (rb + e < a.nr) store_g(a, (fw - a.F) + e * rowstride, make_float2(re[e], im[e]));
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Batches of at most 16 sources over at most SPLIT_PIPE_KC receivers, fused
// kind: a persistent kernel.  Each workgroup walks a contiguous range of
// (frequency, 16-column block) items.  D_{b,k} is split into LDS planes
// [b][r] once per frequency; the next item's R_k fragments and U entries are
// in flight during the current item's products.  Forward: 16x16x32 products,
// the receiver steps spread over the four waves and their partial sums added
// through LDS.  Adjoint: 16x16x16 products over the batch (k = b), each wave
// owning receiver tiles wave, wave + 4, ...; its A operand (conj D, four
// batch rows of one receiver per lane) is read from the same [b][r] planes.
constexpr int SP_WGS = 512;  // persistent workgroups: two per CU (its register use)

template <int PREC>
__global__ __launch_bounds__(256) void k_gemm_spipe(GemmArgs a) {
  using T = SplitT<PREC>;
  using S = SplitK16<PREC>;
  using E = typename T::E;
  using V = typename T::V;
  using V2 = typename T::V2;
  using V4 = typename S::V;
  constexpr int MB = 16, NW = 16, KC = SPLIT_PIPE_KC;
  constexpr int RP = KC + 8;          // D plane row pitch (elements)
  constexpr int RSP = MB + 4;         // residual plane row pitch: [col][b]
  constexpr int KSW = KC / 32 / 4;    // forward k-steps per wave
  constexpr int DPT = MB * (KC / 2) / 256;  // D float4 loads per thread
  __shared__ __align__(16) E s_d[4 * MB * RP];
  __shared__ __align__(16) E s_r[4 * NW * RSP];
  __shared__ float2 s_part[4 * MB * NW];
  __shared__ int s_idx[MB];
  __shared__ long long s_drow[MB];
  __shared__ double s_red[4];
  __shared__ float s_mx[4];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  const int nvb = a.nvb, total = a.nf * nvb;
  const int G = gridDim.x;
  const int rid = (G % 8 == 0) ? (blockIdx.x % 8) * (G / 8) + blockIdx.x / 8 : blockIdx.x;
  const int start = (int)((long long)rid * total / G), end = (int)((long long)(rid + 1) * total / G);
  if (start >= end) return;
  const long long rowstride = (long long)nvb * a.nf * CB;

  if (tid < MB) {
    int s = -1;
    if (tid < a.nb) {
      s = a.idx[tid];
      if (s < 0 || s >= a.ns) s = -1;
    }
    s_idx[tid] = s;
    s_drow[tid] = s >= 0 ? (long long)drow_of(a, tid, s) * a.nrp : -1;  // within one frequency
  }
  __syncthreads();

  auto wave_max = [](float m) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    return m;
  };
  auto dpl = [&](int p, int b, int r) -> E* { return s_d + (p * MB + b) * RP + r; };
  auto rpl = [&](int p, int col, int b) -> E* { return s_r + (p * NW + col) * RSP + b; };

  // R_k rows (wave + 4 q) * 32 + lq * 8 + e of column block cg, lane column lr
  auto load_b = [&](float2 (&dst)[KSW][8], int k, int cg) {
    const float2* base = a.F + ((long long)cg * a.nf + k) * CB + lr;
#pragma unroll
    for (int q = 0; q < KSW; ++q)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int r = (wave + 4 * q) * 32 + lq * 8 + e;
        dst[q][e] = r < a.nr ? base[(long long)r * rowstride] : make_float2(0.f, 0.f);
      }
  };
  const int urow = tid / NW, ucol = tid % NW;  // this thread's residual entry
  auto load_u = [&](int k, int cg) -> float2 {
    const int vs = cg * CB + ucol;
    if (urow < a.nb && vs < a.nvs && s_idx[urow] >= 0)
      return a.Uf[urow_off(a, k, urow, s_idx[urow]) + vs];
    return make_float2(0.f, 0.f);
  };
  // D_{b,k} -> split planes; returns the (fp16) scale and its inverse
  auto stage_d = [&](int k) -> float2 {
    float4 dv[DPT];
#pragma unroll
    for (int q = 0; q < DPT; ++q) {
      const int i = tid + 256 * q;
      const int b = i / (KC / 2), rr = 2 * (i % (KC / 2));
      const long long off = s_drow[b];
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (off >= 0 && rr < a.nr) {
        v = *reinterpret_cast<const float4*>(a.Df + (size_t)k * a.dns * a.nrp + off + rr);
        if (rr + 1 >= a.nr) v.z = v.w = 0.f;
      }
      dv[q] = v;
    }
    float2 sd = make_float2(1.f, 1.f);
    if constexpr (T::F16) sd = pow2_scale_pair(a.dmax[k]);
#pragma unroll
    for (int q = 0; q < DPT; ++q) {
      const int i = tid + 256 * q;
      const int b = i / (KC / 2), rr = 2 * (i % (KC / 2));
#pragma unroll
      for (int h = 0; h < 2; ++h) {  // h = 0: real parts, 1: imaginary parts
        const float x0 = (h ? dv[q].y : dv[q].x) * sd.x, x1 = (h ? dv[q].w : dv[q].z) * sd.x;
        E h0, l0, h1, l1;
        T::split(x0, h0, l0);
        T::split(x1, h1, l1);
        V2 hv, lv;
        hv[0] = h0;
        hv[1] = h1;
        lv[0] = l0;
        lv[1] = l1;
        *reinterpret_cast<V2*>(dpl(2 * h, b, rr)) = hv;
        *reinterpret_cast<V2*>(dpl(2 * h + 1, b, rr)) = lv;
      }
    }
    return sd;
  };

  double lsum = 0.0;
  int cur = start;
  int k = cur / nvb, cg = cur % nvb;
  float2 bfr[KSW][8], bnx[KSW][8];
  load_b(bfr, k, cg);
  float2 up = load_u(k, cg);
  float2 sd = stage_d(k);
  __syncthreads();

  while (true) {
    const int nxt = cur + 1;
    const bool has_next = nxt < end;
    int kn = k, cgn = cg;
    float2 upn = make_float2(0.f, 0.f);
    if (has_next) {  // next item's operands, in flight during this item's products
      kn = nxt / nvb;
      cgn = nxt % nvb;
      load_b(bnx, kn, cgn);
      upn = load_u(kn, cgn);
    }

    // forward: this wave's receiver steps of D_b R_k
    float2 sr = make_float2(1.f, 1.f);
    if constexpr (T::F16) {  // per-wave scale: each wave unscales its own partial sum
      float m = 0.f;
#pragma unroll
      for (int q = 0; q < KSW; ++q)
#pragma unroll
        for (int e = 0; e < 8; ++e) m = fmaxf(m, fmaxf(fabsf(bfr[q][e].x), fabsf(bfr[q][e].y)));
      sr = pow2_scale_pair(wave_max(m));
    }
    floatx4 ar = floatx4{0.f, 0.f, 0.f, 0.f}, ai = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < KSW; ++q) {
      const int kq = wave + 4 * q;
      if (kq * 32 < a.nr) {
        V brh, brl, bih, bil;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          E h, l;
          T::split(bfr[q][e].x * sr.x, h, l);
          brh[e] = h;
          brl[e] = l;
          T::split(bfr[q][e].y * sr.x, h, l);
          bih[e] = h;
          bil[e] = l;
        }
        const int col = kq * 32 + lq * 8;
        const V arh = *reinterpret_cast<const V*>(dpl(0, lr, col));
        const V arl = *reinterpret_cast<const V*>(dpl(1, lr, col));
        const V aih = *reinterpret_cast<const V*>(dpl(2, lr, col));
        const V ail = *reinterpret_cast<const V*>(dpl(3, lr, col));
        cmma3<T>(arh, arl, aih, ail, brh, brl, bih, bil, ar, ai);
      }
    }
    if constexpr (T::F16) {
      ar = (ar * sd.y) * sr.y;
      ai = (ai * sd.y) * sr.y;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) s_part[(wave * MB + lq * 4 + e) * NW + lr] = make_float2(ar[e], ai[e]);
    __syncthreads();

    // residual, float64 loss partial and (fp16) the residual's block scale
    double lpart = 0.0;
    float2 z = s_part[urow * NW + ucol];
#pragma unroll
    for (int w = 1; w < 4; ++w) z = cadd(z, s_part[(w * MB + urow) * NW + ucol]);
    {
      const int vs = cg * CB + ucol;
      const bool ok = urow < a.nb && vs < a.nvs && s_idx[urow] >= 0;
      if (ok) {
        z = csub(z, up);
        const double wk = (k == 0 || 2 * k == a.nt) ? 1.0 : 2.0;
        lpart = wk * ((double)z.x * z.x + (double)z.y * z.y);
      } else {
        z = make_float2(0.f, 0.f);
      }
    }
    float2 ss = make_float2(1.f, 1.f);
    if constexpr (T::F16) {  // the residual's block scale needs every wave's maximum
      lpart = wave_sum(lpart);
      const float zm = wave_max(fmaxf(fabsf(z.x), fabsf(z.y)));
      if (lane == 0) {
        s_red[wave] = lpart;
        s_mx[wave] = zm;
      }
      __syncthreads();
      if (tid == 0) a.loss_part[cur] = ((s_red[0] + s_red[1]) + s_red[2]) + s_red[3];
      ss = pow2_scale_pair(fmaxf(fmaxf(s_mx[0], s_mx[1]), fmaxf(s_mx[2], s_mx[3])));
    } else {  // summed per thread over the workgroup's items, reduced once at the end
      lsum += lpart;
      if (tid == 0) a.loss_part[cur] = 0.0;
    }
    {
      E h, l;
      T::split(z.x * ss.x, h, l);
      *rpl(0, ucol, urow) = h;
      *rpl(1, ucol, urow) = l;
      T::split(z.y * ss.x, h, l);
      *rpl(2, ucol, urow) = h;
      *rpl(3, ucol, urow) = l;
    }
    __syncthreads();

    // adjoint: G_k = D_b^H Res over this wave's receiver tiles, written over R_k
    float2* gbase = a.F + ((long long)cg * a.nf + k) * CB + lr;
    V4 brh, brl, bih, bil;  // Res rows lq*4 .. lq*4+3, column lr
    brh = *reinterpret_cast<const V4*>(rpl(0, lr, lq * 4));
    brl = *reinterpret_cast<const V4*>(rpl(1, lr, lq * 4));
    bih = *reinterpret_cast<const V4*>(rpl(2, lr, lq * 4));
    bil = *reinterpret_cast<const V4*>(rpl(3, lr, lq * 4));
    for (int mt = wave; mt * 16 < a.nr; mt += 4) {
      V4 arh, arl, aih, ail;  // conj D: batch rows lq*4 + i, receiver mt*16 + lr
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int b = lq * 4 + i, r = mt * 16 + lr;
        arh[i] = *dpl(0, b, r);
        arl[i] = *dpl(1, b, r);
        aih[i] = -*dpl(2, b, r);
        ail[i] = -*dpl(3, b, r);
      }
      floatx4 re = floatx4{0.f, 0.f, 0.f, 0.f}, im = floatx4{0.f, 0.f, 0.f, 0.f};
      cmma3<S>(arh, arl, aih, ail, brh, brl, bih, bil, re, im);
      if constexpr (T::F16) {
        re = (re * sd.y) * ss.y;
        im = (im * sd.y) * ss.y;
      }
      const int rb = mt * 16 + lq * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (rb + e < a.nr) store_g(a, (gbase - a.F) + (long long)(rb + e) * rowstride, make_float2(re[e], im[e]));
    }
    if (!has_next) break;
    __syncthreads();  // every wave is done with s_d, s_part, s_r of this item
    if (kn != k) {  // new frequency (rare within one workgroup's range)
      sd = stage_d(kn);
      __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < KSW; ++q)
#pragma unroll
      for (int e = 0; e < 8; ++e) bfr[q][e] = bnx[q][e];
    up = upn;
    cur = nxt;
    k = kn;
    cg = cgn;
  }
  if constexpr (!T::F16) {
    const double tot = block_sum256(lsum, s_red);
    if (tid == 0) a.loss_part[start] = tot;
  }
}

// ---------------------------------------------------------------------------
// 33..64 batch rows, fused kind: a warp-specialised workgroup of twelve waves.
// Eight compute waves use the same LDS planes and 16x16x32 tiling as the tiled
// kernel (each owns one 16-column tile and two of the four row tiles).  Four
// loader waves only stream R_k: they keep WS_DEPTH 64-receiver chunks in flight
// in their registers and hand each to the compute waves through a two-slot LDS
// ring (bf16: already split into hi / lo planes; fp16: float32 values).  D_{b,k}
// chunks are double-buffered as well, so a single barrier separates consecutive
// chunks.  (With one role per wave, each wave has one chunk in flight and waits on
// memory for about half of its time.)  In the barrier-free adjoint all twelve waves
// take receiver tiles.
constexpr int WS_DEPTH = 3;
constexpr int WS_CW = 8;                   // compute waves (two per SIMD)
constexpr int WS_LW = 4;                   // loader waves
constexpr int WS_THREADS = 64 * (WS_CW + WS_LW);

template <int PREC>
__global__ __launch_bounds__(WS_THREADS) void k_gemm_split_ws(GemmArgs a) {
  using C = SCfg<4, 4>;
  using T = SplitT<PREC>;
  using E = typename T::E;
  using V = typename T::V;
  using V2 = typename T::V2;
  constexpr int MB = C::MB, NW = C::NW, KC = C::KCMAX, KSW = C::KSW;
  constexpr int RRP = NW + 2;                 // fp16 ring row pitch (complex values)
  constexpr int RING = KC * RRP;              // fp16: complex values per ring slot
  // bf16: the loader waves split R_k into four planes [re hi, re lo, im hi, im lo] of
  // [column][receiver] bf16 values, so that each B operand is one 16-byte LDS read and
  // every value is split once (fp16 keeps float32 values: its per-chunk scale needs the
  // maximum over all loader waves before any value can be split).
  constexpr bool SPLIT_RING = !T::F16;
  constexpr int RKP = KC + 8;                 // split-ring plane row pitch (elements)
  constexpr int RSLOT = 4 * NW * RKP;         // split ring: elements per slot
  constexpr int NCT = 64 * WS_CW, NLT = 64 * WS_LW;  // compute / loader threads
  constexpr int LPT = KC * NW / 2 / NLT;      // float4 per loader thread per chunk
  constexpr int TPC = C::TPWV * 4 / WS_CW;    // forward 16x16 tiles per compute wave
  constexpr int FPT = MB * (KC / 2) / NCT;    // forward D float4 per compute thread
  static_assert(LPT * NLT == KC * NW / 2 && FPT * NCT == MB * (KC / 2), "split");
  static_assert(WS_DEPTH == 3, "the loader's register rotation is unrolled by three");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  E* s_dsl = reinterpret_cast<E*>(smem_raw);  // two D slots of C::DSZ elements
  float2* s_ring = reinterpret_cast<float2*>(smem_raw + 2 * sizeof(E) * C::DSZ);
  E* s_rpl = reinterpret_cast<E*>(s_ring);    // residual planes; the ring is free by then
  E* s_rsp = reinterpret_cast<E*>(s_ring);    // split ring (bf16)
  static_assert(sizeof(E) * C::RS <= (SPLIT_RING ? sizeof(E) * 2 * RSLOT : sizeof(float2) * 2 * RING),
                "residual planes fit the ring");
  __shared__ int s_idx[MB];
  __shared__ long long s_drow[MB];
  __shared__ double s_red[WS_CW];
  __shared__ float s_rmax[2][WS_LW];  // fp16: per ring slot, per loader wave
  __shared__ float s_max[WS_CW];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool compute = wave < WS_CW;
  const int lr = lane & 15, lq = lane >> 4;
  const int ncg = (a.nvb + 3) / 4;
  const int total = a.nf * ncg;
  const int bid = blockIdx.x, full = (total / 8) * 8;
  const int logical = bid < full ? (bid % 8) * (total / 8) + bid / 8 : bid;
  const int k = logical / ncg, cg = logical % ncg;  // the column groups of one frequency share an XCD
  const int blk0 = cg * 4;
  const long long rowstride = (long long)a.nvb * a.nf * CB;
  const int nc = (a.nr + KC - 1) / KC;
  const int nt_w = wave & 3;            // compute, forward: column tile
  const int rt0 = (wave >> 2) * TPC;    // compute, forward: first of its row tiles
  const int li = tid - NCT;             // loader: thread index within the loaders

  for (int b = tid; b < MB; b += WS_THREADS) {
    int s = -1;
    if (b < a.nb) {
      s = a.idx[b];
      if (s < 0 || s >= a.ns) s = -1;
    }
    s_idx[b] = s;
    s_drow[b] = s >= 0 ? ((long long)k * a.dns + drow_of(a, b, s)) * a.nrp : -1;
  }
  __syncthreads();

  auto wave_max = [](float m) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    return m;
  };
  auto maxn = [](const float* v, int n) {
    float m = v[0];
    for (int i = 1; i < n; ++i) m = fmaxf(m, v[i]);
    return m;
  };
  auto amax4 = [](float4 v) { return fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))); };
  auto dfw = [&](int sl, int p, int b, int r) -> E* { return s_dsl + sl * C::DSZ + (p * MB + b) * C::RP + r; };
  auto rsp = [&](int p, int col, int b) -> E* { return s_rpl + (p * NW + col) * C::BP + b; };
  auto put2 = [&](E* dhi, float x0, float x1, E* dlo) {
    E h0, l0, h1, l1;
    T::split(x0, h0, l0);
    T::split(x1, h1, l1);
    V2 hv, lv;
    hv[0] = h0;
    hv[1] = h1;
    lv[0] = l0;
    lv[1] = l1;
    *reinterpret_cast<V2*>(dhi) = hv;
    *reinterpret_cast<V2*>(dlo) = lv;
  };
  auto put1 = [&](E* dhi, E* dlo, float x) {
    E h, l;
    T::split(x, h, l);
    *dhi = h;
    *dlo = l;
  };
  auto scale_of = [&](const float* v, int n) -> float2 {
    if constexpr (T::F16) return pow2_scale_pair(maxn(v, n));
    else return make_float2(1.f, 1.f);
  };
  // fp16: one power-of-two scale for D_{b,k}, from the frequency's largest |D|
  float2 sdk = make_float2(1.f, 1.f);
  if constexpr (T::F16) sdk = pow2_scale_pair(a.dmax[k]);

  // ---- loader side: R_k chunk c (rows c*KC ..) of the four column blocks.  The
  // loads are unconditional (addresses clamped into the array) so that nothing
  // waits for them before they are written to the ring, where rows beyond nr and
  // blocks beyond nvb become zeros.
  // bf16 split ring: loader thread li owns column pair 2 (li % 32) and the eight rows
  // 8 (li / 32) .. + 7 of each chunk: one 16-byte load per row.
  static_assert(!SPLIT_RING || (LPT == 8 && NLT == (NW / 2) * (KC / 8)), "split-ring mapping");
  const int lcp = 2 * (li & 31), lrg = 8 * (li >> 5);
  const bool lblk_ok = blk0 + lcp / CB < a.nvb;
  const float2* lcol = a.F + ((long long)min(blk0 + lcp / CB, a.nvb - 1) * a.nf + k) * CB + lcp % CB;
  auto issue = [&](float4 (&dst)[LPT], int c) {
    if constexpr (SPLIT_RING) {
#pragma unroll
      for (int q = 0; q < LPT; ++q) {
        const int r = min(c * KC + lrg + q, a.nr - 1);
        dst[q] = stream_load4(lcol + (long long)r * rowstride);
      }
      return;
    }
#pragma unroll
    for (int q = 0; q < LPT; ++q) {
      const int i = li + NLT * q;
      const int rr = i / (NW / 2), cp = 2 * (i % (NW / 2));
      const int r = min(c * KC + rr, a.nr - 1), blk = min(blk0 + cp / CB, a.nvb - 1);
      dst[q] = stream_load4(a.F + (long long)r * rowstride + ((long long)blk * a.nf + k) * CB + cp % CB);
    }
  };
  auto put_ring = [&](const float4 (&src)[LPT], int c) {
    const int slot = c & 1;
    if constexpr (SPLIT_RING) {
      float x[4][8];  // column lcp re, im; column lcp + 1 re, im; rows lrg .. lrg + 7
      if (lblk_ok && c * KC + lrg + LPT <= a.nr) {  // every row real: no selects
#pragma unroll
        for (int q = 0; q < LPT; ++q) {
          x[0][q] = src[q].x;
          x[1][q] = src[q].y;
          x[2][q] = src[q].z;
          x[3][q] = src[q].w;
        }
      } else {
#pragma unroll
        for (int q = 0; q < LPT; ++q) {
          const bool ok = lblk_ok && c * KC + lrg + q < a.nr;
          x[0][q] = ok ? src[q].x : 0.f;
          x[1][q] = ok ? src[q].y : 0.f;
          x[2][q] = ok ? src[q].z : 0.f;
          x[3][q] = ok ? src[q].w : 0.f;
        }
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {  // the two columns
        V ph[2], pl[2];              // [re, im] hi / lo
#pragma unroll
        for (int part = 0; part < 2; ++part)
#pragma unroll
          for (int e = 0; e < 8; e += 2) {
            bf16x2 hv, lv;
            split2_bf16(x[2 * h + part][e], x[2 * h + part][e + 1], hv, lv);
            ph[part][e] = hv[0];
            ph[part][e + 1] = hv[1];
            pl[part][e] = lv[0];
            pl[part][e + 1] = lv[1];
          }
        E* dst = s_rsp + slot * RSLOT + (lcp + h) * RKP + lrg;
        *reinterpret_cast<V*>(dst) = ph[0];
        *reinterpret_cast<V*>(dst + NW * RKP) = pl[0];
        *reinterpret_cast<V*>(dst + 2 * NW * RKP) = ph[1];
        *reinterpret_cast<V*>(dst + 3 * NW * RKP) = pl[1];
      }
      return;
    }
    float m = 0.f;
#pragma unroll
    for (int q = 0; q < LPT; ++q) {
      const int i = li + NLT * q;
      const int rr = i / (NW / 2), cp = 2 * (i % (NW / 2));
      const bool ok = c * KC + rr < a.nr && blk0 + cp / CB < a.nvb;
      const float4 v = ok ? src[q] : make_float4(0.f, 0.f, 0.f, 0.f);
      *reinterpret_cast<float4*>(s_ring + slot * RING + rr * RRP + cp) = v;
      m = fmaxf(m, amax4(v));
    }
    if constexpr (T::F16) {
      m = wave_max(m);
      if (lane == 0) s_rmax[slot][wave - WS_CW] = m;
    }
  };

  // ---- compute side: D chunks for the forward product ([b][r] planes)
  // D loads are unconditional too (a rejected index reads row 0 of the frequency,
  // a receiver beyond nr reads receiver 0); staging zeroes them.
  const long long drow0 = (long long)k * a.dns * a.nrp;
  auto d_at = [&](int b, int r) -> long long {
    const long long off = s_drow[b];
    return (off >= 0 ? off : drow0) + (r < a.nr ? r : 0);
  };
  auto d_ok = [&](int b, int r) { return s_drow[b] >= 0 && r < a.nr; };
  // Each compute thread stages eight consecutive receivers of one batch row per chunk
  // (64 rows x 8 groups = the 512 compute threads): four 16-byte loads, and one 16-byte
  // LDS write per plane.  Its row's address is fixed for the item; receivers at or past
  // nr (only in the last chunk) are zeroed, and a group starting at or past the padded
  // row length loads receiver 0 instead (always in bounds).
  static_assert(FPT == 4 && NCT == MB * (KC / 8), "one row and eight receivers per thread");
  const int db = tid >> 3, dg = (tid & 7) * 8;      // compute threads only
  const bool drow_ok = compute && s_drow[db] >= 0;
  const float2* drow_p = a.Df + (compute && s_drow[db] >= 0 ? s_drow[db] : drow0);
  // Two chunks in flight: chunk c + 3 is requested when chunk c + 1 is staged, two
  // chunks of products before it is needed (a miss in L2 is served from farther away).
  float4 dv[2][FPT];
  auto load_dfwd = [&](float4 (&d)[FPT], int c) {
    const int r0 = c * KC + dg;
    const float4* src = reinterpret_cast<const float4*>(drow_p + (r0 < a.nrp ? r0 : 0));
#pragma unroll
    for (int q = 0; q < FPT; ++q) d[q] = src[q];
  };
  auto stage_dfwd = [&](const float4 (&d)[FPT], int sl, float sd, int c) {
    const int r0 = c * KC + dg;
    float x[16];
#pragma unroll
    for (int q = 0; q < FPT; ++q) {
      x[4 * q] = d[q].x;
      x[4 * q + 1] = d[q].y;
      x[4 * q + 2] = d[q].z;
      x[4 * q + 3] = d[q].w;
    }
    if (!drow_ok || r0 + 8 > a.nr) {
#pragma unroll
      for (int e = 0; e < 8; ++e)
        if (!drow_ok || r0 + e >= a.nr) x[2 * e] = x[2 * e + 1] = 0.f;
    }
    V rh, rl, nih, nil;  // nih, nil: -Im D (cmma3n)
#pragma unroll
    for (int e = 0; e < 8; e += (T::F16 ? 1 : 2)) {
      if constexpr (T::F16) {
        E h, l;
        T::split(x[2 * e] * sd, h, l);
        rh[e] = h;
        rl[e] = l;
        T::split(-x[2 * e + 1] * sd, h, l);
        nih[e] = h;
        nil[e] = l;
      } else {
        bf16x2 hv, lv;
        split2_bf16(x[2 * e], x[2 * e + 2], hv, lv);
        rh[e] = hv[0];
        rh[e + 1] = hv[1];
        rl[e] = lv[0];
        rl[e + 1] = lv[1];
        split2_bf16(-x[2 * e + 1], -x[2 * e + 3], hv, lv);
        nih[e] = hv[0];
        nih[e + 1] = hv[1];
        nil[e] = lv[0];
        nil[e + 1] = lv[1];
      }
    }
    *reinterpret_cast<V*>(dfw(sl, 0, db, dg)) = rh;
    *reinterpret_cast<V*>(dfw(sl, 1, db, dg)) = rl;
    *reinterpret_cast<V*>(dfw(sl, 2, db, dg)) = nih;
    *reinterpret_cast<V*>(dfw(sl, 3, db, dg)) = nil;
  };

  // The two roles run separate loops with the same barriers (2 + nc of them), so
  // that the loaders' in-flight registers and the compute waves' accumulators
  // are not live at the same time in either.
  floatx4 acc_re[TPC], acc_im[TPC], acc_u[TPC];
#pragma unroll
  for (int t = 0; t < TPC; ++t) {
    acc_re[t] = floatx4{0.f, 0.f, 0.f, 0.f};
    acc_im[t] = floatx4{0.f, 0.f, 0.f, 0.f};
    acc_u[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  }
  if (compute) {
    // prologue: D chunk 0 staged, chunks 1 and 2 in flight (chunks past the end load
    // clamped addresses and stage zeros)
    load_dfwd(dv[0], 0);
    load_dfwd(dv[1], 1);
    __syncthreads();
    stage_dfwd(dv[0], 0, sdk.x, 0);
    load_dfwd(dv[0], 2);
    __syncthreads();
    // chunk c: its products, then chunk c + 1 staged from buffer b = (c + 1) % 2 and
    // chunk c + 3 requested into it
    auto chunk = [&](int c, float4 (&dvb)[FPT]) {
      const int sl = c & 1;
      const int len = min(KC, a.nr - c * KC);
      const float2 sd = sdk, sr = scale_of(s_rmax[sl], WS_LW);
      floatx4 cre[TPC], cim[TPC], cu[TPC];
#pragma unroll
      for (int t = 0; t < TPC; ++t) {
        if constexpr (T::F16) {
          cre[t] = floatx4{0.f, 0.f, 0.f, 0.f};
          cim[t] = floatx4{0.f, 0.f, 0.f, 0.f};
          cu[t] = floatx4{0.f, 0.f, 0.f, 0.f};
        } else {
          cre[t] = acc_re[t];
          cim[t] = acc_im[t];
          cu[t] = acc_u[t];
        }
      }
      const float2* ring = s_ring + sl * RING + nt_w * 16 + lr;
      const E* rsp = s_rsp + sl * RSLOT + (nt_w * 16 + lr) * RKP + lq * 8;
#pragma unroll
      for (int q = 0; q < KSW; ++q) {
        if (q * 32 < len) {
          V brh, brl, bih, bil;
          if constexpr (SPLIT_RING) {
            brh = *reinterpret_cast<const V*>(rsp + q * 32);
            brl = *reinterpret_cast<const V*>(rsp + NW * RKP + q * 32);
            bih = *reinterpret_cast<const V*>(rsp + 2 * NW * RKP + q * 32);
            bil = *reinterpret_cast<const V*>(rsp + 3 * NW * RKP + q * 32);
          } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const float2 x = ring[(q * 32 + lq * 8 + e) * RRP];
              E h, l;
              T::split(x.x * sr.x, h, l);
              brh[e] = h;
              brl[e] = l;
              T::split(x.y * sr.x, h, l);
              bih[e] = h;
              bil[e] = l;
            }
          }
#pragma unroll
          for (int t = 0; t < TPC; ++t) {
            const int row = (rt0 + t) * 16 + lr, col = q * 32 + lq * 8;
            const V arh = *reinterpret_cast<const V*>(dfw(sl, 0, row, col));
            const V arl = *reinterpret_cast<const V*>(dfw(sl, 1, row, col));
            const V naih = *reinterpret_cast<const V*>(dfw(sl, 2, row, col));
            const V nail = *reinterpret_cast<const V*>(dfw(sl, 3, row, col));
            cmma3n<T>(arh, arl, naih, nail, brh, brl, bih, bil, cre[t], cim[t], cu[t]);
          }
        }
      }
#pragma unroll
      for (int t = 0; t < TPC; ++t) {
        if constexpr (T::F16) {
          acc_re[t] += (cre[t] * sd.y) * sr.y;
          acc_im[t] += ((cim[t] - cu[t]) * sd.y) * sr.y;
        } else {
          acc_re[t] = cre[t];
          acc_im[t] = cim[t];
          acc_u[t] = cu[t];
        }
      }
      // the next D chunk into the other slot (last read by chunk c - 1); unconditional
      // so that the loads in flight are the same on every path
      stage_dfwd(dvb, sl ^ 1, sdk.x, c + 1);
      load_dfwd(dvb, c + 3);
      __syncthreads();
    };
    int c = 0;
#pragma unroll 1
    for (; c + 1 < nc; c += 2) {
      chunk(c, dv[1]);
      chunk(c + 1, dv[0]);
    }
    if (c < nc) chunk(c, dv[1]);
  } else {
    // prologue: R chunk 0 in the ring, chunks 1 .. 3 in flight
    // Every issue is unconditional (chunks past the end read clamped addresses and
    // are written as zeros) so that the loads in flight are the same on every path
    // and each ring write waits only for its own chunk.
    float4 rq[WS_DEPTH][LPT];
    issue(rq[0], 0);
    issue(rq[1], 1);
    issue(rq[2], 2);
    __syncthreads();
    put_ring(rq[0], 0);
    issue(rq[0], 3);
    __syncthreads();
    int c0 = 0;
#pragma unroll 1
    for (; c0 + WS_DEPTH <= nc; c0 += WS_DEPTH) {
#pragma unroll
      for (int u = 0; u < WS_DEPTH; ++u) {  // R chunk c + 1 into the slot chunk c - 1 used
        const int c = c0 + u;
        put_ring(rq[(u + 1) % WS_DEPTH], c + 1);
        issue(rq[(u + 1) % WS_DEPTH], c + 1 + WS_DEPTH);
        __syncthreads();
      }
    }
#pragma unroll
    for (int u = 0; u < WS_DEPTH - 1; ++u) {  // the last nc % 3 chunks
      const int c = c0 + u;
      if (c < nc) {
        put_ring(rq[(u + 1) % WS_DEPTH], c + 1);
        __syncthreads();
      }
    }
  }

  // residual and float64 loss partial (compute waves)
  double lpart = 0.0;
  float rm = 0.f;
  float2 zr[TPC][4];
  if constexpr (!T::F16) {
#pragma unroll
    for (int t = 0; t < TPC; ++t) acc_im[t] -= acc_u[t];
  }
  if (compute) {
    float2 uv[TPC][4];  // all of this lane's U_b entries in flight at once
#pragma unroll
    for (int t = 0; t < TPC; ++t)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = (rt0 + t) * 16 + lq * 4 + e, vs = blk0 * CB + nt_w * 16 + lr;
        const int s = row < a.nb ? max(s_idx[row], 0) : 0;
        uv[t][e] = a.Uf[urow_off(a, k, row < a.nb ? row : 0, s) + min(vs, a.nvsp - 1)];
      }
#pragma unroll
    for (int t = 0; t < TPC; ++t) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = (rt0 + t) * 16 + lq * 4 + e, col = nt_w * 16 + lr;
        const int vs = blk0 * CB + col;
        float2 z = make_float2(acc_re[t][e], acc_im[t][e]);
        if (row < a.nb && vs < a.nvs && s_idx[row] >= 0) {
          z = csub(z, uv[t][e]);
          lpart += (k == 0 || 2 * k == a.nt ? 1.0 : 2.0) * ((double)z.x * z.x + (double)z.y * z.y);
        } else {
          z = make_float2(0.f, 0.f);
        }
        zr[t][e] = z;
        rm = fmaxf(rm, fmaxf(fabsf(z.x), fabsf(z.y)));
      }
    }
    lpart = wave_sum(lpart);
    rm = wave_max(rm);
    if (lane == 0) {
      s_red[wave] = lpart;
      s_max[wave] = rm;
    }
  }
  __syncthreads();
  if (tid == 0) {
    double tot = 0.0;
    for (int w = 0; w < WS_CW; ++w) tot += s_red[w];
    a.loss_part[logical] = tot;
  }
  const float2 ss = scale_of(s_max, WS_CW);

  // adjoint, without barriers: G_k = D_b^H Res_k.  Every wave (the loader waves too,
  // their ring work being done) owns the receiver tiles wave, wave + WS_CW + WS_LW,
  // ...; it loads its tile's A operand (conj D:
  // eight batch rows of one receiver per lane and k-step) from L2 straight into
  // registers, splitting it there (the next tile's values are in flight during
  // the current tile's products).  The residual planes in LDS are the B operand.
  if (compute) {
#pragma unroll
    for (int t = 0; t < TPC; ++t) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = (rt0 + t) * 16 + lq * 4 + e, col = nt_w * 16 + lr;
        put1(rsp(0, col, row), rsp(1, col, row), zr[t][e].x * ss.x);
        put1(rsp(2, col, row), rsp(3, col, row), zr[t][e].y * ss.x);
      }
    }
  }
  __syncthreads();  // the last barrier: the ring is no longer used
  const int nrt = (a.nr + 15) / 16;
  // This lane's sixteen batch rows (b = kk * 32 + lq * 8 + e) are the same for every
  // tile: their offsets from the frequency's first row (32-bit, a rejected row reading
  // row 0) and whether all of them are real are found once.
  unsigned aoff[2][8];
  bool arows_ok = true;
#pragma unroll
  for (int kk = 0; kk < 2; ++kk)
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const long long off = s_drow[kk * 32 + lq * 8 + e];
      aoff[kk][e] = off >= 0 ? (unsigned)(off - drow0) : 0u;
      arows_ok = arows_ok && off >= 0;
    }
  const float2* dk = a.Df + drow0;
  auto load_tile = [&](float2 (&d)[2][8], int mt, int zero) {  // clamped: always in bounds
    const float2* dr = dk + min(mt * 16 + lr, a.nr - 1) + zero;
#pragma unroll
    for (int kk = 0; kk < 2; ++kk)
#pragma unroll
      for (int e = 0; e < 8; ++e) d[kk][e] = dr[aoff[kk][e]];
  };
  float2 dn[2][8];
  load_tile(dn, min(wave, nrt - 1), 0);
#pragma unroll 1
  for (int mt = wave; mt < nrt; mt += WS_CW + WS_LW) {
    float2 dc[2][8];
#pragma unroll
    for (int kk = 0; kk < 2; ++kk)
#pragma unroll
      for (int e = 0; e < 8; ++e) dc[kk][e] = dn[kk][e];
    const int r = mt * 16 + lr;
    if (!arows_ok || r >= a.nr) {
#pragma unroll
      for (int kk = 0; kk < 2; ++kk)
#pragma unroll
        for (int e = 0; e < 8; ++e)
          if (!d_ok(kk * 32 + lq * 8 + e, r)) dc[kk][e] = make_float2(0.f, 0.f);
    }
    const float2 sd = sdk;
    V arh[2], arl[2], aih[2], ail[2];  // aih, ail: conj D's -Im = Im D (cmma3n)
#pragma unroll
    for (int kk = 0; kk < 2; ++kk)
#pragma unroll
      for (int e = 0; e < 8; e += (T::F16 ? 1 : 2)) {
        if constexpr (T::F16) {
          E h, l;
          T::split(dc[kk][e].x * sd.x, h, l);
          arh[kk][e] = h;
          arl[kk][e] = l;
          T::split(dc[kk][e].y * sd.x, h, l);
          aih[kk][e] = h;
          ail[kk][e] = l;
        } else {
          bf16x2 hv, lv;
          split2_bf16(dc[kk][e].x, dc[kk][e + 1].x, hv, lv);
          arh[kk][e] = hv[0];
          arh[kk][e + 1] = hv[1];
          arl[kk][e] = lv[0];
          arl[kk][e + 1] = lv[1];
          split2_bf16(dc[kk][e].y, dc[kk][e + 1].y, hv, lv);
          aih[kk][e] = hv[0];
          aih[kk][e + 1] = hv[1];
          ail[kk][e] = lv[0];
          ail[kk][e + 1] = lv[1];
        }
      }
    // The next tile's A operand is requested only after this tile's values have arrived:
    // vector-memory loads and stores retire in order under one counter, so a wait for
    // loads issued after the previous tile's G stores would wait for those stores too.
    // The empty asm statement takes the last of this tile's values and yields the zero
    // that the next tile's addresses add, so the compiler cannot issue those loads first.
    int zero = 0;
    asm volatile("" : "+v"(zero) : "v"(dc[1][7].x));
    load_tile(dn, min(mt + WS_CW + WS_LW, nrt - 1), zero);
#pragma unroll 1
    for (int nt = 0; nt < 4; ++nt) {  // not unrolled: the B operands of one column tile at a time
      floatx4 re = floatx4{0.f, 0.f, 0.f, 0.f}, im = floatx4{0.f, 0.f, 0.f, 0.f};
      floatx4 u = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kk = 0; kk < 2; ++kk) {
        const int b = kk * 32 + lq * 8, col = nt * 16 + lr;
        const V brh = *reinterpret_cast<const V*>(rsp(0, col, b));
        const V brl = *reinterpret_cast<const V*>(rsp(1, col, b));
        const V bih = *reinterpret_cast<const V*>(rsp(2, col, b));
        const V bil = *reinterpret_cast<const V*>(rsp(3, col, b));
        cmma3n<T>(arh[kk], arl[kk], aih[kk], ail[kk], brh, brl, bih, bil, re, im, u);
      }
      im -= u;
      if constexpr (T::F16) {
        re = (re * sd.y) * ss.y;
        im = (im * sd.y) * ss.y;
      }
      const int blk = blk0 + nt;
      if (blk < a.nvb) {
        const int rb = mt * 16 + lq * 4;
        float2* fw = a.F + (long long)rb * rowstride + ((long long)blk * a.nf + k) * CB + lr;
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (rb + e < a.nr) store_g_stream(a, (fw - a.F) + e * rowstride, make_float2(re[e], im[e]));
      }
    }
  }
}

template <int PREC>
hipError_t launch_split_ws(const GemmArgs& a, hipStream_t s) {
  using C = SCfg<4, 4>;
  using E = typename SplitT<PREC>::E;
  constexpr size_t ring = SplitT<PREC>::F16 ? sizeof(float2) * 2 * C::KCMAX * (C::NW + 2)
                                            : sizeof(E) * 2 * 4 * C::NW * (C::KCMAX + 8);
  constexpr size_t sm = 2 * sizeof(E) * C::DSZ + ring;
  const int ncg = (a.nvb + 3) / 4;
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gemm_split_ws<PREC>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
  hipLaunchKernelGGL(k_gemm_split_ws<PREC>, dim3(a.nf * ncg), dim3(WS_THREADS), sm, s, a);
  return hipGetLastError();
}

template <int PREC, int NBT, int TNB, int KIND>
hipError_t launch_one(const GemmArgs& a, hipStream_t s) {
  using C = SCfg<NBT, TNB>;
  const int ncg = (a.nvb + TNB - 1) / TNB;
  auto kern = &k_gemm_split<PREC, NBT, TNB, KIND>;
  if (C::SMEM > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)C::SMEM);
  hipLaunchKernelGGL(kern, dim3(a.nf * ncg), dim3(256), C::SMEM, s, a);
  return hipGetLastError();
}

template <int PREC, int NBT, int TNB>
hipError_t launch_split_cfg(int kind, const GemmArgs& a, hipStream_t s) {
  switch (kind) {
    case GK_FUSED: return launch_one<PREC, NBT, TNB, GK_FUSED>(a, s);
    case GK_FWD: return launch_one<PREC, NBT, TNB, GK_FWD>(a, s);
    case GK_ADJ: return launch_one<PREC, NBT, TNB, GK_ADJ>(a, s);
    default: return hipErrorInvalidValue;
  }
}

template <int PREC>
hipError_t launch_split_prec(int kind, const GemmArgs& a, hipStream_t s) {
  if (a.nb <= 16) {
    if (kind != GK_FUSED || a.nr > SPLIT_PIPE_KC) return hipErrorInvalidValue;
    const int total = a.nf * a.nvb;
    int grid = total < SP_WGS ? total : SP_WGS;
    if (grid >= 8) grid -= grid % 8;
    hipLaunchKernelGGL(k_gemm_spipe<PREC>, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
  }
  if (a.nb <= 32) return launch_split_cfg<PREC, 2, 2>(kind, a, s);
  if (kind == GK_FUSED) return launch_split_ws<PREC>(a, s);
  return launch_split_cfg<PREC, 4, 4>(kind, a, s);
}

}  // namespace

// Split forms (bf16x3, fp16x3): 16 < nb <= 64, or the fused kind at nb <= 16 over at
// most SPLIT_PIPE_KC receivers.
hipError_t launch_gemm_split(int kind, int precision, const GemmArgs& a, hipStream_t s) {
  if (a.nb < 1 || a.nb > NB_LIMIT) return hipErrorInvalidValue;
  switch (precision) {
    case MDD_PREC_BF16X3: return launch_split_prec<MDD_PREC_BF16X3>(kind, a, s);
    case MDD_PREC_FP16X3: return launch_split_prec<MDD_PREC_FP16X3>(kind, a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mdd
