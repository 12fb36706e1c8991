// Per-frequency complex products of the MDC operator on MFMA (Theory section,
// matrix form P-_f = P+_f R_f; Appendix A "batched matrix-matrix
// multiplication"), with the residual, the float64 loss partials and the
// adjoint product fused for the mini-batch gradient:
//
//   Res_k = D_{b,k} R_k - U_{b,k}      ([nb x nr] [nr x nvs])
//   G_k   = D_{b,k}^H Res_k            ([nr x nb] [nb x nvs]), written over R_k
//
// Kernels (the split-precision ones for more than 16 batch rows are in
// gemm_split.hip):
//   k_gemm<prec, NBT, TNB, kind>  tiled: a workgroup owns one frequency k and
//       TNB column blocks (16 virtual sources each); the batch rows of D_k are
//       gathered by index into LDS in receiver chunks and the residual block
//       stays in LDS between the two products.  Every kind and precision.
//   k_gemm_pipe   fp32, fused, nb <= 16, nr <= PIPE_KC: persistent, the next
//       item's R_k in flight during the current item's products.
//   k_gemm_ws<kind, prec>  fp32, 33 <= nb <= 64, every kind: loader waves stream R_k
//       through an LDS ring for the compute waves; the adjoint needs no barrier
//       (the adjoint kind reads the batch spectra into the residual planes).
// R_k is read and G_k written exactly once.  G_k goes over R_k, or (the full
// gradient) into, or added to, a second spectra buffer.
//
// There is no complex MFMA: a complex product is four real products
// (Re = Ar Br - Ai Bi, Im = Ar Bi + Ai Br) on v_mfma_f32_16x16x4_f32, or, in
// the split-precision forms, on v_mfma_f32_16x16x32_{bf16,f16} with each
// operand split into hi + lo and hi*hi + hi*lo + lo*hi accumulated in fp32.
// The float32 tiled and warp-specialised kernels use three real products
// instead (cmac3) unless the precision is MDD_PREC_FP32_CGEMM; the persistent
// kernel keeps four.
#include "device_common.h"
#include "mdd_internal.h"

namespace mdd {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ floatx4 mfma4(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Complex multiply-add C += A B on 16x16x4 tiles with three real products instead of
// four: with A = a + ib and B = c + id (lane values of the operand fragments),
//   t1 += a (c + d),  t2 += (a + b) d,  t3 += (b - a) c,
// so that Re C = t1 - t2 and Im C = t1 + t3 (cmac3_finish).  The operand sums are
// vector-unit additions on the lane values; bsum = c + d is shared by the row tiles.
__device__ __forceinline__ void cmac3(float2 av, float2 bv, float bsum, floatx4& t1, floatx4& t2,
                                     floatx4& t3) {
  t1 = mfma4(av.x, bsum, t1);
  t2 = mfma4(av.x + av.y, bv.y, t2);
  t3 = mfma4(av.y - av.x, bv.x, t3);
}

// (t1, t2, t3) -> (Re, Im) in (t1, t2).
__device__ __forceinline__ void cmac3_finish(floatx4& t1, floatx4& t2, const floatx4& t3) {
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const float x = t1[e];
    t1[e] = x - t2[e];
    t2[e] = x + t3[e];
  }
}

// Float32 complex multiply-add in the form the precision asks for: three real
// products (cmac3, accumulators t1 t2 t3) for MDD_PREC_FP32, or the four of a plain
// complex GEMM into (re, im) directly for MDD_PREC_FP32_CGEMM (t3 unused).
template <int PREC>
__device__ __forceinline__ void cmac(float2 av, float2 bv, float bsum, floatx4& re, floatx4& im,
                                     floatx4& t3) {
  if constexpr (PREC == MDD_PREC_FP32) {
    cmac3(av, bv, bsum, re, im, t3);
  } else {
    re = mfma4(av.x, bv.x, re);
    re = mfma4(-av.y, bv.y, re);
    im = mfma4(av.x, bv.y, im);
    im = mfma4(av.y, bv.x, im);
  }
}

template <int PREC>
__device__ __forceinline__ void cmac_finish(floatx4& re, floatx4& im, const floatx4& t3) {
  if constexpr (PREC == MDD_PREC_FP32) cmac3_finish(re, im, t3);
}

template <int PREC>
constexpr bool is_fp32() { return PREC == MDD_PREC_FP32 || PREC == MDD_PREC_FP32_CGEMM; }

// Operand of a 16x16x32 split-precision MFMA: 8 consecutive k values of one
// row (A) or one column (B), real and imaginary parts, hi and lo.
template <int PREC>
struct SplitOp;

template <>
struct SplitOp<MDD_PREC_BF16X3> {
  using V = bf16x8;
  V rh, rl, ih, il;
  __device__ __forceinline__ void set(int e, float2 z) {
    const __bf16 a = (__bf16)z.x, b = (__bf16)z.y;
    rh[e] = a;
    ih[e] = b;
    rl[e] = (__bf16)(z.x - (float)a);
    il[e] = (__bf16)(z.y - (float)b);
  }
  static __device__ __forceinline__ floatx4 mma(V a, V b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

template <>
struct SplitOp<MDD_PREC_BF16> {
  using V = bf16x8;
  V rh, rl, ih, il;
  __device__ __forceinline__ void set(int e, float2 z) {
    rh[e] = (__bf16)z.x;
    ih[e] = (__bf16)z.y;
    rl[e] = (__bf16)0.f;
    il[e] = (__bf16)0.f;
  }
  static __device__ __forceinline__ floatx4 mma(V a, V b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

template <>
struct SplitOp<MDD_PREC_FP16X3> {
  using V = halfx8;
  V rh, rl, ih, il;
  __device__ __forceinline__ void set(int e, float2 z) {  // operands are pre-scaled
    const _Float16 a = (_Float16)z.x, b = (_Float16)z.y;
    rh[e] = a;
    ih[e] = b;
    rl[e] = (_Float16)(z.x - (float)a);
    il[e] = (_Float16)(z.y - (float)b);
  }
  static __device__ __forceinline__ floatx4 mma(V a, V b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

// acc += A * B (complex), or A^H-style when the caller passes conj(A).
template <int PREC, typename Op>
__device__ __forceinline__ void split_cmma(const Op& A, const Op& B, floatx4& re, floatx4& im) {
  using V = typename Op::V;
  const V nih = -A.ih, nil = -A.il;
  if constexpr (PREC == MDD_PREC_BF16) {
    re = Op::mma(A.rh, B.rh, re);
    re = Op::mma(nih, B.ih, re);
    im = Op::mma(A.rh, B.ih, im);
    im = Op::mma(A.ih, B.rh, im);
  } else {
    re = Op::mma(A.rh, B.rh, re);
    re = Op::mma(A.rh, B.rl, re);
    re = Op::mma(A.rl, B.rh, re);
    re = Op::mma(nih, B.ih, re);
    re = Op::mma(nih, B.il, re);
    re = Op::mma(nil, B.ih, re);
    im = Op::mma(A.rh, B.ih, im);
    im = Op::mma(A.rh, B.il, im);
    im = Op::mma(A.rl, B.ih, im);
    im = Op::mma(A.ih, B.rh, im);
    im = Op::mma(A.ih, B.rl, im);
    im = Op::mma(A.il, B.rh, im);
  }
}

// Power-of-two scale bringing max |x| near 2^14 (fp16 split keeps 22 bits
// for entries down to ~2^-8 of the tile maximum).
__device__ __forceinline__ float pow2_scale(float amax) {
  if (!(amax > 0.f) || !(amax < 3.0e38f)) return 1.f;
  int e;
  frexpf(amax, &e);  // amax = m 2^e, m in [0.5, 1)
  return ldexpf(1.f, 14 - e);
}

template <int PREC, int NBT, int TNB>
struct GemmCfg {
  static constexpr int MB = NBT * 16;                 // padded batch rows
  static constexpr int NW = TNB * 16;                 // columns per workgroup
  static constexpr int TILES = NBT * TNB;             // 16x16 output tiles of the forward product
  static constexpr int S = TILES >= 4 ? 1 : 4 / TILES;  // waves splitting K
  static constexpr int G = 4 / S;                     // wave groups over tiles
  static constexpr int TPWV = TILES / G;              // tiles per wave
  static constexpr bool SPLIT = !is_fp32<PREC>();
  static constexpr int KSTEP = SPLIT ? 32 : 4;        // receivers per MFMA
  static constexpr int KCMAX = NBT == 1 ? (SPLIT ? 256 : 224) : (NBT == 2 ? 128 : 64);  // receiver chunk
  static constexpr int KSW = KCMAX / KSTEP / S;       // k-steps per wave per chunk
  static constexpr int BREG = SPLIT ? 8 : 1;          // right-operand values per lane per k-step
  static constexpr int DST = KCMAX + 2;               // LDS row stride of D (16-byte aligned)
  static constexpr int RST = NW + 1;                  // LDS row stride of the residual
  static constexpr int RED_SZ = S > 1 ? S * MB * NW : 0;
  static constexpr size_t SMEM = sizeof(float2) * ((size_t)MB * DST + RED_SZ + (size_t)MB * RST);
  static_assert(TILES % G == 0 && KCMAX % (KSTEP * S) == 0, "tiling");
  // Tiles of one wave share their column tile when TILES >= 4 (tile = g + t * G).
  static_assert(S > 1 || G % TNB == 0, "a wave's tiles must share one column tile");
};

template <int PREC, int NBT, int TNB, int KIND>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs a) {
  using C = GemmCfg<PREC, NBT, TNB>;
  constexpr int MB = C::MB, NW = C::NW, KCMAX = C::KCMAX, KSTEP = C::KSTEP;
  extern __shared__ float2 smem[];
  float2* s_d = smem;                       // D_{b,k} chunk [MB][DST]
  float2* s_part = s_d + MB * C::DST;       // split-K partials [S][MB][NW] (S > 1)
  float2* s_res = s_part + C::RED_SZ;       // residual [MB][RST]
  __shared__ int s_idx[MB];
  __shared__ long long s_drow[MB];          // element offset of row idx[b] of D_k (or -1)
  __shared__ double s_red[4];
  __shared__ float s_scale[4];              // fp16 split: per-chunk max-abs exchange

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lq = lane >> 4;

  // Map the linear workgroup id so that the column groups of one frequency run
  // on the same XCD (dispatch is round-robin over the 8 XCDs): they share D_k.
  const int ncg = (a.nvb + TNB - 1) / TNB;
  const int total = a.nf * ncg;
  const int bid = blockIdx.x;
  const int full = (total / 8) * 8;
  const int logical = bid < full ? (bid % 8) * (total / 8) + bid / 8 : bid;
  const int k = logical / ncg, cg = logical % ncg;
  const int blk0 = cg * TNB;
  const int nchunks = (a.nr + KCMAX - 1) / KCMAX;
  const double wk = (k == 0 || 2 * k == a.nt) ? 1.0 : 2.0;
  // F element (r, blk, k, c) is at r * rowstride + (blk * nf + k) * CB + c.
  const long long rowstride = (long long)a.nvb * a.nf * CB;

  auto fill_idx = [&]() {
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
  };
  if constexpr (KIND == GK_ADJ) fill_idx();

  // Rows r0 .. r0 + lenp of D_{b,k} -> s_d (zero beyond nr and for bad indices).
  auto load_d_chunk = [&](int r0, int lenp) {
    constexpr int PAIRS = KCMAX / 2;
    for (int i = tid; i < MB * PAIRS; i += 256) {
      const int b = i / PAIRS, rr = 2 * (i % PAIRS);
      if (rr >= lenp) continue;
      const long long off = s_drow[b];
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (off >= 0 && r0 + rr < a.nr) v = *reinterpret_cast<const float4*>(a.Df + off + r0 + rr);
      s_d[b * C::DST + rr] = make_float2(v.x, v.y);
      s_d[b * C::DST + rr + 1] = make_float2(v.z, v.w);
    }
  };

  auto block_amax_scale = [&](float m) -> float {  // fp16 split: power-of-two scale of a block
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    if (lane == 0) s_scale[wave] = m;
    __syncthreads();
    const float amax = fmaxf(fmaxf(s_scale[0], s_scale[1]), fmaxf(s_scale[2], s_scale[3]));
    __syncthreads();
    return pow2_scale(amax);
  };
  auto lds_amax = [&](const float2* base, int rows, int stride, int cols) -> float {
    float m = 0.f;
    for (int i = tid; i < rows * cols; i += 256) {
      const float2 z = base[(i / cols) * stride + (i % cols)];
      m = fmaxf(m, fmaxf(fabsf(z.x), fabsf(z.y)));
    }
    return m;
  };

  int last_r0 = -1;  // receiver chunk resident in s_d

  // ------------------------------------------------------------ forward
  if constexpr (KIND != GK_ADJ) {
    const int g = wave % C::G, ks = wave / C::G;
    const int nt_w = g % TNB;                       // column tile of this wave (S == 1)
    // Right operand (R_k rows of this wave's k-steps), straight from HBM into
    // registers: each load instruction reads 4 rows x 16 columns = 4 x 128 B.
    // With S > 1 every wave uses the single column tile 0.
    float2 bfr[C::KSW][C::BREG];
    const int ncol_blk = blk0 + (C::S == 1 ? nt_w : 0);
    auto load_b = [&](int r0, int len) {
      const int rr0 = ks * KSTEP + (C::SPLIT ? lq * 8 : lq);
      const float2* fb =
          a.F + (r0 + rr0) * rowstride + ((long long)ncol_blk * a.nf + k) * CB + lr;
      const bool colok = ncol_blk < a.nvb;
#pragma unroll
      for (int q = 0; q < C::KSW; ++q) {
#pragma unroll
        for (int e = 0; e < C::BREG; ++e) {
          const int dr = q * C::S * KSTEP + e;     // row offset from rr0
          float2 v = make_float2(0.f, 0.f);
          if (colok && rr0 + dr < len) v = fb[dr * rowstride];
          bfr[q][e] = v;
        }
      }
    };
    load_b(0, min(KCMAX, a.nr));   // issued before the batch indices are known
    fill_idx();
    float2 upre[C::TPWV][4];                        // data entries subtracted later (S == 1)
    float2 upre_s[(MB * NW + 255) / 256];           // the same for S > 1
    if constexpr (KIND == GK_FUSED && C::S > 1) {
#pragma unroll
      for (int q = 0; q < (MB * NW + 255) / 256; ++q) {
        const int i = tid + 256 * q;
        const int row = i / NW, col = i % NW;
        const int vs = blk0 * CB + col;
        upre_s[q] = make_float2(0.f, 0.f);
        if (i < MB * NW && row < a.nb && vs < a.nvs && s_idx[row] >= 0)
          upre_s[q] = a.Uf[urow_off(a, k, row, s_idx[row]) + vs];
      }
    }
    if constexpr (KIND == GK_FUSED && C::S == 1) {
#pragma unroll
      for (int t = 0; t < C::TPWV; ++t) {
        const int mt = (g + t * C::G) / TNB;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = mt * 16 + lq * 4 + e, vs = (blk0 + nt_w) * CB + lr;
          upre[t][e] = make_float2(0.f, 0.f);
          if (row < a.nb && vs < a.nvs && s_idx[row] >= 0)
            upre[t][e] = a.Uf[urow_off(a, k, row, s_idx[row]) + vs];
        }
      }
    }
    floatx4 acc_re[C::TPWV], acc_im[C::TPWV];
    floatx4 acc_3[C::SPLIT ? 1 : C::TPWV];         // float32: the third product of cmac3
#pragma unroll
    for (int t = 0; t < C::TPWV; ++t) {
      acc_re[t] = floatx4{0.f, 0.f, 0.f, 0.f};
      acc_im[t] = floatx4{0.f, 0.f, 0.f, 0.f};
      if constexpr (!C::SPLIT) acc_3[t] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
    for (int r0 = 0; r0 < a.nr; r0 += KCMAX) {
      const int len = min(KCMAX, a.nr - r0);
      const int lenp = (len + 31) & ~31;
      if (r0 > 0) {
        load_b(r0, len);
        __syncthreads();
      }
      load_d_chunk(r0, lenp);
      last_r0 = r0;
      __syncthreads();
      float fp16_sd = 1.f, fp16_sr = 1.f;
      floatx4 cre[C::TPWV], cim[C::TPWV];             // fp16 split: per-chunk accumulators
      if constexpr (PREC == MDD_PREC_FP16X3) {
        fp16_sd = block_amax_scale(lds_amax(s_d, MB, C::DST, lenp));
        float m = 0.f;
#pragma unroll
        for (int q = 0; q < C::KSW; ++q)
#pragma unroll
          for (int e = 0; e < C::BREG; ++e)
            m = fmaxf(m, fmaxf(fabsf(bfr[q][e].x), fabsf(bfr[q][e].y)));
        fp16_sr = block_amax_scale(m);
#pragma unroll
        for (int t = 0; t < C::TPWV; ++t) {
          cre[t] = floatx4{0.f, 0.f, 0.f, 0.f};
          cim[t] = floatx4{0.f, 0.f, 0.f, 0.f};
        }
      }
#pragma unroll
      for (int q = 0; q < C::KSW; ++q) {
        const int kk = ks + q * C::S;
        if (kk * KSTEP >= lenp) break;
        if constexpr (!C::SPLIT) {
          const float2 rv = bfr[q][0];
          const float rsum = rv.x + rv.y;
#pragma unroll
          for (int t = 0; t < C::TPWV; ++t) {
            const int mt = (g + t * C::G) / TNB;
            cmac<PREC>(s_d[(mt * 16 + lr) * C::DST + kk * 4 + lq], rv, rsum, acc_re[t], acc_im[t],
                       acc_3[t]);
          }
        } else {
          using Op = SplitOp<PREC>;
          Op B;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            float2 rv = bfr[q][e];
            if constexpr (PREC == MDD_PREC_FP16X3) rv = cscale(rv, fp16_sr);
            B.set(e, rv);
          }
#pragma unroll
          for (int t = 0; t < C::TPWV; ++t) {
            const int mt = (g + t * C::G) / TNB;
            Op A;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              float2 dv = s_d[(mt * 16 + lr) * C::DST + kk * 32 + lq * 8 + e];
              if constexpr (PREC == MDD_PREC_FP16X3) dv = cscale(dv, fp16_sd);
              A.set(e, dv);
            }
            if constexpr (PREC == MDD_PREC_FP16X3) split_cmma<PREC>(A, B, cre[t], cim[t]);
            else split_cmma<PREC>(A, B, acc_re[t], acc_im[t]);
          }
        }
      }
      if constexpr (PREC == MDD_PREC_FP16X3) {
        const float inv = 1.f / (fp16_sd * fp16_sr);
#pragma unroll
        for (int t = 0; t < C::TPWV; ++t) {
          acc_re[t] += cre[t] * inv;
          acc_im[t] += cim[t] * inv;
        }
      }
    }

    if constexpr (!C::SPLIT) {
#pragma unroll
      for (int t = 0; t < C::TPWV; ++t) cmac_finish<PREC>(acc_re[t], acc_im[t], acc_3[t]);
    }

    // Residual (or predicted data) and the loss partial.
    double lpart = 0.0;
    if constexpr (C::S == 1) {
#pragma unroll
      for (int t = 0; t < C::TPWV; ++t) {
        const int mt = (g + t * C::G) / TNB;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = mt * 16 + lq * 4 + e, col = nt_w * 16 + lr;
          const int vs = blk0 * CB + col;
          const bool ok = row < a.nb && vs < a.nvs && s_idx[row] >= 0;
          float2 z = make_float2(acc_re[t][e], acc_im[t][e]);
          if constexpr (KIND == GK_FUSED) {
            if (ok) {
              z = csub(z, upre[t][e]);
              lpart += wk * ((double)z.x * z.x + (double)z.y * z.y);
            } else {
              z = make_float2(0.f, 0.f);
            }
            s_res[row * C::RST + col] = z;
          } else {
            if (row < a.nb && blk0 + nt_w < a.nvb)
              a.Bsp[(((size_t)row * a.nvb + blk0 + nt_w) * a.nf + k) * CB + lr] =
                  ok ? z : make_float2(0.f, 0.f);
          }
        }
      }
    } else {
#pragma unroll
      for (int t = 0; t < C::TPWV; ++t) {
        const int tile = g + t * C::G;
        const int mt = tile / TNB, nt = tile % TNB;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = mt * 16 + lq * 4 + e, col = nt * 16 + lr;
          s_part[(ks * MB + row) * NW + col] = make_float2(acc_re[t][e], acc_im[t][e]);
        }
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < (MB * NW + 255) / 256; ++q) {
        const int i = tid + 256 * q;
        if (i >= MB * NW) break;
        const int row = i / NW, col = i % NW;
        float2 z = s_part[row * NW + col];
#pragma unroll
        for (int s = 1; s < C::S; ++s) z = cadd(z, s_part[(s * MB + row) * NW + col]);
        const int vs = blk0 * CB + col;
        const bool ok = row < a.nb && vs < a.nvs && s_idx[row] >= 0;
        if constexpr (KIND == GK_FUSED) {
          if (ok) {
            z = csub(z, upre_s[q]);
            lpart += wk * ((double)z.x * z.x + (double)z.y * z.y);
          } else {
            z = make_float2(0.f, 0.f);
          }
          s_res[row * C::RST + col] = z;
        } else {
          const int blk = blk0 + col / 16;
          if (row < a.nb && blk < a.nvb)
            a.Bsp[(((size_t)row * a.nvb + blk) * a.nf + k) * CB + (col & 15)] =
                ok ? z : make_float2(0.f, 0.f);
        }
      }
    }
    if constexpr (KIND == GK_FUSED) {
      const double tot = block_sum256(lpart, s_red);
      if (tid == 0) a.loss_part[logical] = tot;
    }
    if constexpr (KIND == GK_FWD) return;
  } else {
    // Adjoint only: the batch spectra V_k are the right-hand operand.
    for (int i = tid; i < MB * NW; i += 256) {
      const int row = i / NW, col = i % NW;
      const int blk = blk0 + col / 16;
      float2 z = make_float2(0.f, 0.f);
      if (row < a.nb && blk < a.nvb && s_idx[row] >= 0)
        z = a.Bsp[(((size_t)row * a.nvb + blk) * a.nf + k) * CB + (col & 15)];
      s_res[row * C::RST + col] = z;
    }
  }
  __syncthreads();

  // ------------------------------------------------------------ adjoint
  float fp16_ss = 1.f;
  if constexpr (PREC == MDD_PREC_FP16X3)
    fp16_ss = block_amax_scale(lds_amax(s_res, MB, C::RST, NW));
  for (int r0 = 0; r0 < a.nr; r0 += KCMAX) {
    const int len = min(KCMAX, a.nr - r0);
    const int lenp = (len + 31) & ~31;
    if (!(nchunks == 1 && last_r0 == r0)) {   // the single chunk is still resident
      if (r0 > 0) __syncthreads();
      load_d_chunk(r0, lenp);
      __syncthreads();
    }
    float fp16_sd = 1.f;
    if constexpr (PREC == MDD_PREC_FP16X3) fp16_sd = block_amax_scale(lds_amax(s_d, MB, C::DST, lenp));
    for (int mt = wave; mt * 16 < len; mt += 4) {
#pragma unroll
      for (int nt = 0; nt < TNB; ++nt) {
        floatx4 re = floatx4{0.f, 0.f, 0.f, 0.f}, im = floatx4{0.f, 0.f, 0.f, 0.f};
        if constexpr (!C::SPLIT) {
          floatx4 t3 = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int kk = 0; kk < MB / 4; ++kk) {
            const float2 sv = s_res[(kk * 4 + lq) * C::RST + nt * 16 + lr];
            cmac<PREC>(cconj(s_d[(kk * 4 + lq) * C::DST + mt * 16 + lr]), sv, sv.x + sv.y, re, im,
                       t3);
          }
          cmac_finish<PREC>(re, im, t3);
        } else {
          using Op = SplitOp<PREC>;
#pragma unroll
          for (int kk = 0; kk < (MB + 31) / 32; ++kk) {
            Op A, B;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const int b = kk * 32 + lq * 8 + e;
              float2 dv = make_float2(0.f, 0.f), sv = make_float2(0.f, 0.f);
              if (b < MB) {
                dv = cconj(s_d[b * C::DST + mt * 16 + lr]);
                sv = s_res[b * C::RST + nt * 16 + lr];
              }
              if constexpr (PREC == MDD_PREC_FP16X3) {
                dv = cscale(dv, fp16_sd);
                sv = cscale(sv, fp16_ss);
              }
              A.set(e, dv);
              B.set(e, sv);
            }
            split_cmma<PREC>(A, B, re, im);
          }
          if constexpr (PREC == MDD_PREC_FP16X3) {
            const float inv = 1.f / (fp16_sd * fp16_ss);
            re *= inv;
            im *= inv;
          }
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

// s <- s + x with the rounding error of that addition added to the compensation e
// (Dekker's Fast2Sum on each lane value: the error term is exact when |s| >= |x|,
// which holds once the running total dominates one chunk's sum; when it does not,
// the sum itself is still the rounded one).
__device__ __forceinline__ void two_sum(floatx4& s, floatx4& e, const floatx4& x) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float t = s[i] + x[i];
    e[i] += x[i] - (t - s[i]);
    s[i] = t;
  }
}

// Float32 fused products for 33..64 batch rows: a warp-specialised workgroup of
// twelve waves.  Four loader waves keep three 64-receiver chunks of R_k (96 KB)
// in flight in their registers and pass each through a two-slot LDS ring; eight
// compute waves stage D_{b,k} chunks (double-buffered) and run the forward
// 16x16x4 products, one barrier per chunk.  The adjoint has no barrier: each
// compute wave owns receiver tiles and loads its A operand (conj D, one batch
// row group per k-step) from L2 straight into registers.  All loads are
// unconditional (addresses clamped into the arrays, zeros applied where the
// values are used), so that each wait covers only the loads it needs.
constexpr int WF_DEPTH = 3;
constexpr int WF_CW = 8;                      // compute waves (two per SIMD)
constexpr int WF_LW = 4;                      // loader waves
constexpr int WF_THREADS = 64 * (WF_CW + WF_LW);
constexpr int WF_KC = 64;                     // receivers per chunk
constexpr int WF_DP = WF_KC + 4;              // D slot row pitch [b][r] (complex)
constexpr int WF_RP = 64 + 16;                // ring / residual row pitch [r or b][col]
constexpr size_t WF_SMEM = sizeof(float2) * (2 * 64 * WF_DP + 2 * WF_KC * WF_RP);

template <int KIND, int PREC>
__global__ __launch_bounds__(WF_THREADS) void k_gemm_ws(GemmArgs a) {
  constexpr int MB = 64, NW = 64, KC = WF_KC;
  constexpr int NCT = 64 * WF_CW, NLT = 64 * WF_LW;
  constexpr int LPT = KC * NW / 2 / NLT;      // float4 per loader thread per chunk
  constexpr int FPT = MB * (KC / 2) / NCT;    // D float4 per compute thread per chunk
  constexpr int TPC = 2;                      // forward row tiles per compute wave
  constexpr int RING = KC * WF_RP, DSL = MB * WF_DP;
  static_assert(LPT * NLT == KC * NW / 2 && FPT * NCT == MB * (KC / 2), "split");
  extern __shared__ float2 smem_f2[];
  float2* s_d = smem_f2;                      // two D slots [b][r]
  float2* s_ring = smem_f2 + 2 * DSL;         // two R slots [r][col]
  float2* s_res = s_ring;                     // residual [b][col], after the forward
  __shared__ int s_idx[MB];
  __shared__ long long s_drow[MB];
  __shared__ double s_red[WF_CW];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool compute = wave < WF_CW;
  const int lr = lane & 15, lq = lane >> 4;
  const int ncg = (a.nvb + 3) / 4;
  const int total = a.nf * ncg;
  const int bid = blockIdx.x, full = (total / 8) * 8;
  const int logical = bid < full ? (bid % 8) * (total / 8) + bid / 8 : bid;
  const int k = logical / ncg, cg = logical % ncg;  // the column groups of one frequency share an XCD
  const int blk0 = cg * 4;
  const long long rowstride = (long long)a.nvb * a.nf * CB;
  const int nc = (a.nr + KC - 1) / KC;
  const int nt_w = wave & 3, rt0 = (wave >> 2) * TPC;
  const int li = tid - NCT;

  for (int b = tid; b < MB; b += WF_THREADS) {
    int s = -1;
    if (b < a.nb) {
      s = a.idx[b];
      if (s < 0 || s >= a.ns) s = -1;
    }
    s_idx[b] = s;
    s_drow[b] = s >= 0 ? ((long long)k * a.dns + drow_of(a, b, s)) * a.nrp : -1;
  }
  __syncthreads();

  const long long drow0 = (long long)k * a.dns * a.nrp;
  auto d_at = [&](int b, int r) -> long long {  // always in bounds
    const long long off = s_drow[b];
    return (off >= 0 ? off : drow0) + (r < a.nr ? r : 0);
  };
  auto d_ok = [&](int b, int r) { return s_drow[b] >= 0 && r < a.nr; };

  if constexpr (KIND == GK_ADJ) {  // the residual planes are the batch spectra V_k
    if (compute) {
      for (int i = tid; i < MB * NW; i += NCT) {
        const int row = i / NW, col = i % NW, blk = blk0 + col / CB;
        float2 z = make_float2(0.f, 0.f);
        if (row < a.nb && blk0 * CB + col < a.nvs && s_idx[row] >= 0)
          z = a.Bsp[(((size_t)row * a.nvb + blk) * a.nf + k) * CB + (col & 15)];
        s_res[row * WF_RP + col] = z;
      }
    }
  } else if (compute) {
    float4 dv[FPT];
    auto load_d = [&](int c) {
#pragma unroll
      for (int q = 0; q < FPT; ++q) {
        const int i = tid + NCT * q;
        dv[q] = *reinterpret_cast<const float4*>(a.Df + d_at(i / (KC / 2), c * KC + 2 * (i % (KC / 2))));
      }
    };
    auto stage_d = [&](int sl, int c) {
#pragma unroll
      for (int q = 0; q < FPT; ++q) {
        const int i = tid + NCT * q;
        const int b = i / (KC / 2), rr = 2 * (i % (KC / 2)), r = c * KC + rr;
        float4 v = d_ok(b, r) ? dv[q] : make_float4(0.f, 0.f, 0.f, 0.f);
        if (r + 1 >= a.nr) v.z = v.w = 0.f;
        *reinterpret_cast<float4*>(s_d + sl * DSL + b * WF_DP + rr) = v;
      }
    };
    // per tile: (re, im) and the third accumulator of cmac3 (unused by the cgemm form),
    // and their compensation terms
    floatx4 ar[TPC], ai[TPC], a3[TPC], er[TPC], ei[TPC], e3[TPC];
#pragma unroll
    for (int t = 0; t < TPC; ++t) {
      ar[t] = floatx4{0.f, 0.f, 0.f, 0.f};
      ai[t] = floatx4{0.f, 0.f, 0.f, 0.f};
      a3[t] = floatx4{0.f, 0.f, 0.f, 0.f};
      er[t] = floatx4{0.f, 0.f, 0.f, 0.f};
      ei[t] = floatx4{0.f, 0.f, 0.f, 0.f};
      e3[t] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
    load_d(0);
    __syncthreads();
    stage_d(0, 0);
    load_d(1);
    __syncthreads();
#pragma unroll 1
    for (int c = 0; c < nc; ++c) {
      const int sl = c & 1;
      const float2* ring = s_ring + sl * RING + lq * WF_RP + nt_w * 16 + lr;
      const float2* dsl = s_d + sl * DSL + (rt0 * 16 + lr) * WF_DP + lq;
      // two-level sum: each chunk's 16 k-steps start from zero and the chunk's sum is
      // added to the total with its rounding error carried in a compensation term
      // (TwoSum), so the products' rounding grows with the chunk length, not with nr
      floatx4 cr[TPC], ci[TPC], c3[TPC];
#pragma unroll
      for (int t = 0; t < TPC; ++t) {
        cr[t] = floatx4{0.f, 0.f, 0.f, 0.f};
        ci[t] = floatx4{0.f, 0.f, 0.f, 0.f};
        c3[t] = floatx4{0.f, 0.f, 0.f, 0.f};
      }
#pragma unroll
      for (int ks = 0; ks < KC / 4; ++ks) {  // rows past nr are zeros in both operands
        const float2 bv = ring[ks * 4 * WF_RP];
        const float bsum = bv.x + bv.y;
#pragma unroll
        for (int t = 0; t < TPC; ++t)
          cmac<PREC>(dsl[t * 16 * WF_DP + ks * 4], bv, bsum, cr[t], ci[t], c3[t]);
      }
#pragma unroll
      for (int t = 0; t < TPC; ++t) {
        two_sum(ar[t], er[t], cr[t]);
        two_sum(ai[t], ei[t], ci[t]);
        two_sum(a3[t], e3[t], c3[t]);
      }
      stage_d(sl ^ 1, c + 1);  // the next chunk into the slot chunk c - 1 used
      load_d(c + 2);
      __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < TPC; ++t) {
      ar[t] += er[t];
      ai[t] += ei[t];
      a3[t] += e3[t];
      cmac_finish<PREC>(ar[t], ai[t], a3[t]);
    }

    if constexpr (KIND == GK_FWD) {  // P_k = D_b R_k -> batch spectra
#pragma unroll
      for (int t = 0; t < TPC; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = (rt0 + t) * 16 + lq * 4 + e, col = nt_w * 16 + lr, blk = blk0 + nt_w;
          if (row < a.nb && blk < a.nvb) {
            const bool ok = blk0 * CB + col < a.nvs && s_idx[row] >= 0;
            a.Bsp[(((size_t)row * a.nvb + blk) * a.nf + k) * CB + lr] =
                ok ? make_float2(ar[t][e], ai[t][e]) : make_float2(0.f, 0.f);
          }
        }
    } else {
    // residual and float64 loss partial
    float2 uv[TPC][4];
#pragma unroll
    for (int t = 0; t < TPC; ++t)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = (rt0 + t) * 16 + lq * 4 + e, vs = blk0 * CB + nt_w * 16 + lr;
        const int s = row < a.nb ? max(s_idx[row], 0) : 0;
        uv[t][e] = a.Uf[urow_off(a, k, row < a.nb ? row : 0, s) + min(vs, a.nvsp - 1)];
      }
    double lpart = 0.0;
#pragma unroll
    for (int t = 0; t < TPC; ++t) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = (rt0 + t) * 16 + lq * 4 + e, col = nt_w * 16 + lr;
        const int vs = blk0 * CB + col;
        float2 z = make_float2(ar[t][e], ai[t][e]);
        if (row < a.nb && vs < a.nvs && s_idx[row] >= 0) {
          z = csub(z, uv[t][e]);
          lpart += (k == 0 || 2 * k == a.nt ? 1.0 : 2.0) * ((double)z.x * z.x + (double)z.y * z.y);
        } else {
          z = make_float2(0.f, 0.f);
        }
        s_res[row * WF_RP + col] = z;  // the ring is no longer read
      }
    }
    lpart = wave_sum(lpart);
    if (lane == 0) s_red[wave] = lpart;
    }
  } else {
    float4 rq[WF_DEPTH][LPT];
    auto issue = [&](float4 (&dst)[LPT], int c) {
#pragma unroll
      for (int q = 0; q < LPT; ++q) {
        const int i = li + NLT * q;
        const int rr = i / (NW / 2), cp = 2 * (i % (NW / 2));
        const int r = min(c * KC + rr, a.nr - 1), blk = min(blk0 + cp / CB, a.nvb - 1);
        dst[q] = *reinterpret_cast<const float4*>(a.F + (long long)r * rowstride +
                                                  ((long long)blk * a.nf + k) * CB + cp % CB);
      }
    };
    auto put_ring = [&](const float4 (&src)[LPT], int c) {
#pragma unroll
      for (int q = 0; q < LPT; ++q) {
        const int i = li + NLT * q;
        const int rr = i / (NW / 2), cp = 2 * (i % (NW / 2));
        const bool ok = c * KC + rr < a.nr && blk0 + cp / CB < a.nvb;
        *reinterpret_cast<float4*>(s_ring + (c & 1) * RING + rr * WF_RP + cp) =
            ok ? src[q] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    };
    issue(rq[0], 0);
    issue(rq[1], 1);
    issue(rq[2], 2);
    __syncthreads();
    put_ring(rq[0], 0);
    issue(rq[0], 3);
    __syncthreads();
    int c0 = 0;
#pragma unroll 1
    for (; c0 + WF_DEPTH <= nc; c0 += WF_DEPTH) {
#pragma unroll
      for (int u = 0; u < WF_DEPTH; ++u) {  // chunk c + 1 into the slot chunk c - 1 used
        const int c = c0 + u;
        put_ring(rq[(u + 1) % WF_DEPTH], c + 1);
        issue(rq[(u + 1) % WF_DEPTH], c + 1 + WF_DEPTH);
        __syncthreads();
      }
    }
#pragma unroll
    for (int u = 0; u < WF_DEPTH - 1; ++u) {
      const int c = c0 + u;
      if (c < nc) {
        put_ring(rq[(u + 1) % WF_DEPTH], c + 1);
        __syncthreads();
      }
    }
  }
  __syncthreads();  // residual complete; the last barrier of the loader waves
  if constexpr (KIND == GK_FUSED) {
    if (tid == 0) {
      double tot = 0.0;
      for (int w = 0; w < WF_CW; ++w) tot += s_red[w];
      a.loss_part[logical] = tot;
    }
  }
  if (KIND == GK_FWD) return;

  // adjoint: G_k = D_b^H Res over this wave's receiver tiles, written over R_k; the
  // loader waves, their ring work done, take tiles too
  const int nrt = (a.nr + 15) / 16;
  auto load_tile = [&](float2 (&d)[16], int mt) {  // conj D operand: b = ks*4 + lq
    const int r = min(mt * 16 + lr, a.nr - 1);
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) d[ks] = a.Df[d_at(ks * 4 + lq, r)];
  };
  float2 dn[16];
  load_tile(dn, min(wave, nrt - 1));
#pragma unroll 1
  for (int mt = wave; mt < nrt; mt += WF_CW + WF_LW) {
    float2 dc[16];
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) dc[ks] = dn[ks];
    load_tile(dn, min(mt + WF_CW + WF_LW, nrt - 1));
    const int r = mt * 16 + lr;
#pragma unroll
    for (int ks = 0; ks < 16; ++ks)
      if (!d_ok(ks * 4 + lq, r)) dc[ks] = make_float2(0.f, 0.f);
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) dc[ks].y = -dc[ks].y;  // conj D
#pragma unroll 1
    for (int nt = 0; nt < 4; ++nt) {
      floatx4 re = floatx4{0.f, 0.f, 0.f, 0.f}, im = floatx4{0.f, 0.f, 0.f, 0.f};
      floatx4 t3 = floatx4{0.f, 0.f, 0.f, 0.f};
      const float2* res = s_res + lq * WF_RP + nt * 16 + lr;
#pragma unroll
      for (int ks = 0; ks < 16; ++ks) {
        const float2 sv = res[ks * 4 * WF_RP];
        cmac<PREC>(dc[ks], sv, sv.x + sv.y, re, im, t3);
      }
      cmac_finish<PREC>(re, im, t3);
      const int blk = blk0 + nt;
      if (blk < a.nvb) {
        const int rb = mt * 16 + lq * 4;
        float2* fw = a.F + (long long)rb * rowstride + ((long long)blk * a.nf + k) * CB + lr;
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (rb + e < a.nr) store_g(a, (fw - a.F) + e * rowstride, make_float2(re[e], im[e]));
      }
    }
  }
}

// Persistent, software-pipelined form of the fused product for float32, at most
// 16 batch rows and at most PIPE_KC receivers (one chunk).  Each workgroup walks a
// contiguous range of (frequency, column group) items: while one item's products
// run, the next item's R_k fragments and data entries are already in flight, and
// D_{b,k} stays in LDS for as long as the frequency does not change.
constexpr int PIPE_KC = 224;
constexpr int PIPE_WGS = 768;   // 3 workgroups on each of the 256 CUs (registers capped to fit)

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_gemm_pipe(GemmArgs a) {
  constexpr int MB = 16, NW = 16, DST = PIPE_KC + 2, RST = NW + 1;
  constexpr int KSW = PIPE_KC / 4 / 4;        // k-steps per wave (4 waves split K)
  constexpr int PAIRS = PIPE_KC / 2;          // float4 pairs per D row
  constexpr int DPT = MB * PAIRS / 256;       // D float4 per thread
  static_assert(KSW == 14, "the wait for the next item's operands names each of them");
  __shared__ float2 s_d[MB * DST];
  __shared__ float2 s_part[4 * MB * NW];
  __shared__ float2 s_res[MB * RST];
  __shared__ int s_idx[MB];
  __shared__ long long s_drow[MB];
  __shared__ double s_red[4];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  const int nvb = a.nvb, total = a.nf * nvb;
  const int G = gridDim.x;
  const int rid = (G % 8 == 0) ? (blockIdx.x % 8) * (G / 8) + blockIdx.x / 8 : blockIdx.x;
  const int start = (int)((long long)rid * total / G), end = (int)((long long)(rid + 1) * total / G);
  if (start >= end) return;
  const long long rowstride = (long long)nvb * a.nf * CB;
  const int lenp = (a.nr + 31) & ~31;

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

  // this thread's residual entry
  const int urow = tid / NW, ucol = tid % NW;
  // R_k / G_k of column group cg live at F + (cg * nf + k) * CB (uniform) plus a
  // 32-bit per-lane offset r * rowstride + lane column.
  const unsigned rs32 = (unsigned)rowstride;
  const unsigned lane_off = (unsigned)(wave * 4 + lq) * rs32 + lr;
  auto load_b = [&](float2 (&dst)[KSW], int k, int cg) {
    const float2* base = a.F + ((long long)cg * a.nf + k) * CB;
#pragma unroll
    for (int q = 0; q < KSW; ++q) {
      const int rr = wave * 4 + lq + q * 16;
      dst[q] = rr < a.nr ? base[lane_off + (unsigned)q * 16u * rs32] : make_float2(0.f, 0.f);
    }
  };
  auto load_u = [&](int k, int cg) -> float2 {
    const int vs = cg * CB + ucol;
    if (urow < a.nb && vs < a.nvs && s_idx[urow] >= 0)
      return a.Uf[urow_off(a, k, urow, s_idx[urow]) + vs];
    return make_float2(0.f, 0.f);
  };
  // D_{b,k} rows -> LDS.  The loads are unconditional (a rejected row reads row 0, a
  // pair past the row reads its last pair) and all in flight at once; what they should
  // not have read is zeroed when it is written to LDS.
  auto stage_d = [&](int k) {
    float4 v[DPT];
#pragma unroll
    for (int q = 0; q < DPT; ++q) {
      const int i = tid + 256 * q;
      const int b = i / PAIRS, rr = 2 * (i % PAIRS);
      const long long off = s_drow[b];
      v[q] = *reinterpret_cast<const float4*>(a.Df + (size_t)k * a.dns * a.nrp + (off >= 0 ? off : 0) +
                                              min(rr, a.nrp - 2));
    }
#pragma unroll
    for (int q = 0; q < DPT; ++q) {
      const int i = tid + 256 * q;
      const int b = i / PAIRS, rr = 2 * (i % PAIRS);
      if (!(s_drow[b] >= 0 && rr < a.nr)) v[q] = make_float4(0.f, 0.f, 0.f, 0.f);
      s_d[b * DST + rr] = make_float2(v[q].x, v[q].y);
      s_d[b * DST + rr + 1] = make_float2(v[q].z, v[q].w);
    }
  };

  double lsum = 0.0;
  int cur = start;
  int k = cur / nvb, cg = cur % nvb;
  float2 bfr[KSW], bnx[KSW];
#pragma unroll
  for (int q = 0; q < KSW; ++q) bnx[q] = make_float2(0.f, 0.f);
  load_b(bfr, k, cg);
  float2 up = load_u(k, cg);
  stage_d(k);
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

    // forward: Res = D_b R_k (split over the 4 waves), then the residual and the loss
    floatx4 ar = floatx4{0.f, 0.f, 0.f, 0.f}, ai = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < KSW; ++q) {
      const int kk = wave + 4 * q;
      if (kk * 4 < lenp) {
        const float2 rv = bfr[q];
        const float2 dv = s_d[lr * DST + kk * 4 + lq];
        ar = mfma4(dv.x, rv.x, ar);
        ar = mfma4(-dv.y, rv.y, ar);
        ai = mfma4(dv.x, rv.y, ai);
        ai = mfma4(dv.y, rv.x, ai);
      }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
      s_part[(wave * MB + lq * 4 + e) * NW + lr] = make_float2(ar[e], ai[e]);
    __syncthreads();
    double lpart = 0.0;
    {
      float2 z = s_part[urow * NW + ucol];
#pragma unroll
      for (int w = 1; w < 4; ++w) z = cadd(z, s_part[(w * MB + urow) * NW + ucol]);
      const int vs = cg * CB + ucol;
      const bool ok = urow < a.nb && vs < a.nvs && s_idx[urow] >= 0;
      if (ok) {
        z = csub(z, up);
        const double wk = (k == 0 || 2 * k == a.nt) ? 1.0 : 2.0;
        lpart = wk * ((double)z.x * z.x + (double)z.y * z.y);
      } else {
        z = make_float2(0.f, 0.f);
      }
      s_res[urow * RST + ucol] = z;
    }
    // The loss is summed per thread over the workgroup's items (a fixed range) and
    // reduced once at the end into the partial of its first item; the others are 0.
    lsum += lpart;
    if (tid == 0) a.loss_part[cur] = 0.0;
    __syncthreads();    // publishes s_res
    // The next item's operands are waited for here, before this item's G stores are
    // issued: loads and stores retire in order under one counter, so a wait at the top
    // of the next iteration would wait for every store of this one as well.
    asm volatile("" ::"v"(bnx[0].x), "v"(bnx[1].x), "v"(bnx[2].x), "v"(bnx[3].x), "v"(bnx[4].x),
                 "v"(bnx[5].x), "v"(bnx[6].x), "v"(bnx[7].x), "v"(bnx[8].x), "v"(bnx[9].x),
                 "v"(bnx[10].x), "v"(bnx[11].x), "v"(bnx[12].x), "v"(bnx[13].x), "v"(upn.x));

    // adjoint: G_k = D_b^H Res over this wave's receiver tiles, written over R_k
    for (int mt = wave; mt * 16 < a.nr; mt += 4) {
      floatx4 re = floatx4{0.f, 0.f, 0.f, 0.f}, im = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kk = 0; kk < MB / 4; ++kk) {
        const float2 dv = s_d[(kk * 4 + lq) * DST + mt * 16 + lr];
        const float2 sv = s_res[(kk * 4 + lq) * RST + lr];
        re = mfma4(dv.x, sv.x, re);
        re = mfma4(dv.y, sv.y, re);
        im = mfma4(dv.x, sv.y, im);
        im = mfma4(-dv.y, sv.x, im);
      }
      const int rb = mt * 16 + lq * 4;
      float2* base = a.F + ((long long)cg * a.nf + k) * CB;
      const unsigned o = (unsigned)rb * rs32 + lr;
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (rb + e < a.nr) store_g(a, (base - a.F) + o + (unsigned)e * rs32, make_float2(re[e], im[e]));
    }
    if (!has_next) break;
    __syncthreads();  // every wave is done with s_d, s_part, s_res of this item
    if (kn != k) {   // new frequency (rare within one workgroup's range)
      stage_d(kn);
      __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < KSW; ++q) bfr[q] = bnx[q];
    up = upn;
    cur = nxt;
    k = kn;
    cg = cgn;
  }
  const double tot = block_sum256(lsum, s_red);
  if (tid == 0) a.loss_part[start] = tot;
}

template <int KIND, int PREC>
hipError_t launch_ws(const GemmArgs& a, hipStream_t s) {
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gemm_ws<KIND, PREC>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)WF_SMEM);
  const int ncg = (a.nvb + 3) / 4;
  hipLaunchKernelGGL((k_gemm_ws<KIND, PREC>), dim3(a.nf * ncg), dim3(WF_THREADS), WF_SMEM, s, a);
  return hipGetLastError();
}

template <int PREC, int NBT, int TNB>
hipError_t launch_cfg(int kind, const GemmArgs& a, hipStream_t s) {
  using C = GemmCfg<PREC, NBT, TNB>;
  const int ncg = (a.nvb + TNB - 1) / TNB;
  const dim3 grid(a.nf * ncg), block(256);
  const size_t sm = C::SMEM;
  switch (kind) {
    case GK_FUSED:
      if (sm > 65536)
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gemm<PREC, NBT, TNB, GK_FUSED>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
      hipLaunchKernelGGL((k_gemm<PREC, NBT, TNB, GK_FUSED>), grid, block, sm, s, a);
      break;
    case GK_FWD:
      if (sm > 65536)
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gemm<PREC, NBT, TNB, GK_FWD>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
      hipLaunchKernelGGL((k_gemm<PREC, NBT, TNB, GK_FWD>), grid, block, sm, s, a);
      break;
    case GK_ADJ:
      if (sm > 65536)
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gemm<PREC, NBT, TNB, GK_ADJ>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
      hipLaunchKernelGGL((k_gemm<PREC, NBT, TNB, GK_ADJ>), grid, block, sm, s, a);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int PREC>
hipError_t launch_prec(int kind, const GemmArgs& a, hipStream_t s) {
  if constexpr (is_fp32<PREC>()) {  // four real products per complex one in this kernel
    if (kind == GK_FUSED && a.nb <= 16 && a.nr <= PIPE_KC) {
      const int total = a.nf * a.nvb;
      int grid = total < PIPE_WGS ? total : PIPE_WGS;
      if (grid >= 8) grid -= grid % 8;
      hipLaunchKernelGGL(k_gemm_pipe, dim3(grid), dim3(256), 0, s, a);
      return hipGetLastError();
    }
  }
  if constexpr (PREC == MDD_PREC_BF16X3 || PREC == MDD_PREC_FP16X3) {
    if (a.nb > 16 || (kind == GK_FUSED && a.nr <= SPLIT_PIPE_KC))
      return launch_gemm_split(kind, PREC, a, s);  // operands split once, in LDS
  }
  if (a.nb <= 16) return launch_cfg<PREC, 1, 1>(kind, a, s);
  if constexpr (PREC == MDD_PREC_BF16X3 || PREC == MDD_PREC_FP16X3) {
    return hipErrorInvalidValue;  // not reached: nb > 16 went to launch_gemm_split
  } else {
    if (a.nb <= 32) return launch_cfg<PREC, 2, 2>(kind, a, s);
    if constexpr (is_fp32<PREC>()) {
      switch (kind) {
        case GK_FUSED: return launch_ws<GK_FUSED, PREC>(a, s);
        case GK_FWD: return launch_ws<GK_FWD, PREC>(a, s);
        case GK_ADJ: return launch_ws<GK_ADJ, PREC>(a, s);
        default: return hipErrorInvalidValue;
      }
    }
    return launch_cfg<PREC, 4, 4>(kind, a, s);
  }
}

}  // namespace

hipError_t launch_gemm(int kind, int precision, const GemmArgs& a, hipStream_t s) {
  if (a.nb <= 0 || a.nb > NB_LIMIT) return hipErrorInvalidValue;
  switch (precision) {
    case MDD_PREC_FP32: return launch_prec<MDD_PREC_FP32>(kind, a, s);
    case MDD_PREC_BF16X3: return launch_prec<MDD_PREC_BF16X3>(kind, a, s);
    case MDD_PREC_FP16X3: return launch_prec<MDD_PREC_FP16X3>(kind, a, s);
    case MDD_PREC_BF16: return launch_prec<MDD_PREC_BF16>(kind, a, s);
    case MDD_PREC_FP32_CGEMM: return launch_prec<MDD_PREC_FP32_CGEMM>(kind, a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mdd
