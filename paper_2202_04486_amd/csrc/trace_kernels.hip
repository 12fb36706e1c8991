// Time <-> frequency kernels over traces: the model / data transforms of the
// MDC operator (Appendix A: Fourier transform along time before, inverse
// transform after, the per-frequency products) fused with the causality mask,
// the float64 gradient norm and the optimiser update.
//
// A real trace of nt samples is transformed as a complex sequence of
// N2 = nt/2 points z[n] = x[2n] + i x[2n+1] (then split into the one-sided
// spectrum), with a radix-8 Stockham FFT held in registers: each lane owns 8
// points n = j + L r (L = N2/8 lanes per trace, r < 8), passes exchange data
// through a wave-private LDS region.  A workgroup owns one tile of 16 traces
// (half of one in the gradient and update modes of long traces) whose spectra
// form one contiguous [nf][16] block in HBM, staged in LDS so both the time
// side (whole traces) and the frequency side (whole blocks) are read and
// written with contiguous accesses.
#include "device_common.h"
#include "mdd_internal.h"

namespace mdd {
namespace {


// Streaming access to the model and optimiser state: each element is read and
// written once per step and the whole state is larger than the last-level
// cache, so these accesses are marked non-temporal.  That keeps the spectra
// (written here, read by the next step's products, and the reverse) resident
// in the cache.
typedef float stream2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 stream_load(const float2* p) {
  const stream2 v = __builtin_nontemporal_load(reinterpret_cast<const stream2*>(p));
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ void stream_store(float2 x, float2* p) {
  const stream2 v = {x.x, x.y};
  __builtin_nontemporal_store(v, reinterpret_cast<stream2*>(p));
}

template <bool INV>
__device__ __forceinline__ float2 rot(float2 a) {  // * -i (forward) or * +i (inverse)
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

template <bool INV>
__device__ __forceinline__ float2 twid(const float2* tw, int m) {
  const float2 w = tw[m];
  return INV ? make_float2(w.x, -w.y) : w;
}

// In-register 8-point DFT (radix-2 decomposition), sign by direction.
template <bool INV>
__device__ __forceinline__ void dft8(float2 (&v)[8]) {
  const float h = 0.70710678118654752440f;
  const float2 a0 = cadd(v[0], v[4]), a1 = csub(v[0], v[4]);
  const float2 a2 = cadd(v[2], v[6]), a3 = csub(v[2], v[6]);
  const float2 a4 = cadd(v[1], v[5]), a5 = csub(v[1], v[5]);
  const float2 a6 = cadd(v[3], v[7]), a7 = csub(v[3], v[7]);
  const float2 e0 = cadd(a0, a2), e2 = csub(a0, a2);
  const float2 e1 = cadd(a1, rot<INV>(a3)), e3 = csub(a1, rot<INV>(a3));
  const float2 o0 = cadd(a4, a6), o2 = csub(a4, a6);
  const float2 o1 = cadd(a5, rot<INV>(a7)), o3 = csub(a5, rot<INV>(a7));
  float2 t1, t3;
  if (!INV) {
    t1 = make_float2(h * (o1.x + o1.y), h * (o1.y - o1.x));
    t3 = make_float2(h * (o3.y - o3.x), -h * (o3.x + o3.y));
  } else {
    t1 = make_float2(h * (o1.x - o1.y), h * (o1.x + o1.y));
    t3 = make_float2(-h * (o3.x + o3.y), h * (o3.x - o3.y));
  }
  const float2 t2 = rot<INV>(o2);
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cadd(e1, t1);
  v[5] = csub(e1, t1);
  v[2] = cadd(e2, t2);
  v[6] = csub(e2, t2);
  v[3] = cadd(e3, t3);
  v[7] = csub(e3, t3);
}

__device__ __forceinline__ int pidx(int i) { return i + (i >> 3); }  // LDS padding

template <int N2>
struct FftShape {
  static constexpr int L = N2 / 8;
  static constexpr int NP8 = N2 >= 512 ? 3 : 2;                 // radix-8 passes
  static constexpr int REM = N2 / (NP8 == 3 ? 512 : 64);         // 1, 2 or 4: tail radix
  static constexpr int SC = N2 + N2 / 8;                         // padded scratch per trace
  // Twiddle table (LDS): [0, N2) exp(-2 pi i k / nt) for the real split; then per
  // pass the factors laid out [r-1][k] so that lanes read consecutive entries.
  static constexpr int TW_P1 = N2;                               // W_64^{r k},  k < 8
  static constexpr int TW_P2 = TW_P1 + 7 * 8;                    // W_512^{r k}, k < 64
  static constexpr int TW_Q = TW_P2 + (NP8 == 3 ? 7 * 64 : 0);   // W_N2^{q j},  j < 64
  static constexpr int TW_SIZE = TW_Q + (REM - 1) * 64;
  static_assert(N2 == 64 || N2 == 128 || N2 == 256 || N2 == 512, "unsupported length");
};

// Complex FFT of N2 = NT/2 points of one trace.  On entry lane j holds
// v[r] = a[j + L r]; on exit v[r] = A[j + L r] (natural order, unnormalised).
template <int NT, bool INV>
__device__ __forceinline__ void fft_half(float2 (&v)[8], int j, float2* sc, const float2* tw) {
  constexpr int N2 = NT / 2;
  using S = FftShape<N2>;
  constexpr int L = S::L;
#pragma unroll
  for (int p = 0; p < S::NP8; ++p) {
    const int Ns = p == 0 ? 1 : (p == 1 ? 8 : 64);
    if (p > 0) {
      const float2* t = tw + (p == 1 ? S::TW_P1 : S::TW_P2) + (j & (Ns - 1));
#pragma unroll
      for (int r = 1; r < 8; ++r) v[r] = cmul(v[r], twid<INV>(t, (r - 1) * Ns));
    }
    dft8<INV>(v);
    const bool last = (p == S::NP8 - 1) && (S::REM == 1);
    if (!last) {
      const int base = (j / Ns) * Ns * 8 + (j & (Ns - 1));
      wave_sync();
#pragma unroll
      for (int r = 0; r < 8; ++r) sc[pidx(base + r * Ns)] = v[r];
      wave_sync();
#pragma unroll
      for (int r = 0; r < 8; ++r) v[r] = sc[pidx(j + r * L)];
    }
  }
  if constexpr (S::REM == 4) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int jj = j + L * h;
      float2 x0 = v[h], x1 = v[h + 2], x2 = v[h + 4], x3 = v[h + 6];
      x1 = cmul(x1, twid<INV>(tw, S::TW_Q + jj));
      x2 = cmul(x2, twid<INV>(tw, S::TW_Q + 64 + jj));
      x3 = cmul(x3, twid<INV>(tw, S::TW_Q + 128 + jj));
      const float2 s02 = cadd(x0, x2), d02 = csub(x0, x2);
      const float2 s13 = cadd(x1, x3), d13 = rot<INV>(csub(x1, x3));
      v[h] = cadd(s02, s13);
      v[h + 4] = csub(s02, s13);
      v[h + 2] = cadd(d02, d13);
      v[h + 6] = csub(d02, d13);
    }
  } else if constexpr (S::REM == 2) {
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int jj = j + L * h;
      const float2 x0 = v[h];
      const float2 x1 = cmul(v[h + 4], twid<INV>(tw, S::TW_Q + jj));
      v[h] = cadd(x0, x1);
      v[h + 4] = csub(x0, x1);
    }
  }
}

// Split the half-length complex spectrum Z into the one-sided spectrum of the
// real trace: X[k] = (Z[k] + conj Z[N2-k])/2 - i W^k (Z[k] - conj Z[N2-k])/2,
// W = exp(-2 pi i / nt).  On exit v[r] = X[j + L r]; lane j = 0 also returns
// the Nyquist bin X[N2].
template <int NT>
__device__ __forceinline__ void rfft_split(float2 (&v)[8], int j, int lane, const float2* tw,
                                           float2& xnyq) {
  constexpr int N2 = NT / 2;
  constexpr int L = N2 / 8;
  const int pj = (L - j) & (L - 1);
  const int plane = lane - j + pj;
  float2 zp[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const float2 a = v[7 - r];
    const float2 b = v[(8 - r) & 7];
    float2 s;
    s.x = __shfl(a.x, plane, 64);
    s.y = __shfl(a.y, plane, 64);
    zp[r] = (j == 0) ? b : s;
  }
  xnyq = make_float2(v[0].x - v[0].y, 0.f);
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int k = j + L * r;
    const float2 A = v[r], B = cconj(zp[r]);
    const float2 E = cscale(cadd(A, B), 0.5f);
    const float2 Dh = cscale(csub(A, B), 0.5f);
    const float2 O = make_float2(Dh.y, -Dh.x);  // -i * Dh
    v[r] = cadd(E, cmul(tw[k], O));
  }
  if (j == 0) v[0].y = 0.f;
}

// Inverse of rfft_split: from the one-sided spectrum column c of a staged tile
// (bins >= nf are zero) build Z[k] = E[k] + i O[k] for k = j + L r.
template <int NT, int SPS>
__device__ __forceinline__ void irfft_merge(float2 (&v)[8], int j, const float2* spec, int c,
                                            int nf, const float2* tw) {
  constexpr int N2 = NT / 2;
  constexpr int L = N2 / 8;
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int k = j + L * r;
    const int km = N2 - k;
    float2 X = k < nf ? spec[k * SPS + c] : make_float2(0.f, 0.f);
    float2 Xm = km < nf ? spec[km * SPS + c] : make_float2(0.f, 0.f);
    if (k == 0) {  // the imaginary parts of the DC and Nyquist bins of a real trace are dropped
      X.y = 0.f;
      Xm.y = 0.f;
    }
    const float2 B = cconj(Xm);
    const float2 E = cscale(cadd(X, B), 0.5f);
    const float2 O = cmul(cscale(csub(X, B), 0.5f), cconj(tw[k]));
    v[r] = make_float2(E.x - O.y, E.y + O.x);
  }
}

template <int NT, int MODE>
struct TraceCfg {
  static constexpr int N2 = NT / 2;
  static constexpr int L = FftShape<N2>::L;
  static constexpr int TPW = 64 / L;              // traces per wavefront at a time
  // The gradient and update modes of long traces give each workgroup half of a
  // 16-column spectral block (CW = 8 traces, four wavefronts): three such
  // workgroups fit a CU where one full-block workgroup of eight wavefronts did
  // (registers and LDS), and the grid's last partial round is half as long.
  // The two halves of a block run on the same XCD, so its L2 serves both.
  static constexpr bool UPD = MODE == TM_GRAD || MODE == TM_SGD || MODE == TM_ADAM ||
                              MODE == TM_NSGD;
  static constexpr int SPLIT = (UPD && NT >= 512) ? 2 : 1;
  static constexpr int CW = CB / SPLIT;           // columns (traces) per workgroup
  static constexpr int NWAVES = NT == 1024 ? 8 / SPLIT : CW / TPW;
  static constexpr int ITERS = CW / (NWAVES * TPW);
  static constexpr int THREADS = 64 * NWAVES;
  static constexpr int SPS = CW + 1;              // LDS row stride of the spectral tile (odd)
  static_assert(ITERS * NWAVES * TPW == CW, "tile");
};

// Deterministic sum over the workgroup of one double per thread (result in thread 0).
template <int NWAVES>
__device__ __forceinline__ double tile_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < NWAVES; ++w) s += red[w];
  return s;
}

// One workgroup per tile of CB traces, one wavefront per trace (or several
// traces per wavefront for short traces).  Update modes request a trace's model
// and optimiser state just before its inverse transform (the loads are in flight
// while it runs) and store them right after the update.
template <int NT, int MODE>
__global__ __launch_bounds__((TraceCfg<NT, MODE>::THREADS)) void k_trace(TraceArgs a) {
  using C = TraceCfg<NT, MODE>;
  constexpr int N2 = C::N2, L = C::L, TPW = C::TPW, NW = C::NWAVES, NTH = C::THREADS;
  constexpr int CW = C::CW, SPS = C::SPS;
  using S = FftShape<N2>;
  constexpr bool UPDATE = MODE == TM_SGD || MODE == TM_ADAM || MODE == TM_NSGD;
  extern __shared__ float2 smem[];
  float2* s_tw = smem;
  float2* s_sc = smem + S::TW_SIZE;
  float2* s_spec = s_sc + NW * TPW * S::SC;
  __shared__ double s_red[NW];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int p = lane / L, j = lane % L;
  // workgroup -> (tile, part): a group of 8 * SPLIT consecutive ids holds every
  // part of 8 tiles, ids w, w + 8, ... (one XCD under round-robin dispatch) the
  // parts of one tile.
  int tile = blockIdx.x, half = 0;
  if constexpr (C::SPLIT > 1) {
    const int g = blockIdx.x / (8 * C::SPLIT), w = blockIdx.x % (8 * C::SPLIT);
    const int m = min(8, a.rows * a.ncb - 8 * g);  // tiles in this group
    tile = 8 * g + w % m;
    half = w / m;
  }
  const int row = tile / a.ncb, cb = tile % a.ncb;
  const int nf = a.nf;
  float2* gspec = a.spec + row * a.s_row + cb * a.s_cb + half * CW;
  auto column = [&](int it) { return it * NW * TPW + wave * TPW + p; };  // trace within the half

  // Model / optimiser state of the lane's trace in iteration `it`.
  float2 rv[8], m0[8], m1[8];
  auto load_state = [&](int it) {
    if constexpr (UPDATE) {
      const int col = cb * CB + half * CW + column(it);
      const bool valid = col < a.ncols;
      const long long trace = (long long)row * a.ncols + col;
      const float2* R = reinterpret_cast<const float2*>(a.model + trace * NT);
      const float2* M0 = reinterpret_cast<const float2*>(a.st0 + trace * NT);
      const float2* M1 = reinterpret_cast<const float2*>(a.st1 + trace * NT);
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        rv[r] = valid ? stream_load(R + j + L * r) : make_float2(0.f, 0.f);
        if constexpr (MODE != TM_SGD) m0[r] = valid ? stream_load(M0 + j + L * r) : make_float2(0.f, 0.f);
        if constexpr (MODE == TM_ADAM) m1[r] = valid ? stream_load(M1 + j + L * r) : make_float2(0.f, 0.f);
      }
    }
  };

  for (int i = tid; i < S::TW_SIZE; i += NTH) s_tw[i] = a.tw[i];
  if (MODE != TM_RFFT) {
    for (int i = tid; i < nf * (CW / 2); i += NTH) {
      const int k = i / (CW / 2), c2 = 2 * (i % (CW / 2));
      const float4 z = *reinterpret_cast<const float4*>(gspec + k * a.s_k + c2);
      s_spec[k * SPS + c2] = make_float2(z.x, z.y);
      s_spec[k * SPS + c2 + 1] = make_float2(z.z, z.w);
    }
  }
  __syncthreads();

  float2* sc = s_sc + (wave * TPW + p) * S::SC;
  double part = 0.0;

#pragma unroll 1
  for (int it = 0; it < C::ITERS; ++it) {
    const int c = column(it);
    const int col = cb * CB + half * CW + c;
    const bool valid = col < a.ncols;
    const long long trace = (long long)row * a.ncols + col;
    float2 v[8];

    if constexpr (MODE == TM_RFFT) {
      const float2* x = reinterpret_cast<const float2*>(a.x_in + trace * NT);
      const float2* x2 = reinterpret_cast<const float2*>(a.x_in2 + trace * NT);
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        float2 z = make_float2(0.f, 0.f);
        if (valid) {
          z = stream_load(x + j + L * r);
          if (a.x_in2) {
            const float2 y = stream_load(x2 + j + L * r);
            z.x += a.mu2 * y.x;
            z.y += a.mu2 * y.y;
          }
        }
        v[r] = z;
      }
      fft_half<NT, false>(v, j, sc, s_tw);
      float2 xn;
      rfft_split<NT>(v, j, lane, s_tw, xn);
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int k = j + L * r;
        if (k < nf) s_spec[k * SPS + c] = v[r];
      }
      if (j == 0 && nf > N2) s_spec[N2 * SPS + c] = xn;
      if (a.part && valid) {  // energy in the bins that are not retained
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          const int k = j + L * r;
          if (k >= nf) part += 2.0 * ((double)v[r].x * v[r].x + (double)v[r].y * v[r].y);
        }
        if (j == 0 && nf <= N2) part += (double)xn.x * xn.x;
      }
    } else {
      load_state(it);  // in flight during the inverse transform
      irfft_merge<NT, SPS>(v, j, s_spec, c, nf, s_tw);
      fft_half<NT, true>(v, j, sc, s_tw);
      const float inv_n2 = 1.0f / float(N2);
#pragma unroll
      for (int r = 0; r < 8; ++r) v[r] = cscale(v[r], inv_n2);  // time samples 2n, 2n+1

      if constexpr (MODE == TM_IRFFT) {
        if (valid) {
          float2* y = reinterpret_cast<float2*>(a.x_out + trace * NT);
#pragma unroll
          for (int r = 0; r < 8; ++r) y[j + L * r] = v[r];
        }
      } else {
        const int t0 = (a.onset && valid) ? a.onset[trace] : 0;
        if (t0 > 0) {
#pragma unroll
          for (int r = 0; r < 8; ++r) {
            const int t = 2 * (j + L * r);
            if (t < t0) v[r].x = 0.f;
            if (t + 1 < t0) v[r].y = 0.f;
          }
        }
        if (valid) {
#pragma unroll
          for (int r = 0; r < 8; ++r) part += (double)v[r].x * v[r].x + (double)v[r].y * v[r].y;
        }
        if constexpr (MODE == TM_GRAD) {
          if (valid) {
            float2* y = reinterpret_cast<float2*>(a.x_out + trace * NT);
#pragma unroll
            for (int r = 0; r < 8; ++r) y[j + L * r] = v[r];
          }
        } else if constexpr (UPDATE) {
          // v[r] holds the masked gradient; it is replaced by the next evaluation point.
#pragma unroll
          for (int r = 0; r < 8; ++r) {
            const float2 g = v[r];
            float2 x = rv[r];
            float2 ev;
            if constexpr (MODE == TM_SGD) {
              x.x -= a.lr * g.x;
              x.y -= a.lr * g.y;
            } else if constexpr (MODE == TM_ADAM) {
              float2 m = m0[r], q = m1[r];
              m.x = a.beta1 * m.x + a.omb1 * g.x;
              m.y = a.beta1 * m.y + a.omb1 * g.y;
              q.x = a.beta2 * q.x + a.omb2 * (g.x * g.x);
              q.y = a.beta2 * q.y + a.omb2 * (g.y * g.y);
              // hardware square root and reciprocal (each within 1 ulp)
              x.x -= a.lr * (m.x * a.inv_bc1) *
                     __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(q.x * a.inv_bc2) + a.eps);
              x.y -= a.lr * (m.y * a.inv_bc1) *
                     __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(q.y * a.inv_bc2) + a.eps);
              m0[r] = m;
              m1[r] = q;
            } else {  // Nesterov: velocity <- mu velocity - lr g; R <- R + velocity
              const int t = 2 * (j + L * r);
              float2 vel = m0[r];
              vel.x = a.mu * vel.x - a.lr * g.x;
              vel.y = a.mu * vel.y - a.lr * g.y;
              if (t < t0) vel.x = 0.f;
              if (t + 1 < t0) vel.y = 0.f;
              x.x += vel.x;
              x.y += vel.y;
              m0[r] = vel;
              ev = make_float2(x.x + a.mu * vel.x, x.y + a.mu * vel.y);
            }
            const int t = 2 * (j + L * r);
            if (t < t0) x.x = 0.f;
            if (t + 1 < t0) x.y = 0.f;
            rv[r] = x;
            if constexpr (MODE == TM_NSGD) {
              if (t < t0) ev.x = 0.f;
              if (t + 1 < t0) ev.y = 0.f;
              v[r] = ev;
            } else {
              v[r] = x;
            }
          }
          if (valid) {
            float2* R = reinterpret_cast<float2*>(a.model + trace * NT);
            float2* M0 = reinterpret_cast<float2*>(a.st0 + trace * NT);
            float2* M1 = reinterpret_cast<float2*>(a.st1 + trace * NT);
#pragma unroll
            for (int r = 0; r < 8; ++r) {
              stream_store(rv[r], R + j + L * r);
              if constexpr (MODE != TM_SGD) stream_store(m0[r], M0 + j + L * r);
              if constexpr (MODE == TM_ADAM) stream_store(m1[r], M1 + j + L * r);
            }
          }
          if (a.store_spec) {  // spectra of the next evaluation point, over this column
            fft_half<NT, false>(v, j, sc, s_tw);
            float2 xn;
            rfft_split<NT>(v, j, lane, s_tw, xn);
#pragma unroll
            for (int r = 0; r < 8; ++r) {
              const int k = j + L * r;
              if (k < nf) s_spec[k * SPS + c] = v[r];
            }
            if (j == 0 && nf > N2) s_spec[N2 * SPS + c] = xn;
          }
        }
      }
    }
  }

  if (a.part) {
    const double tot = tile_sum<NW>(part, s_red);
    if (tid == 0) a.part[blockIdx.x] = tot;
  }
  if (MODE == TM_RFFT || (UPDATE && a.store_spec)) {
    __syncthreads();
    for (int i = tid; i < nf * (CW / 2); i += NTH) {
      const int k = i / (CW / 2), c2 = 2 * (i % (CW / 2));
      const float2 z0 = s_spec[k * SPS + c2], z1 = s_spec[k * SPS + c2 + 1];
      *reinterpret_cast<float4*>(gspec + k * a.s_k + c2) = make_float4(z0.x, z0.y, z1.x, z1.y);
    }
  }
}

// Builds the twiddle table of FftShape for nt (float64 angles, rounded once).
__global__ void k_twiddles(float2* tw, int nt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n2 = nt / 2;
  const int np8 = n2 >= 512 ? 3 : 2;
  const int rem = n2 / (np8 == 3 ? 512 : 64);
  const int p1 = n2, p2 = p1 + 56, q0 = p2 + (np8 == 3 ? 448 : 0), total = q0 + (rem - 1) * 64;
  if (i >= total) return;
  double num, den;  // angle = -2 pi num / den
  if (i < p1) {
    num = i;
    den = nt;
  } else if (i < p2) {
    num = (double)((i - p1) / 8 + 1) * ((i - p1) % 8);
    den = 64.0;
  } else if (i < q0) {
    num = (double)((i - p2) / 64 + 1) * ((i - p2) % 64);
    den = 512.0;
  } else {
    num = (double)((i - q0) / 64 + 1) * ((i - q0) % 64);
    den = n2;
  }
  double s, c;
  sincospi(-2.0 * num / den, &s, &c);
  tw[i] = make_float2((float)c, (float)s);
}

template <int NT, int MODE>
size_t trace_smem(int nf) {
  using C = TraceCfg<NT, MODE>;
  using S = FftShape<C::N2>;
  return sizeof(float2) * ((size_t)S::TW_SIZE + (size_t)C::NWAVES * C::TPW * S::SC +
                           (size_t)nf * C::SPS);
}

template <int NT, int MODE>
hipError_t launch_mode(const TraceArgs& a, hipStream_t s) {
  using C = TraceCfg<NT, MODE>;
  const dim3 grid(a.rows * a.ncb * C::SPLIT), block(C::THREADS);
  const size_t sm = trace_smem<NT, MODE>(a.nf);
  if (sm > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_trace<NT, MODE>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
  hipLaunchKernelGGL((k_trace<NT, MODE>), grid, block, sm, s, a);
  return hipGetLastError();
}

template <int NT>
hipError_t launch_nt(int mode, const TraceArgs& a, hipStream_t s) {
  switch (mode) {
    case TM_RFFT: return launch_mode<NT, TM_RFFT>(a, s);
    case TM_IRFFT: return launch_mode<NT, TM_IRFFT>(a, s);
    case TM_GRAD: return launch_mode<NT, TM_GRAD>(a, s);
    case TM_SGD: return launch_mode<NT, TM_SGD>(a, s);
    case TM_ADAM: return launch_mode<NT, TM_ADAM>(a, s);
    case TM_NSGD: return launch_mode<NT, TM_NSGD>(a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_twiddles(float2* tw, int nt, hipStream_t s) {
  hipLaunchKernelGGL(k_twiddles, dim3((2 * nt + 255) / 256), dim3(256), 0, s, tw, nt);
  return hipGetLastError();
}

int trace_update_split(int nt) {
  switch (nt) {
    case 128: return TraceCfg<128, TM_ADAM>::SPLIT;
    case 256: return TraceCfg<256, TM_ADAM>::SPLIT;
    case 512: return TraceCfg<512, TM_ADAM>::SPLIT;
    case 1024: return TraceCfg<1024, TM_ADAM>::SPLIT;
    default: return 1;
  }
}

hipError_t launch_trace(int mode, const TraceArgs& a, hipStream_t s) {
  if (a.rows <= 0 || a.ncb <= 0) return hipSuccess;
  switch (a.nt) {
    case 128: return launch_nt<128>(mode, a, s);
    case 256: return launch_nt<256>(mode, a, s);
    case 512: return launch_nt<512>(mode, a, s);
    case 1024: return launch_nt<1024>(mode, a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mdd
