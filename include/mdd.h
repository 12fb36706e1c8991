/*
 * mdd.h -- C ABI of the MI355X (gfx950) stochastic multi-dimensional
 * deconvolution library (Ravasi, Selvan and Luiken, "Stochastic
 * Multi-Dimensional Deconvolution").
 *
 * The library computes, on one GPU, the stochastic gradient of the finite-sum
 * time-domain MDD misfit over a batch of sources and the optimiser step that
 * uses it.  Notation follows the paper's Theory section:
 *
 *   d  [ns][nr][nt]   down-going wavefield p+ (the kernel), float32, time
 *   R  [nr][nvs][nt]  local reflection response (the unknown), float32, time
 *   u  [ns][nvs][nt]  up-going wavefield p-, float32, time
 *
 * all C order with time fastest (traces stacked as in the vectors r_t, p-_t).
 * The operator P+ is the multi-dimensional convolution: per frequency f the
 * matrix product P-_f = P+_f R_f ([ns x nr] times [nr x nvs]); in time it is
 * a circular convolution over nt samples summed over receivers.
 *
 * Conventions (the paper leaves them open): forward DFT exp(-2 pi i k t / nt)
 * unnormalised, inverse with 1/nt, nfft = nt (circular, no padding), unit
 * quadrature weights, and only the one-sided bins k < nf are kept (nf <=
 * nt/2 + 1), which is the operator with the kernel band-limited to those
 * bins.  The loss is reported in the time domain (Parseval: in-band residual
 * energy plus the data's fixed out-of-band energy).
 *
 * Memory.  Every pointer argument is a DEVICE pointer unless its name ends in
 * _host.  The caller allocates and owns all device memory, including the
 * workspace; the library never allocates device memory.  A plan stores
 * pointers into the workspace only.  Inputs passed to mdd_set_* must stay
 * valid until that work has run on the plan's stream.
 *
 * Streams.  All work is enqueued asynchronously on the plan's stream (a
 * hipStream_t passed as void*; NULL is the default stream).  One plan serves
 * one stream and is not thread-safe.  Output scalars (loss, gradient norm)
 * are written to device memory and are valid once the stream has reached
 * them.
 *
 * Errors.  Every call validates its arguments on the host before enqueuing
 * anything: an invalid call enqueues no work and returns a negative status.
 * A failed HIP call returns MDD_EHIP; its hipError_t is kept by the plan
 * (mdd_plan_last_hip_error).  Faults inside kernels surface at the next
 * synchronising call.  Nothing is printed and no exception crosses the ABI.
 * Batch indices must lie in [0, ns); kernels treat an index outside that
 * range as a source whose wavefields are zero (it contributes nothing).
 */
#ifndef MDD_H
#define MDD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mdd_status;

#define MDD_OK 0
#define MDD_EINVAL (-1)       /* NULL pointer, unknown enum value, bad scalar */
#define MDD_ESHAPE (-2)       /* inconsistent sizes (nf > nt/2+1, nb > nb_max, nt unsupported) */
#define MDD_ENOMEM (-3)       /* workspace NULL, misaligned or smaller than needed */
#define MDD_EHIP (-4)         /* a HIP runtime call failed */
#define MDD_EUNSUPPORTED (-5) /* precision or optimiser not available */
#define MDD_ESTATE (-6)       /* kernel / data not set before a call that needs them */
#define MDD_ELIMIT (-7)       /* sizes beyond the library's static workspace (the _noalloc call) */

/* Arithmetic of the two per-frequency complex products.  With one virtual source
 * (nvs = 1) the products are matrix-vector products bound by the bytes of D_b and
 * run in float32 on the vector units whatever the setting (Appendix A: the
 * matrix-matrix product reduces to a matrix-vector product there). */
#define MDD_PREC_FP32 0   /* float32 MFMA, float32 accumulate.  Each complex product is formed
                             from three real ones, except in the fused gradient / step at
                             most 16 batch rows over at most 224 receivers, which uses four */
#define MDD_PREC_BF16X3 1 /* bf16 hi+lo split, hi*hi + hi*lo + lo*hi, float32 accumulate */
#define MDD_PREC_FP16X3 2 /* fp16 hi+lo split with power-of-two tile scaling, float32 accumulate */
#define MDD_PREC_BF16 3   /* single bf16 product (diagnostic: expected to miss 1e-3) */
#define MDD_PREC_FP32_CGEMM 4 /* float32 with four real products per complex one everywhere,
                                 as a plain complex GEMM does (a comparison form) */

/* Plan flags. */
#define MDD_FLAG_STORE_RF 1 /* mdd_step also writes the spectra of the updated model so the
                               next mdd_step on the same R skips its forward transform */
#define MDD_FLAG_FULL_GRAD 2 /* reserve a second spectra buffer and the list of all sources
                                for mdd_full_grad / mdd_full_step */
#define MDD_FLAG_STREAM_KERNEL 4 /* keep no kernel spectra for all sources: the caller stages
                                    each batch's rows with mdd_stage_kernel (the kernel may
                                    then live out of device memory); not with FULL_GRAD.
                                    Lifts the 4096 limit on ns to 1048576 */
#define MDD_FLAG_STREAM_DATA 8   /* with MDD_FLAG_STREAM_KERNEL: keep no data spectra for all
                                    sources either; the caller stages each batch's data rows
                                    with mdd_stage_data.  The workspace then does not grow
                                    with ns */

/* Sizes.  ns sources (at most 4096, or 1048576 with MDD_FLAG_STREAM_KERNEL), nr
 * receivers and nvs virtual sources (at most 4096), nt time samples (128, 256, 512
 * or 1024), nf retained one-sided frequency bins (1..nt/2+1), nb_max the largest
 * batch any call on this plan will use (1..ns, <= 64). */
typedef struct mdd_dims {
  int32_t ns, nr, nvs, nt, nf, nb_max;
  int32_t precision; /* MDD_PREC_* */
  int32_t flags;     /* MDD_FLAG_* */
} mdd_dims;

/* Optimiser of mdd_step. */
#define MDD_OPT_SGD 0   /* R <- M (R - lr g)  (Theory section: SGD iterations) */
#define MDD_OPT_ADAM 1  /* Adam with bias correction, model kept masked */
#define MDD_OPT_NSGD 2  /* Nesterov momentum, Sutskever form: gradient at R + mu s0;
                           s0 <- mu s0 - lr g; R <- R + s0 */

typedef struct mdd_opt {
  int32_t kind;    /* MDD_OPT_* */
  int32_t reserved;
  double lr;       /* step size alpha (> 0) */
  double beta1;    /* Adam first-moment decay, in [0, 1) */
  double beta2;    /* Adam second-moment decay, in [0, 1) */
  double eps;      /* Adam denominator guard (> 0) */
  double mu;       /* Nesterov momentum, in [0, 1) */
  int64_t t;       /* Adam: number of this step, >= 1 */
} mdd_opt;

typedef struct mdd_plan mdd_plan;

/* Bytes of device workspace a plan with these sizes needs (256-byte aligned
 * regions), or 0 if the sizes are invalid.  Pure host computation. */
size_t mdd_workspace_bytes(const mdd_dims* dims);

/* Validate dims, lay the plan out in the caller's workspace (device memory of
 * at least mdd_workspace_bytes bytes, 256-byte aligned) and initialise its
 * tables on `stream`.  *out receives a host-allocated plan object.
 * Errors: EINVAL (NULL), ESHAPE (sizes), ENOMEM (workspace), EUNSUPPORTED
 * (precision), EHIP. */
mdd_status mdd_plan_create(const mdd_dims* dims, void* workspace, size_t ws_bytes, void* stream,
                           mdd_plan** out);

/* Release the host plan object (the workspace stays the caller's). */
mdd_status mdd_plan_destroy(mdd_plan* plan);

/* Change the stream later calls are enqueued on. */
mdd_status mdd_plan_set_stream(mdd_plan* plan, void* stream);

/* Kernel of the operator (Theory section, the down-going wavefield P+):
 * d [ns][nr][nt] float32.  Computes and stores its spectra D_k, k < nf
 * (layout [nf][ns][nr] complex, rows padded to 16 entries). */
mdd_status mdd_set_kernel(mdd_plan* plan, const float* d);

/* Up-going data p- (Theory section): u [ns][nvs][nt] float32.  Stores its
 * spectra U_k, k < nf, and each source's energy outside the retained bins
 * (float64), which the time-domain loss adds to the in-band residual energy. */
mdd_status mdd_set_data(mdd_plan* plan, const float* u);

/* Causality preconditioner C_c (Theory section): onset [nr][nvs] int32; sample
 * t of trace (r, vs) of the gradient and of the model is kept iff
 * t >= onset[r][vs].  NULL removes the mask. */
mdd_status mdd_set_mask(mdd_plan* plan, const int32_t* onset);

/* Forward MDC on a batch (Theory section, matrix form of the MDC integral,
 * applied in the time domain as in Appendix A: transform, per-frequency
 * product, inverse transform): U_out[b] = P+_{idx[b]} R, U_out [nb][nvs][nt]
 * float32.  R [nr][nvs][nt]; idx [nb] int32 device array; 1 <= nb <= nb_max.
 * Needs mdd_set_kernel. */
mdd_status mdc_forward(mdd_plan* plan, const float* R, const int32_t* idx, int32_t nb,
                       float* U_out);

/* Adjoint MDC on a batch (Theory section: the adjoint P+^H that the mini-batch
 * gradient, Eq. (6), applies to the residual; per frequency the product with the
 * conjugate transpose of the kernel rows, Appendix A): G_out = sum_b
 * P+_{idx[b]}^H V[b], G_out [nr][nvs][nt] float32, V [nb][nvs][nt].  No mask is
 * applied.  Needs mdd_set_kernel. */
mdd_status mdc_adjoint(mdd_plan* plan, const float* V, const int32_t* idx, int32_t nb,
                       float* G_out);

/* The same operators with the reciprocity preconditioner C_r of the preconditioned
 * functional (Theory section; C_r R = (R + R^T) / 2 over receiver and virtual source):
 *   mdc_forward_rec: U_out = P+_b C_r R;    mdc_adjoint_rec: G_out = C_r P+_b^H V.
 * C_r is applied to the retained spectra of R (after its transform) or of the adjoint
 * product (before the inverse transform), which equals applying it to the traces since
 * the transform acts on each trace alone; it reads and writes nr * nvs * nf complex
 * values instead of the traces.  Needs nr == nvs (MDD_ESHAPE otherwise) and
 * mdd_set_kernel; arguments, layouts and errors as for mdc_forward / mdc_adjoint. */
mdd_status mdc_forward_rec(mdd_plan* plan, const float* R, const int32_t* idx, int32_t nb,
                           float* U_out);
mdd_status mdc_adjoint_rec(mdd_plan* plan, const float* V, const int32_t* idx, int32_t nb,
                           float* G_out);

/* Mini-batch gradient of the finite-sum functional (Theory section):
 *   loss = 1/2 sum_{b} || p-_{idx[b]} - P+_{idx[b]} R ||^2        (float64)
 *   G    = C_c [ - sum_{b} P+_{idx[b]}^H (p-_{idx[b]} - P+_{idx[b]} R) ]
 *   gnorm2 = || G ||^2                                              (float64)
 * The gradient is the SUM over the batch as printed; repeated indices count
 * twice.  G_out [nr][nvs][nt] float32; loss_out and gnorm2_out are device
 * float64 scalars (either may be NULL).  Needs kernel and data. */
mdd_status mdd_stoch_grad(mdd_plan* plan, const float* R, const int32_t* idx, int32_t nb,
                          float* G_out, double* loss_out, double* gnorm2_out);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): the mini-batch gradient of
 * mdd_stoch_grad, with the plan's set-up (mdd_set_kernel, mdd_set_data,
 * mdd_set_mask) done in the same call, on a plan laid out in a workspace the library
 * itself holds: one static device array of MDD_NOALLOC_WORKSPACE_BYTES per GPU,
 * resident from the library's first use on that GPU until the process ends.  No
 * device or host memory is allocated.  dims as for mdd_plan_create (flags
 * MDD_FLAG_STREAM_KERNEL and MDD_FLAG_FULL_GRAD are rejected); d, u, onset (may be
 * NULL), R, idx, nb, G_out, loss_out, gnorm2_out as for mdd_set_kernel,
 * mdd_set_data, mdd_set_mask and mdd_stoch_grad.  `stream` must belong to the
 * current device.  Every call on one GPU uses that GPU's array: calls that overlap
 * in time on one GPU (other streams, other threads) race and must be serialised by
 * the caller; a call's results do not depend on what an earlier call left there.
 * Errors: EINVAL (NULL, flags, a stream of another device), ESHAPE, EUNSUPPORTED,
 * ELIMIT (mdd_workspace_bytes(dims) above MDD_NOALLOC_WORKSPACE_BYTES), EHIP. */
#define MDD_NOALLOC_WORKSPACE_BYTES (64u << 20)
mdd_status mdd_stoch_grad_noalloc(const mdd_dims* dims, const float* d, const float* u,
                                  const int32_t* onset, const float* R, const int32_t* idx,
                                  int32_t nb, float* G_out, double* loss_out, double* gnorm2_out,
                                  void* stream);

/* Kernel rows of one batch, for a plan with MDD_FLAG_STREAM_KERNEL (Examples and
 * Appendix A: with 3D acquisitions the kernel may not fit in memory; a step only
 * uses the nb rows of its batch).  d_rows [nb][nr][nt] float32 device: row b is
 * the down-going wavefield of the source the next call's idx[b] names.  The
 * following mdc_forward / mdc_adjoint / mdd_stoch_grad / mdd_step on this plan
 * must pass a batch of the same length nb, and take D row b from here (U still
 * from idx[b]; an index outside [0, ns) still acts as a zero source).  d_rows may
 * be reused once the stream has passed this call.  mdd_set_kernel, mdd_sigma_max2
 * and the full gradient need every source and return ESTATE on such a plan.
 * Errors: EINVAL (NULL), ESTATE (plan without the flag), ESHAPE (nb outside
 * [1, nb_max]), EHIP. */
mdd_status mdd_stage_kernel(mdd_plan* plan, const float* d_rows, int32_t nb);

/* Data rows of one batch, for a plan with MDD_FLAG_STREAM_DATA (the same concern
 * as mdd_stage_kernel: with 10^3 - 10^5 sources the up-going data need not stay in
 * device memory either).  u_rows [nb][nvs][nt] float32 device: row b is the up-going
 * wavefield of the source the next call's idx[b] names.  Computes their spectra and
 * out-of-band energies in place of mdd_set_data's; the following mdd_stoch_grad /
 * mdd_step must pass a batch of the same length nb and take U row b and its energy
 * from here (an index outside [0, ns) still acts as a zero source).  mdd_set_data
 * returns ESTATE on such a plan.  Errors: EINVAL (NULL), ESTATE (plan without the
 * flag), ESHAPE (nb outside [1, nb_max]), EHIP. */
mdd_status mdd_stage_data(mdd_plan* plan, const float* u_rows, int32_t nb);

/* Host-side check of a batch before it is enqueued: idx_host [nb] in host memory.
 * The device entry points treat an index outside [0, ns) as a source with zero
 * wavefields; callers that want such an index to be an error check the batch here.
 * Returns EINVAL (NULL, or an index outside [0, ns)) or ESHAPE (nb outside
 * [1, nb_max]).  Calls no HIP function. */
mdd_status mdd_check_batch_host(const int32_t* idx_host, int32_t nb, int32_t ns, int32_t nb_max);

/* One stochastic step in place (Theory section: the SGD iteration r <- r - alpha g
 * on the batch gradient of Eq. (6), and its Nesterov-momentum form N-SGD; Adam is
 * not in the paper): the gradient of mdd_stoch_grad at R (or, for
 * MDD_OPT_NSGD, at R + mu s0), then the update of R and of the optimiser state
 * s0, s1 ([nr][nvs][nt] float32 each): SGD uses neither (may be NULL), NSGD
 * uses s0 (velocity), ADAM uses s0 (first moment) and s1 (second moment).
 * The masked samples of R stay zero.  loss_out / gnorm2_out as above (the
 * values at the point where the gradient was taken). */
mdd_status mdd_step(mdd_plan* plan, float* R, float* s0, float* s1, const mdd_opt* opt,
                    const int32_t* idx, int32_t nb, double* loss_out, double* gnorm2_out);

/* Gradient of the whole finite-sum functional (Theory section: the batch is every
 * source; Appendix A: one such iteration costs what one stochastic epoch costs,
 * less the per-batch model transforms):
 *   loss = 1/2 sum_{s < ns} || p-_s - P+_s R ||^2                  (float64)
 *   G    = C_c [ - sum_{s < ns} P+_s^H (p-_s - P+_s R) ],  gnorm2 = || G ||^2
 * The sources are taken in order in batches of nb_max; R is transformed once and
 * the batches' adjoint products accumulate in the second spectra buffer.
 * G_out [nr][nvs][nt] float32; loss_out / gnorm2_out device float64 (may be NULL).
 * Needs kernel, data and MDD_FLAG_FULL_GRAD (MDD_ESTATE otherwise). */
mdd_status mdd_full_grad(mdd_plan* plan, const float* R, float* G_out, double* loss_out,
                         double* gnorm2_out);

/* One full-gradient iteration in place: the gradient of mdd_full_grad at R (for
 * MDD_OPT_NSGD at R + mu s0), then the update of mdd_step.  With MDD_OPT_SGD and
 * lr = kappa 2 / sigma_max^2 this is the Landweber iteration of Appendix B.
 * Needs kernel, data and MDD_FLAG_FULL_GRAD. */
mdd_status mdd_full_step(mdd_plan* plan, float* R, float* s0, float* s1, const mdd_opt* opt,
                         double* loss_out, double* gnorm2_out);

/* Reciprocity preconditioner C_r (Theory section): out = (z + z^T) / 2, the
 * transpose swapping the first two axes of z [n][n][nt] float32 (receivers and
 * virtual sources, which then coincide).  C_r is self-adjoint, so the same call
 * is its adjoint.  z and out are device pointers, 16-byte aligned; out may be z
 * (in place), otherwise the two must not overlap.  No plan: enqueued on `stream`.
 * Errors: EINVAL (NULL or misaligned), ESHAPE (n outside [1, 4096], nt not one of
 * 128, 256, 512, 1024), EHIP. */
mdd_status mdd_reciprocity(const float* z, float* out, int32_t n, int32_t nt, void* stream);

/* Forget stored model spectra (MDD_FLAG_STORE_RF): call after changing R
 * other than through mdd_step. */
mdd_status mdd_invalidate_model_spectra(mdd_plan* plan);

/* Largest squared singular value of the kernel at each retained frequency,
 * lam_out [nf] device float64, by `iters` power iterations on D_k^H D_k over
 * all ns sources (Appendix B: the operator's largest singular value is the
 * kernel's, max over k).  Needs mdd_set_kernel. */
mdd_status mdd_sigma_max2(mdd_plan* plan, int32_t iters, double* lam_out);

/* Kernel timing with HIP events on the plan's stream.  enable != 0 starts
 * recording (the plan keeps up to `capacity` launches, host memory);
 * mdd_profile_read returns, per kernel class (see MDD_KC_*), the summed
 * milliseconds and launch counts of the launches recorded so far.  It
 * synchronises the plan's stream. */
#define MDD_KC_FFT_MODEL 0   /* forward transform of the model */
#define MDD_KC_GEMM 1        /* per-frequency products (+ residual, loss) */
#define MDD_KC_UPDATE 2      /* inverse transform + mask + update (+ model transform) */
#define MDD_KC_REDUCE 3      /* float64 reductions */
#define MDD_KC_DATA_FFT 4    /* transforms of batch data (forward / adjoint operators) */
#define MDD_KC_RECIPROCITY 5 /* C_r on spectra (mdc_forward_rec / mdc_adjoint_rec) */
#define MDD_KC_COUNT 6
mdd_status mdd_profile_enable(mdd_plan* plan, int32_t enable, int32_t capacity);
mdd_status mdd_profile_read(mdd_plan* plan, double* ms_host, int64_t* count_host);

/* Measurement aid, not a step of the method: moves the HBM bytes of one Adam update
 * launch (R, s0, s1 [rows][ncols][nt] float32 read and written in place, and the
 * spectra spec [rows][ceil(ncols/16)][nf][16] complex float32 read and written in
 * place) without its transforms, so that its duration is the floor the memory
 * system sets for the update kernel at these sizes.  variant 0: the update kernel's
 * grid, workgroup mapping, spectra staging and 8-byte per-lane accesses; 1: the same
 * with 16-byte per-lane accesses; 2: flat streams over the three arrays and the
 * spectra (two launches); 3: the spectra alone as a flat stream (the bytes the
 * per-frequency products read and write besides D_b and U_b).  The arrays' contents
 * are overwritten with meaningless
 * values.  Pointers 16-byte aligned; enqueued on `stream`.  Errors: EINVAL (NULL,
 * misaligned, variant), ESHAPE (rows or ncols outside [1, 4096], nt not one of
 * 128, 256, 512, 1024, nf outside [1, nt/2 + 1]), EHIP. */
mdd_status mdd_calibrate_update(float* R, float* s0, float* s1, float* spec, int32_t rows,
                                int32_t ncols, int32_t nt, int32_t nf, int32_t variant,
                                void* stream);

/* Measurement aid, not a step of the method: reads the batch's kernel rows, row idx[b]
 * of D_k for every frequency k and batch entry b (D [nf][ns][round16(nr)] complex
 * float32, idx nb int32 on the device; an index outside [0, ns) reads row 0), with the
 * grid of the one-virtual-source products (nf x groups workgroups, batch entries split
 * into groups of ceil(nb / groups)) but none of their arithmetic, reductions or
 * barriers, and writes one partial per (frequency, group, receiver pair) to out
 * (nf * groups * round16(nr) / 2 float4).  Its duration is the floor of that access
 * pattern.  groups 0 takes the number the products kernel uses for (nb, nf).  Pointers
 * D and out 16-byte aligned; enqueued on `stream`.  Errors: EINVAL (NULL, misaligned),
 * ESHAPE (nb outside [1, 64], ns outside [1, 2^20], nr outside [1, 4096], nf outside
 * [1, 2049], groups outside [1, nb]), EHIP. */
mdd_status mdd_calibrate_rows(const float* D, const int32_t* idx, float* out, int32_t nb,
                              int32_t nf, int32_t ns, int32_t nr, int32_t groups, void* stream);

/* Static description of a status code. */
const char* mdd_status_string(mdd_status status);

/* The hipError_t of the last failed HIP call on this plan (0 if none). */
int32_t mdd_plan_last_hip_error(const mdd_plan* plan);

#ifdef __cplusplus
}
#endif
#endif /* MDD_H */
