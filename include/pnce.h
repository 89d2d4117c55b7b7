/*
 * pnce.h -- PN-sequence correlation channel estimation on AMD Instinct MI355X
 * (gfx950): the C ABI of libpnce.so.
 *
 * Method (arXiv 2206.05506, Sections II-A and II-B): T transmitters send the
 * same m-sequence s of length N = 2^d - 1 at once, transmitter t delayed by
 * t*L samples (Eq. 7-8 with the shift spacing equal to the CIR length L).
 * Receive antenna r hears one frame y_r of N samples (cyclic prefix removed).
 * Correlating y_r with s at the K = T*L lags those transmitters occupy gives
 * every (transmitter, antenna) L-tap CIR at once (Eq. 3, Eq. 10):
 *
 *     H[b][r][k] = (1/N) * sum_{n<N} Y[b][r][n] * s[(n - k) mod N],  k < K,
 *
 * i.e. the dense contraction H = Y P / N with P[n][k] = s[(n-k) mod N] a
 * Toeplitz +-1 slice of the circulant of Eq. 2. Transmitter t's CIR is the
 * view H[b][r][t*L : (t+1)*L] (Eq. 10). The library never stores P: the
 * kernels expand it from the sequence bits on chip.
 *
 * Plans made by pnce_create_ex may instead delay transmitter t by
 * floor(N/T)*t samples (Eq. 8's circular shift, PNCE_LAGS_EQ8): column
 * k = t*L + l of H then holds lag lag(k) = floor(N/T)*t + l, P[n][k] =
 * s[(n - lag(k)) mod N], and every "k" in the formulas below reads lag(k).
 * They may also use another primitive polynomial, i.e. another m-sequence of
 * the same length, as a neighbouring cell would (Section II-B).
 *
 * Conventions for every entry point
 *  - Tensor pointers are DEVICE memory owned by the caller, dense row-major,
 *    with the shapes stated per call. Complex numbers are interleaved
 *    (re, im) float pairs ("c64") or double pairs ("c128"). Each pointer is
 *    aligned to its element: 8 bytes for c64, 16 for c128, 8 for buffers of
 *    16-bit codes, 4 for e4m3 codes and for scales; a misaligned pointer is
 *    refused with PNCE_E_INVALID.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Compute calls only enqueue work and return; results are ready when the
 *    stream is. Faults of enqueued kernels surface at the caller's next sync.
 *  - Return value: 0 = PNCE_OK; > 0 = a warning, the call did its work;
 *    < 0 = an error, nothing was enqueued and no output was touched. The
 *    text of the last error on the calling thread is pnce_last_error().
 *  - A plan (and an uneven-batch plan) belongs to the device that was
 *    current when it was made: its sequence tables live there. Compute calls
 *    made while another device is current return PNCE_E_INVALID.
 *  - An empty batch (batch == 0) is valid: once the plan and the other
 *    scalar arguments (precision, format, cp, steps) pass their checks, the
 *    call returns PNCE_OK without reading its tensor pointers, which may be
 *    NULL, and enqueues nothing.
 *  - Compute calls allocate nothing, set no memory with a memset and do not
 *    synchronise: each enqueues kernels only, so a sequence of them can be
 *    captured into a hipGraph and replayed. pnce_varlen_tune and
 *    pnce_varlen_set_tuning are not compute calls: they rebuild and upload
 *    an uneven-batch plan's work list, allocating and synchronising.
 *  - No C++ exception and no abort crosses this boundary.
 *  - A plan is immutable after pnce_create; calls on one plan from several
 *    host threads or streams are safe, except that pnce_refine uses the
 *    workspace its caller passes. An uneven-batch plan changes only in
 *    pnce_varlen_tune and pnce_varlen_set_tuning, which must not overlap any
 *    other use of that plan, including its launches still in flight.
 */
#ifndef PNCE_H
#define PNCE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pnce_plan pnce_plan;   /* opaque, owned by the library */
typedef int pnce_status;

#define PNCE_OK 0
#define PNCE_W_LAG_ALIAS 1      /* T*L > N: lags are taken mod N, so some   */
                                /* columns of H repeat (Eq. 7 violated)      */
#define PNCE_E_INVALID (-1)     /* null pointer, size <= 0, bad enum value   */
#define PNCE_E_UNSUPPORTED (-2) /* N is not 2^d - 1 with 2 <= d <= 16        */
#define PNCE_E_NOMEM (-3)       /* device or host allocation failed          */
#define PNCE_E_HIP (-4)         /* a HIP runtime call failed                 */

/* Arithmetic of a contraction (estimate / adjoint). */
#define PNCE_PREC_F32 0   /* FP32 matrix cores: v_mfma_f32_32x32x2_f32        */
#define PNCE_PREC_F32S 1  /* FP32-accurate on bf16 matrix cores: each FP32    */
                          /* operand split into three bf16 parts (exact, the  */
                          /* other operand being +-1), FP32 accumulation      */
#define PNCE_PREC_BF16 2  /* operand rounded once to bf16 (round to nearest   */
                          /* even), bf16 matrix cores, FP32 accumulation      */
#define PNCE_PREC_F64 3   /* FP64 vector ALU on c128 buffers (for gradient    */
                          /* checks; not a throughput path)                   */
#define PNCE_PREC_F64ACC 4 /* c64 buffers, FP64 sums on FP64 matrix cores    */
                           /* (v_mfma_f64_16x16x4_f64), one rounding to FP32  */
#define PNCE_PREC_EXACT 5  /* c64 buffers, exact sums: each input row in      */
                           /* fixed point (62 bits below a power of two above */
                           /* the row's largest |re| or |im|) cut into eight  */
                           /* 8-bit digits, each digit's sum exact in int32   */
                           /* on int8 matrix cores (v_mfma_i32_32x32x32_i8),  */
                           /* combined and scaled in FP64; alpha and beta in  */
                           /* FP64, one rounding to FP32. Exact for elements  */
                           /* within 2^38 of their row's largest magnitude,   */
                           /* smaller ones rounded at 2^-62 of the row bound; */
                           /* at most 65535 terms per output (else            */
                           /* PNCE_E_UNSUPPORTED); a row holding inf or NaN   */
                           /* gives NaN outputs.                              */
#define PNCE_PREC_EXACT32 6 /* as PNCE_PREC_EXACT with 30 bits cut into four  */
                            /* digits (half the matrix work), and no FP64     */
                            /* arithmetic: the digit sums combined exactly in */
                            /* int64, rounded once to FP32, alpha and beta    */
                            /* applied in FP32. Exact for elements within 2^6 */
                            /* of their row's largest magnitude, smaller ones */
                            /* rounded to a multiple of 2^-30 of the row      */
                            /* bound (the power of two above that magnitude): */
                            /* an error of at most 2^-30 max|x| per term      */

/* Reduced-precision storage formats of Y (the half-precision conversion
 * before correlation, Section III-B). */
#define PNCE_FMT_BF16 1
#define PNCE_FMT_F16 2
#define PNCE_FMT_E4M3 3   /* OCP e4m3fn, saturating at +-448 */

/* Where transmitter t's L lags sit (the circular shift of its sequence). */
#define PNCE_LAGS_ADJACENT 0 /* t*L + l: blocks side by side, K = T*L lags    */
#define PNCE_LAGS_EQ8 1      /* floor(N/T)*t + l: Eq. 8, with floor(N/T) - L  */
                             /* guard lags after each block                   */

/*
 * Create a plan for sequence length N, T multiplexed transmitters, L taps
 * and R receive antennas (Sections II-A, II-B). Builds the m-sequence on the
 * host (degree d = log2(N+1); fixed primitive polynomial per degree; LFSR
 * state 1,0,...,0; bit 0 sent as +1 and bit 1 as -1) and uploads its bits
 * (a few KiB) to the current device. Synchronous.
 * Errors: plan == NULL or T, L, R <= 0 -> PNCE_E_INVALID; N not 2^d - 1 with
 * 2 <= d <= 16, one frame too large for 32-bit offsets
 * ((R + 32) * (max(N, T*L) + 1) * 8 >= 2^31), or a sequence bit stream of
 * N + max(N, T*L) + 352 bits that does not fit a workgroup's 160 KiB of LDS
 * next to the kernels' stages (only d = 16 with T*L above about 14 N)
 * -> PNCE_E_UNSUPPORTED;
 * T*L > 16*N or R > 65535 -> PNCE_E_INVALID. Warning: T*L > N (Eq. 7's bound N_batch <= floor(N/L)
 * broken) -> PNCE_W_LAG_ALIAS, with a valid plan. On error *plan = NULL.
 */
pnce_status pnce_create(pnce_plan **plan, int N, int T, int L, int R);

/*
 * pnce_create with a choice of sequence and lag layout (Section II-B, Eq. 8).
 * feedback: 0 for the built-in polynomial, else the taps of the feedback
 *   polynomial x^d + sum_{bit i set} x^i (bits below d; the LFSR computes
 *   b[n+d] = XOR over set bits i of b[n+i] from the start 1,0,...,0). It must
 *   be primitive, so that the sequence has length N and the two-level
 *   autocorrelation of Eq. 1; neighbouring cells take different ones.
 * spacing: PNCE_LAGS_ADJACENT (as pnce_create) or PNCE_LAGS_EQ8.
 * Every entry point taking the plan follows its lags (estimate, packed and
 * cyclic-prefix estimates, least squares, adjoint, refinement).
 * Errors: as pnce_create, plus -> PNCE_E_INVALID for an unknown spacing,
 * PNCE_LAGS_EQ8 with T*L > N (Eq. 7: the blocks would overlap), feedback
 * bits at or above d, or a feedback polynomial that is not primitive.
 */
pnce_status pnce_create_ex(pnce_plan **plan, int N, int T, int L, int R, unsigned feedback,
                           int spacing);

/* The plan's lags as T*L host ints: lags_host[t*L + l] = t*D + l with D = L
 * (PNCE_LAGS_ADJACENT) or floor(N/T) (PNCE_LAGS_EQ8). */
pnce_status pnce_get_lags(const pnce_plan *plan, int *lags_host);

/* The feedback taps of the plan's sequence (the built-in ones when the plan
 * was made with feedback 0). */
pnce_status pnce_get_feedback(const pnce_plan *plan, unsigned *feedback);

/* Free a plan and its device tables. NULL is a no-op. Synchronous: the
 * caller must not destroy a plan that enqueued work still uses. */
pnce_status pnce_destroy(pnce_plan *plan);

/* Copy the plan's sequence as N host bytes of +1 / -1 (Eq. 1). */
pnce_status pnce_get_sequence(const pnce_plan *plan, signed char *s_host);

/* Plan geometry: writes N, T, L, R (any pointer may be NULL). */
pnce_status pnce_get_shape(const pnce_plan *plan, int *N, int *T, int *L, int *R);

/*
 * Correlator (Eq. 3, Eq. 10) on complex input.
 *   H = alpha * s_b * (Y P) + beta * H,  s_b = scales ? scales[b] : 1,
 *   (Y P)[b][r][k] = sum_{n<N} Y[b][r][n] s[(n - k) mod N].
 * alpha = 1/N is the correlator of Eq. 3; alpha = 1 gives P^T applied to Y
 * (the backward of the receive model P x). alpha and beta are applied in
 * FP32 (FP64 for PNCE_PREC_F64).
 * Y: [batch][R][N] c64 (c128 when precision == PNCE_PREC_F64);
 * H: [batch][R][T*L] c64 (c128 for PNCE_PREC_F64), read only if beta != 0;
 * scales: NULL or `batch` device floats. Y and H must not overlap.
 * precision: PNCE_PREC_F32, _F32S, _BF16, _F64, _F64ACC, _EXACT (alpha and
 * beta then in FP64) or _EXACT32.
 * Errors: null Y/H, batch < 0, unknown precision -> PNCE_E_INVALID.
 */
pnce_status pnce_estimate(const pnce_plan *plan, void *stream, const void *Y,
                          void *H, int batch, int precision, double alpha,
                          const float *scales, double beta);

/*
 * Quantise a complex64 batch for storage (the conversion to half precision
 * before correlation, Section III-B) with a per-frame power-of-two scale.
 * scale_b is the smallest 2^e with maxabs_b <= target * 2^e, maxabs_b the
 * largest |re| or |im| in frame b, target 1 (bf16, f16) or 448 (e4m3);
 * a frame of zeros or with a non-finite maxabs gets 1. Each value is
 * multiplied by 1/scale_b in FP32 and rounded to nearest even.
 * Y: [batch][R][N] c64. Yq: [batch][R][2][N+1] codes, 2 bytes each for
 * bf16/f16 and 1 byte for e4m3: per antenna the real plane then the
 * imaginary plane, each padded with one zero sample. scales: [batch] float.
 * Runs two kernels (per-frame max, then convert) on `stream`.
 * Errors: null pointer, batch < 0, bad format -> PNCE_E_INVALID.
 */
pnce_status pnce_pack(const pnce_plan *plan, void *stream, const void *Y,
                      void *Yq, float *scales, int batch, int format);

/*
 * pnce_pack_cp (cp = 0: pnce_pack) with a workspace from the caller, which
 * lets every frame be read from HBM once (the conversion to half precision
 * ahead of the correlation, Section III-B): frames above 1 MiB (and batches
 * under 256 frames) are cut into slices of 16,384 samples held in registers
 * by consecutive workgroups until the frame's maximum is gathered, then
 * converted (one launch after a clear of the workspace); the codes and
 * scales equal pnce_pack's. Batches of 256+ frames of at most 1 MiB take
 * pnce_pack's one-launch path, and frames of more than half as many slices
 * as the GPU holds workgroups at once (about 4 million samples on MI355X)
 * its two-pass path; both leave work unused but for the flag below.
 * work: device memory of at least PNCE_PACK_WORK_BYTES(batch) bytes, 4-byte
 * aligned, owned by the caller, overwritten by the call (no content needed
 * before it; 4 KiB per frame keeps the frames' synchronisation words on
 * separate memory channels); concurrent calls need separate workspaces.
 * After the call has run, the 32-bit word at index 1024 * batch of work
 * (the last one; every launch plan writes it) is nonzero only if a
 * slice's wait for the rest of its frame ran past its bound (about a second;
 * never expected: the launch is sized so that a frame's workgroups run
 * together); the codes of that call are then not valid.
 * Errors: as for pnce_pack_cp; work NULL, misaligned or too small ->
 * PNCE_E_INVALID.
 */
#define PNCE_PACK_WORK_BYTES(batch) (4096 * (size_t)(batch) + 4)
pnce_status pnce_pack_ws(const pnce_plan *plan, void *stream, const void *Y_raw, int cp,
                         void *Yq, float *scales, int batch, int format, void *work,
                         size_t work_bytes);

/*
 * Correlator on a quantised batch (layout of pnce_pack) with FP32
 * accumulation on bf16 / f16 / fp8 matrix cores; the +-1 operand is exact in
 * every format. H = (scales[b] / N) * (Yq P) + beta * H, H [batch][R][T*L]
 * c64. scales may be NULL (all 1).
 * Errors: null Yq/H, batch < 0, bad format -> PNCE_E_INVALID.
 */
pnce_status pnce_estimate_packed(const pnce_plan *plan, void *stream,
                                 const void *Yq, const float *scales, void *H,
                                 int batch, int format, double beta);

/*
 * Adjoint of the correlator: a circular convolution with the sequence,
 *   A = alpha * (G P^T) + beta * C,  (G P^T)[b][r][n] = sum_{k<T*L}
 *   G[b][r][k] s[(n - k) mod N].
 * alpha and beta are applied in FP32 (FP64 for PNCE_PREC_F64).
 * With alpha = 1/N it is the transpose of pnce_estimate (the backward of
 * the correlator); with alpha = -1, beta = 1, C = y and G a CIR stack it is
 * the residual y - P h of the receive model of Eq. 9.
 * G: [batch][R][T*L]; A, C: [batch][R][N]; c64, or c128 for
 * PNCE_PREC_F64. C may equal A, or be NULL when beta == 0. G must not
 * overlap A. precision: PNCE_PREC_F32, _F32S, _BF16, _F64, _F64ACC, _EXACT
 * (alpha and beta then in FP64) or _EXACT32.
 */
pnce_status pnce_adjoint(const pnce_plan *plan, void *stream, const void *G,
                         void *A, const void *C, int batch, int precision,
                         double alpha, double beta);

/*
 * Least-squares refinement of a CIR estimate (the correlator's bias floor
 * comes from the -1/M term of Eq. 1; each step removes part of it):
 *   repeat `steps` times:  r = y - P x;  x = x + P^T r / N.
 * The correlations and the inner steps' residuals are summed on four int8
 * digits (PNCE_PREC_EXACT32: exact to 2^-30 of each row's largest element,
 * then an FP32 epilogue; no FP64 arithmetic); the last residual is exact
 * (PNCE_PREC_EXACT: r is y - P x rounded once to FP32, FP64 only there). Residual sums of more than 65535
 * terms are FP32-accurate (PNCE_PREC_F32S) in the inner steps and
 * accumulated in FP64 (PNCE_PREC_F64ACC) in the last.
 * y: [batch][R][N] c64 (the original, unquantised frames);
 * X: [batch][R][T*L] c64, in: the starting estimate, out: refined;
 * work: device scratch of batch*R*N*8 bytes (the residual). steps >= 0.
 */
pnce_status pnce_refine(const pnce_plan *plan, void *stream, const void *y,
                        void *X, void *work, int batch, int steps);

/*
 * pnce_refine for callers that cannot allocate device memory (code under
 * stream capture, serving loops, harnesses that forbid hipMalloc): the same
 * kernels and steps, with the residual kept in a fixed array of
 * PNCE_NOALLOC_SCRATCH_MIB MiB of device memory that the library holds on
 * each GPU it runs on until the process ends; no memory is allocated or
 * freed by the call. Frames are refined in groups of
 * floor(PNCE_NOALLOC_SCRATCH_MIB MiB / (R*N*8)) (each frame's result equals
 * that of pnce_refine up to FP32 rounding of the kernels' launch shape).
 * y, X: as for pnce_refine (device memory owned by the caller).
 * Every call on one GPU shares that GPU's array: calls that overlap in time
 * on one GPU (on different streams, or from several threads) race and give
 * wrong results; calls on one stream are ordered and safe. The array keeps
 * the last call's residuals; nothing in it needs to start at zero.
 * Errors: PNCE_E_UNSUPPORTED when one frame's residual (R*N*8 bytes) exceeds
 * the array; otherwise as for pnce_refine.
 */
#define PNCE_NOALLOC_SCRATCH_MIB 64
pnce_status pnce_refine_noalloc(const pnce_plan *plan, void *stream, const void *y,
                                void *X, int batch, int steps);

/*
 * Raw received blocks (Section II-A, Section III-B): each antenna row holds
 * the cyclic prefix of cp samples followed by the N samples of the sequence
 * period; the prefix is removed by addressing alone (rows are cp + N
 * samples apart), in the same launch as the correlation or the conversion.
 * Y_raw: [batch][R][cp + N] complex64 (complex128 for PNCE_PREC_F64);
 * pnce_estimate_cp computes H = scales_b * (Y P) / N as pnce_estimate with
 * alpha = 1/N, beta = 0; pnce_pack_cp writes the codes and scales of
 * pnce_pack. cp >= 0; raw frames must stay below 2 GiB
 * (PNCE_E_UNSUPPORTED), other errors as for pnce_estimate / pnce_pack.
 */
pnce_status pnce_estimate_cp(const pnce_plan *plan, void *stream, const void *Y_raw, int cp,
                             void *H, int batch, int precision, const float *scales);
pnce_status pnce_pack_cp(const pnce_plan *plan, void *stream, const void *Y_raw, int cp,
                         void *Yq, float *scales, int batch, int format);

/*
 * pnce_estimate_cp on raw blocks that sit in host memory, with their copies
 * to the device overlapped with the estimates (the host-to-device transfer
 * that the frame latency of Section IV-C includes). Frames are taken in
 * chunks of `chunk`: chunk i is copied on copy_stream into half (i & 1) of
 * the staging buffer while chunk i - 1 is estimated on `stream`; events
 * order each copy after the estimate that last read its half and each
 * estimate after its copy. Every copy waits for the work already queued on
 * `stream` when the call is made, and `stream` waits for every copy, so once
 * `stream` reaches the end of this call's work, H is complete and staging and
 * Y_host are free again. Results equal pnce_estimate_cp on the same frames
 * bit for bit.
 * Y_host: [frames][R][cp + N] complex64 (complex128 for PNCE_PREC_F64) in
 *   host memory; page-locked (hipHostMalloc) for the copies to overlap, else
 *   the runtime stages them and they do not. Must not change until `stream`
 *   has finished this call's work.
 * H: [frames][R][T*L] complex64 (complex128 for PNCE_PREC_F64), device.
 * staging: device memory owned by the caller, 16-byte aligned, of at least
 *   PNCE_HOST_STAGING_BYTES(R, N, cp, min(chunk, frames), precision) bytes;
 *   its contents on return are unspecified.
 * copy_stream may equal stream (the copies then do not overlap).
 * Unlike the compute calls, this call creates and destroys four HIP events
 * (hipEventDisableTiming) and enqueues copies: it is not meant for stream
 * capture.
 * Errors: PNCE_E_INVALID for chunk < 1, a NULL pointer with frames > 0 or a
 * staging buffer that is too small; otherwise as for pnce_estimate_cp. An
 * error after the first chunk was queued leaves H partly written.
 */
#define PNCE_HOST_STAGING_BYTES(R, N, cp, chunk, precision)                         \
  (2 * (size_t)(chunk) * (size_t)(R) * ((size_t)(N) + (size_t)(cp)) *             \
   ((precision) == PNCE_PREC_F64 ? 16 : 8))
pnce_status pnce_estimate_host(const pnce_plan *plan, void *stream, void *copy_stream,
                               const void *Y_host, int cp, void *H, int frames, int chunk,
                               int precision, void *staging, size_t staging_bytes);

/*
 * Least-squares CIRs in closed form. The two-level autocorrelation of the
 * sequence (Eq. 1) gives P^T P = (N+1) I - J (J all-ones, K = T*L <= N), so
 * (P^T P)^-1 = (I + J / (N+1-K)) / (N+1), and from correlator outputs
 * H = P^T y / N (Eq. 3, Eq. 10) every row (frame, antenna) becomes
 *   H <- N/(N+1) * (H + (sum_k H[k]) / (N+1-K)),
 * the exact least-squares solution: it removes the -sum(h)/N bias that the
 * -1 off-peak autocorrelation leaves in Eq. 3 (noiseless frames are
 * recovered to rounding). In place on H: [batch][R][T*L] complex64 device;
 * the row sums are accumulated in FP64. Errors: PNCE_E_UNSUPPORTED when
 * T*L > N (least squares is not unique); the usual plan/batch/pointer checks.
 */
pnce_status pnce_debias(const pnce_plan *plan, void *stream, void *H, int batch);

/*
 * pnce_estimate (alpha = 1/N, beta = 0) followed by pnce_debias: the
 * correction is applied in the correlator's epilogue when one workgroup
 * holds every lag of a row (T*L <= 512 and enough frames to fill the chip),
 * otherwise by a second launch. precision: PNCE_PREC_F32, _F32S or _BF16.
 * scales: optional per-frame factors as for pnce_estimate. Same errors as
 * pnce_debias and pnce_estimate.
 */
pnce_status pnce_estimate_ls(const pnce_plan *plan, void *stream, const void *Y, void *H,
                             int batch, int precision, const float *scales);

/* ---------------------------------------------------------------------------
 * Uneven batches (the batching form): frames of different (R, N, T, L) drawn
 * from the ranges of Table I, estimated in ONE persistent launch whose work
 * list is built on the host, with tile widths chosen by an autotuner.
 * ------------------------------------------------------------------------- */
typedef struct {
  int R, N, T, L;     /* frame shape; N = 2^d - 1 with 2 <= d <= 16          */
  long long y_off;    /* first code of the frame in Yq, in codes; a multiple  */
                      /* of 8. The frame holds [R][2][N+1] codes (the layout  */
                      /* of pnce_pack for one frame)                          */
  long long h_off;    /* first complex64 element of the frame's CIRs in H,    */
                      /* which hold [R][T*L] values                           */
} pnce_frame_desc;

typedef struct pnce_varlen_plan pnce_varlen_plan;   /* opaque */

/*
 * Build a plan for `nframes` frames described by the host array `frames`
 * (copied). format: PNCE_FMT_BF16 or PNCE_FMT_F16. Every frame uses the
 * built-in m-sequence of its length and adjacent lag blocks (the lags of
 * pnce_create). Builds one m-sequence per distinct N, the frame table and a
 * work list: units of (frame, 32-antenna
 * block) carrying all their column tiles, dealt to persistent workgroups
 * longest-first. Column width per (N, T*L) class defaults to 128, 64 or 32
 * lags per wave by T*L; pnce_varlen_tune replaces it with measured choices.
 * Synchronous (uploads the tables). Errors: PNCE_E_INVALID for a bad frame,
 * offset or format, PNCE_E_UNSUPPORTED for a bad N or a frame whose codes
 * ((R + 32) * 2 * (N + 1) * 2 bytes) reach 2 GiB. Warning
 * PNCE_W_LAG_ALIAS if some frame has T*L > N.
 */
pnce_status pnce_varlen_create(pnce_varlen_plan **vplan, const pnce_frame_desc *frames,
                               int nframes, int format);

/* Free a varlen plan. NULL is a no-op. */
pnce_status pnce_varlen_destroy(pnce_varlen_plan *vplan);

/*
 * The correlator of Eq. 3 / Eq. 10 for every frame, one persistent launch:
 *   H_f = (scales[f] / N_f) * (Yq_f P_f), scales may be NULL (all 1).
 * Yq: device codes of all frames (at their y_off); H: device complex64 (at
 * their h_off); the caller keeps the frames' regions disjoint. The launch
 * reads only plan-owned static tables, so it can be captured in a hipGraph.
 * The device work list is allocated once, by pnce_varlen_create, at its
 * largest possible size, and pnce_varlen_tune / pnce_varlen_set_tuning copy
 * the new list over it in place: a graph captured before tuning keeps valid
 * addresses and its replays run the current schedule.
 */
pnce_status pnce_varlen_estimate(const pnce_varlen_plan *vplan, void *stream, const void *Yq,
                                 const float *scales, void *H);

/* The same result through one launch per frame (the reference schedule);
 * each frame uses the column width of the plan, so results are identical. */
pnce_status pnce_varlen_estimate_each(const pnce_varlen_plan *vplan, void *stream,
                                      const void *Yq, const float *scales, void *H);

/*
 * Autotuner: for each (N, T*L) class and each column width (32, 64 and 128
 * lags per wave) it measures the marginal time of one (frame, 32-antenna)
 * unit in a full persistent launch: the units of up to 16 frames of the
 * class, repeated to give every workgroup slot about 2 and then 4 of them,
 * are timed (`reps` launches each, HIP events on `stream`), and the
 * difference divided by the extra units per slot cancels launch and start
 * overheads. From these it builds candidate work lists (the plan's current
 * one; the fastest widths with measured costs; the default widths with
 * measured costs; the fastest widths with the default cost model), times
 * each on the whole batch and keeps the fastest, so tuning does not lose to
 * the plan's previous schedule beyond timing noise. Synchronous. Writes H
 * (the repeated units write the same values). Replaces the plan's work
 * list: no launch of this plan may be in flight.
 */
pnce_status pnce_varlen_tune(pnce_varlen_plan *vplan, void *stream, const void *Yq,
                             const float *scales, void *H, int reps);

/*
 * Read (n_classes only when the arrays are NULL) or install the per-class
 * choice: sequence length N, T*L, lags per wave / 32 (1, 2 or 4) and cost in
 * microseconds per unit. set_tuning rebuilds and uploads the work list
 * (synchronous; no launch of this plan may be in flight); classes not
 * listed keep their choice. Lets a caller cache tuning results.
 */
pnce_status pnce_varlen_get_tuning(const pnce_varlen_plan *vplan, int *n_classes, int *N,
                                   int *K, int *nc, float *us_per_unit);
pnce_status pnce_varlen_set_tuning(pnce_varlen_plan *vplan, int n_classes, const int *N,
                                   const int *K, const int *nc, const float *us_per_unit);

/* Work-list statistics: persistent workgroups, tiles, and the largest and
 * mean per-workgroup cost (microseconds, by the plan's cost model). */
pnce_status pnce_varlen_stats(const pnce_varlen_plan *vplan, int *n_workgroups, int *n_tiles,
                              float *max_cost, float *mean_cost);

/* Text of a status code (static storage). */
const char *pnce_status_string(pnce_status status);

/* Detail of the last error returned on the calling thread ("" if none). */
const char *pnce_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PNCE_H */
