/*
 * tacaw.h -- C ABI of the TACAW spectral hot path on MI355X (gfx950).
 *
 * The library reduces, for every probe position, a time series of exit waves
 * psi(k, t) to the ultra-low-loss spectrum S(k, omega) and its detector
 * integrals (paper: Sec. I Eq. 1 for |FT_t psi|^2; Sec. II.B.2 for the Welch
 * chunking "s_{n+1} = s_n + L/nu" and the window; Eq. 2 for the chunk average
 * united over scan batches; the DetectorSet paragraphs of Sec. II.B.1 and
 * App. B for mask integration).
 *
 * Conventions shared by every entry point:
 *  - Pixels k run over a ny x nx reciprocal-space grid, row-major, contiguous.
 *  - Frequency bins are in FFT order: bin m holds nu_m = m / (L dt) for
 *    m < L/2 and (m - L) / (L dt) otherwise; the forward kernel is
 *    exp(-2 pi i m t / L) (Sec. III.B transform sign), so exp(+2 pi i nu t)
 *    lands at +nu. A plan with an energy window (omega_half = M > 0) keeps only
 *    the bins of signed index -M..M, in ascending order (row r = M + signed m).
 *    "n_omega" below is the number of output bins, L or 2M + 1.
 *  - All device pointers are caller-owned HIP device memory (e.g. torch
 *    tensors) unless stated otherwise. Work is enqueued on the plan's HIP
 *    stream in call order; an input buffer must stay alive until the stream has
 *    passed the call that reads it. Calls return after enqueueing.
 *  - Return value: 0 (TACAW_OK) or a negative TACAW_ERR_* code; no exception
 *    crosses the ABI. tacaw_last_error() gives a thread-local message.
 *    Argument, shape and state checks run on the host before any HIP call.
 *  - A plan is not thread-safe; distinct plans may run on distinct streams.
 */
#ifndef TACAW_H
#define TACAW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---------------------------------------------------- */
#define TACAW_OK 0
#define TACAW_ERR_INVALID_ARG (-1) /* bad value, null pointer, misaligned pointer */
#define TACAW_ERR_SHAPE (-2)       /* sizes inconsistent with the plan            */
#define TACAW_ERR_STATE (-3)       /* call not allowed in the plan's state         */
#define TACAW_ERR_OOM (-4)         /* device allocation failed or size too large   */
#define TACAW_ERR_HIP (-5)         /* a HIP runtime call failed                    */
#define TACAW_ERR_UNSUPPORTED (-6) /* valid but not implemented combination        */
#define TACAW_ERR_NONFINITE (-7)   /* finalize with TACAW_FLAG_CHECK_FINITE found NaN  */
                                   /* or Inf in S or D_p (the plan is finalized)     */

/* ---- window w(t), t = 0..L-1 (Sec. II.B.2; Sec. III.A) ------------------ */
#define TACAW_WIN_HANN 0       /* periodic Hann 1/2 - 1/2 cos(2 pi t / L) (default)   */
#define TACAW_WIN_RECT 1       /* no window (all ones)                                */
#define TACAW_WIN_HANN_WIDTH 2 /* width-r Hann: 1/2 + 1/2 cos(2 pi (t - L/2)/(r L))    */
                               /* for |t - L/2| <= r L / 2, else 0; r = window_param  */
#define TACAW_WIN_TUKEY 3      /* periodic Tukey, window_param = alpha (taper share)  */
#define TACAW_WIN_CUSTOM 4     /* caller-supplied values h_window[0..L-1] (e.g. the   */
                               /* Blackman-Harris, Kaiser and Dolph-Chebyshev windows */
                               /* of App. A)                                          */

/* ---- elastic-mean handling (the mean is removed before the window) ------ */
#define TACAW_MEAN_GLOBAL 0      /* mean over the frames that enter a chunk (default) */
#define TACAW_MEAN_PER_SEGMENT 1 /* unweighted mean of each chunk's own L frames       */
                                 /* (scipy's detrend='constant'), removed exactly in   */
                                 /* FP64; needs the FFT or bf16 GEMM transform, a      */
                                 /* window whose DFT lives on bins 0 and +-1,          */
                                 /* hop >= L/4 and n_frames                            */
                                 /* < 2^31, else UNSUPPORTED                           */
#define TACAW_MEAN_NONE 2        /* keep the zero-loss peak (the paper's behaviour)   */

/* ---- time transform ------------------------------------------------------ */
#define TACAW_FFT_F32 0     /* radix FFT in FP32, staged in LDS                      */
#define TACAW_GEMM_BF16X3 1 /* DFT as a GEMM on MFMA, bf16 hi/lo split x3, FP32 acc;  */
                            /* L = 128..1024 (powers of two). With a window whose DFT */
                            /* lives on bins 0 and +-1 it streams like the FFT form   */
                            /* (pushes of any size, rings, exact mean correction);    */
                            /* otherwise each probe's series comes in one push        */
#define TACAW_GEMM_F16X3 2  /* DFT as a GEMM on MFMA, scaled fp16 hi/lo split x3;     */
                            /* L = 128..1024; each probe's whole series in one push   */
                            /* (its operand scale and the exact mean are pre-passes)  */

/* ---- input element type -------------------------------------------------- */
#define TACAW_C64 0  /* complex64: interleaved float (re, im), 8 bytes           */
#define TACAW_C128 1 /* complex128: interleaved double (re, im), 16 bytes        */

/* ---- reduction over probes (Eq. 2: union of scan batches) --------------- */
#define TACAW_PROBE_MEAN 0 /* S = average over probes (default)                 */
#define TACAW_PROBE_SUM 1  /* S = sum over probes                                */

typedef struct tacaw_plan_s* tacaw_plan_t;

/* Plan descriptor. Chunk (segment) s covers frames [s*hop, s*hop + seg_len);
 * only full chunks are used: N_s = (n_frames - seg_len) / hop + 1, and frames
 * at or beyond (N_s - 1) * hop + seg_len are accepted and ignored. */
typedef struct {
  int32_t n_probe;        /* probes (scan positions) in this plan, >= 1              */
  int32_t ny, nx;         /* reciprocal-space grid, ny * nx pixels                   */
  int64_t n_frames;       /* frames that will be pushed per probe (N_t >= seg_len)   */
  int32_t seg_len;        /* L: power of two in [64, 1024], or 200 (Sec. III.A's     */
                          /* chunk length; FFT transform, forward only)              */
  int32_t hop;            /* H = L / nu with integer division, 1 <= H <= L           */
  int32_t window;         /* TACAW_WIN_*                                             */
  double window_param;    /* r for HANN_WIDTH (> 0), alpha for TUKEY ([0, 1])        */
  int32_t mean_mode;      /* TACAW_MEAN_*                                            */
  int32_t transform;      /* TACAW_FFT_F32 or TACAW_GEMM_*                           */
  int32_t in_dtype;       /* TACAW_C64 or TACAW_C128                                 */
  int32_t probe_reduce;   /* TACAW_PROBE_MEAN or TACAW_PROBE_SUM                     */
  double dt_fs;           /* frame interval in fs (> 0; axis helpers only)           */
  int32_t n_det;          /* detector masks given at plan time (0..8)                */
  const double* d_masks;  /* device [n_det][ny][nx] float64 weights, or NULL if      */
                          /* n_det == 0; copied into the plan. Needed for per-probe  */
                          /* detector spectra (STEM images), which are fused into    */
                          /* the push.                                               */
  int32_t max_probes_in_flight; /* probes with a partially pushed series at once    */
                                /* (streaming ring capacity); 0 = n_probe            */
  int32_t flags;          /* TACAW_FLAG_* bits                                       */
  double temperature_K;   /* > 0: multiply bin m by the quantum-statistics factor    */
                          /* beta E_m / (1 - exp(-beta E_m)) of Eq. 1, beta = 1/kT,  */
                          /* E_m = h nu_m (dt_fs sets nu_m; +nu is energy loss);     */
                          /* 0: no factor                                            */
  const double* h_window; /* host array of seg_len window values (TACAW_WIN_CUSTOM)  */
                          /* copied at plan creation; NULL otherwise                 */
  int64_t ring_frames;    /* streaming ring depth D per in-flight probe: 0 = seg_len,*/
                          /* chunks are processed by the push that completes them;   */
                          /* D > seg_len (a multiple of 64; D - seg_len >= every     */
                          /* push) = deferred mode: pushes are copied into the ring  */
                          /* and completed chunks are processed from it in batches,  */
                          /* when the ring would overwrite them and at the end of    */
                          /* each probe's series (fewer, larger launches; FFT or     */
                          /* bf16 GEMM form, compact windows)                        */
  int64_t k_row_stride;   /* k-space window (the k-ROI of Sec. II.B): elements       */
                          /* between the input's pixel rows, >= nx (0 = nx). The    */
                          /* ny x nx pixels reduced are then a window of a wider     */
                          /* grid, read in place by pushes and the adjoint.          */
  int32_t omega_half;     /* energy window (the centred +-ROI of Sec. II.B / App. B):*/
                          /* 0 = all seg_len bins in FFT order; M in [1, L/2 - 1] =  */
                          /* only the 2M + 1 bins of signed index -M..M (frequency   */
                          /* m / (L dt)), stored in ascending order, row r = m + M.  */
                          /* S, D, D_p and their gradients then have n_omega = 2M+1  */
                          /* rows, and the DFT-GEMM form computes only these rows.   */
} tacaw_plan_desc;

/* flags: record HIP events around the chunk kernel of every push; the duration
 * of the last push's chunk launches (or of the last ingest and its commit) is
 * reported in tacaw_plan_info.last_chunk_kernel_ms (reading it synchronizes with
 * the plan's stream; -1 if that push completed no chunk). */
#define TACAW_FLAG_TIME_KERNELS 1
/* flags: deferred ring mode (ring_frames > 0, hop = seg_len/2) with the ring
 * stored per pixel tile of the chunk kernel, [slot][tile][row][tile pixels],
 * instead of per frame: a tile's chunk is then contiguous in memory, so the
 * chunk kernel needs a few address translations per chunk instead of one per
 * frame (large frames, e.g. 1024^2 pixels, otherwise miss the translation
 * caches on most loads). Pushes, or a producer writing through
 * tacaw_ingest_frames_tiled (tacaw_ingest_frames fails with STATE on such a
 * plan). */
#define TACAW_FLAG_TILED_RING 2
/* flags: finalize counts the non-finite values of S and of the per-probe detector
 * spectra after normalisation (NaN or Inf exit waves propagate into them; without
 * the flag nothing checks). If any is found, finalize still completes (S written,
 * the plan finalized) but returns TACAW_ERR_NONFINITE; tacaw_plan_info.nonfinite
 * holds the count. The check synchronizes with the plan's stream. */
#define TACAW_FLAG_CHECK_FINITE 4

typedef struct {
  int32_t n_segments;     /* N_s                                                     */
  int32_t n_omega;        /* output bins: seg_len, or 2 omega_half + 1               */
  int64_t frames_used;    /* (N_s - 1) * hop + seg_len                               */
  int64_t frames_dropped; /* frames pushed so far beyond frames_used (all probes)    */
  int64_t device_bytes;   /* device memory currently owned by the plan               */
  int32_t state;          /* 0 open, 1 finalized                                     */
  int32_t probes_complete;/* probes whose whole series has been pushed               */
  double window_sum_sq;   /* sum_t w(t)^2                                            */
  int32_t tile_pixels;    /* pixels per workgroup tile of the push kernel            */
  int32_t nonfinite;      /* non-finite values in S and D_p at finalize (flag        */
                          /* TACAW_FLAG_CHECK_FINITE; clipped to 2^31 - 1), else 0    */
  double last_chunk_kernel_ms; /* last push's chunk kernel in ms (flag set), or -1   */
} tacaw_plan_info;

/* Create a plan: validates desc on the host (no HIP call on failure), then
 * allocates the plan's FP64 accumulators on the current HIP device and records
 * hip_stream (a hipStream_t; NULL = default stream) for all later work.
 * Errors: INVALID_ARG, UNSUPPORTED, OOM, HIP. *out is NULL on error. */
int tacaw_plan(const tacaw_plan_desc* desc, void* hip_stream, tacaw_plan_t* out);

/* Host-only validation of a descriptor (the checks tacaw_plan runs first). */
int tacaw_plan_check(const tacaw_plan_desc* desc);

/* Push the next n_frames frames of probes [probe0, probe0 + n_probes) in time
 * order (Sec. II.B: exit waves are processed on the fly as they are produced).
 * Element (i, n, ky, kx) of the push, for probe probe0 + i, frame cursor + n and
 * pixel (ky, kx), is at d_frames + i * probe_stride + n * frame_stride +
 * ky * R + kx, strides in ELEMENTS of in_dtype, R = k_row_stride (nx if 0), and
 * frame_stride >= (ny - 1) R + nx. All probes of one push must have
 * received the same number of frames before. Every chunk completed by this push
 * is windowed, transformed, squared and accumulated in FP64; frames that later
 * chunks still need are copied into a plan-owned ring (last L frames per probe
 * in flight), so a series may arrive in any number of pieces. The result does
 * not depend on how frames or probes are split into pushes (App. B: batch shape
 * does not influence the results). A thermalisation period is discarded by
 * pointing d_frames at the first kept frame, and every s-th stored snapshot
 * is kept by passing s times the frame pitch as frame_stride (Sec. III.A drops
 * the first picoseconds of each trajectory before chunking); no copy is made.
 * Errors: INVALID_ARG (null/misaligned pointer, bad stride), SHAPE (probe range
 * or frame count beyond the plan), STATE (plan finalized, probes at different
 * frame cursors, ring capacity exceeded), OOM, HIP. */
int tacaw_push_frames(tacaw_plan_t plan, const void* d_frames, int32_t probe0, int32_t n_probes,
                      int64_t n_frames, int64_t probe_stride, int64_t frame_stride);

/* Zero-copy ingest (deferred ring mode only): a producer writes the next n_frames
 * frames of probes [probe0, probe0 + n_probes) straight into the plan's ring
 * instead of pushing a buffer (so frames never exist twice in HBM). On return
 * *d_dst points at frame cursor of probe probe0; element (i, n, k) goes to
 * *d_dst + i * (*probe_stride) + n * (*frame_stride) + k (elements of in_dtype,
 * contiguous ny * nx frames). Chunk launches that must read the overwritten
 * rows first are enqueued before returning, so the producer writes on the
 * plan's stream (or after synchronizing with it), then calls
 * tacaw_commit_frames with the same arguments; no other push, ingest or finalize
 * may come in between. Conditions: 1 <= n_frames <= ring_frames - seg_len; the
 * rows do not wrap (cursor mod ring_frames + n_frames <= ring_frames); probe0 mod
 * max_probes_in_flight + n_probes <= max_probes_in_flight; frames end at or
 * before frames_used.
 * Errors: INVALID_ARG, STATE (not deferred, ingest open, cursors differ, ring
 * slots taken), SHAPE (sizes above), OOM, HIP. */
int tacaw_ingest_frames(tacaw_plan_t plan, int32_t probe0, int32_t n_probes, int64_t n_frames,
                        void** d_dst, int64_t* probe_stride, int64_t* frame_stride);

/* Zero-copy ingest for plans whose ring is stored per pixel tile
 * (TACAW_FLAG_TILED_RING): as tacaw_ingest_frames, but element (i, n, k) goes to
 * *d_dst + i * (*probe_stride) + (k / T) * (*tile_stride) + n * (*frame_stride)
 * + k mod T, with T = *tile_pixels (elements of in_dtype): each tile of T
 * adjacent pixels holds its frames contiguously. Conditions and errors as
 * tacaw_ingest_frames (STATE also for a plan without the tiled ring, and for
 * the per-chunk mean, whose FP64 pass reads per-frame rows); commit with
 * tacaw_commit_frames. */
int tacaw_ingest_frames_tiled(tacaw_plan_t plan, int32_t probe0, int32_t n_probes,
                              int64_t n_frames, void** d_dst, int64_t* probe_stride,
                              int64_t* frame_stride, int64_t* tile_stride, int32_t* tile_pixels);

/* Mark the frames handed out by the open tacaw_ingest_frames as written: at the
 * end of a series, its remaining chunks run. Errors: STATE (no matching ingest), HIP. */
int tacaw_commit_frames(tacaw_plan_t plan, int32_t probe0, int32_t n_probes, int64_t n_frames);

/* Finish the reduction once every probe's series has been pushed: applies the
 * exact elastic-mean correction, normalises per voxel by 1 / (L sum_t w^2) and
 * averages over chunks (and probes, Eq. 2). Writes S(m, k) as float64
 * [n_omega][ny][nx] to d_S when d_S is not NULL (caller-owned device buffer);
 * the plan keeps its own copy for tacaw_detector_spectra and tacaw_backward.
 * Errors: STATE (already finalized, or a probe's series incomplete), HIP. */
int tacaw_finalize(tacaw_plan_t plan, double* d_S);

/* Detector (energy-filtered) spectra from a finalized plan:
 * D_j(m) = sum_k M_j(k) S(m, k) into d_D [n_det][n_omega] (float64, device).
 * d_masks_or_null: device [n_det][ny][nx] float64 masks, or NULL to use the
 * plan's masks (then n_det must equal the plan's). d_Dp_or_null: device
 * [n_det][n_probe][n_omega] float64 per-probe spectra (one STEM-EELS image per
 * detector and bin); requires the plan's own masks.
 * Errors: STATE (not finalized), INVALID_ARG, HIP. */
int tacaw_detector_spectra(tacaw_plan_t plan, const double* d_masks_or_null, int32_t n_det,
                           double* d_D, double* d_Dp_or_null);

/* Adjoint of the finalized plan's outputs with respect to the input series and
 * the window parameter. Upstream gradients (any may be NULL, all device
 * float64): d_gS [n_omega][ny][nx] (dLoss/dS), d_gD [n_det][n_omega]
 * (dLoss/dD_j, plan masks), d_gDp [n_det][n_probe][n_omega] (dLoss/dD_{j,p}).
 * d_frames: the complete series of probes [probe0, probe0 + n_probes) again
 * (same layout rules as tacaw_push_frames, all frames_used frames present);
 * chunk transforms are recomputed, not stored. The elastic mean, and for
 * windows whose DFT lives on bins 0 and +-1 the mean term of the gradient, are
 * taken from the forward pass's FP64 sums, so d_frames must hold the frames
 * that were pushed. d_grad_frames: output, same
 * dtype and strides as d_frames, d/dRe + i d/dIm convention; it is fully
 * written for frames < frames_used and left untouched beyond. d_grad_wparam:
 * device float64 scalar that receives (+=) dLoss/d(window_param) for
 * HANN_WIDTH plans (may be NULL). All mean modes; with PER_SEGMENT each
 * chunk's mean is taken from the forward pass too.
 * Errors: STATE (not finalized), INVALID_ARG, UNSUPPORTED, HIP. */
int tacaw_backward(tacaw_plan_t plan, const void* d_frames, int32_t probe0, int32_t n_probes,
                   int64_t probe_stride, int64_t frame_stride, const double* d_gS,
                   const double* d_gD, const double* d_gDp, void* d_grad_frames,
                   double* d_grad_wparam);

/* Allocation-free form of tacaw_backward, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc). Same arguments, results and errors as tacaw_backward,
 * whose kernels it runs; their scratch (16 bytes per probe and pixel of the call
 * plus 16 bytes per pixel tile) comes from a fixed library-owned device array of
 * TACAW_STATIC_SCRATCH_BYTES per GPU (held until the process ends) instead of
 * plan memory, and no device memory is allocated or freed. The plan's device
 * must be current. A call needing more scratch fails with SHAPE (split the
 * probes over several calls). Every call on one GPU shares that array and
 * writes each scratch value before reading it: calls that overlap in time on
 * one GPU (other streams or threads) race and must be serialised by the caller.
 * Errors: as tacaw_backward, plus SHAPE (scratch limit) and INVALID_ARG (the
 * plan's device is not current). */
#define TACAW_STATIC_SCRATCH_BYTES (16 << 20)
int tacaw_backward_static(tacaw_plan_t plan, const void* d_frames, int32_t probe0,
                          int32_t n_probes, int64_t probe_stride, int64_t frame_stride,
                          const double* d_gS, const double* d_gD, const double* d_gDp,
                          void* d_grad_frames, double* d_grad_wparam);

/* Zero every accumulator and frame cursor so the plan can take a new series of
 * the same shape (buffers are kept). */
int tacaw_reset(tacaw_plan_t plan);

/* Checkpoint and resume of a long run. The result is a sum over chunks and
 * probe batches, each batch adding its share to a stored array (Sec. II.B's
 * Calculator paragraph, Eq. 2), so the accumulators after some probes are the
 * complete state of the run: a job that stops there can carry on in a new
 * process from a copy of them.
 *
 * tacaw_plan_export writes that state to the host buffer h_buf (caller-owned,
 * buf_bytes long): a header (format tag, a fingerprint of the descriptor fields,
 * window and detector masks the state depends on, the sizes, frames dropped),
 * the frame cursor of every probe, then S, the per-probe mean references, mean
 * and correction sums, the per-probe detector spectra and, with the per-chunk
 * mean, its correction sums, references and chunk means, as stored on the
 * device (FP64). The format is for the same library build and byte order.
 * It synchronises the plan's stream. *bytes_needed (if not NULL) receives the
 * size; with h_buf NULL only the size is returned (any state). Allowed only on
 * an open plan at a probe boundary: every probe untouched or complete (cursor 0
 * or >= frames_used), no ingest open. Errors: INVALID_ARG (NULL plan), SHAPE
 * (buffer too small), STATE (finalized, or a probe partially pushed), HIP.
 *
 * tacaw_plan_import loads such a state into a plan built from the same
 * descriptor and mask values (the pointers and stream may differ) that has had
 * no frames pushed since its creation or last reset; the plan then continues
 * as the exporting one would: pushing the remaining probes as an uninterrupted
 * run does gives bitwise its S, and its detector spectra up to the order of
 * their FP64 atomic sums (which varies between any two runs). Errors:
 * INVALID_ARG (NULL, not a
 * state, or a cursor off a probe boundary), SHAPE (another descriptor, or bytes
 * shorter than the state), STATE (finalized, frames pushed, ingest open), HIP;
 * on an error the plan is unchanged, except after HIP (reset it). */
int tacaw_plan_export(tacaw_plan_t plan, void* h_buf, int64_t buf_bytes, int64_t* bytes_needed);
int tacaw_plan_import(tacaw_plan_t plan, const void* h_buf, int64_t bytes);

/* Union of two exported states over disjoint probe sets (Eq. 2: S of a scan is
 * the sum over its batches), e.g. shards of the probes reduced in separate
 * processes or on separate GPUs: the accumulators are added element-wise in
 * FP64 (an untouched probe's entries are zero in an export), the cursors of the
 * probes pushed in either state are kept and the dropped-frame counts added.
 * Importing the result and finalizing gives the spectra of all those probes, up
 * to the FP64 rounding order of the sums. Host memory only, no device call:
 * h_a, h_b and h_out are caller-owned buffers of `bytes` bytes each (h_out may
 * be h_a or h_b). Errors: INVALID_ARG (NULL, not a state, a probe pushed in
 * both), SHAPE (different descriptors or sizes, or bytes not the states' size). */
int tacaw_state_merge(const void* h_a, const void* h_b, void* h_out, int64_t bytes);

/* Replace the stream used for subsequent calls. */
int tacaw_set_stream(tacaw_plan_t plan, void* hip_stream);

/* Sizes and counters of a plan (host call, no device work). */
int tacaw_plan_get_info(tacaw_plan_t plan, tacaw_plan_info* info);

/* Free every plan-owned device buffer (waits for the plan's stream). */
void tacaw_destroy(tacaw_plan_t plan);

/* Message of the last error on this thread ("" if none). */
const char* tacaw_last_error(void);

/* Library version string. */
const char* tacaw_version(void);

/* ---- fused producer (synthetic exit waves) ------------------------------ */
/* Synthetic exit-wave series written straight into a ring (through the ingest
 * calls above) or any strided complex64 buffer, standing in for the multislice
 * producer whose frames the paper reduces as they are produced (Sec. II.B). Per
 * probe p, frame n and pixel k:
 *   psi = elastic + sum_{j < n_terms} amplitude (x_j(n) + i y_j(n))
 *         + noise_sigma (g_r + i g_i),
 * term j a tone of quantised frequency f_j (2^20 phase steps per cycle, energy
 * from one of the probe's n_lines Lorentzian lines with centres uniform in
 * [line_lo_mev, line_hi_mev] and half widths in [hwhm_lo_mev, hwhm_hi_mev], or
 * uniform in [e_lo_mev, e_hi_mev] when n_lines = 0; dt_fs the frame step),
 * advanced frame by frame by a float32 rotation that restarts from the
 * tabulated phase every 64 frames. All random draws come from Philox4x32-10
 * (Salmon et al., SC 2011) keyed by seed and counted by (probe, pixel or
 * frame, term), so any frame range can be produced in any order. The tables
 * are caller-owned device arrays: d_cos, d_sin = cos, sin (2 pi q / 2^20),
 * q < 2^20 (float32); d_normal = 2^12 standard normals (float32); d_tan =
 * tan(pi (u - 1/2)), u = (i + 1/2) / 2^16 (float64). */
typedef struct {
  int32_t ny, nx;
  int32_t n_terms;  /* 0 .. 16 */
  int32_t n_lines;  /* 0: uniform energy band */
  uint32_t seed;
  int32_t reserved;
  double amplitude, noise_sigma, elastic_re, elastic_im;
  double e_lo_mev, e_hi_mev, line_lo_mev, line_hi_mev, hwhm_lo_mev, hwhm_hi_mev;
  double dt_fs;
  const float* d_cos;
  const float* d_sin;
  const float* d_normal;
  const double* d_tan;
} tacaw_synth_desc;

/* Frames [frame0, frame0 + n_frames) of probes [probe0, probe0 + n_probes) as
 * complex64: element (i, n, k) at d_dst + i * probe_stride + (k / tile_pixels)
 * * tile_stride + n * frame_stride + k mod tile_pixels (elements; tile_pixels >=
 * ny * nx means a plain frame layout, tile_stride then ignored), i.e. the
 * layouts tacaw_ingest_frames and tacaw_ingest_frames_tiled hand out. One
 * kernel on hip_stream; nothing is allocated. Errors: INVALID_ARG (null
 * pointers, tables, strides, alignment), SHAPE (ranges), HIP. */
int tacaw_synth_frames(const tacaw_synth_desc* desc, void* d_dst, int32_t probe0,
                       int32_t n_probes, int64_t frame0, int64_t n_frames, int64_t probe_stride,
                       int64_t frame_stride, int64_t tile_stride, int32_t tile_pixels,
                       void* hip_stream);

/* Measured HBM read ceiling (measurement support, not a step of the method):
 * reads every byte of the device buffer d_buf once with 16-byte vector loads
 * and stores the wrapping (mod 2^64) sum of its little-endian 64-bit words in
 * the device scalar *d_sum, so the reads cannot be elided and the result is
 * checkable. Timing the call (HIP events on hip_stream) over a buffer far larger
 * than the caches gives the read bandwidth the chunk transform's exit-wave
 * rate is compared with, next to the datasheet HBM peak. n_bytes must be a
 * positive multiple of 16 and d_buf 16-byte aligned; stream-ordered, nothing
 * is allocated. Errors: INVALID_ARG, HIP. */
int tacaw_read_probe(const void* d_buf, int64_t n_bytes, void* hip_stream, uint64_t* d_sum);

/* The same measurement for the access pattern of the chunk transform: the
 * device buffer is n_rows rows (frames) of row_bytes, read once column by
 * column, seg_bytes wide (a pixel tile: 128 = 16 complex64 pixels), with 8-byte
 * loads, so that one wave load takes seg_bytes from each of 512 / seg_bytes
 * rows. *d_sum receives the same wrapping 64-bit sum as tacaw_read_probe gives
 * for the whole buffer. seg_bytes in {64, 128, 256, 512}, row_bytes a multiple
 * of it (at most 65535 columns), 8-byte alignment; nothing is allocated.
 * Errors: INVALID_ARG, HIP. */
int tacaw_read_probe_columns(const void* d_buf, int64_t n_rows, int64_t row_bytes,
                             int32_t seg_bytes, void* hip_stream, uint64_t* d_sum);

#ifdef __cplusplus
}
#endif

#endif /* TACAW_H */
