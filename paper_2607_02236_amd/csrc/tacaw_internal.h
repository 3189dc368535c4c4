// Internal interface between the plan runtime (tacaw_plan.hip) and the kernel
// translation units. Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tacaw {

constexpr int kMaxDet = 8;   // detector masks per plan
constexpr int kMaxCorr = 3;  // bins where the window's DFT is non-zero (Hann: 0, 1, L-1)

// Thread-local error message of the C ABI (tacaw_last_error): set_error stores
// msg and returns code; clear_error empties it.
int set_error(int code, const char* msg);
void clear_error();

// Element offset of pixel k inside one input frame whose ny rows of nx pixels are
// rs elements apart (rs = nx: contiguous; rs > nx: a k-space window of a wider grid).
__host__ __device__ __forceinline__ int64_t pix_off(int64_t k, int32_t nx, int64_t rs) {
  return rs == nx ? k : (k / nx) * rs + k % nx;
}

// Arguments of the fused chunk kernels (FFT and GEMM forms).
struct SegArgs {
  const void* in;          // push buffer, element (i, n, k) at in + i*pstride + n*fstride +
                           // pix_off(k, nx, row_stride)
  int64_t pstride;         // elements
  int64_t fstride;         // elements
  int64_t row_stride;      // elements between the input's pixel rows (ring: nx)
  int32_t nx;
  int64_t push_begin;      // absolute frame index of the push buffer's frame 0
  const void* ring;        // [n_slots][D][n_k] frames pushed earlier, slot = probe % n_slots,
                           // frame f at row f mod D
  int64_t ring_depth;      // D (>= L, < 2^30)
  int32_t ring_row_lo;     // (s_lo * hop) mod D: ring row of the launch's first chunk
  int32_t from_ring;       // whole-series variant: every chunk is read from the ring
  int32_t ring_tiles;      // > 0: the ring is stored per pixel tile, [n_slots][ring_tiles][D][W]
                           // (W = the chunk kernel's tile width); 0: [n_slots][D][n_k]
  int32_t n_slots;
  int32_t n_k;
  int32_t probe0;          // first probe of the push
  int32_t n_probes;        // probes in the push
  int32_t s_lo, s_hi;      // chunks [s_lo, s_hi) are completed by this push
  int32_t hop;
  int32_t track_mean;      // accumulate sum(psi - c) and sum_s X'_s at the correction bins
  int32_t corr_skip;       // leave the correction bins out of S (the per-chunk mean kernel
                           // supplies their whole FP64 value)
  int32_t n_corr;          // 1 (rectangular) or 3 (Hann)
  int32_t corr_rows[kMaxCorr];  // output rows of the correction bins 0, 1, L-1 (GEMM form)
  const float* win_t;      // window, transposed per thread: [N2][N1] (t = N2*n1 + n2)
  const float2* tw;        // inter-pass twiddles exp(-2 pi i n2 k1 / L): [N2][N1]
  double2* cref;           // [n_probe][n_k] reference subtracted before the window; with
                           // track_mean the launch holding a probe's first chunk writes it
  double2* msum;           // [n_probe][n_k] FP64 sum of (psi - c) over counted frames
  double2* xs;             // [n_probe][kMaxCorr][n_k] FP64 sum over chunks of X'(bin)
  double* S;               // [n_om][n_k] FP64 accumulator of sum |X'|^2
  int32_t s_store;         // 1: first launch since reset, S is written (not read and added)
  int32_t n_om;            // output rows: L, or 2 roi_half + 1
  int32_t roi_half;        // energy window M (0 = all bins); bin m -> row (m + M) mod L
  int32_t n_det;           // per-probe detector partials (0 = off)
  const double* masks;     // [n_det][n_k]
  const int32_t* pair_slot;// [n_tiles][n_det] slot in dpart of (tile, detector), -1 if the
                           // detector's mask is zero on the tile; slots are grouped by detector
  double* dpart;           // [n_pairs][n_probes][n_om]
  const float* gscale;     // GEMM form: [n_probe][n_k] power-of-two scale of psi - mu
};

// Launchers (return hipError_t of the launch).
hipError_t launch_seg_fft(int L, int in_dtype, bool sub64, const SegArgs& a, int n_tiles,
                          hipStream_t st);
// the whole-series variant reading every frame from the ring (a.from_ring, 2 hop = L)
hipError_t launch_seg_fft_ring(int L, int in_dtype, bool sub64, const SegArgs& a, int n_tiles,
                               hipStream_t st);
int seg_fft_tile_pixels(int L);
void seg_fft_split(int L, int* n1, int* n2);  // L = N1 * N2 of the push kernel's tables
bool seg_fft_supported(int L);

// fmat: [2][m_rows][2L] hi and lo parts of the window-folded DFT rows of the
// output bins (row 2r + c), m_rows = 2 n_om rounded up to a multiple of 32
hipError_t launch_seg_gemm(int L, int in_dtype, bool sub64, int prec, const SegArgs& a,
                           const void* fmat, int m_rows, int n_tiles, hipStream_t st);
int seg_gemm_tile_pixels(int L, int n_om);  // pixels per workgroup for n_om output rows
bool seg_gemm_supported(int L);
hipError_t launch_gemm_scale(const void* in, int in_dtype, int64_t pstride, int64_t fstride,
                             int32_t nx, int64_t rs, int64_t n_used, int32_t probe0,
                             int32_t n_probes, int32_t n_k, int prec, const double2* cref,
                             float* scale, hipStream_t st);

// Auxiliary kernels (tacaw_aux.hip).
hipError_t launch_fill_zero(void* p, int64_t bytes, hipStream_t st);
hipError_t launch_read_probe(const void* p, int64_t bytes, uint64_t* sum, hipStream_t st);
hipError_t launch_read_probe_columns(const void* p, int64_t n_rows, int64_t row_bytes,
                                     int32_t seg_bytes, uint64_t* sum, hipStream_t st);
// frames sampled for a probe's reference: frame t[r] of the push (relative to its
// first frame) with weight wt[r]; c = inv_sum * sum_r wt[r] psi(t[r])
constexpr int kRefSamples = 16;
struct RefSamples {
  int32_t n;
  int32_t round32;  // round c to FP32 (complex64 input: the chunk kernel subtracts in FP32)
  int32_t t[kRefSamples];
  double wt[kRefSamples];
  double inv_sum;
};
// nx, rs: pixel rows of the input frames (see pix_off)
hipError_t launch_ref_sampled(const void* in, int in_dtype, int64_t pstride, int64_t fstride,
                              int32_t nx, int64_t rs, const RefSamples& smp, int32_t probe0,
                              int32_t n_probes, int32_t n_k, double2* cref, hipStream_t st);
hipError_t launch_ref_mean(const void* in, int in_dtype, int64_t pstride, int64_t fstride,
                           int32_t nx, int64_t rs, int64_t n_used, int32_t probe0,
                           int32_t n_probes, int32_t n_k, double2* cref, hipStream_t st);
// the ring holds contiguous frames (pixel k at row offset k)
hipError_t launch_ring_store(const void* in, int in_dtype, int64_t pstride, int64_t fstride,
                             int32_t nx, int64_t rs, int64_t push_begin, int64_t f_lo,
                             int64_t f_hi, int32_t probe0, int32_t n_probes, int32_t n_slots,
                             int64_t depth, int32_t n_k, int32_t tile_w, void* ring,
                             hipStream_t st);
// det_off[d] .. det_off[d + 1]: the dpart slots of detector d (n_det + 1 entries)
struct DetSlots {
  int32_t off[kMaxDet + 1];
};
hipError_t launch_dpart_reduce(const double* dpart, const DetSlots& slots, int32_t n_probes,
                               int32_t n_det, int32_t n_om, int32_t probe0, int32_t n_probe_total,
                               double* Dp, hipStream_t st);

struct CorrArgs {
  int32_t n_k, n_probe, n_om, n_corr, mean_global;
  int32_t rows[kMaxCorr];  // output rows of the correction bins
  double2 wbin[kMaxCorr];  // W(bin) = sum_t w(t) exp(-2 pi i bin t / L)
  double inv_nused;        // 1 / frames_used
  double n_seg;            // N_s
  const double2* cref;
  const double2* msum;
  const double2* xs;
  const double* pcorr;  // [P][3][n_k] per-chunk mean: sum_s |X_s(b)|^2 (null unless that mode)
};
// S[i] <- kappa * q[(i / inner) % n_om] * S[i] (q may be null), copied to out when given
hipError_t launch_finalize_S(double* S, double* out, int64_t n_elem, double kappa, const double* q,
                             int64_t inner, int32_t n_om, hipStream_t st);
hipError_t launch_correct_S(const CorrArgs& c, double* S, double* out, double kappa, hipStream_t st);
hipError_t launch_correct_Dp(const CorrArgs& c, const double* masks, int32_t n_det, double* Dp,
                             hipStream_t st);
hipError_t launch_scale(double* p, int64_t n, double k, hipStream_t st);

// Per-chunk mean (tacaw_aux.hip): streams the frames [f_lo, f_hi) of a push once
// and keeps, per (probe, pixel) and open chunk, the FP64 sums the exact correction needs.
constexpr int kMaxPsegOpen = 4;  // chunks that may contain one frame: ceil(L / H)
struct PsegArgs {
  const void* in;          // frames of the push; element of absolute frame n at (n - base) * fstride
  int64_t pstride, fstride, rs;
  int32_t nx, n_k, probe0, n_probes;
  int64_t base, f_lo, f_hi;
  int32_t L, H, Ns, n_corr, V;
  double2 wbin[kMaxCorr];  // W(bin)
  const double2* tw;       // [3][L]: w(t) exp(-2 pi i bin t / L), bins 0, 1, L - 1 (rows 0, 1 read)
  const double2* cref;     // [P][n_k] reference c of these FP64 sums (the first frame)
  double2* open;           // [P][V][4][n_k]: open chunk sums (layout in pseg_kernel)
  double* pcorr;           // [P][3][n_k]: sum_s |X_s(b)|^2 of the closed chunks
  double2* cmean;          // [P][Ns][n_k]: each chunk's FP64 mean c + sum_t y' / L
};
hipError_t launch_pseg(const PsegArgs& a, int32_t in_dtype, hipStream_t st);
hipError_t launch_detector(const double* S, const double* masks, int32_t n_det, int32_t L,
                           int32_t n_k, double* D, hipStream_t st);

// Adjoint (tacaw_adjoint.hip).
// Tile of this workgroup. Workgroups are dealt to the 8 XCDs round-robin
// (workgroup b runs on XCD b mod 8); this gives each XCD a contiguous range of
// tiles, so neighbouring tiles (adjacent pixels of the same frame rows) go
// through the same L2. A bijection of [0, gridDim.x).
__device__ __forceinline__ int xcd_tile() {
  const int b = blockIdx.x, n = gridDim.x, q = n / 8, r = n % 8, x = b % 8;
  return x * q + (x < r ? x : r) + b / 8;
}

struct BwdArgs {
  const void* in;
  int64_t pstride, fstride;
  int64_t row_stride;      // pixel rows of in and grad (see pix_off)
  int32_t nx;
  void* grad;              // same layout as in
  int32_t n_k, probe0, n_probes, n_probe_total, n_seg, hop, n_det;
  int32_t n_om, roi_half;  // output rows and energy window (bin m -> row (m + M) mod L)
  int32_t mean_global;
  int32_t per_chunk;       // per-chunk mean: chunk s subtracts cmean[p][s][k]
  const double2* cmean;    // [n_probe][n_seg][n_k] chunk means from the forward pass
  double inv_nused;
  int64_t n_used;
  const float* win_t;      // [N2][N1]
  const float* dwin_t;     // [N2][N1] d w / d r (HANN_WIDTH) or null
  const float2* tw;        // [N2][N1]
  const double2* cref;     // [n_probe][n_k] reference c (the chunk kernel's, or the exact mean)
  const double2* msum;     // [n_probe][n_k] FP64 sum over the used frames of psi - c
  const double2* xs;       // [n_probe][kMaxCorr][n_k] FP64 sum over chunks of X' at bins 0, 1, L-1
  int32_t n_corr;          // bins where the window's DFT is nonzero (1 or 3), 0 = any bin
  double2 wbin[kMaxCorr];  // the window's DFT at bins 0, 1, L-1
  const double* gS;        // [n_om][n_k] or null
  const double* gD;        // [n_det][n_om] or null
  const double* gDp;       // [n_det][n_probe][n_om] or null
  const double* masks;     // [n_det][n_k]
  double kappa_S, kappa_p; // normalisations of S and S_p
  const double* qfac;      // [n_om] quantum-statistics factor per row, or null
  double2* gmean;          // [n_probes][n_k] sum over chunks and t of w * grad_y (mean term)
  double* dwpart;          // [n_tiles][2] partial sums: r-derivative term, loss value
};
hipError_t launch_bwd(int L, int in_dtype, const BwdArgs& a, int n_tiles, hipStream_t st);
int bwd_tile_pixels(int L);
int bwd_pass1_size(int L);
hipError_t launch_bwd_mean_fix(const BwdArgs& a, int in_dtype, hipStream_t st);
hipError_t launch_bwd_wparam(const double* part, int n, double c, double* out, hipStream_t st);
hipError_t launch_mean_exact(const void* in, int in_dtype, int64_t pstride, int64_t fstride,
                             int32_t nx, int64_t rs, int64_t n_used, int32_t probe0,
                             int32_t n_probes, int32_t n_k, double2* mu, hipStream_t st);
hipError_t launch_dot_gS(const double* S, const double* gS, int64_t n, double* out,
                         hipStream_t st);
hipError_t launch_sum(const double* p, int64_t n, double* out, hipStream_t st);
// *cnt += the count of NaN and Inf values in x[0..n) (the caller zeroes *cnt)
hipError_t launch_count_nonfinite(const double* x, int64_t n, unsigned long long* cnt,
                                  hipStream_t st);

}  // namespace tacaw
