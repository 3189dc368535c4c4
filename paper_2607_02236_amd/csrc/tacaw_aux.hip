// Auxiliary kernels of the plan: zero fills, per-probe references, the exact
// FP64 mean pre-pass, ring stores for streamed series, per-probe detector
// partial reduction, the exact elastic-mean correction, normalisation and the
// masked detector reduction D_j(m) = sum_k M_j(k) S(m, k) (DetectorSet,
// Sec. II.B.1 of the paper).
#include <type_traits>

#include "tacaw_internal.h"

namespace tacaw {

static inline int blocks_for(int64_t n, int bs, int cap = 65535 * 8) {
  int64_t b = (n + bs - 1) / bs;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}

__global__ void fill_zero_kernel(uint4* p, int64_t n16, unsigned char* tail, int ntail) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
  if (blockIdx.x == 0 && (int)threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

hipError_t launch_fill_zero(void* p, int64_t bytes, hipStream_t st) {
  if (bytes <= 0) return hipSuccess;
  const int64_t n16 = bytes / 16;
  const int ntail = (int)(bytes - n16 * 16);
  hipLaunchKernelGGL(fill_zero_kernel, dim3(blocks_for(n16, 256, 8192)), dim3(256), 0, st,
                     (uint4*)p, n16, (unsigned char*)p + n16 * 16, ntail);
  return hipGetLastError();
}

// Reference c(k) of a probe: the window-weighted mean of up to kRefSamples
// frames spread over the first chunk (FP64 sum, rounded to FP32 for complex64
// input so that the chunk kernel subtracts exactly this value). Any c keeps the
// mean correction exact; one close to the chunks' own mean keeps the FP32
// transform of psi - c small at bins 0 and +-1, where the correction cancels.
template <typename InT>
__global__ void ref_sampled_kernel(const InT* in, int64_t pstride, int64_t fstride, int32_t nx,
                                   int64_t rs, RefSamples smp, int32_t probe0, int32_t n_probes,
                                   int32_t n_k, double2* cref) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (k >= n_k || i >= n_probes) return;
  const InT* src = in + (int64_t)i * pstride + pix_off(k, nx, rs);
  double sx = 0.0, sy = 0.0;
  for (int r = 0; r < smp.n; ++r) {
    const InT v = src[(int64_t)smp.t[r] * fstride];
    sx += smp.wt[r] * (double)v.x;
    sy += smp.wt[r] * (double)v.y;
  }
  sx *= smp.inv_sum;
  sy *= smp.inv_sum;
  if (smp.round32) {
    sx = (double)(float)sx;
    sy = (double)(float)sy;
  }
  cref[(int64_t)(probe0 + i) * n_k + k] = make_double2(sx, sy);
}

hipError_t launch_ref_sampled(const void* in, int in_dtype, int64_t pstride, int64_t fstride,
                              int32_t nx, int64_t rs, const RefSamples& smp, int32_t probe0,
                              int32_t n_probes, int32_t n_k, double2* cref, hipStream_t st) {
  dim3 g((n_k + 255) / 256, n_probes);
  if (in_dtype == 1)
    hipLaunchKernelGGL(ref_sampled_kernel<double2>, g, dim3(256), 0, st, (const double2*)in,
                       pstride, fstride, nx, rs, smp, probe0, n_probes, n_k, cref);
  else
    hipLaunchKernelGGL(ref_sampled_kernel<float2>, g, dim3(256), 0, st, (const float2*)in,
                       pstride, fstride, nx, rs, smp, probe0, n_probes, n_k, cref);
  return hipGetLastError();
}

// Exact FP64 time mean over frames [0, n_used) of each (probe, pixel).
template <typename InT>
__global__ void mean_kernel(const InT* in, int64_t pstride, int64_t fstride, int32_t nx, int64_t rs,
                            int64_t n_used, int32_t probe0, int32_t n_probes, int32_t n_k,
                            double2* out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (k >= n_k || i >= n_probes) return;
  const InT* p = in + (int64_t)i * pstride + pix_off(k, nx, rs);
  double sx = 0.0, sy = 0.0;
  for (int64_t n = 0; n < n_used; ++n) {
    const InT v = p[n * fstride];
    sx += (double)v.x;
    sy += (double)v.y;
  }
  out[(int64_t)(probe0 + i) * n_k + k] = make_double2(sx / (double)n_used, sy / (double)n_used);
}

hipError_t launch_mean_exact(const void* in, int in_dtype, int64_t pstride, int64_t fstride,
                             int32_t nx, int64_t rs, int64_t n_used, int32_t probe0,
                             int32_t n_probes, int32_t n_k, double2* mu, hipStream_t st) {
  dim3 g((n_k + 255) / 256, n_probes);
  if (in_dtype == 1)
    hipLaunchKernelGGL(mean_kernel<double2>, g, dim3(256), 0, st, (const double2*)in, pstride,
                       fstride, nx, rs, n_used, probe0, n_probes, n_k, mu);
  else
    hipLaunchKernelGGL(mean_kernel<float2>, g, dim3(256), 0, st, (const float2*)in, pstride,
                       fstride, nx, rs, n_used, probe0, n_probes, n_k, mu);
  return hipGetLastError();
}

hipError_t launch_ref_mean(const void* in, int in_dtype, int64_t pstride, int64_t fstride,
                           int32_t nx, int64_t rs, int64_t n_used, int32_t probe0,
                           int32_t n_probes, int32_t n_k, double2* cref, hipStream_t st) {
  return launch_mean_exact(in, in_dtype, pstride, fstride, nx, rs, n_used, probe0, n_probes, n_k,
                           cref, st);
}

// ring[slot][f % D][k] = in[i][f - push_begin][k] for f in [f_lo, f_hi); each
// thread copies 16 bytes (two complex64 or one complex128 element).
template <typename InT>
__global__ void ring_store_kernel(const InT* in, int64_t pstride, int64_t fstride, int32_t nx,
                                  int64_t rs, int64_t push_begin, int64_t f_lo, int32_t n_f,
                                  int32_t probe0, int32_t n_slots, int64_t depth, int32_t n_k,
                                  InT* ring) {
  constexpr int V = 16 / (int)sizeof(InT);  // elements per thread
  const int64_t k0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * V;
  const int fi = blockIdx.y;
  const int i = blockIdx.z;
  if (k0 >= n_k || fi >= n_f) return;
  const int64_t f = f_lo + fi;
  const int slot = (probe0 + i) % n_slots;
  InT* dst = ring + ((int64_t)slot * depth + (f % depth)) * n_k;
  const InT* src = in + (int64_t)i * pstride + (f - push_begin) * fstride;
#pragma unroll
  for (int v = 0; v < V; ++v)
    if (k0 + v < n_k) dst[k0 + v] = src[pix_off(k0 + v, nx, rs)];
}

// The same into a ring stored per pixel tile: element (slot, row, k) at
// ((slot * n_tiles + k / W) * D + row) * W + k % W. A block copies R consecutive
// frames (R = 16, or the largest power of two dividing D; the first frame aligned
// to R in absolute frame index) of 256 V / R pixels, so it reads R runs of 256 V / R pixels and
// writes R consecutive rows, R W elements in a row, of each of its tiles: long
// runs on both sides instead of one tile row (64 bytes at W = 8) per tile.
#ifndef TACAW_RING_VEC
#define TACAW_RING_VEC 16  // bytes each thread of the tiled ring store copies per frame
#endif
template <typename InT>
__global__ void ring_store_tiled_kernel(const InT* in, int64_t pstride, int64_t fstride,
                                        int32_t nx, int64_t rs, int64_t push_begin, int64_t f_lo,
                                        int64_t f_hi, int32_t R, int32_t probe0, int32_t n_slots,
                                        int64_t depth, int32_t n_k, int32_t tile_w,
                                        int32_t n_tiles, InT* ring) {
  constexpr int V = TACAW_RING_VEC / (int)sizeof(InT);  // elements per thread
  const int tpr = 256 / R;                               // threads per frame
  const int r = threadIdx.x / tpr;
  const int64_t k0 = ((int64_t)blockIdx.x * tpr + threadIdx.x % tpr) * V;
  const int64_t f = (f_lo - f_lo % R) + (int64_t)blockIdx.y * R + r;
  const int i = blockIdx.z;
  if (k0 >= n_k || f < f_lo || f >= f_hi) return;
  const int slot = (probe0 + i) % n_slots;
  const InT* src = in + (int64_t)i * pstride + (f - push_begin) * fstride;
  const int64_t t = k0 / tile_w;  // tile_w is a multiple of V: the V elements share a tile row
  InT* dst = ring + (((int64_t)slot * n_tiles + t) * depth + (f % depth)) * tile_w + (k0 - t * tile_w);
#pragma unroll
  for (int v = 0; v < V; ++v)
    if (k0 + v < n_k) dst[v] = src[pix_off(k0 + v, nx, rs)];
}

hipError_t launch_ring_store(const void* in, int in_dtype, int64_t pstride, int64_t fstride,
                             int32_t nx, int64_t rs, int64_t push_begin, int64_t f_lo,
                             int64_t f_hi, int32_t probe0, int32_t n_probes, int32_t n_slots,
                             int64_t depth, int32_t n_k, int32_t tile_w, void* ring,
                             hipStream_t st) {
  const int64_t nf = f_hi - f_lo;
  if (nf <= 0) return hipSuccess;
  if (tile_w > 0) {
    const int V = TACAW_RING_VEC / (in_dtype == 1 ? 16 : 8);
#ifndef TACAW_RING_ROWS
#define TACAW_RING_ROWS 16  // frames per block of the tiled ring store (tuning parameter)
#endif
    int R = TACAW_RING_ROWS;  // halved until it divides D
    while (depth % R != 0) R /= 2;
    if (tile_w % V != 0) return hipErrorInvalidValue;
    const int32_t n_tiles = (n_k + tile_w - 1) / tile_w;
    const int64_t fb = f_lo - f_lo % R;
    dim3 g((unsigned)((n_k + (256 / R) * V - 1) / ((256 / R) * V)),
           (unsigned)((f_hi - fb + R - 1) / R), n_probes);
    if (in_dtype == 1)
      hipLaunchKernelGGL(ring_store_tiled_kernel<double2>, g, dim3(256), 0, st, (const double2*)in,
                         pstride, fstride, nx, rs, push_begin, f_lo, f_hi, R, probe0, n_slots,
                         depth, n_k, tile_w, n_tiles, (double2*)ring);
    else
      hipLaunchKernelGGL(ring_store_tiled_kernel<float2>, g, dim3(256), 0, st, (const float2*)in,
                         pstride, fstride, nx, rs, push_begin, f_lo, f_hi, R, probe0, n_slots,
                         depth, n_k, tile_w, n_tiles, (float2*)ring);
    return hipGetLastError();
  }
  const int V = in_dtype == 1 ? 1 : 2;
  dim3 g((unsigned)((n_k + 256 * V - 1) / (256 * V)), (unsigned)nf, n_probes);
  if (in_dtype == 1)
    hipLaunchKernelGGL(ring_store_kernel<double2>, g, dim3(256), 0, st, (const double2*)in,
                       pstride, fstride, nx, rs, push_begin, f_lo, (int32_t)nf, probe0, n_slots,
                       depth, n_k, (double2*)ring);
  else
    hipLaunchKernelGGL(ring_store_kernel<float2>, g, dim3(256), 0, st, (const float2*)in, pstride,
                       fstride, nx, rs, push_begin, f_lo, (int32_t)nf, probe0, n_slots, depth,
                       n_k, (float2*)ring);
  return hipGetLastError();
}

// Per-probe detector spectra from the cumulative (tile, detector) partials:
// Dp[d][probe0 + i][m] += sum over the slots s of detector d of
// (part[s][i][m] - part[s][i-1][m]). Block (m-range, d, g) sums a group of at
// most `per` slots, reads every partial once and adds its per-probe differences
// atomically (groups run in parallel).
__global__ void dpart_reduce_kernel(const double* part, DetSlots so, int32_t per,
                                    int32_t n_probes, int32_t n_om, int32_t probe0,
                                    int32_t n_probe_total, double* Dp) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  const int d = blockIdx.y;
  const int g = blockIdx.z;
  if (m >= n_om) return;
  const int s0 = so.off[d] + g * per, s1 = min(so.off[d + 1], s0 + per);
  if (s0 >= s1) return;
  const int64_t per_slot = (int64_t)n_probes * n_om;
  double prev = 0.0;
  for (int i = 0; i < n_probes; ++i) {
    const double* base = part + (int64_t)i * n_om + m;
    double cur = 0.0;
    for (int s = s0; s < s1; ++s) cur += base[s * per_slot];
    atomicAdd(&Dp[((int64_t)d * n_probe_total + probe0 + i) * n_om + m], cur - prev);
    prev = cur;
  }
}

hipError_t launch_dpart_reduce(const double* dpart, const DetSlots& so, int32_t n_probes,
                               int32_t n_det, int32_t n_om, int32_t probe0, int32_t n_probe_total,
                               double* Dp, hipStream_t st) {
  int most = 0;
  for (int d = 0; d < n_det; ++d) most = max(most, so.off[d + 1] - so.off[d]);
  if (most == 0) return hipSuccess;
  int per = 8;  // slots per block: enough blocks to fill the chip, few atomics per value
  if ((most + per - 1) / per > 1024) per = (most + 1023) / 1024;
  dim3 g((n_om + 127) / 128, n_det, (most + per - 1) / per);
  hipLaunchKernelGGL(dpart_reduce_kernel, g, dim3(128), 0, st, dpart, so, per, n_probes, n_om,
                     probe0, n_probe_total, Dp);
  return hipGetLastError();
}

// ---- exact elastic-mean correction -----------------------------------------
// For chunk spectra of the reference-subtracted series X'_s and the true
// mean-subtracted X_s = X'_s - delta W (delta = mu - c):
//   sum_s |X_s|^2 = sum_s |X'_s|^2 - 2 Re(conj(delta W) sum_s X'_s) + N_s |delta W|^2
__device__ __forceinline__ double corr_term(const CorrArgs& c, int p, int64_t k, int b) {
  if (c.pcorr) return c.pcorr[((int64_t)p * kMaxCorr + b) * c.n_k + k];
  const double2 cr = c.cref[(int64_t)p * c.n_k + k];
  double2 delta;
  if (c.mean_global) {
    const double2 ms = c.msum[(int64_t)p * c.n_k + k];
    delta = make_double2(ms.x * c.inv_nused, ms.y * c.inv_nused);
  } else {
    delta = make_double2(-cr.x, -cr.y);
  }
  const double2 w = c.wbin[b];
  const double2 dw = make_double2(delta.x * w.x - delta.y * w.y, delta.x * w.y + delta.y * w.x);
  const double2 xs = c.xs[((int64_t)p * kMaxCorr + b) * c.n_k + k];
  // Re(conj(dw) * xs) = dw.x xs.x + dw.y xs.y
  return -2.0 * (dw.x * xs.x + dw.y * xs.y) + c.n_seg * (dw.x * dw.x + dw.y * dw.y);
}

__global__ void correct_S_kernel(const CorrArgs c, double* S) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= c.n_k) return;
  for (int b = 0; b < c.n_corr; ++b) {
    double sum = 0.0;
    for (int p = 0; p < c.n_probe; ++p) sum += corr_term(c, p, k, b);
    S[(int64_t)c.rows[b] * c.n_k + k] += sum;
  }
}

hipError_t launch_correct_S(const CorrArgs& c, double* S, double* /*out*/, double /*kappa*/,
                            hipStream_t st) {
  hipLaunchKernelGGL(correct_S_kernel, dim3((c.n_k + 255) / 256), dim3(256), 0, st, c, S);
  return hipGetLastError();
}

// Dp[d][p][bin_b] += sum_k M_d(k) corr_p(b, k)
__global__ void correct_Dp_kernel(const CorrArgs c, const double* masks, int32_t n_det,
                                  double* Dp) {
  const int p = blockIdx.y;
  __shared__ double red[256];
  double accd[kMaxDet * kMaxCorr];
#pragma unroll
  for (int i = 0; i < kMaxDet * kMaxCorr; ++i) accd[i] = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < c.n_k;
       k += (int64_t)gridDim.x * blockDim.x) {
    double ct[kMaxCorr];
#pragma unroll
    for (int b = 0; b < kMaxCorr; ++b) ct[b] = (b < c.n_corr) ? corr_term(c, p, k, b) : 0.0;
#pragma unroll
    for (int d = 0; d < kMaxDet; ++d) {
      if (d < n_det) {
        const double m = masks[(int64_t)d * c.n_k + k];
#pragma unroll
        for (int b = 0; b < kMaxCorr; ++b) accd[d * kMaxCorr + b] += m * ct[b];
      }
    }
  }
  for (int d = 0; d < n_det; ++d) {
    for (int b = 0; b < c.n_corr; ++b) {
      red[threadIdx.x] = accd[d * kMaxCorr + b];
      __syncthreads();
      for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
      }
      if (threadIdx.x == 0)
        atomicAdd(&Dp[((int64_t)d * c.n_probe + p) * c.n_om + c.rows[b]], red[0]);
      __syncthreads();
    }
  }
}

hipError_t launch_correct_Dp(const CorrArgs& c, const double* masks, int32_t n_det, double* Dp,
                             hipStream_t st) {
  const int gx = (int)((c.n_k + 256 * 16 - 1) / (256 * 16));
  hipLaunchKernelGGL(correct_Dp_kernel, dim3(gx > 0 ? gx : 1, c.n_probe), dim3(256), 0, st, c,
                     masks, n_det, Dp);
  return hipGetLastError();
}

// ---- per-chunk mean --------------------------------------------------------
// With its own mean mu_s subtracted, chunk s has at a correction bin b
//   X_s(b) = A_s(b) - delta_s W(b),  A_s(b) = sum_t w(t) e^{-2 pi i b t / L} y'(s H + t),
// where y' = psi - c and delta_s = mu_s - c = (1/L) sum_t y'(s H + t). The chunk
// kernel leaves these bins out of S in this mode; this kernel adds the whole
// sum_s |X_s(b)|^2, formed in FP64 from exact FP64 sums.
// One thread per (probe, pixel) walks the push's frames in time order; the V
// chunks that can hold a frame live in V register slots (chunk s in slot s mod V),
// a chunk's sums are cleared at its first frame and turned into its correction
// at its last. Open sums persist in `open` between pushes.
#ifndef TACAW_PSEG_U
#define TACAW_PSEG_U 16
#endif
template <typename InT, int V, bool FAST>
__global__ void __launch_bounds__(256) pseg_kernel(const PsegArgs a) {
  // Slot state (four double2): the chunk sum of y'; A(0); (P, Q); (R, T) with
  // P = sum e_r y_r, Q = sum e_i y_i, R = sum e_r y_i, T = sum e_i y_r and
  // e = w(t) exp(-2 pi i t / L). The window is real, so bins 1 and L - 1 share
  // them: A(1) = (P - Q, R + T), A(L - 1) = conj(e) y summed = (P + Q, R - T).
  constexpr int Q = 4;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (k >= a.n_k || i >= a.n_probes) return;
  const int p = a.probe0 + i;
  const InT* src = (const InT*)a.in + (int64_t)i * a.pstride + pix_off(k, a.nx, a.rs);
  const double2 c = a.cref[(int64_t)p * a.n_k + k];
  double2* op = a.open + (int64_t)p * V * Q * a.n_k + k;
  double* cp = a.pcorr + (int64_t)p * kMaxCorr * a.n_k + k;
  double2 st[V][Q];
  double cor[kMaxCorr];
#pragma unroll
  for (int r = 0; r < V; ++r)
#pragma unroll
    for (int q = 0; q < Q; ++q) st[r][q] = op[(int64_t)(r * Q + q) * a.n_k];
#pragma unroll
  for (int b = 0; b < kMaxCorr; ++b) cor[b] = cp[(int64_t)b * a.n_k];
  const bool three = a.n_corr == 3;
  const double inv_l = 1.0 / (double)a.L;
  const double* w0 = (const double*)a.tw;  // w(t) = Re tw[0][t], stride 2
  const double2* e1 = a.tw + a.L;         // w(t) exp(-2 pi i t / L)
  constexpr int U = TACAW_PSEG_U;         // frames in flight per thread
  // add chunk s's correction from its finished sums and keep its mean
  auto close = [&](const double2 (&z)[Q], int s) {
    const double dx = z[0].x * inv_l, dy = z[0].y * inv_l;
    a.cmean[((int64_t)p * a.Ns + s) * a.n_k + k] = make_double2(c.x + dx, c.y + dy);
    double2 A[kMaxCorr];
    A[0] = z[1];
    A[1] = make_double2(z[2].x - z[2].y, z[3].x + z[3].y);
    A[2] = make_double2(z[2].x + z[2].y, z[3].x - z[3].y);
#pragma unroll
    for (int b = 0; b < kMaxCorr; ++b) {
      if (b == 0 || three) {
        const double2 wb = a.wbin[b];
        const double wx = dx * wb.x - dy * wb.y, wy = dx * wb.y + dy * wb.x;
        const double xr = A[b].x - wx, xi = A[b].y - wy;  // X_s(b) = A_s(b) - delta_s W(b)
        cor[b] += xr * xr + xi * xi;
      }
    }
  };
  if constexpr (FAST) {
    // H divides L (FAST is chosen when L = V H): frame n = j H + u lies in chunks
    // j - q, q = 0..V-1, at t = q H + u, so inside a hop block every frame updates
    // the same V sums with no bookkeeping; chunk j starts at u = 0 and chunk
    // j - V + 1 ends after u = H - 1. Register sq[q] holds chunk j - q (HBM slot
    // (j - q) mod V); sums of chunks that do not exist (j - q < 0, or past the
    // last chunk) are never closed.
    double2 sq[V][Q];
    const int jb = (int)(a.f_lo / a.H);
#pragma unroll
    for (int q = 0; q < V; ++q) {
      const int slot = ((jb - q) % V + V) % V;
#pragma unroll
      for (int z = 0; z < Q; ++z) sq[q][z] = st[0][z];
#pragma unroll
      for (int r = 1; r < V; ++r)
        if (slot == r)
#pragma unroll
          for (int z = 0; z < Q; ++z) sq[q][z] = st[r][z];
    }
    int64_t n = a.f_lo;
    while (n < a.f_hi) {
      const int j = (int)(n / a.H);
      const int u0 = (int)(n - (int64_t)j * a.H);
      const int u1 = (int)min<int64_t>(a.H, u0 + (a.f_hi - n));
      if (u0 == 0) {
#pragma unroll
        for (int z = 0; z < Q; ++z) sq[0][z] = make_double2(0.0, 0.0);
      }
      const InT* fp = src + (n - a.base) * a.fstride;
      for (int u = u0; u < u1; u += U) {
        InT v[U];
#pragma unroll
        for (int x = 0; x < U; ++x)
          if (u + x < u1) v[x] = fp[(int64_t)(u + x - u0) * a.fstride];
#pragma unroll
        for (int x = 0; x < U; ++x) {
          if (u + x >= u1) continue;
          const double yr = (double)v[x].x - c.x, yi = (double)v[x].y - c.y;
#pragma unroll
          for (int q = 0; q < V; ++q) {
            const int t = q * a.H + u + x;
            const double w = w0[2 * t];
            sq[q][0].x += yr;
            sq[q][0].y += yi;
            sq[q][1].x += w * yr;
            sq[q][1].y += w * yi;
            if (three) {
              const double2 e = e1[t];
              sq[q][2].x += e.x * yr;
              sq[q][2].y += e.y * yi;
              sq[q][3].x += e.x * yi;
              sq[q][3].y += e.y * yr;
            }
          }
        }
      }
      n += u1 - u0;
      if (u1 == a.H) {  // hop block j is complete
        const int s_end = j - (V - 1);
        if (s_end >= 0 && s_end < a.Ns) close(sq[V - 1], s_end);
#pragma unroll
        for (int q = V - 1; q > 0; --q)
#pragma unroll
          for (int z = 0; z < Q; ++z) sq[q][z] = sq[q - 1][z];
      }
    }
    // back to HBM slots: register q now holds chunk je - q
    const int je = (int)(a.f_hi / a.H);
#pragma unroll
    for (int q = 0; q < V; ++q) {
      const int slot = ((je - q) % V + V) % V;
#pragma unroll
      for (int z = 0; z < Q; ++z) op[(int64_t)(slot * Q + z) * a.n_k] = sq[q][z];
    }
#pragma unroll
    for (int b = 0; b < kMaxCorr; ++b) cp[(int64_t)b * a.n_k] = cor[b];
    return;
  } else {
  for (int64_t n0 = a.f_lo; n0 < a.f_hi; n0 += U) {
    InT v[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (n0 + u < a.f_hi) v[u] = src[(n0 + u - a.base) * a.fstride];
    // uniform bookkeeping: frame n = n0 + u lies after chunk start sl * H + rem
    int sl = (int)(n0 / a.H);
    int rem = (int)(n0 - (int64_t)sl * a.H);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (n0 + u >= a.f_hi) break;
      const int n = (int)(n0 + u);  // frames below 2^31 (checked by the plan)
      const double yr = (double)v[u].x - c.x, yi = (double)v[u].y - c.y;
      const int smax = min(a.Ns - 1, sl);  // the latest chunk that has started
#pragma unroll
      for (int r = 0; r < V; ++r) {
        const int s = smax - (((smax - r) % V) + V) % V;  // the chunk in slot r
        const int t = n - s * a.H;
        if (s < 0 || t >= a.L) continue;  // no chunk of slot r holds frame n
        if (t == 0) {
#pragma unroll
          for (int q = 0; q < Q; ++q) st[r][q] = make_double2(0.0, 0.0);
        }
        const double w = w0[2 * t];
        st[r][0].x += yr;
        st[r][0].y += yi;
        st[r][1].x += w * yr;
        st[r][1].y += w * yi;
        if (three) {
          const double2 e = e1[t];
          st[r][2].x += e.x * yr;
          st[r][2].y += e.y * yi;
          st[r][3].x += e.x * yi;
          st[r][3].y += e.y * yr;
        }
        if (t == a.L - 1) close(st[r], s);
      }
      if (++rem == a.H) {
        rem = 0;
        ++sl;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < V; ++r)
#pragma unroll
    for (int q = 0; q < Q; ++q) op[(int64_t)(r * Q + q) * a.n_k] = st[r][q];
#pragma unroll
  for (int b = 0; b < kMaxCorr; ++b) cp[(int64_t)b * a.n_k] = cor[b];
  }
}

hipError_t launch_pseg(const PsegArgs& a, int32_t in_dtype, hipStream_t st) {
  if (a.f_hi <= a.f_lo || a.n_probes < 1) return hipSuccess;
  if (a.V < 1 || a.V > kMaxPsegOpen) return hipErrorInvalidValue;
  dim3 g((a.n_k + 255) / 256, a.n_probes);
  const bool fast = a.L == a.V * a.H;
  auto go = [&](auto vt) {
    constexpr int V = decltype(vt)::value;
    if (in_dtype == 1) {
      if (fast)
        hipLaunchKernelGGL((pseg_kernel<double2, V, true>), g, dim3(256), 0, st, a);
      else
        hipLaunchKernelGGL((pseg_kernel<double2, V, false>), g, dim3(256), 0, st, a);
    } else {
      if (fast)
        hipLaunchKernelGGL((pseg_kernel<float2, V, true>), g, dim3(256), 0, st, a);
      else
        hipLaunchKernelGGL((pseg_kernel<float2, V, false>), g, dim3(256), 0, st, a);
    }
  };
  switch (a.V) {
    case 1: go(std::integral_constant<int, 1>{}); break;
    case 2: go(std::integral_constant<int, 2>{}); break;
    case 3: go(std::integral_constant<int, 3>{}); break;
    default: go(std::integral_constant<int, 4>{}); break;
  }
  return hipGetLastError();
}

// ---- HBM read ceiling ------------------------------------------------------
// Grid-stride read of 16-byte words, TACAW_READ_U independent loads per thread
// and trip, summed as 64-bit words (wrapping); one atomic per block.
#ifndef TACAW_READ_U
#define TACAW_READ_U 16
#endif
__global__ void __launch_bounds__(256) read_probe_kernel(const uint4* __restrict__ p, int64_t n16,
                                                         unsigned long long* sum) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long acc = 0;
  auto add = [&](const uint4 v) {
    acc += ((unsigned long long)v.y << 32 | v.x) + ((unsigned long long)v.w << 32 | v.z);
  };
  constexpr int U = TACAW_READ_U;
  for (; i + (U - 1) * stride < n16; i += U * stride) {
    uint4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = p[i + u * stride];
#pragma unroll
    for (int u = 0; u < U; ++u) add(v[u]);
  }
  for (; i < n16; i += stride) add(p[i]);
  __shared__ unsigned long long red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(sum, red[0]);
}

hipError_t launch_read_probe(const void* p, int64_t bytes, uint64_t* sum, hipStream_t st) {
  hipError_t e = launch_fill_zero(sum, 8, st);
  if (e != hipSuccess) return e;
  const int64_t n16 = bytes / 16;
  const int64_t want = (n16 + TACAW_READ_U * 256 - 1) / (TACAW_READ_U * 256);
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(want, 256 * 32));
  hipLaunchKernelGGL(read_probe_kernel, dim3(blocks), dim3(256), 0, st, (const uint4*)p, n16,
                     (unsigned long long*)sum);
  return hipGetLastError();
}

// Column pattern, the chunk transform's loads without its arithmetic: the rows
// (frames) of row_bytes are cut into columns seg_bytes wide (pixel tiles). One
// 512-thread workgroup per column walks all rows; a thread takes 8 bytes,
// seg_bytes / 8 lanes share a row, so a wave load spans 64 / (seg_bytes / 8) rows,
// and 8 row passes are in flight. The workgroup reserves most of the LDS so
// that, like the chunk transform, one runs per CU.
constexpr int kColThreads = 512;
constexpr int kColLds = 96 * 1024;
__global__ void __launch_bounds__(kColThreads) read_probe_columns_kernel(
    const char* __restrict__ p, int64_t n_rows, int64_t row_bytes, int32_t lanes,
    unsigned long long* sum) {
  constexpr int U = 8;
  __shared__ unsigned long long red[kColLds / 8];  // only the first kColThreads are used
  const int rows_per_pass = kColThreads / lanes;
  const int lane = threadIdx.x % lanes, r_off = threadIdx.x / lanes;
  const char* colp = p + (int64_t)blockIdx.x * lanes * 8 + lane * 8;
  unsigned long long acc = 0;
  for (int64_t r0 = r_off; r0 < n_rows; r0 += (int64_t)U * rows_per_pass) {
    unsigned long long v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t r = r0 + (int64_t)u * rows_per_pass;
      v[u] = r < n_rows ? *(const unsigned long long*)(colp + r * row_bytes) : 0ull;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc += v[u];
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kColThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(sum, red[0]);
}

hipError_t launch_read_probe_columns(const void* p, int64_t n_rows, int64_t row_bytes,
                                     int32_t seg_bytes, uint64_t* sum, hipStream_t st) {
  hipError_t e = launch_fill_zero(sum, 8, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(read_probe_columns_kernel, dim3((unsigned)(row_bytes / seg_bytes)),
                     dim3(kColThreads), 0, st, (const char*)p, n_rows, row_bytes,
                     seg_bytes / 8, (unsigned long long*)sum);
  return hipGetLastError();
}

// S[i] <- kappa q(r) S[i], row r = (i / inner) % n_om (q null: factor 1); copy to out if given
__global__ void scale_copy_kernel(double* S, double* out, int64_t n, double kappa, const double* q,
                                  int64_t inner, int32_t n_om) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double f = q ? kappa * q[(i / inner) % n_om] : kappa;
    const double v = S[i] * f;
    S[i] = v;
    if (out) out[i] = v;
  }
}

hipError_t launch_finalize_S(double* S, double* out, int64_t n_elem, double kappa, const double* q,
                             int64_t inner, int32_t n_om, hipStream_t st) {
  hipLaunchKernelGGL(scale_copy_kernel, dim3(blocks_for(n_elem, 256, 8192)), dim3(256), 0, st, S,
                     out, n_elem, kappa, q, inner, n_om);
  return hipGetLastError();
}

hipError_t launch_scale(double* p, int64_t n, double k, hipStream_t st) {
  return launch_finalize_S(p, nullptr, n, k, nullptr, 1, 1, st);
}

// D[d][m] += sum over a pixel chunk of M_d(k) S(m, k): each block takes kDetBins
// bins and a chunk of pixels (coalesced rows of S), reduces across each wave
// with lane shuffles and adds one value per (wave, bin, detector) atomically.
constexpr int kDetBins = 4;
template <int ND>
__global__ void detector_kernel(const double* S, const double* masks, int32_t L, int32_t n_k,
                                int32_t chunk, double* D) {
  const int m0 = blockIdx.y * kDetBins;
  const int64_t k0 = (int64_t)blockIdx.x * chunk;
  const int64_t k1 = (k0 + chunk < n_k) ? k0 + chunk : n_k;
  double acc[kDetBins][ND];
#pragma unroll
  for (int b = 0; b < kDetBins; ++b)
#pragma unroll
    for (int d = 0; d < ND; ++d) acc[b][d] = 0.0;
  for (int64_t k = k0 + threadIdx.x; k < k1; k += blockDim.x) {
    double mk[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) mk[d] = masks[(int64_t)d * n_k + k];
#pragma unroll
    for (int b = 0; b < kDetBins; ++b) {
      const double sv = (m0 + b < L) ? S[(int64_t)(m0 + b) * n_k + k] : 0.0;
#pragma unroll
      for (int d = 0; d < ND; ++d) acc[b][d] += mk[d] * sv;
    }
  }
#pragma unroll
  for (int b = 0; b < kDetBins; ++b) {
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      double v = acc[b][d];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      if ((threadIdx.x & 63) == 0 && m0 + b < L) atomicAdd(&D[(int64_t)d * L + m0 + b], v);
    }
  }
}

template <int ND>
static void launch_det_nd(const double* S, const double* masks, int32_t L, int32_t n_k,
                          double* D, hipStream_t st) {
  const int chunk = 16384;
  dim3 g((n_k + chunk - 1) / chunk, (L + kDetBins - 1) / kDetBins);
  hipLaunchKernelGGL((detector_kernel<ND>), g, dim3(256), 0, st, S, masks, L, n_k, chunk, D);
}

hipError_t launch_detector(const double* S, const double* masks, int32_t n_det, int32_t L,
                           int32_t n_k, double* D, hipStream_t st) {
  switch (n_det) {
    case 1: launch_det_nd<1>(S, masks, L, n_k, D, st); break;
    case 2: launch_det_nd<2>(S, masks, L, n_k, D, st); break;
    case 3: launch_det_nd<3>(S, masks, L, n_k, D, st); break;
    case 4: launch_det_nd<4>(S, masks, L, n_k, D, st); break;
    case 5: launch_det_nd<5>(S, masks, L, n_k, D, st); break;
    case 6: launch_det_nd<6>(S, masks, L, n_k, D, st); break;
    case 7: launch_det_nd<7>(S, masks, L, n_k, D, st); break;
    case 8: launch_det_nd<8>(S, masks, L, n_k, D, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// out[0] += sum_i a[i] * b[i]
__global__ void dot_kernel(const double* a, const double* b, int64_t n, double* out) {
  __shared__ double red[256];
  double s = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    s += a[i] * (b ? b[i] : 1.0);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(out, red[0]);
}

hipError_t launch_dot_gS(const double* S, const double* gS, int64_t n, double* out,
                         hipStream_t st) {
  hipLaunchKernelGGL(dot_kernel, dim3(blocks_for(n, 256, 1024)), dim3(256), 0, st, S, gS, n, out);
  return hipGetLastError();
}

hipError_t launch_sum(const double* p, int64_t n, double* out, hipStream_t st) {
  return launch_dot_gS(p, nullptr, n, out, st);
}

// *cnt += number of non-finite values (NaN or +-Inf) in x[0..n)
__global__ void count_nonfinite_kernel(const double* __restrict__ x, int64_t n,
                                       unsigned long long* cnt) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  unsigned long long c = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    c += isfinite(x[i]) ? 0ull : 1ull;
  if (c) atomicAdd(cnt, c);
}

hipError_t launch_count_nonfinite(const double* x, int64_t n, unsigned long long* cnt,
                                  hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(count_nonfinite_kernel, dim3(blocks_for(n, 256, 4096)), dim3(256), 0, st, x,
                     n, cnt);
  return hipGetLastError();
}

}  // namespace tacaw
