// Fused producer: synthetic exit waves written straight into a destination with
// the layout of a plan's ring (or any strided buffer), so that streamed frames
// exist once in HBM. It stands in for the multislice producer of the paper's
// pipeline (Sec. II.B: exit waves are reduced as they are produced).
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC 2011), a
// counter-based generator: ten rounds, each two 32 x 32 -> 64-bit products of
// counter words with fixed multipliers and xors with the key, the key advanced
// by two Weyl constants between rounds. Signal model (complex64, per probe p,
// frame n, pixel k):
//   psi = e0 + sum_j a (x_j(n) + i y_j(n)) + sigma (g_r + i g_i),
// term j rotating by its quantised frequency f_j (Q = 2^20 steps per cycle):
// (x, y) <- (x c - y s, x s + y c), (c, s) = (cos, sin)(2 pi f_j / Q) from a
// table, restarted every kBlock frames from the tabulated phase f_j n + phi_j,
// so a frame's value depends only on its kBlock-frame block and not on how the
// frames are split into calls. Every product and sum is one IEEE float32
// operation in a fixed order (no contraction), so the CPU twin computes the
// same bits (this file is compiled with -ffp-contract=off, and the kernels
// say so too). f_j, phi_j: Philox((p, k, j, 0), (seed, 0x21)); line centres and
// half widths: Philox((p, l, 0, 0), (seed, 0x11)); noise: word n mod 4 of
// Philox((p, n / 4, k, 0), (seed, 0x41)), the low 12 bits of its two 16-bit
// halves indexing a table of 2^12 standard normals.
#include <stdint.h>

#include "../../include/tacaw.h"
#include "tacaw_internal.h"

namespace tacaw {

constexpr int kQ = 1 << 20;
constexpr int kBlock = 64;
constexpr int kMaxTerms = 16;
constexpr int kNormals = 1 << 12;  // standard normals in the noise table
constexpr int kMaxLines = 1 << 20;

struct Philox4 {
  uint32_t x[4];
};

__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                 uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n1 = (uint32_t)p1;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    const uint32_t n3 = (uint32_t)p0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
  }
  return Philox4{{c0, c1, c2, c3}};
}

__device__ __forceinline__ double unit32(uint32_t r) { return (double)r * (1.0 / 4294967296.0); }

struct SynthArgs {
  tacaw_synth_desc d;
  double cyc_per_mev;
  void* dst;
  int32_t probe0, n_probes;
  int64_t frame0, n_frames;
  int64_t pstride, fstride, tstride;
  int32_t tile_px;
  int32_t n_k;
};

// line l of probe p: centre and half width in meV
__device__ __forceinline__ void probe_line(const tacaw_synth_desc& d, uint32_t p, uint32_t l,
                                           double& centre, double& hwhm) {
#pragma clang fp contract(off)
  const Philox4 r = philox4x32_10(p, l, 0u, 0u, d.seed, 0x11u);
  centre = d.line_lo_mev + (d.line_hi_mev - d.line_lo_mev) * unit32(r.x[0]);
  hwhm = d.hwhm_lo_mev + (d.hwhm_hi_mev - d.hwhm_lo_mev) * unit32(r.x[1]);
}

// one thread per (pixel, probe); frames [frame0, frame0 + n_frames) in order;
// T terms (compile-time, so the term state stays in registers)
template <int T>
__global__ void __launch_bounds__(256) synth_frames_kernel(const SynthArgs a) {
#pragma clang fp contract(off)
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  const tacaw_synth_desc& d = a.d;
  // the normal table in LDS (two random reads per value would otherwise go to L2)
  __shared__ float s_normal[kNormals];
  if (d.noise_sigma != 0.0) {
    for (int e = threadIdx.x; e < kNormals; e += blockDim.x) s_normal[e] = d.d_normal[e];
    __syncthreads();
  }
  if (k >= a.n_k) return;
  const uint32_t p = (uint32_t)(a.probe0 + i);
  // the pixel's terms: rotation per frame and phase step
  float rc[T > 0 ? T : 1], rs[T > 0 ? T : 1];
  uint32_t fq[T > 0 ? T : 1], phq[T > 0 ? T : 1];
#pragma unroll
  for (int j = 0; j < T; ++j) {
    const Philox4 r = philox4x32_10(p, (uint32_t)k, (uint32_t)j, 0u, d.seed, 0x21u);
    double e;
    if (d.n_lines > 0) {
      double centre, hwhm;
      probe_line(d, p, r.x[0] % (uint32_t)d.n_lines, centre, hwhm);
      e = centre + hwhm * d.d_tan[r.x[1] >> 16];
      e = fmin(fmax(e, -400.0), 400.0);
    } else {
      e = d.e_lo_mev + (d.e_hi_mev - d.e_lo_mev) * unit32(r.x[0]);
    }
    const int64_t f = (int64_t)floor(e * a.cyc_per_mev + 0.5);
    fq[j] = (uint32_t)(f & (kQ - 1));
    phq[j] = r.x[2] & (uint32_t)(kQ - 1);
    rc[j] = d.d_cos[fq[j]];
    rs[j] = d.d_sin[fq[j]];
  }
  const float amp = (float)d.amplitude, sig = (float)d.noise_sigma;
  const float e_re = (float)d.elastic_re, e_im = (float)d.elastic_im;
  const bool noisy = d.noise_sigma != 0.0;
  float2* out = (float2*)a.dst + (int64_t)i * a.pstride + (k / a.tile_px) * a.tstride + k % a.tile_px;
  const int64_t n_end = a.frame0 + a.n_frames;
  float x[T > 0 ? T : 1], y[T > 0 ? T : 1];
  Philox4 nz{};
  for (int64_t n = (a.frame0 / kBlock) * kBlock; n < n_end; ++n) {
    if (n % kBlock == 0) {  // restart the rotations from the table
#pragma unroll
      for (int j = 0; j < T; ++j) {
        const uint32_t idx = (uint32_t)(((uint64_t)fq[j] * (uint64_t)n + phq[j]) & (kQ - 1));
        x[j] = d.d_cos[idx];
        y[j] = d.d_sin[idx];
      }
    }
    if (n >= a.frame0) {
      float re = e_re, im = e_im;
#pragma unroll
      for (int j = 0; j < T; ++j) {
        re = re + x[j] * amp;
        im = im + y[j] * amp;
      }
      if (noisy) {
        if ((n & 3) == 0 || n == a.frame0)
          nz = philox4x32_10(p, (uint32_t)(n >> 2), (uint32_t)k, 0u, d.seed, 0x41u);
        const int q = (int)(n & 3);
        const uint32_t w = q == 0 ? nz.x[0] : q == 1 ? nz.x[1] : q == 2 ? nz.x[2] : nz.x[3];
        re = re + s_normal[w & (kNormals - 1)] * sig;
        im = im + s_normal[(w >> 16) & (kNormals - 1)] * sig;
      }
      out[(n - a.frame0) * a.fstride] = make_float2(re, im);
    }
#pragma unroll
    for (int j = 0; j < T; ++j) {
      const float xn = x[j] * rc[j] - y[j] * rs[j];
      const float yn = x[j] * rs[j] + y[j] * rc[j];
      x[j] = xn;
      y[j] = yn;
    }
  }
}

template <int T>
static void launch_synth(const SynthArgs& a, dim3 g, hipStream_t st) {
  if constexpr (T > 0) {
    if (a.d.n_terms < T) return launch_synth<T - 1>(a, g, st);
  }
  hipLaunchKernelGGL(synth_frames_kernel<T>, g, dim3(256), 0, st, a);
}

}  // namespace tacaw

extern "C" int tacaw_synth_frames(const tacaw_synth_desc* d, void* d_dst, int32_t probe0,
                                  int32_t n_probes, int64_t frame0, int64_t n_frames,
                                  int64_t probe_stride, int64_t frame_stride, int64_t tile_stride,
                                  int32_t tile_pixels, void* hip_stream) {
  using namespace tacaw;
  clear_error();
  if (!d || !d_dst) return set_error(TACAW_ERR_INVALID_ARG, "desc and destination must be given");
  if (d->ny < 1 || d->nx < 1 || (int64_t)d->ny * d->nx > 0x7FFFFFFF)
    return set_error(TACAW_ERR_SHAPE, "grid must be 1 .. 2^31 - 1 pixels");
  if (d->n_terms < 0 || d->n_terms > kMaxTerms || d->n_lines < 0 || d->n_lines > kMaxLines)
    return set_error(TACAW_ERR_INVALID_ARG, "n_terms must be 0 .. 16 and n_lines >= 0");
  if (!d->d_cos || !d->d_sin || (d->noise_sigma != 0.0 && !d->d_normal) ||
      (d->n_lines > 0 && !d->d_tan))
    return set_error(TACAW_ERR_INVALID_ARG, "tables must be given");
  if (n_probes < 1 || probe0 < 0 || frame0 < 0 || n_frames < 0 || frame0 + n_frames > 0xFFFFFFFFLL ||
      (int64_t)probe0 + n_probes > 0x7FFFFFFFLL)
    return set_error(TACAW_ERR_SHAPE, "probe or frame range out of bounds");
  const int64_t n_k = (int64_t)d->ny * d->nx;
  if (tile_pixels < 1 || (tile_pixels < n_k && tile_stride < 1) || frame_stride < 1 ||
      (n_probes > 1 && probe_stride < 1))
    return set_error(TACAW_ERR_INVALID_ARG, "bad destination strides");
  if ((uintptr_t)d_dst % 8 != 0) return set_error(TACAW_ERR_INVALID_ARG, "destination not 8-byte aligned");
  if (n_frames == 0) return TACAW_OK;
  SynthArgs a{};
  a.d = *d;
  a.cyc_per_mev = 1e-3 / (6.62607015e-34 / 1.602176634e-19) * d->dt_fs * 1e-15 * kQ;
  a.dst = d_dst;
  a.probe0 = probe0;
  a.n_probes = n_probes;
  a.frame0 = frame0;
  a.n_frames = n_frames;
  a.pstride = probe_stride;
  a.fstride = frame_stride;
  a.tstride = tile_pixels < n_k ? tile_stride : 0;
  a.tile_px = tile_pixels < n_k ? tile_pixels : (int32_t)n_k;
  a.n_k = (int32_t)n_k;
  dim3 g((unsigned)((n_k + 255) / 256), (unsigned)n_probes);
  launch_synth<kMaxTerms>(a, g, (hipStream_t)hip_stream);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(TACAW_ERR_HIP, hipGetErrorString(e));
  return TACAW_OK;
}
