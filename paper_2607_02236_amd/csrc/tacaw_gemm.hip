// Chunk transform as a dense GEMM on MFMA with split-precision operands.
//
// X(m, k) = sum_t F(m, t) y(t, k),  F(m, t) = w(t) exp(-2 pi i m t / L), written as a
// real GEMM with M = 2 n_om rows (re/im of each output bin interleaved; n_om = L,
// or the 2M + 1 bins of an energy window, whose other rows are never computed),
// K = 2L (re/im of each frame interleaved) and N = pixels:
//   [Xr]   [ Fr  -Fi ] [yr]
//   [Xi] = [ Fi   Fr ] [yi]
// Both operands are split into a high and a low half-precision part
// (bf16 or fp16), and X ~= A_hi B_hi + A_hi B_lo + A_lo B_hi is accumulated in
// FP32 by v_mfma_f32_32x32x16_{bf16,f16}; |X|^2 is accumulated in FP64.
// y = s (psi - mu) with the exact FP64 mean mu (a pre-pass) and a power-of-two
// scale s per (probe, pixel) that keeps the fp16 low parts in the normal range
// (s = 1 for bf16). The power is divided by s^2 before accumulation.
//
// Workgroup: 8 waves, a tile of 32 pixels (the MFMA N dimension) and all
// rows; wave w owns row blocks {w, w + 8, ...} of 32 rows. Frames are staged
// through LDS in chunks of KC frames, already converted to the operand order.
#include "tacaw_internal.h"

namespace tacaw {

typedef __attribute__((__vector_size__(8 * sizeof(short)))) short h8;  // 8 x 16-bit
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int kGemmPx = 32;      // pixels per workgroup (MFMA N)
constexpr int kGemmWaves = 8;
constexpr int kGemmKC = 256;     // frames per LDS chunk

__device__ __forceinline__ unsigned short bf16_rne(float x) {
  unsigned u = __builtin_bit_cast(unsigned, x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(unsigned short h) {
  return __builtin_bit_cast(float, ((unsigned)h) << 16);
}

// split x into hi + lo of the chosen half type (bit patterns)
template <int PREC>
__device__ __forceinline__ void split2(float x, unsigned short& hi, unsigned short& lo) {
  if constexpr (PREC == 0) {  // bf16
    hi = bf16_rne(x);
    lo = bf16_rne(x - bf16_to_f(hi));
  } else {  // fp16
    const _Float16 h = (_Float16)x;
    const _Float16 l = (_Float16)(x - (float)h);
    hi = __builtin_bit_cast(unsigned short, h);
    lo = __builtin_bit_cast(unsigned short, l);
  }
}

template <int PREC>
__device__ __forceinline__ f32x16 mfma(h8 a, h8 b, f32x16 c) {
  if constexpr (PREC == 0) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  } else {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a),
                                                  __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
  }
}

// fmat layout: [2][m_rows][2L] 16-bit (hi then lo), row 2r + c (c = 0 real, 1 imag) of
// output row r (bin (r - roi_half) mod L), zero rows up to m_rows (a multiple of 32);
// column 2t + c' (c' = 0 multiplies Re y, 1 multiplies Im y).
// gscale: [n_probe][n_k] float, the power-of-two scale s of y.
// MBW: row blocks per wave (at most); NB: 32-pixel column blocks per workgroup. Fewer
// rows (an energy window) leave room for more columns, so each DFT-matrix fragment
// read from L2 feeds NB products.
template <int L, typename InT, int PREC, bool DP, int MBW, int NB>
__global__ void __launch_bounds__(64 * kGemmWaves)
    seg_gemm_kernel(const SegArgs a, const unsigned short* __restrict__ fmat, int m_rows,
                    const float* __restrict__ gscale) {
  constexpr int NT = 64 * kGemmWaves;
  constexpr int PX = kGemmPx * NB;              // pixels per workgroup
  constexpr int KC = L < kGemmKC / NB ? L : kGemmKC / NB;  // frames per LDS stage
  constexpr int KSTEPS = KC / 8;                // 16 real K (8 frames) per MFMA
  constexpr int K2 = 2 * L;
  constexpr int SG = NT / PX;                   // staging groups of 4 frames
  static_assert(MBW >= 1 && MBW * kGemmWaves * 32 <= 2 * L, "row blocks per wave");
  static_assert(L % KC == 0 && SG >= 1, "staging");

  // B operand staging: [nb][hi, lo][kstep][lane][8], 16-bit
  __shared__ __attribute__((aligned(16))) unsigned short bst[NB * 2 * KSTEPS * 64 * 8];
  __shared__ double s_mask[DP ? kMaxDet * PX : 1];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int tile = blockIdx.x;
  const int n_k = a.n_k;
  const int col = lane & 31;      // pixel of this lane in MFMA operands and results
  const int half = lane >> 5;
  const int n_blocks = m_rows / 32;  // row blocks of this plan (energy window)
  const int n_om = a.n_om;
  int64_t kcol[NB];
  bool cvalid[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    kcol[nb] = (int64_t)tile * PX + kGemmPx * nb + col;
    cvalid[nb] = kcol[nb] < n_k;
  }

  if constexpr (DP) {
    for (int i = tid; i < kMaxDet * PX; i += NT) {
      const int d = i / PX, x = i % PX;
      const int64_t kk = (int64_t)tile * PX + x;
      s_mask[i] = (d < a.n_det && kk < n_k) ? a.masks[(int64_t)d * n_k + kk] : 0.0;
    }
  }

  // staging role: thread handles pixel sp of the tile and frame groups of 4
  const int sp = tid % PX;
  const int sgrp = tid / PX;
  const int snb = sp / kGemmPx, s32 = sp % kGemmPx;
  const int64_t ks = (int64_t)tile * PX + sp;
  const int64_t ksc = ks < n_k ? ks : (int64_t)n_k - 1;

  double acc64[MBW][NB][8];
#pragma unroll
  for (int b = 0; b < MBW; ++b)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int q = 0; q < 8; ++q) acc64[b][nb][q] = 0.0;

  for (int i = 0; i < a.n_probes; ++i) {
    const int p = a.probe0 + i;
    const double2 mu = a.cref[(int64_t)p * n_k + ksc];
    const float sc = gscale[(int64_t)p * n_k + ksc];
    float inv2[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const float sc_col = gscale[(int64_t)p * n_k + (cvalid[nb] ? kcol[nb] : (int64_t)n_k - 1)];
      inv2[nb] = 1.0f / (sc_col * sc_col);
    }
    const InT* inb = (const InT*)a.in + (int64_t)i * a.pstride + pix_off(ksc, a.nx, a.row_stride);

    for (int s = a.s_lo; s < a.s_hi; ++s) {
      const int64_t seg0 = (int64_t)s * a.hop - a.push_begin;
      f32x16 acc[MBW][NB];
#pragma unroll
      for (int b = 0; b < MBW; ++b)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
          for (int v = 0; v < 16; ++v) acc[b][nb][v] = 0.0f;

      for (int c0 = 0; c0 < L; c0 += KC) {
        __syncthreads();  // previous stage's operand reads are complete
        // stage frames [c0, c0 + KC) of this chunk: groups of 4 frames per lane slot
        for (int g4 = sgrp; g4 < KC / 4; g4 += SG) {
          const int t0 = c0 + 4 * g4;
          unsigned short hv[8], lv[8];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const InT x = inb[(seg0 + t0 + u) * a.fstride];
            const float yr = (float)(((double)x.x - mu.x) * (double)sc);
            const float yi = (float)(((double)x.y - mu.y) * (double)sc);
            split2<PREC>(yr, hv[2 * u], lv[2 * u]);
            split2<PREC>(yi, hv[2 * u + 1], lv[2 * u + 1]);
          }
          const int tl = 4 * g4;                    // frame within the stage
          const int kst = tl / 8, hh = (tl % 8) / 4;
          const int lanep = s32 + 32 * hh;          // operand lane holding these 8 K values
          const int hslot = (((snb * 2 + 0) * KSTEPS + kst) * 64 + lanep) * 8;
          const int lslot = (((snb * 2 + 1) * KSTEPS + kst) * 64 + lanep) * 8;
          uint4 H, Lw;
          H.x = hv[0] | ((unsigned)hv[1] << 16);
          H.y = hv[2] | ((unsigned)hv[3] << 16);
          H.z = hv[4] | ((unsigned)hv[5] << 16);
          H.w = hv[6] | ((unsigned)hv[7] << 16);
          Lw.x = lv[0] | ((unsigned)lv[1] << 16);
          Lw.y = lv[2] | ((unsigned)lv[3] << 16);
          Lw.z = lv[4] | ((unsigned)lv[5] << 16);
          Lw.w = lv[6] | ((unsigned)lv[7] << 16);
          *reinterpret_cast<uint4*>(&bst[hslot]) = H;
          *reinterpret_cast<uint4*>(&bst[lslot]) = Lw;
        }
        __syncthreads();
        for (int kst = 0; kst < KSTEPS; ++kst) {
          h8 bh[NB], bl[NB];
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) {
            bh[nb] = *reinterpret_cast<const h8*>(&bst[(((nb * 2 + 0) * KSTEPS + kst) * 64 + lane) * 8]);
            bl[nb] = *reinterpret_cast<const h8*>(&bst[(((nb * 2 + 1) * KSTEPS + kst) * 64 + lane) * 8]);
          }
          const int kcol2 = 2 * c0 + 16 * kst + 8 * half;  // first of the lane's 8 K columns
#pragma unroll
          for (int b = 0; b < MBW; ++b) {
            if (wave + kGemmWaves * b < n_blocks) {  // uniform per wave
              const int row = 32 * (wave + kGemmWaves * b) + col;
              const h8 ah = *reinterpret_cast<const h8*>(fmat + (int64_t)row * K2 + kcol2);
              const h8 al =
                  *reinterpret_cast<const h8*>(fmat + (int64_t)(m_rows + row) * K2 + kcol2);
#pragma unroll
              for (int nb = 0; nb < NB; ++nb) {
                acc[b][nb] = mfma<PREC>(ah, bh[nb], acc[b][nb]);
                acc[b][nb] = mfma<PREC>(ah, bl[nb], acc[b][nb]);
                acc[b][nb] = mfma<PREC>(al, bh[nb], acc[b][nb]);
              }
            }
          }
        }
      }
      // |X|^2: accumulator v of a lane holds row 8 (v / 4) + 4 half + (v % 4) of
      // its 32-row block, column col; rows (2m', 2m'+1) are (Re, Im) of one bin
#pragma unroll
      for (int b = 0; b < MBW; ++b) {
        if (wave + kGemmWaves * b < n_blocks) {
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) {
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              const int v = 4 * (q / 2) + 2 * (q % 2);
              const float pw = acc[b][nb][v] * acc[b][nb][v] + acc[b][nb][v + 1] * acc[b][nb][v + 1];
              acc64[b][nb][q] += (double)(pw * inv2[nb]);
            }
          }
        }
      }
    }

    if constexpr (DP) {
      // cumulative detector partials through LDS, two halves of the rows
      double* sd = reinterpret_cast<double*>(bst);
      // n_om <= 128 MBW rows, so a half holds at most 64 MBW rows of PX pixels
      static_assert(sizeof(bst) >= (size_t)64 * MBW * PX * 8, "LDS for partials");
      const int32_t* slots = a.pair_slot + (int64_t)tile * a.n_det;
      const int hrows = (n_om + 1) / 2;
      for (int hb = 0; hb < 2; ++hb) {
        __syncthreads();
#pragma unroll
        for (int b = 0; b < MBW; ++b) {
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const int rblk = wave + kGemmWaves * b;
            const int r = 16 * rblk + 4 * (q / 2) + 2 * half + (q % 2);
            if (r < n_om && (r >= hrows) == (hb == 1)) {
#pragma unroll
              for (int nb = 0; nb < NB; ++nb)
                sd[(r - hb * hrows) * PX + kGemmPx * nb + col] = acc64[b][nb][q];
            }
          }
        }
        __syncthreads();
        const int r0 = hb * hrows, nr = hb ? n_om - hrows : hrows;
        for (int rr = tid; rr < nr; rr += NT) {
          for (int d = 0; d < a.n_det; ++d) {
            const int slot = slots[d];  // -1: this detector's mask is zero on the tile
            if (slot < 0) continue;
            double dsum = 0.0;
#pragma unroll
            for (int x = 0; x < PX; ++x) dsum += s_mask[d * PX + x] * sd[rr * PX + x];
            // cumulative over probes 0..i
            a.dpart[((int64_t)slot * a.n_probes + i) * n_om + r0 + rr] = dsum;
          }
        }
      }
    }
  }

#pragma unroll
  for (int b = 0; b < MBW; ++b) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int rblk = wave + kGemmWaves * b;
      const int r = 16 * rblk + 4 * (q / 2) + 2 * half + (q % 2);
      if (r < n_om) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          if (cvalid[nb]) {
            double* sp = a.S + (int64_t)r * n_k + kcol[nb];
            *sp = a.s_store ? acc64[b][nb][q] : *sp + acc64[b][nb][q];
          }
        }
      }
    }
  }
}

// column blocks for a plan: the fewer 32-row blocks per wave, the more columns
static int gemm_nb(int L, int n_om) {
  const int mbw = (((2 * n_om + 31) / 32) + kGemmWaves - 1) / kGemmWaves;  // row blocks per wave
  (void)L;
  return mbw <= 1 ? 4 : (mbw == 2 ? 2 : 1);
}

template <int L, typename InT, int PREC, int MBW, int NB>
static hipError_t launch_g4(const SegArgs& a, const void* fmat, int m_rows, const float* gscale,
                            int n_tiles, hipStream_t st) {
  if (a.n_det > 0)
    hipLaunchKernelGGL((seg_gemm_kernel<L, InT, PREC, true, MBW, NB>), dim3(n_tiles),
                       dim3(64 * kGemmWaves), 0, st, a, (const unsigned short*)fmat, m_rows, gscale);
  else
    hipLaunchKernelGGL((seg_gemm_kernel<L, InT, PREC, false, MBW, NB>), dim3(n_tiles),
                       dim3(64 * kGemmWaves), 0, st, a, (const unsigned short*)fmat, m_rows, gscale);
  return hipGetLastError();
}

template <int L, typename InT, int PREC>
static hipError_t launch_g3(const SegArgs& a, const void* fmat, int m_rows, const float* gscale,
                            int n_tiles, hipStream_t st) {
  const int nb = gemm_nb(L, a.n_om);
  if (nb == 4) return launch_g4<L, InT, PREC, 1, 4>(a, fmat, m_rows, gscale, n_tiles, st);
  if constexpr (L >= 256) {
    if (nb == 2) return launch_g4<L, InT, PREC, 2, 2>(a, fmat, m_rows, gscale, n_tiles, st);
  }
  if constexpr (L >= 512) {
    return launch_g4<L, InT, PREC, L / 128, 1>(a, fmat, m_rows, gscale, n_tiles, st);
  }
  return hipErrorInvalidValue;
}

template <int L>
static hipError_t launch_g2(int in_dtype, int prec, const SegArgs& a, const void* fmat,
                            int m_rows, const float* gscale, int n_tiles, hipStream_t st) {
  if (m_rows < 32 || m_rows % 32 != 0 || m_rows > 2 * L || m_rows < 2 * a.n_om)
    return hipErrorInvalidValue;
  if (in_dtype == 1)
    return prec ? launch_g3<L, double2, 1>(a, fmat, m_rows, gscale, n_tiles, st)
                : launch_g3<L, double2, 0>(a, fmat, m_rows, gscale, n_tiles, st);
  return prec ? launch_g3<L, float2, 1>(a, fmat, m_rows, gscale, n_tiles, st)
              : launch_g3<L, float2, 0>(a, fmat, m_rows, gscale, n_tiles, st);
}

bool seg_gemm_supported(int L) { return L == 128 || L == 256 || L == 512; }
int seg_gemm_tile_pixels(int L, int n_om) { return kGemmPx * gemm_nb(L, n_om); }

hipError_t launch_seg_gemm(int L, int in_dtype, bool /*sub64*/, int prec, const SegArgs& a,
                           const void* fmat, int m_rows, int n_tiles, hipStream_t st) {
  const float* gscale = a.gscale;
  switch (L) {
    case 128: return launch_g2<128>(in_dtype, prec, a, fmat, m_rows, gscale, n_tiles, st);
    case 256: return launch_g2<256>(in_dtype, prec, a, fmat, m_rows, gscale, n_tiles, st);
    case 512: return launch_g2<512>(in_dtype, prec, a, fmat, m_rows, gscale, n_tiles, st);
  }
  return hipErrorInvalidValue;
}

// Per (probe, pixel) power-of-two scale s = 2^-e with 2^e > 2 max_n |psi_n - c|
// over frames [0, n_used) (c = the subtracted reference), so |s (psi - c)| < 1/2
// and fp16 low parts stay normal; s = 1 for bf16.
template <typename InT>
__global__ void gemm_scale_kernel(const InT* in, int64_t pstride, int64_t fstride, int32_t nx,
                                  int64_t rs, int64_t n_used, int32_t probe0, int32_t n_probes,
                                  int32_t n_k, int32_t prec, const double2* cref, float* scale) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (k >= n_k || i >= n_probes) return;
  const InT* p = in + (int64_t)i * pstride + pix_off(k, nx, rs);
  const double2 c = cref[(int64_t)(probe0 + i) * n_k + k];
  double mx = 0.0;
  for (int64_t n = 0; n < n_used; ++n) {
    const InT v = p[n * fstride];
    mx = fmax(mx, fmax(fabs((double)v.x - c.x), fabs((double)v.y - c.y)));
  }
  float s = 1.0f;
  if (prec == 1 && mx > 0.0) {
    int e = 0;
    frexp(2.0 * mx, &e);  // 2 mx < 2^e
    e = e < -100 ? -100 : (e > 100 ? 100 : e);
    s = ldexpf(1.0f, -e);
  }
  scale[(int64_t)(probe0 + i) * n_k + k] = s;
}

hipError_t launch_gemm_scale(const void* in, int in_dtype, int64_t pstride, int64_t fstride,
                             int32_t nx, int64_t rs, int64_t n_used, int32_t probe0,
                             int32_t n_probes, int32_t n_k, int prec, const double2* cref,
                             float* scale, hipStream_t st) {
  dim3 g((n_k + 255) / 256, n_probes);
  if (in_dtype == 1)
    hipLaunchKernelGGL(gemm_scale_kernel<double2>, g, dim3(256), 0, st, (const double2*)in, pstride,
                       fstride, nx, rs, n_used, probe0, n_probes, n_k, prec, cref, scale);
  else
    hipLaunchKernelGGL(gemm_scale_kernel<float2>, g, dim3(256), 0, st, (const float2*)in, pstride,
                       fstride, nx, rs, n_used, probe0, n_probes, n_k, prec, cref, scale);
  return hipGetLastError();
}

}  // namespace tacaw
