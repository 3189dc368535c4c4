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
// y = s (psi - mu), mu the exact FP64 mean (a pre-pass) or, in the streaming form,
// a reference c with the exact mean correction at finalize; s is a power-of-two
// scale per (probe, pixel) that keeps the fp16 low parts in the normal range
// (s = 1 for bf16). The power is divided by s^2 before accumulation.
#include "tacaw_internal.h"

namespace tacaw {

typedef __attribute__((__vector_size__(8 * sizeof(short)))) short h8;  // 8 x 16-bit
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int kGemmPx = 32;      // pixels per MFMA column block (MFMA N)
constexpr int kGemmWaves = 4;    // one wave per SIMD
constexpr int kGemmKC = 256;     // frames per LDS stage (divided by the column blocks)

typedef __attribute__((__vector_size__(2 * sizeof(float)))) float f32x2;
typedef __attribute__((__vector_size__(2 * sizeof(__bf16)))) __bf16 bf16x2;
typedef __attribute__((__vector_size__(2 * sizeof(_Float16)))) _Float16 f16x2;

// split the pair (a, b) into hi + lo of the chosen half type, each a packed pair
// (a in the low 16 bits): hi = RNE(x), lo = RNE(x - hi), where x - hi is exact in
// FP32. One packed conversion per part (v_cvt_pk_{bf16,f16}_f32).
template <int PREC>
__device__ __forceinline__ void split_pair(float a, float b, unsigned& hi, unsigned& lo) {
  const f32x2 x = {a, b};
  if constexpr (PREC == 0) {  // bf16
    const unsigned h = __builtin_bit_cast(unsigned, __builtin_convertvector(x, bf16x2));
    const f32x2 r = {a - __builtin_bit_cast(float, h << 16),
                     b - __builtin_bit_cast(float, h & 0xFFFF0000u)};
    hi = h;
    lo = __builtin_bit_cast(unsigned, __builtin_convertvector(r, bf16x2));
  } else {  // fp16
    const f16x2 h = __builtin_convertvector(x, f16x2);
    const f32x2 r = {a - (float)h[0], b - (float)h[1]};
    hi = __builtin_bit_cast(unsigned, h);
    lo = __builtin_bit_cast(unsigned, __builtin_convertvector(r, f16x2));
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
// gscale: [n_probe][n_k] float, the power-of-two scale s of y (fp16; 1 for bf16).
//
// Workgroup: 4 waves (one per SIMD), a tile of PX = 32 NB pixels and one row group
// of the GEMM: wave w owns row block blk_lo + w (32 rows) of its group and holds
// NB accumulator tiles of 32 x 32; as many groups as the rows need at 4 blocks
// each. Frames are staged through LDS in stages of KC frames, converted to operand
// order, in two alternating buffers (one barrier per stage).
// Every load runs a whole stage ahead of its use, so that no wait on a load
// (vector loads complete in issue order) stalls the MFMAs: during stage st, group u
// of stage st + 1 is converted into the other buffer at k-step u KSTEPS / G4N and
// its registers refilled with group u of stage st + 2, and the wave's DFT-matrix
// fragment of k-step k is refilled with stage st + 1 right after k-step k's MFMAs.
// SRC: 0 every frame from the push buffer; 1 frames before push_begin from the
// per-frame ring (immediate and deferred streaming); 2 every frame from the ring
// stored per tile of PX pixels ([slot][tile][row][PX]).
// TRACK: the reference c is subtracted instead of the exact mean (streaming form):
// the launch holding a probe's first chunk fixes c (the window-weighted mean of 16
// frames spread over that chunk), and the FP64 sums of psi - c (each frame once) and
// of X' at the correction bins feed the exact correction at finalize, as in the
// FFT form; the correction bins are squared in FP64. bf16 only (fp16 needs the
// whole-series scale pre-pass).
template <int L, typename InT, int PREC, bool DP, int NB, bool TRACK, int SRC>
__global__ void __launch_bounds__(64 * kGemmWaves)
    seg_gemm_kernel(const SegArgs a, const unsigned short* __restrict__ fmat, int m_rows,
                    const float* __restrict__ gscale, int n_groups) {
  static_assert(!TRACK || PREC == 0, "the streaming form is bf16");
  constexpr int NT = 64 * kGemmWaves;
  constexpr int PX = kGemmPx * NB;              // pixels per workgroup
  constexpr int KC = L < kGemmKC / NB ? L : kGemmKC / NB;  // frames per LDS stage
  constexpr int KSTEPS = KC / 8;                // 16 real K (8 frames) per MFMA
  constexpr int K2 = 2 * L;
  constexpr int SG = NT / PX;                   // staging groups of 4 frames
  constexpr int G4N = (KC / 4) / SG;            // groups per thread and stage
  constexpr int SPC = L / KC;                   // stages per chunk
  constexpr int BUF = NB * 2 * KSTEPS * 64 * 8; // 16-bit values per stage buffer
  constexpr int N1 = 16, N2 = L / N1;           // the window table's split (reference samples)
  static_assert(L % KC == 0 && (KC / 4) % SG == 0 && G4N >= 1 && G4N <= KSTEPS, "staging");

  // B operand stages: [2][nb][hi, lo][kstep][lane][8], 16-bit; reused at the end of a
  // probe for the FP64 reductions
  constexpr int RED = 16 * kGemmWaves * PX * 4;  // 16-bit slots of the partials' rows
  __shared__ __attribute__((aligned(16))) unsigned short bst[2 * BUF > RED ? 2 * BUF : RED];
  __shared__ double s_mask[DP ? kMaxDet * PX : 1];
  __shared__ double2 s_ref[TRACK ? PX : 1];
  __shared__ double2 s_xs[TRACK ? kMaxCorr * PX : 1];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int n_k = a.n_k;
  // Workgroup ids go round robin over the 8 XCDs. The row groups of a tile take ids
  // of one XCD that are adjacent in its order, so the frames every group stages are
  // read from HBM once and then hit that XCD's L2.
  const int xcd = blockIdx.x % 8, slot = blockIdx.x / 8;
  const int tile = (slot / n_groups) * 8 + xcd;
  const int grp = slot % n_groups;
  if ((int64_t)tile * PX >= n_k) return;  // padding of the last round of 8 tiles
  const int col = lane & 31;      // pixel of this lane in MFMA operands and results
  const int half = lane >> 5;
  const int n_om = a.n_om;
  // row blocks of this workgroup's group: [blk_lo, blk_hi); this wave's: blk
  const int n_blocks = m_rows / 32;
  const int bpg = (n_blocks + n_groups - 1) / n_groups;
  const int blk_lo = grp * bpg;
  const int blk_hi = min(n_blocks, blk_lo + bpg);
  const int blk = blk_lo + wave;
  const bool active = blk < blk_hi;  // uniform per wave
  const bool lead = grp == 0;        // the group that keeps the mean sums
  int kcol[NB];  // n_k < 2^31
  bool cvalid[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    kcol[nb] = tile * PX + kGemmPx * nb + col;
    cvalid[nb] = kcol[nb] < n_k;
  }
  if constexpr (DP) {
    for (int i = tid; i < kMaxDet * PX; i += NT) {
      const int d = i / PX, x = i % PX;
      const int64_t kk = (int64_t)tile * PX + x;
      s_mask[i] = (d < a.n_det && kk < n_k) ? a.masks[(int64_t)d * n_k + kk] : 0.0;
    }
  }
  // correction rows owned by this group (output row r is GEMM rows 2r, 2r + 1)
  int crow[kMaxCorr];
  bool cown[kMaxCorr];
#pragma unroll
  for (int b = 0; b < kMaxCorr; ++b) {
    crow[b] = b < a.n_corr ? a.corr_rows[b] : -1;
    cown[b] = TRACK && crow[b] >= 0 && (2 * crow[b]) / 32 >= blk_lo && (2 * crow[b]) / 32 < blk_hi;
  }

  // staging role: pixel sp of the tile, frame groups sgrp + SG u of each stage
  const int sp = tid % PX;
  static_assert(PX % 64 == 0, "a wave stages one frame group row");
  const int sgrp = __builtin_amdgcn_readfirstlane(tid / PX);  // uniform per wave
  const int snb = sp / kGemmPx, s32 = sp % kGemmPx;
  const int64_t ks = (int64_t)tile * PX + sp;
  const int64_t ksc = ks < n_k ? ks : (int64_t)n_k - 1;
  const int64_t poff = pix_off(ksc, a.nx, a.row_stride);
  const int H = a.hop;
  // this lane's DFT-matrix row; a wave without a block reads a valid one and its
  // results are dropped (its SIMD has no other wave, so this costs no MFMA time)
  const int64_t arow = 32 * (int64_t)min(blk, n_blocks - 1) + col;

  // frame f (absolute) of probe i at pixel k
  auto fetch = [&](int i, int64_t f, int64_t k) -> InT {
    if constexpr (SRC == 0) {
      return ((const InT*)a.in)[(int64_t)i * a.pstride + (f - a.push_begin) * a.fstride +
                                pix_off(k, a.nx, a.row_stride)];
    } else {
      const int64_t slot = (a.probe0 + i) % a.n_slots;
      const int64_t row = f % a.ring_depth;
      if constexpr (SRC == 2) {
        return ((const InT*)a.ring)[((slot * a.ring_tiles + k / PX) * a.ring_depth + row) * PX +
                                    k % PX];
      } else {
        if (f >= a.push_begin)
          return ((const InT*)a.in)[(int64_t)i * a.pstride + (f - a.push_begin) * a.fstride +
                                    pix_off(k, a.nx, a.row_stride)];
        return ((const InT*)a.ring)[(slot * a.ring_depth + row) * n_k + k];
      }
    }
  };

  double acc64[NB][8];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int q = 0; q < 8; ++q) acc64[nb][q] = 0.0;

  for (int i = 0; i < a.n_probes; ++i) {
    const int p = a.probe0 + i;
    __syncthreads();  // the previous probe's reductions through bst / s_ref / s_xs are done
    double2 mu;       // subtracted before splitting: the exact mean, or the reference c
    if constexpr (TRACK) {
      if (a.s_lo == 0) {
        // the probe's first chunk fixes c (every row group computes the same value)
        if (tid < PX) {
          const int64_t kk = (int64_t)tile * PX + tid;
          const int64_t kr = kk < n_k ? kk : (int64_t)n_k - 1;
          double sx = 0.0, sy = 0.0, sw = 0.0, px_ = 0.0, py_ = 0.0;
#pragma unroll 1
          for (int n1 = 0; n1 < N1; ++n1) {
            const InT x = fetch(i, (int64_t)N2 * n1 + N2 / 2, kr);
            const double w = fabs((double)a.win_t[(N2 / 2) * N1 + n1]);
            sx += w * (double)x.x;
            sy += w * (double)x.y;
            px_ += (double)x.x;
            py_ += (double)x.y;
            sw += w;
          }
          if (!(sw > 0.0)) {
            sx = px_;
            sy = py_;
            sw = (double)N1;
          }
          double2 c = make_double2(sx / sw, sy / sw);
          if constexpr (sizeof(InT) == 8) c = make_double2((double)(float)c.x, (double)(float)c.y);
          s_ref[tid] = c;
          if (lead && kk < n_k) a.cref[(int64_t)p * n_k + kk] = c;
        }
        __syncthreads();
        mu = s_ref[sp];
      } else {
        mu = a.cref[(int64_t)p * n_k + ksc];
      }
      for (int e = tid; e < kMaxCorr * PX; e += NT) s_xs[e] = make_double2(0.0, 0.0);
    } else {
      mu = a.cref[(int64_t)p * n_k + ksc];
    }
    const float2 muh = make_float2((float)mu.x, (float)mu.y);
    const float2 mul = make_float2((float)(mu.x - (double)muh.x), (float)(mu.y - (double)muh.y));
    // fp16: the power-of-two operand scale of the pre-pass; bf16 needs none
    const float sc = PREC == 0 ? 1.0f : gscale[(int64_t)p * n_k + ksc];
    float inv2[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const float sc_col =
          PREC == 0 ? 1.0f : gscale[(int64_t)p * n_k + (cvalid[nb] ? kcol[nb] : n_k - 1)];
      inv2[nb] = 1.0f / (sc_col * sc_col);
    }
    double2 msum = make_double2(0.0, 0.0);

    const int n_stages = (a.s_hi - a.s_lo) * SPC;
    // this probe's column of the staging pixel: push buffer and ring (per-frame
    // rows of n_k values, or per-tile rows of PX values)
    const InT* colp = (const InT*)a.in + (int64_t)i * a.pstride + poff;
    const InT* colr = nullptr;
    int64_t rstride = 0;
    if constexpr (SRC != 0) {
      const int64_t slot = (a.probe0 + i) % a.n_slots;
      if constexpr (SRC == 2) {
        colr = (const InT*)a.ring + (slot * a.ring_tiles + ksc / PX) * a.ring_depth * PX + ksc % PX;
        rstride = PX;
      } else {
        colr = (const InT*)a.ring + slot * a.ring_depth * n_k + ksc;
        rstride = n_k;
      }
    }
    InT raw[4 * G4N];
    // group u (4 frames) of stage st of this thread's pixel into raw group u
    auto load_group = [&](int st, int u) {
      const int64_t fs = (int64_t)(a.s_lo + st / SPC) * H + (st % SPC) * KC;  // first frame
      if constexpr (SRC == 0) {
        const InT* b = colp + (fs - a.push_begin) * a.fstride;
#pragma unroll
        for (int v = 0; v < 4; ++v)
          raw[4 * u + v] = b[(int64_t)(4 * (sgrp + SG * u) + v) * a.fstride];
      } else {
        const int64_t r0 = fs % a.ring_depth;  // ring row of the stage's first frame
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int off = 4 * (sgrp + SG * u) + v;  // < KC <= ring depth
          int64_t row = r0 + off;
          row -= row >= a.ring_depth ? a.ring_depth : 0;
          const InT* src = (SRC == 1 && fs + off >= a.push_begin)
                               ? colp + (fs + off - a.push_begin) * a.fstride
                               : colr + row * rstride;
          raw[4 * u + v] = *src;
        }
      }
    };
    // convert raw group u (stage st) and store it into LDS buffer par; the mean sums
    // take its frames only when counted
    auto store_group = [&](int st, int u, int par, bool counted) {
      const int s = a.s_lo + st / SPC, c0 = (st % SPC) * KC;
      unsigned short* bb = bst + par * BUF;
      const int g4 = sgrp + SG * u;
      unsigned hw[4], lw[4];
      // frames counted in the mean sums (each once: in chunk 0, or new in its chunk),
      // as weights 0 or 1 that are uniform per wave (t0 is): no branches
      const int t0 = c0 + 4 * g4;
      float2 y[4];
      float wc[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const InT x = raw[4 * u + v];
        wc[v] = (counted && (s == 0 || t0 + v >= L - H)) ? 1.0f : 0.0f;
        if constexpr (sizeof(InT) == 16) {  // complex128: the difference in FP64
          const double dx = x.x - mu.x, dy = x.y - mu.y;
          if constexpr (TRACK) {
            msum.x += dx * (double)wc[v];
            msum.y += dy * (double)wc[v];
          }
          y[v] = make_float2((float)dx, (float)dy);
        } else {
          // FP32: (x - mu_hi) - mu_lo, mu = mu_hi + mu_lo; the tracked c is an FP32
          // value (mu_lo = 0), and the FP64 mean sum takes the same difference
          if constexpr (TRACK)
            y[v] = make_float2(x.x - muh.x, x.y - muh.y);
          else
            y[v] = make_float2((x.x - muh.x) - mul.x, (x.y - muh.y) - mul.y);
        }
      }
      if constexpr (TRACK && sizeof(InT) == 8) {
        // at most 4 terms in FP32 (exact weights) before the FP64 sum: their
        // rounding errors are random and far below the operand split's
        float gx = y[0].x * wc[0], gy = y[0].y * wc[0];
#pragma unroll
        for (int v = 1; v < 4; ++v) {
          gx += y[v].x * wc[v];
          gy += y[v].y * wc[v];
        }
        msum.x += (double)gx;
        msum.y += (double)gy;
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if constexpr (PREC == 1) {  // power-of-two scale: exact
          y[v].x *= sc;
          y[v].y *= sc;
        }
        split_pair<PREC>(y[v].x, y[v].y, hw[v], lw[v]);
      }
      const int tl = 4 * g4;                    // frame within the stage
      const int kst = tl / 8, hh = (tl % 8) / 4;
      const int lanep = s32 + 32 * hh;          // operand lane holding these 8 K values
      const int hslot = (((snb * 2 + 0) * KSTEPS + kst) * 64 + lanep) * 8;
      const int lslot = (((snb * 2 + 1) * KSTEPS + kst) * 64 + lanep) * 8;
      *reinterpret_cast<uint4*>(&bb[hslot]) = make_uint4(hw[0], hw[1], hw[2], hw[3]);
      *reinterpret_cast<uint4*>(&bb[lslot]) = make_uint4(lw[0], lw[1], lw[2], lw[3]);
    };
    // DFT-matrix fragment slot k: k-step k of stage st (the lane's 8 K columns)
    h8 ah[KSTEPS], al[KSTEPS];
    auto a_load = [&](int st, int k) {
      const int kc2 = 2 * (st % SPC) * KC + 16 * k + 8 * half;
      ah[k] = *reinterpret_cast<const h8*>(fmat + arow * K2 + kc2);
      al[k] = *reinterpret_cast<const h8*>(fmat + (m_rows + arow) * K2 + kc2);
    };

    f32x16 acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[nb][v] = 0.0f;

    if (n_stages > 0) {
#pragma unroll
      for (int u = 0; u < G4N; ++u) load_group(0, u);
#pragma unroll
      for (int k = 0; k < KSTEPS; ++k) a_load(0, k);
#pragma unroll
      for (int u = 0; u < G4N; ++u) store_group(0, u, 0, true);
#pragma unroll
      for (int u = 0; u < G4N; ++u) load_group(min(1, n_stages - 1), u);
      __syncthreads();
    }
    // The k-step sequence has no branches (which would make the compiler's waits on
    // loads conservative): the last stages reload the last stage's frames and DFT
    // fragments (valid addresses) and convert them into the idle buffer uncounted.
    for (int st = 0; st < n_stages; ++st) {
      const unsigned short* bb = bst + (st & 1) * BUF;
      const bool next = st + 1 < n_stages;
      const int st1 = min(st + 1, n_stages - 1), st2 = min(st + 2, n_stages - 1);
      // B fragments from LDS, one k-step ahead within the stage
      h8 bh[2][NB], bl[2][NB];
      auto b_load = [&](int k) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          bh[k & 1][nb] = *reinterpret_cast<const h8*>(&bb[(((nb * 2 + 0) * KSTEPS + k) * 64 + lane) * 8]);
          bl[k & 1][nb] = *reinterpret_cast<const h8*>(&bb[(((nb * 2 + 1) * KSTEPS + k) * 64 + lane) * 8]);
        }
      };
      b_load(0);
#pragma unroll
      for (int kst = 0; kst < KSTEPS; ++kst) {
        if (kst + 1 < KSTEPS) b_load(kst + 1);
        const int c = kst & 1;
        // each product over the column blocks in turn: an MFMA's accumulator comes
        // from the one NB MFMAs earlier, past its latency
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb] = mfma<PREC>(ah[kst], bh[c][nb], acc[nb]);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb] = mfma<PREC>(ah[kst], bl[c][nb], acc[nb]);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb] = mfma<PREC>(al[kst], bh[c][nb], acc[nb]);
        a_load(st1, kst);
#pragma unroll
        for (int u = 0; u < G4N; ++u) {
          if (u * KSTEPS / G4N == kst) {
            store_group(st1, u, (st + 1) & 1, next);
            load_group(st2, u);
          }
        }
      }
      // one wave per SIMD issues in order: interleave the conversion (VALU) with the
      // MFMAs, so that it runs while the matrix core works, and issue the next
      // k-step's B fragments (2 NB LDS reads) before this k-step's 3 NB MFMAs, which
      // then hide their latency (each read placed just before its MFMA waited for it)
#pragma unroll
      for (int kst = 0; kst < KSTEPS; ++kst) {
        if (kst == 0) __builtin_amdgcn_sched_group_barrier(0x100, (KSTEPS > 1 ? 4 : 2) * NB, 0);
        else if (kst + 1 < KSTEPS) __builtin_amdgcn_sched_group_barrier(0x100, 2 * NB, 0);
#pragma unroll
        for (int i = 0; i < 3 * NB; ++i) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
          __builtin_amdgcn_sched_group_barrier(0x002, 4, 0);  // VALU
        }
      }
      if (st % SPC == SPC - 1 && active) {
        // chunk complete: |X|^2 into the FP64 accumulators. Accumulator v of a lane
        // holds row 8 (v / 4) + 4 half + (v % 4) of its 32-row block, column col;
        // rows (2m', 2m'+1) are (Re, Im) of output row m'
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const int v = 4 * (q / 2) + 2 * (q % 2);
            const float xr = acc[nb][v], xi = acc[nb][v + 1];
            bool corr = false;
            if constexpr (TRACK) {
              const int r = 16 * blk + 4 * (q / 2) + 2 * half + (q % 2);
#pragma unroll
              for (int cb = 0; cb < kMaxCorr; ++cb) {
                if (cown[cb] && r == crow[cb]) {
                  corr = true;
                  double2* xp = &s_xs[cb * PX + kGemmPx * nb + col];
                  xp->x += (double)xr;
                  xp->y += (double)xi;
                }
              }
            }
            if (corr) {
              // the per-chunk mean kernel supplies these rows' whole FP64 value
              if (!a.corr_skip) acc64[nb][q] += (double)xr * (double)xr + (double)xi * (double)xi;
            } else {
              const float pw = xr * xr + xi * xi;
              acc64[nb][q] += (double)(pw * inv2[nb]);
            }
          }
#pragma unroll
          for (int v = 0; v < 16; ++v) acc[nb][v] = 0.0f;
        }
      }
      __syncthreads();
    }

    if constexpr (TRACK) {
      // this probe's FP64 sums: psi - c over the staged frames (lead group), and X' at
      // the correction rows it owns
      double2* red = reinterpret_cast<double2*>(bst);
      red[tid] = msum;
      __syncthreads();
      if (tid < PX) {
        const int64_t kk = (int64_t)tile * PX + tid;
        if (kk < n_k) {
          if (lead) {
            double2 t = make_double2(0.0, 0.0);
            for (int g = 0; g < SG; ++g) {
              t.x += red[g * PX + tid].x;
              t.y += red[g * PX + tid].y;
            }
            double2* ms = a.msum + (int64_t)p * n_k + kk;
            ms->x += t.x;
            ms->y += t.y;
          }
#pragma unroll
          for (int cb = 0; cb < kMaxCorr; ++cb) {
            if (cown[cb]) {  // slots: bins 0, 1, L - 1
              double2* xp = a.xs + ((int64_t)p * kMaxCorr + cb) * n_k + kk;
              xp->x += s_xs[cb * PX + tid].x;
              xp->y += s_xs[cb * PX + tid].y;
            }
          }
        }
      }
    }

    if constexpr (DP) {
      // cumulative detector partials of this group's output rows
      __syncthreads();
      double* sd = reinterpret_cast<double*>(bst);  // [group rows][PX]
      const int r_lo = 16 * blk_lo, r_hi = min(n_om, 16 * blk_hi);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int r = 16 * blk + 4 * (q / 2) + 2 * half + (q % 2);
        if (active && r < r_hi) {
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) sd[(r - r_lo) * PX + kGemmPx * nb + col] = acc64[nb][q];
        }
      }
      __syncthreads();
      const int32_t* slots = a.pair_slot + (int64_t)tile * a.n_det;
      for (int rr = tid; rr < r_hi - r_lo; rr += NT) {
        for (int d = 0; d < a.n_det; ++d) {
          const int slot = slots[d];  // -1: this detector's mask is zero on the tile
          if (slot < 0) continue;
          double dsum = 0.0;
#pragma unroll
          for (int x = 0; x < PX; ++x) dsum += s_mask[d * PX + x] * sd[rr * PX + x];
          // cumulative over probes 0..i
          a.dpart[((int64_t)slot * a.n_probes + i) * n_om + r_lo + rr] = dsum;
        }
      }
    }
  }

#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int r = 16 * blk + 4 * (q / 2) + 2 * half + (q % 2);
    if (active && r < n_om) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        if (cvalid[nb]) {
          double* sp_ = a.S + (int64_t)r * n_k + kcol[nb];
          *sp_ = a.s_store ? acc64[nb][q] : *sp_ + acc64[nb][q];
        }
      }
    }
  }
}

// 4 column blocks (128 pixels) per workgroup, so each DFT-matrix fragment feeds 12
// MFMAs; rows beyond 4 waves x 32 go to more row groups, each staging the same
// frames (from L2 after the first)
constexpr int kGemmNB = 4;
static int gemm_groups(int n_om) {
  const int blocks = (2 * n_om + 31) / 32;
  return (blocks + kGemmWaves - 1) / kGemmWaves;
}

template <int L, typename InT, int PREC, bool TRACK, int SRC>
static hipError_t launch_g5(const SegArgs& a, const void* fmat, int m_rows, const float* gscale,
                            int n_groups, hipStream_t st) {
  // 1-D grid: the tiles padded to a multiple of 8 (one per XCD), times the groups
  constexpr int NB = kGemmNB;
  const int64_t n_tiles = (a.n_k + 32 * NB - 1) / (32 * NB);
  const dim3 grid((unsigned)(((n_tiles + 7) / 8) * 8 * n_groups));
  if (a.n_det > 0)
    hipLaunchKernelGGL((seg_gemm_kernel<L, InT, PREC, true, NB, TRACK, SRC>), grid,
                       dim3(64 * kGemmWaves), 0, st, a, (const unsigned short*)fmat, m_rows, gscale,
                       n_groups);
  else
    hipLaunchKernelGGL((seg_gemm_kernel<L, InT, PREC, false, NB, TRACK, SRC>), grid,
                       dim3(64 * kGemmWaves), 0, st, a, (const unsigned short*)fmat, m_rows, gscale,
                       n_groups);
  return hipGetLastError();
}

template <int L, typename InT, int PREC>
static hipError_t launch_g3(const SegArgs& a, const void* fmat, int m_rows, const float* gscale,
                            int n_tiles, hipStream_t st) {
  (void)n_tiles;  // the grid follows from n_k and the tile width
  const int n_groups = gemm_groups(a.n_om);
  const int src = a.from_ring ? (a.ring_tiles > 0 ? 2 : 1)
                              : ((int64_t)a.s_lo * a.hop >= a.push_begin ? 0 : 1);
  if (a.track_mean) {
    if constexpr (PREC == 0) {
      if (src == 2) return launch_g5<L, InT, PREC, true, 2>(a, fmat, m_rows, gscale, n_groups, st);
      if (src == 1) return launch_g5<L, InT, PREC, true, 1>(a, fmat, m_rows, gscale, n_groups, st);
      return launch_g5<L, InT, PREC, true, 0>(a, fmat, m_rows, gscale, n_groups, st);
    }
    return hipErrorInvalidValue;
  }
  if (src != 0) return hipErrorInvalidValue;  // the exact-mean form takes whole series
  return launch_g5<L, InT, PREC, false, 0>(a, fmat, m_rows, gscale, n_groups, st);
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

bool seg_gemm_supported(int L) { return L == 128 || L == 256 || L == 512 || L == 1024; }
int seg_gemm_tile_pixels(int L, int n_om) {
  (void)L;
  (void)n_om;
  return kGemmPx * kGemmNB;
}

hipError_t launch_seg_gemm(int L, int in_dtype, bool /*sub64*/, int prec, const SegArgs& a,
                           const void* fmat, int m_rows, int n_tiles, hipStream_t st) {
  const float* gscale = a.gscale;
  switch (L) {
    case 128: return launch_g2<128>(in_dtype, prec, a, fmat, m_rows, gscale, n_tiles, st);
    case 256: return launch_g2<256>(in_dtype, prec, a, fmat, m_rows, gscale, n_tiles, st);
    case 512: return launch_g2<512>(in_dtype, prec, a, fmat, m_rows, gscale, n_tiles, st);
    case 1024: return launch_g2<1024>(in_dtype, prec, a, fmat, m_rows, gscale, n_tiles, st);
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
