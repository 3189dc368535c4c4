// Fused chunk kernel, FFT form: ingest -> reference subtraction -> window ->
// L-point FP32 FFT along time (two passes, one LDS exchange) -> |X|^2 -> FP64
// accumulation over chunks and probes, plus the state of the exact elastic-mean
// correction and per-probe detector partials.
//
// What is computed (paper Sec. II.B.2 and Eq. 1, 2): for chunk s of probe p and
// pixel k, X'_s(m, k) = sum_t w(t) (psi(sH + t, k) - c(k)) exp(-2 pi i m t / L),
// and S(m, k) += |X'_s(m, k)|^2. c is a per-(probe, pixel) reference (a
// window-weighted mean of frames sampled over the first chunk, or the exact
// mean); the difference to the elastic mean mu is restored exactly afterwards
// from FP64 sums (finalize), because for the supported compact windows
// W(m) = sum_t w(t) exp(-2 pi i m t / L) vanishes outside bins {0, 1, L-1}.
// At those bins |X'|^2 is squared in FP64 (the correction cancels most of it).
//
// Work decomposition (one workgroup = a tile of W adjacent pixels, all probes
// and all chunks of the push):
//   L = N1 * N2. Thread (px, n2) owns pixel k0 + px and the N1 samples
//   t = N2 * n1 + n2; it loads them with lanes running along pixels (coalesced
//   rows of W * 8 bytes), does the N1-point DFT over n1 in registers, applies
//   the twiddle exp(-2 pi i n2 k1 / L), exchanges through LDS, and then as
//   thread (px, j) does the N1 / N2 remaining N2-point DFTs over n2 for
//   k1 = j + N2 q. Output bin m = k1 + N1 k2.
//   With 50 % overlap (H = L/2) the second half of a chunk's samples (n1 >=
//   N1/2) is the first half of the next chunk's, so every frame is read from
//   memory once per push; other hops reload each chunk.
#pragma once

#include <type_traits>

#include "buffer_io.h"
#include "regfft.h"
#include "tacaw_internal.h"

namespace tacaw {

// |z|^2 in FP64. At the correction bins the exact mean correction cancels most of
// sum_s |X'_s|^2, so it is formed from the FP32 transform values without the
// FP32 rounding of the square.
__device__ __forceinline__ double sq64(float2 z) {
  const double x = (double)z.x, y = (double)z.y;
  return x * x + y * y;
}

template <int L>
struct FftShape;
template <>
struct FftShape<64> {
  static constexpr int N1 = 8, W = 16;
};
template <>
struct FftShape<128> {
  static constexpr int N1 = 16, W = 16;
};
template <>
struct FftShape<256> {
  static constexpr int N1 = 16, W = 16;
};
#ifndef TACAW_TILE_W512
#define TACAW_TILE_W512 16  // pixels per workgroup at L = 512 (tuning parameter)
#endif
template <>
struct FftShape<512> {
  static constexpr int N1 = 16, W = TACAW_TILE_W512;
};
#ifndef TACAW_TILE_W1024
#define TACAW_TILE_W1024 8  // pixels per workgroup at L = 1024 (tuning parameter)
#endif
template <>
struct FftShape<1024> {
  static constexpr int N1 = 16, W = TACAW_TILE_W1024;
};
// L = 200 (the chunk length of the paper's worked example): 10-point DFTs
// (prime-factor 2 x 5) in both passes; 32 pixels so that a wave's 64 lanes hold
// two pass-2 roles of the same fold half
template <>
struct FftShape<200> {
  static constexpr int N1 = 10, W = 32;
};

// LEAN: every chunk of the launch lies inside the push buffer and H = L/2 or
// H = L, so all loads use uniform row bases and the frames to count in the mean
// sum are known per n1 at compile time. The general variant also reads the ring, takes
// any hop and decides per lane.
// MODE 4: MODE 2 with the ring stored per pixel tile, [slot][tile][row][W], so
// that a tile's chunk is contiguous (few address translations per chunk).
// MODE 0: general (any hop; frames before the push from the ring, per lane);
// MODE 1: whole-series variant reading the push buffer; MODE 2: whole-series
// variant reading every frame from the ring (deferred streaming); MODE 3: MODE 1
// when a whole chunk of frames spans less than 2 GiB, so one buffer descriptor per
// chunk serves all row groups through a scalar offset (fewer scalar registers).
#ifndef TACAW_XBUF_TILES
#define TACAW_XBUF_TILES 2  // exchange tiles: 2 = alternate per chunk (one barrier), 1 = two barriers
#endif
#ifndef TACAW_WAVES_PER_EU
#define TACAW_WAVES_PER_EU 1  // minimum waves per SIMD the register allocation must allow
#endif
// FULL (whole-series variants only): hop = L, no overlap; otherwise hop = L/2 there.
template <int L, typename InT, bool SUB64, bool DP, int MODE, bool FULL = false>
__global__ void __launch_bounds__(FftShape<L>::W*(L / FftShape<L>::N1))
    __attribute__((amdgpu_waves_per_eu(TACAW_WAVES_PER_EU)))
    seg_fft_kernel(const SegArgs a) {
  constexpr bool LEAN = MODE != 0;
  static_assert(LEAN || !FULL, "hop = L is a whole-series variant");
  constexpr bool TILED = MODE == 4;
  constexpr bool RING = MODE == 2 || TILED;
  constexpr bool NARROW = MODE == 3;
  constexpr int N1 = FftShape<L>::N1;
  constexpr int W = FftShape<L>::W;
  constexpr int N2 = L / N1;
  constexpr int NT = W * N2;
  constexpr int HALF = N1 / 2;
  constexpr int ESZ = (int)sizeof(InT);
  constexpr int BATCH = HALF;             // loads in flight per thread and batch
  constexpr int R = N2 <= N1 ? N1 / N2 : 1;  // pass-2 DFTs per thread (N2 <= N1)
  constexpr int G = N2 > N1 ? N2 / N1 : 1;   // threads per pass-2 DFT (N2 > N1)
  constexpr int PADK = W;                  // LDS padding per k1 row (bank spread)
  constexpr int KROW = N2 * W + PADK;      // float2 per k1 row of the exchange tile
  static_assert(N1 % N2 == 0 || N2 % N1 == 0, "pass-2 split");
  static_assert(G == 1 || G == 2 || G == 4, "pass-2 split factor");

  // two exchange tiles [k1][n2][px] used by alternate chunks, so one barrier per
  // chunk suffices; tile 0 is reused for the per-probe reductions
  constexpr int NBUF = TACAW_XBUF_TILES;
  __shared__ float2 xbuf2[NBUF * N1 * KROW];
  float2* const xbuf = xbuf2;
  __shared__ float2 s_tw[L];          // [n2][k1]
  __shared__ float s_win[L];          // [n2][n1]
  __shared__ double s_mask[DP ? kMaxDet * W : 1];
  __shared__ double2 s_ref[W];        // reference of the probe's pixels (first chunk)

  const int tid = threadIdx.x;
  const int px = tid % W;
  const int n2 = tid / W;  // pass 1: time residue; pass 2: role j
  const int tile = xcd_tile();
  const int n_k = a.n_k;
  const int64_t k = (int64_t)tile * W + px;
  const bool kvalid = k < n_k;
  const int64_t kc = kvalid ? k : (int64_t)n_k - 1;

  for (int i = tid; i < L; i += NT) {
    s_tw[i] = a.tw[i];
    s_win[i] = a.win_t[i];
  }
  if constexpr (DP) {
    for (int i = tid; i < kMaxDet * W; i += NT) {
      const int d = i / W, x = i % W;
      const int64_t kk = (int64_t)tile * W + x;
      s_mask[i] = (d < a.n_det && kk < n_k) ? a.masks[(int64_t)d * n_k + kk] : 0.0;
    }
  }
  __syncthreads();

  // pass-2 role: output bins owned by this thread are m = k1 + N1 k2 with
  //   R-mode: k1 = j + N2 q (q < R), k2 = 0..N2-1         (acc index q*N2 + k2)
  //   G-mode: k1 = j % N1, k2 = G r + g, g = j / N1      (acc index r)
  const int j = n2;
  const int k1g = j % N1;
  const int gg = j / N1;  // uniform per wave (W * 4 lanes share it)

  double acc[N1];  // FP64 sum of |X'|^2 over this launch's chunks and probes
#pragma unroll
  for (int i = 0; i < N1; ++i) acc[i] = 0.0;

  const int H = a.hop;
  const bool half_hop = (2 * H == L);
  const bool track = a.track_mean != 0;
  // correction bins: 0 -> thread j = 0 value 0; 1 -> j = 1 value 0; L-1 -> j = N2-1, last value
  const int corr_b = (j == 0) ? 0 : (j == 1 ? 1 : 2);
  const bool corr_own = track && (j == 0 || (a.n_corr == 3 && (j == 1 || j == N2 - 1)));
  const int64_t row_bytes = a.fstride * ESZ;
  // pixel kc inside an input frame (a k-space window may have wider pixel rows)
  const int64_t kin = pix_off(kc, a.nx, a.row_stride);
  // per-lane byte offset inside a frame row group: (n2 rows down, kc pixels across)
  const uint32_t lane_off = (uint32_t)(((int64_t)n2 * a.fstride + kin) * ESZ);
  // bytes addressable from a row-group base: N2 - 1 full frames plus the span of
  // the last frame's pixels (the host checks that this fits in 32 bits)
  const int64_t span = pix_off((int64_t)n_k - 1, a.nx, a.row_stride) + 1;
  const uint32_t group_bytes = (uint32_t)((int64_t)(N2 - 1) * row_bytes + span * ESZ);

  // LEAN: raw samples of the next chunk, loaded one chunk ahead (software prefetch)
  InT pre[LEAN ? N1 : 1];
  // MODE 4: the ring is stored per pixel tile ([slot][tile][row][W]), so a row
  // group of a tile is N2 consecutive rows of W pixels
  const uint32_t tiled_off = (uint32_t)(((int64_t)n2 * W + px) * ESZ);
  constexpr uint32_t tiled_bytes = (uint32_t)(N2 * W * ESZ);
  // MODE 3: a chunk's frames lie within 2 GiB of its first row
  const uint32_t chunk_bytes =
      NARROW ? (uint32_t)((int64_t)(L - N2) * row_bytes + (int64_t)group_bytes) : 0u;
  auto fetch_at = [&](int ii, int ss, int n1) -> InT {
    const char* rb;
    if constexpr (NARROW) {
      const char* cb = (const char*)a.in + (int64_t)ii * a.pstride * ESZ +
                       ((int64_t)ss * H - a.push_begin) * row_bytes;
      return buffer_load_so<InT>(cb, chunk_bytes, lane_off, (uint32_t)(N2 * n1 * row_bytes));
    } else if constexpr (RING) {
      // ring rows (ss H + N2 n1) mod D of probe probe0 + ii; D and H are multiples of
      // N2, so a row group never wraps (row_bytes is one frame of the ring here)
      // the chunks of one launch span at most D frames, so from the first chunk's row
      // (ring_row_lo, from the host) each chunk and row group wraps at most once
      const int D = (int)a.ring_depth;
      int row = a.ring_row_lo + (ss - a.s_lo) * H;
      if (row >= D) row -= D;
      row += N2 * n1;
      if (row >= D) row -= D;
      const int64_t slot = (a.probe0 + ii) % a.n_slots;
      if constexpr (TILED) {
        int64_t tb = (int64_t)W * ESZ;  // bytes per tile row, formed next to the load
        asm volatile("" : "+s"(tb));
        rb = (const char*)a.ring + ((slot * a.ring_tiles + tile) * D + row) * tb;
        return buffer_load<InT>(rb, tiled_bytes, tiled_off);
      }
      int64_t rbytes = row_bytes;  // formed next to the load (see the push case below)
      asm volatile("" : "+s"(rbytes));
      rb = (const char*)a.ring + (slot * D + row) * rbytes;
    } else {
      // the row-group stride passes through an empty asm so that the 16 per-group
      // offsets are formed next to each load instead of being kept (and spilled)
      int64_t gstride = (int64_t)N2 * row_bytes;
      asm volatile("" : "+s"(gstride));
      rb = (const char*)a.in + (int64_t)ii * a.pstride * ESZ +
           ((int64_t)ss * H - a.push_begin) * row_bytes + n1 * gstride;
    }
    return buffer_load<InT>(rb, group_bytes, lane_off);
  };
  if constexpr (LEAN) {
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) pre[n1] = fetch_at(0, a.s_lo, n1);
  }

  int cc = 0;  // chunks processed by this thread block (selects the exchange tile)
  for (int i = 0; i < a.n_probes; ++i) {
    const int p = a.probe0 + i;
    // reference c: fixed by the probe's first chunk (make_ref below) or read back
    double2 cr = make_double2(0.0, 0.0);
    if (!(track && a.s_lo == 0)) cr = a.cref[(int64_t)p * n_k + kc];
    float2 cf = make_float2((float)cr.x, (float)cr.y);
    const char* in_probe = (const char*)a.in + (int64_t)i * a.pstride * ESZ;
    const InT* ringb =
        a.ring ? (const InT*)a.ring + ((int64_t)(p % a.n_slots) * a.ring_depth) * n_k + kc : nullptr;
    double2 msum = make_double2(0.0, 0.0);
    double2 xsum = make_double2(0.0, 0.0);
    float2 kept[HALF];
    bool have_kept = false;

    for (int s = a.s_lo; s < a.s_hi; ++s) {
      const int64_t seg0 = (int64_t)s * H;
      const bool fast = LEAN || seg0 >= a.push_begin;
      float2 v[N1];

      // subtract the reference; add the frame to the FP64 mean sum when it is
      // counted (each frame once, in the first chunk that contains it).
      // CM: 0 = not tracked, 1 = every loaded frame counts, 2 = per-lane test
      // t >= L - H, 3 = t >= L/2 (H = L/2), which is n1 >= N1/2 for every lane
      auto take = [&](int n1, InT x, auto cmode) -> float2 {
        constexpr int CM = decltype(cmode)::value;
        const int tau = N2 * n1 + n2;
        const bool count = CM == 1 || (CM == 2 && tau >= L - H) || (CM == 3 && n1 >= HALF);
        float2 z;
        double dx, dy;
        if constexpr (SUB64) {
          dx = (double)x.x - cr.x;
          dy = (double)x.y - cr.y;
          z = make_float2((float)dx, (float)dy);
        } else {
          z = make_float2((float)x.x - cf.x, (float)x.y - cf.y);
          dx = (double)z.x;
          dy = (double)z.y;
        }
        if constexpr (CM == 1) {
          msum.x += dx;
          msum.y += dy;
        } else if constexpr (CM != 0) {
          msum.x += count ? dx : 0.0;
          msum.y += count ? dy : 0.0;
        }
        return z;
      };
      // The probe's first chunk fixes c: the window-weighted mean of the N1 frames
      // t = N2 n1 + N2 / 2, spread evenly over the chunk, which thread n2 = N2 / 2
      // holds (FP64 sum, rounded to FP32 for complex64 input, so that the c
      // subtracted in FP32 below is the c the correction uses). Every value of c
      // keeps the mean correction exact; one near the chunks' own mean keeps |X'|
      // small at bins 0 and +-1,
      // where the correction cancels. It depends only on the series, not on how
      // it was pushed.
      // raw(n1): the thread's raw sample n1 of the chunk, from a register array
      // (unrolled loop) or a load (rolled loop: once per probe, few registers)
      auto make_ref = [&](auto raw, auto unroll) {
        if (n2 == N2 / 2) {
          double sx = 0.0, sy = 0.0, sw = 0.0, px_ = 0.0, py_ = 0.0;
          auto add = [&](int n1) {
            const InT x = raw(n1);
            const double w = fabs((double)s_win[n2 * N1 + n1]);
            sx += w * (double)x.x;
            sy += w * (double)x.y;
            px_ += (double)x.x;
            py_ += (double)x.y;
            sw += w;
          };
          if constexpr (decltype(unroll)::value) {
#pragma unroll
            for (int n1 = 0; n1 < N1; ++n1) add(n1);
          } else {
#pragma unroll 1
            for (int n1 = 0; n1 < N1; ++n1) add(n1);
          }
          if (!(sw > 0.0)) {  // a window that vanishes at every sample: plain mean
            sx = px_;
            sy = py_;
            sw = (double)N1;
          }
          sx /= sw;
          sy /= sw;
          if constexpr (ESZ == 8) {
            sx = (double)(float)sx;
            sy = (double)(float)sy;
          }
          s_ref[px] = make_double2(sx, sy);
          if (kvalid) a.cref[(int64_t)p * n_k + k] = make_double2(sx, sy);
        }
        __syncthreads();
        cr = s_ref[px];
        cf = make_float2((float)cr.x, (float)cr.y);
      };
      auto fetch_fast = [&](int n1) -> InT {
        // uniform base of the row group N2 * n1 .. N2 * n1 + N2 - 1 of this chunk;
        // one 32-bit lane offset (n2 rows, kc pixels) shared by every load
        int64_t gstride = (int64_t)N2 * row_bytes;  // formed next to the load (see fetch_at)
        asm volatile("" : "+s"(gstride));
        const char* rb = in_probe + (seg0 - a.push_begin) * row_bytes + n1 * gstride;
        return buffer_load<InT>(rb, group_bytes, lane_off);
      };
      auto fetch_any = [&](int n1) -> InT {
        const int64_t f = seg0 + N2 * n1 + n2;
        if (f >= a.push_begin)
          return *(const InT*)(in_probe + (f - a.push_begin) * row_bytes + kin * ESZ);
        return ringb[(f % a.ring_depth) * (int64_t)n_k];
      };
      auto load_range = [&](int lo, auto fetch, auto cmode) {
#pragma unroll
        for (int b0 = 0; b0 < N1; b0 += BATCH) {
          if (b0 >= lo) {
            InT raw[BATCH];
#pragma unroll
            for (int u = 0; u < BATCH; ++u) raw[u] = fetch(b0 + u);
#pragma unroll
            for (int u = 0; u < BATCH; ++u) v[b0 + u] = take(b0 + u, raw[u], cmode);
          }
        }
      };
      using C0 = std::integral_constant<int, 0>;
      using C1 = std::integral_constant<int, 1>;
      using C2 = std::integral_constant<int, 2>;
      using C3 = std::integral_constant<int, 3>;

      // the thread's window values, read before the samples are taken
      float wv[N1];
#pragma unroll
      for (int n1 = 0; n1 < N1; ++n1) wv[n1] = s_win[n2 * N1 + n1];
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (LEAN) {
        // H = L/2, chunk s: frames with t >= L/2 (n1 >= HALF) are new; t < L/2 are new
        // only for s = 0. H = L: every frame of every chunk is new.
        auto take_pre = [&](int lo, auto cmode) {
#pragma unroll
          for (int n1 = 0; n1 < N1; ++n1)
            if (n1 >= lo) v[n1] = take(n1, pre[n1], cmode);
        };
        if (have_kept) {
#pragma unroll
          for (int n1 = 0; n1 < HALF; ++n1) v[n1] = kept[n1];
          if (track) take_pre(HALF, C1{});
          else take_pre(HALF, C0{});
        } else if (!track) {
          take_pre(0, C0{});
        } else if (s == 0 || FULL) {
          if (s == 0) make_ref([&](int n1) { return pre[n1]; }, std::true_type{});
          take_pre(0, C1{});
        } else {
          take_pre(0, C3{});
        }
        // prefetch the next chunk's new samples (or the next probe's first chunk)
        const bool next_chunk = s + 1 < a.s_hi;
        if (next_chunk || i + 1 < a.n_probes) {
          const int ii = next_chunk ? i : i + 1;
          const int ss = next_chunk ? s + 1 : a.s_lo;
#pragma unroll
          for (int n1 = 0; n1 < N1; ++n1)
            if (n1 >= HALF || !next_chunk || FULL) pre[n1] = fetch_at(ii, ss, n1);
        }
      } else if (have_kept && half_hop) {
        // the kept half was counted in the previous chunk; the new half all counts
#pragma unroll
        for (int n1 = 0; n1 < HALF; ++n1) v[n1] = kept[n1];
        if (fast) {
          if (track) load_range(HALF, fetch_fast, C1{});
          else load_range(HALF, fetch_fast, C0{});
        } else {
          if (track) load_range(HALF, fetch_any, C1{});
          else load_range(HALF, fetch_any, C0{});
        }
      } else {
        if (!track) {
          if (fast) load_range(0, fetch_fast, C0{});
          else load_range(0, fetch_any, C0{});
        } else if (s == 0) {
          // thread n2 = N2 / 2 loads its samples for the reference (and again below)
          make_ref(fetch_any, std::false_type{});
          if (fast) load_range(0, fetch_fast, C1{});
          else load_range(0, fetch_any, C1{});
        } else {
          if (fast) load_range(0, fetch_fast, C2{});
          else load_range(0, fetch_any, C2{});
        }
      }
      if constexpr (!FULL) {
#pragma unroll
        for (int n1 = HALF; n1 < N1; ++n1) kept[n1 - HALF] = v[n1];
        have_kept = true;  // (the general variant also tests half_hop itself)
      }

      // window (table stored per thread: s_win[n2 * N1 + n1] = w(N2 n1 + n2))
#pragma unroll
      for (int n1 = 0; n1 < N1; ++n1) {
        v[n1].x *= wv[n1];
        v[n1].y *= wv[n1];
      }
      // pass 1: DFT over n1, then twiddle exp(-2 pi i n2 k1 / L); the twiddles are
      // read first, so that their LDS latency passes during the DFT
      float2 twv[N1];
#pragma unroll
      for (int k1 = 1; k1 < N1; ++k1) twv[k1] = s_tw[n2 * N1 + k1];
      __builtin_amdgcn_sched_barrier(0);
      dft_inplace<N1>(v);
#pragma unroll
      for (int k1 = 1; k1 < N1; ++k1) v[k1] = cmul(v[k1], twv[k1]);

      // tile (cc & 1), cc counting this thread block's chunks: the reads of
      // chunk cc - 2 from it finished before the barrier of chunk cc - 1, so only
      // the barrier after the writes is needed
      float2* const xb = xbuf2 + (NBUF == 2 ? (cc & 1) : 0) * (N1 * KROW);
      ++cc;
      if constexpr (NBUF == 1) __syncthreads();  // the previous chunk's reads are done
#pragma unroll
      for (int k1 = 0; k1 < N1; ++k1) xb[k1 * KROW + n2 * W + px] = v[k1];
      __syncthreads();

      if constexpr (G == 1) {
        // R-mode: thread j transforms over n2 for k1 = j + N2 q
#pragma unroll
        for (int q = 0; q < R; ++q) {
          float2 X[N2];
          const float2* col = xb + (j + N2 * q) * KROW + px;
#pragma unroll
          for (int r = 0; r < N2; ++r) X[r] = col[r * W];
          // all reads issued before the first use (the general variant has no
          // registers to spare for that)
          if constexpr (LEAN) __builtin_amdgcn_sched_barrier(0);
          dft_inplace<N2>(X);
#pragma unroll
          for (int k2 = 0; k2 < N2; ++k2) {
            // the correction bins (bin 0, 1: q = 0, k2 = 0 of threads j = 0, 1; bin
            // L - 1: q = R - 1, k2 = N2 - 1 of thread j = N2 - 1) are added below
            const bool cand = (q == 0 && k2 == 0) || (q == R - 1 && k2 == N2 - 1);
            if (!(cand && corr_own && (k2 == 0 ? j <= 1 : j == N2 - 1 && j > 1))) {
              const float pw = X[k2].x * X[k2].x + X[k2].y * X[k2].y;
              acc[q * N2 + k2] += (double)pw;
            }
          }
          // (the correction bins: their FP64 sum, and their square in FP64 unless
          // the per-chunk mean kernel supplies them)
          if (corr_own) {
            if (q == 0 && j <= 1) {
              xsum.x += (double)X[0].x;
              xsum.y += (double)X[0].y;
              if (!a.corr_skip) acc[0] += sq64(X[0]);
            }
            if (q == R - 1 && j == N2 - 1 && j > 1) {
              xsum.x += (double)X[N2 - 1].x;
              xsum.y += (double)X[N2 - 1].y;
              if (!a.corr_skip) acc[q * N2 + N2 - 1] += sq64(X[N2 - 1]);
            }
          }
        }
      } else {
        // G-mode: G threads share the N2-point DFT of k1 = j % N1
        const float2* col = xb + k1g * KROW + px;
        float2 X[N1];
        if constexpr (G == 2 && LEAN) {
          // all 32 reads first, so that their latencies overlap
          float2 c[N2];
#pragma unroll
          for (int n = 0; n < N2; ++n) c[n] = col[n * W];
          __builtin_amdgcn_sched_barrier(0);
          auto cr = [&](int n) { return c[n]; };
          if (gg == 0) dif_combine<N1, 2, 0>(cr, X);
          else dif_combine<N1, 2, 1>(cr, X);
        } else if constexpr (G == 2) {
          // the general variant has no registers to spare: read as used
          auto cl = [&](int n) { return col[n * W]; };
          if (gg == 0) dif_combine<N1, 2, 0>(cl, X);
          else dif_combine<N1, 2, 1>(cl, X);
        } else if constexpr (!LEAN) {
          auto cl = [&](int n) { return col[n * W]; };
          if (gg == 0) dif_combine<N1, 4, 0>(cl, X);
          else if (gg == 1) dif_combine<N1, 4, 1>(cl, X);
          else if (gg == 2) dif_combine<N1, 4, 2>(cl, X);
          else dif_combine<N1, 4, 3>(cl, X);
        } else {
          // G = 4: the 64 values are read and folded in two halves of 32 (all 64
          // at once would exceed the register budget)
          constexpr int HN = N1 / 2;
          auto fold_half = [&](auto h) {
            constexpr int H0 = decltype(h)::value * HN;
            float2 c[4 * HN];
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
              for (int n = 0; n < HN; ++n) c[q * HN + n] = col[(H0 + n + N1 * q) * W];
            __builtin_amdgcn_sched_barrier(0);
            auto cr = [&](int m) { return c[(m / N1) * HN + m % N1 - H0]; };
            if (gg == 0) dif_fold_part<N1, 4, 0, H0, H0 + HN>(cr, X);
            else if (gg == 1) dif_fold_part<N1, 4, 1, H0, H0 + HN>(cr, X);
            else if (gg == 2) dif_fold_part<N1, 4, 2, H0, H0 + HN>(cr, X);
            else dif_fold_part<N1, 4, 3, H0, H0 + HN>(cr, X);
          };
          fold_half(std::integral_constant<int, 0>{});
          fold_half(std::integral_constant<int, 1>{});
          if (gg == 1) TwiddleRow<N1, N2, 1>::apply(X);
          else if (gg == 2) TwiddleRow<N1, N2, 2>::apply(X);
          else if (gg == 3) TwiddleRow<N1, N2, 3>::apply(X);
        }
        dft_inplace<N1>(X);
#pragma unroll
        for (int r = 0; r < N1; ++r) {
          // correction bins: r = 0 of threads j = 0, 1 (bins 0, 1) and r = N1 - 1 of
          // thread j = N2 - 1 (bin L - 1) are added below
          if (!((r == 0 || r == N1 - 1) && corr_own && (r == 0 ? j <= 1 : j > 1))) {
            const float pw = X[r].x * X[r].x + X[r].y * X[r].y;
            acc[r] += (double)pw;
          }
        }
        // (the correction bins: their FP64 sum, and their square in FP64 unless the
        // per-chunk mean kernel supplies them)
        if (corr_own) {
          if (j <= 1) {
            xsum.x += (double)X[0].x;
            xsum.y += (double)X[0].y;
            if (!a.corr_skip) acc[0] += sq64(X[0]);
          } else {
            xsum.x += (double)X[N1 - 1].x;
            xsum.y += (double)X[N1 - 1].y;
            if (!a.corr_skip) acc[N1 - 1] += sq64(X[N1 - 1]);
          }
        }
      }
    }

    if (track) {
      __syncthreads();
      double2* red = reinterpret_cast<double2*>(xbuf);
      red[tid] = msum;
      __syncthreads();
      if (n2 == 0 && kvalid) {
        double2 t = make_double2(0.0, 0.0);
#pragma unroll
        for (int r = 0; r < N2; ++r) {
          t.x += red[r * W + px].x;
          t.y += red[r * W + px].y;
        }
        double2* ms = a.msum + (int64_t)p * n_k + k;
        double2 o = *ms;
        o.x += t.x;
        o.y += t.y;
        *ms = o;
      }
      if (corr_own && kvalid) {
        double2* xp = a.xs + ((int64_t)p * kMaxCorr + corr_b) * n_k + k;
        double2 o = *xp;
        o.x += xsum.x;
        o.y += xsum.y;
        *xp = o;
      }
    }

    if constexpr (DP) {
      // detector partials: the mask-weighted tile sum of the FP64 accumulator,
      // cumulative over this launch's probes (the reduce kernel differences them)
      __syncthreads();
      double* sp = reinterpret_cast<double*>(xbuf);  // [L][W]
#pragma unroll
      for (int t = 0; t < N1; ++t) {
        const int m = (G == 1) ? (j + N2 * (t / N2)) + N1 * (t % N2) : k1g + N1 * (G * t + gg);
        sp[m * W + px] = acc[t];
      }
      __syncthreads();
      const int n_om = a.n_om;
      const int32_t* slots = a.pair_slot + (int64_t)tile * a.n_det;
      for (int r = tid; r < n_om; r += NT) {
        int m = r - a.roi_half;  // output row r holds bin m
        if (m < 0) m += L;
        double pv[W];
#pragma unroll
        for (int x = 0; x < W; ++x) pv[x] = sp[m * W + x];
#pragma unroll 1
        for (int d = 0; d < a.n_det; ++d) {
          const int slot = slots[d];  // uniform; -1: this detector's mask is zero here
          if (slot < 0) continue;
          double dsum = 0.0;
#pragma unroll
          for (int x = 0; x < W; ++x) dsum += s_mask[d * W + x] * pv[x];
          // cumulative over the launch's probes 0..i
          a.dpart[((int64_t)slot * a.n_probes + i) * n_om + r] = dsum;
        }
      }
    }
    // the reductions above used tile 0, which a later chunk writes
    __syncthreads();
  }

  if (kvalid) {
#pragma unroll
    for (int t = 0; t < N1; ++t) {
      const int m = (G == 1) ? (j + N2 * (t / N2)) + N1 * (t % N2) : k1g + N1 * (G * t + gg);
      int row = m + a.roi_half;  // rows >= n_om lie outside the energy window
      if (row >= L) row -= L;
      if (row < a.n_om) {
        double* sp = a.S + (int64_t)row * n_k + k;
        *sp = a.s_store ? acc[t] : *sp + acc[t];
      }
    }
  }
}

}  // namespace tacaw
