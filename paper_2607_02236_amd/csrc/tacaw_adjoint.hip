// Adjoint of the spectral reduction (vector-Jacobian product), chunk by chunk
// with recomputation: no chunk spectra are stored.
//
// For Lval = sum_{p,s,m,k} G_p(m,k) |X_{p,s}(m,k)|^2, X = DFT_t(w (psi - mu)):
//   g_y(t)  = 2 sum_m G(m) X(m) exp(+2 pi i m t / L)      (d/dRe + i d/dIm)
//   g_z(t)  = w(t) g_y(t)
//   grad psi(n) = sum over the chunks holding n of g_z(n - sH)
//                 - [n < N_used] (1 / N_used) sum_s sum_t g_z_s(t)   (GLOBAL mean)
//   dLval/dr = sum Re[conj(g_y) z] dw/dr - 2 Lval sum_t w dw/dr / sum_t w^2
// with G_p(m,k) = kappa_S (gS(m,k) + sum_j gD_j(m) M_j(k)) + kappa_p sum_j gDp_{j,p}(m) M_j(k).
// The mean-term sum is sum_s sum_m 2 G(m) X_s(m) conj(W(m)), W the window's DFT.
// For a window whose W vanishes outside bins {0, 1, L-1} it needs only the FP64
// chunk sums of X at those bins, which the forward pass kept for its exact mean
// correction (sum_s X_s = sum_s X'_s - N_s delta W, delta = mu - c); the term is
// then subtracted as each frame is stored. Otherwise the sum is accumulated here
// and a second pass subtracts it. mu = c + (FP64 sum of psi - c) / N_used, also
// from the forward pass.
//
// Transforms (L = N1 N2, t = N2 n1 + n2, m = k1 + N1 k2): the forward one is the
// chunk kernel's (N1-point DFTs over n1 in registers, inter-pass twiddle, one LDS
// exchange, N2-point DFTs over n2, as G = N2 / N1 threads with a folded
// decimation-in-frequency stage when N2 > N1). The inverse runs the same steps
// in reverse order on conj(G X):
//   conj(U(k1, n2)) = sum_k2 conj(Z(k1 + N1 k2)) exp(-2 pi i k2 n2 / N2)   (Z = G X)
//   conj(g_y(t)) / 2 = sum_k1 conj(U(k1, n2)) exp(-2 pi i k1 n2 / L) exp(-2 pi i k1 n1 / N1)
// The first line is computed by the threads that hold the bins (with G threads
// per k1: thread g forms C_g(n) = exp(-2 pi i g n / N2) DFT_N1(conj Z_g)(n), and
// conj(U(k1, n + N1 j)) = sum_g exp(-2 pi i g j / G) C_g(n)); one LDS exchange
// brings the columns back to the time layout for the second line. Two exchanges
// and two barriers per chunk.
#include <type_traits>

#include "buffer_io.h"
#include "regfft.h"
#include "tacaw_internal.h"

namespace tacaw {

template <int L>
struct BwdShape;
template <>
struct BwdShape<64> {
  static constexpr int N1 = 8, W = 16;
};
template <>
struct BwdShape<128> {
  static constexpr int N1 = 16, W = 16;
};
template <>
struct BwdShape<256> {
  static constexpr int N1 = 16, W = 16;
};
template <>
struct BwdShape<512> {
  static constexpr int N1 = 16, W = 16;
};
template <>
struct BwdShape<1024> {
  static constexpr int N1 = 16, W = 8;
};
// L = 200 (the paper's chunk length): the forward's 10 x 20 split (prime-factor
// 10-point DFTs); 32 pixels so that every wave holds two bin roles of one fold
// half (the fold half is then uniform per wave)
template <>
struct BwdShape<200> {
  static constexpr int N1 = 10, W = 32;
};

// x exp(-2 pi i e / G), G in {2, 4}
template <int G>
__device__ __forceinline__ float2 rot_g(float2 x, int e) {
  e %= G;
  if (e == 0) return x;
  if (G == 2 || e == 2) return make_float2(-x.x, -x.y);
  return e == 1 ? make_float2(x.y, -x.x) : make_float2(-x.y, x.x);
}

// DW: the window-parameter derivative is wanted (dwin_t set). It needs the
// centred samples again after both transforms: for complex64 input with
// L <= 512 they stay in registers through the transforms (KEEP_Z); otherwise
// (complex128, L = 1024) they are re-read from memory at the end of the chunk.
// MT: mean term. 0: none (no mean subtracted); 1: accumulate its sum for the
// separate pass; 2: from the forward pass's bin sums, subtracted at the stores;
// 3: per-chunk means (chunk s subtracts its own mean mu_s, from the forward
// pass): the frames of chunk s get 2 w g_s - M_s / L with
// M_s = 2 sum_b G(b) conj(W(b)) X_s(b) over the bins where W != 0, posted by the
// bin-role threads that hold those bins.
template <int L, typename InT, bool DW, int MT>
__global__ void __launch_bounds__(BwdShape<L>::W*(L / BwdShape<L>::N1))
    bwd_kernel(const BwdArgs a) {
  constexpr int N1 = BwdShape<L>::N1;
  constexpr int W = BwdShape<L>::W;
  constexpr int N2 = L / N1;
  constexpr int NT = W * N2;
  constexpr int HALF = N1 / 2;
  constexpr int R = N2 <= N1 ? N1 / N2 : 1;  // pass-2 DFTs per thread (N2 <= N1)
  constexpr int G = N2 > N1 ? N2 / N1 : 1;   // threads per pass-2 DFT (N2 > N1)
  constexpr int KROW = N2 * W + W;           // float2 per k1 row of an exchange tile
  constexpr int TILE = N1 * KROW;
  static_assert(G == 1 || G == 2 || G == 4, "pass-2 split");

  __shared__ float2 xbuf2[2 * TILE];  // forward exchange tile, inverse exchange tile
  __shared__ float2 s_tw[L];          // [n2][k1] exp(-2 pi i n2 k1 / L)
  __shared__ float s_win[L];          // [n2][n1]
  __shared__ float s_dwin[DW ? L : 1];
  __shared__ double red[2 * NT];
  __shared__ float s_mk[kMaxDet * W];  // detector masks of the tile's pixels
  __shared__ double2 s_mt[MT == 3 ? kMaxCorr * W : 1];  // MT 3: M_s terms per bin and pixel
  float2* const xa = xbuf2;
  float2* const xi = xbuf2 + TILE;

  const int tid = threadIdx.x;
  const int px = tid % W;
  const int n2 = tid / W;  // time role: residue n2; bin role: j = n2
  const int j = n2;
  const int k1g = j % N1;
  const int gg = j / N1;   // uniform per wave
  const int tile = xcd_tile();
  const int n_k = a.n_k;
  const int64_t k = (int64_t)tile * W + px;
  const bool kvalid = k < n_k;
  const int64_t kc = kvalid ? k : (int64_t)n_k - 1;
  for (int i = tid; i < L; i += NT) {
    s_tw[i] = a.tw[i];
    s_win[i] = a.win_t[i];
    if constexpr (DW) s_dwin[i] = a.dwin_t[i];
  }
  for (int e = tid; e < kMaxDet * W; e += NT) {
    const int d = e / W;
    const int64_t kk = (int64_t)tile * W + e % W;
    s_mk[e] = (d < a.n_det && kk < n_k) ? (float)a.masks[(int64_t)d * n_k + kk] : 0.0f;
  }
  __syncthreads();

  // bin m held as value t by this thread in the bin role
  auto bin = [&](int t) -> int {
    if constexpr (G == 1) return (j + N2 * (t / N2)) + N1 * (t % N2);
    else return k1g + N1 * (G * t + gg);
  };
  // upstream weight G_p(m, k) of this pixel; bins outside the energy window
  // have no output row and weight 0
  auto weight = [&](int m, int p) -> double {
    int r = m + a.roi_half;  // output row of bin m
    if (r >= L) r -= L;
    const int n_om = a.n_om;
    // the row passes through an empty asm so that the 16 bins' addresses are
    // formed on each call instead of being hoisted out of the probe loop (and spilled)
    asm volatile("" : "+v"(r));
    double g = 0.0;
    if (r < n_om) {
      if (a.gS) g += a.kappa_S * a.gS[(int64_t)r * n_k + kc];
      for (int d = 0; d < a.n_det; ++d) {
        double c = 0.0;
        if (a.gD) c += a.kappa_S * a.gD[(int64_t)d * n_om + r];
        if (a.gDp) c += a.kappa_p * a.gDp[((int64_t)d * a.n_probe_total + p) * n_om + r];
        g += c * (double)s_mk[d * W + px];
      }
      if (a.qfac) g *= a.qfac[r];
    }
    return g;
  };

  const int H = a.hop;
  const bool half_hop = (2 * H == L);
  double dA = 0.0, dLval = 0.0;
  float Gt[N1];  // weights of the thread's bins (they change per probe only through gDp)

  // frames and gradient: raw buffer accesses, one 32-bit lane offset (n2 rows,
  // pixel kc) from a uniform row-group base (rows N2 n1 .. N2 n1 + N2 - 1 of a
  // chunk; the host checks that a group spans less than 2 GiB)
  constexpr int ESZ = (int)sizeof(InT);
  const int64_t row_bytes = a.fstride * ESZ;
  const int64_t kin = pix_off(kc, a.nx, a.row_stride);
  const uint32_t lane_off = (uint32_t)(((int64_t)n2 * a.fstride + kin) * ESZ);
  const int64_t span = pix_off((int64_t)n_k - 1, a.nx, a.row_stride) + 1;
  const uint32_t group_bytes = (uint32_t)((int64_t)(N2 - 1) * row_bytes + span * ESZ);
  auto group = [&](const void* base, int ii, int ss, int n1) -> char* {
    int64_t gstride = (int64_t)N2 * row_bytes;  // formed next to each access, not kept
    asm volatile("" : "+s"(gstride));
    return (char*)base + (int64_t)ii * a.pstride * ESZ + (int64_t)ss * H * row_bytes + n1 * gstride;
  };
  // raw samples of the next chunk, loaded one chunk ahead
  InT pre[N1];
#pragma unroll
  for (int n1 = 0; n1 < N1; ++n1) pre[n1] = buffer_load<InT>(group(a.in, 0, 0, n1), group_bytes, lane_off);

  for (int i = 0; i < a.n_probes; ++i) {
    const int p = a.probe0 + i;
    if (i == 0 || a.gDp) {
#pragma unroll
      for (int t = 0; t < N1; ++t) Gt[t] = (float)weight(bin(t), p);
    }
    // mu = c + delta, delta = (sum over the used frames of psi - c) / N_used
    double2 mu = make_double2(0.0, 0.0), delta = make_double2(0.0, 0.0);
    if constexpr (MT == 1 || MT == 2) {
      const double2 cr = a.cref[(int64_t)p * n_k + kc];
      const double2 ms = a.msum[(int64_t)p * n_k + kc];
      delta = make_double2(ms.x * a.inv_nused, ms.y * a.inv_nused);
      mu = make_double2(cr.x + delta.x, cr.y + delta.y);
    }
    // MT 2: the mean term of this probe and pixel, divided by N_used
    float2 fix = make_float2(0.f, 0.f);
    double2 fixd = make_double2(0.0, 0.0);
    if constexpr (MT == 2) {
      double2 gm = make_double2(0.0, 0.0);
      for (int b = 0; b < a.n_corr; ++b) {
        const int m = b == 0 ? 0 : (b == 1 ? 1 : L - 1);
        const double g = 2.0 * (double)(float)weight(m, p);  // the FP32 weight the transform uses
        const double2 wb = a.wbin[b];
        const double2 x = a.xs[((int64_t)p * kMaxCorr + b) * n_k + kc];
        // sum_s X_s(m) = sum_s X'_s(m) - N_s delta W(m)
        const double sx = x.x - a.n_seg * (delta.x * wb.x - delta.y * wb.y);
        const double sy = x.y - a.n_seg * (delta.x * wb.y + delta.y * wb.x);
        gm.x += g * (wb.x * sx + wb.y * sy);  // g conj(W) (sx + i sy)
        gm.y += g * (wb.x * sy - wb.y * sx);
      }
      fixd = make_double2(gm.x * a.inv_nused, gm.y * a.inv_nused);
      fix = make_float2((float)fixd.x, (float)fixd.y);
    }
    float2 carry[HALF];
#pragma unroll
    for (int u = 0; u < HALF; ++u) carry[u] = make_float2(0.f, 0.f);
    double2 gsum = make_double2(0.0, 0.0);

    for (int s = 0; s < a.n_seg; ++s) {
      auto centre = [&](const InT& x) -> float2 {
        return make_float2((float)((double)x.x - mu.x), (float)((double)x.y - mu.y));
      };
      // MT 3: this chunk's mean (read here rather than carried through the transforms)
      if constexpr (MT == 3) mu = a.cmean[((int64_t)p * a.n_seg + s) * n_k + kc];
      float2 v[N1];
      // DW (complex64): the centred samples stay in registers for the r-derivative
      // (re-reading them at the end of the chunk missed the L2 and doubled the reads)
      constexpr bool KEEP_Z = DW && sizeof(InT) == 8 && L <= 512;
      float2 zk[KEEP_Z ? N1 : 1];
#pragma unroll
      for (int n1 = 0; n1 < N1; ++n1) {
        const float2 z = centre(pre[n1]);
        if constexpr (KEEP_Z) zk[n1] = z;
        const float w = s_win[n2 * N1 + n1];
        v[n1] = make_float2(w * z.x, w * z.y);
      }
      // prefetch the next chunk (or the next probe's first chunk)
      {
        const bool next_chunk = s + 1 < a.n_seg;
        if (next_chunk || i + 1 < a.n_probes) {
          const int ii = next_chunk ? i : i + 1;
          const int ss = next_chunk ? s + 1 : 0;
#pragma unroll
          for (int n1 = 0; n1 < N1; ++n1)
            pre[n1] = buffer_load<InT>(group(a.in, ii, ss, n1), group_bytes, lane_off);
        }
      }
      // ---- forward transform: time layout -> bin layout X[t] = X(bin(t)); the
      // twiddles are read first, so that their LDS latency passes during the DFT
      float2 twv[N1];
#pragma unroll
      for (int k1 = 1; k1 < N1; ++k1) twv[k1] = s_tw[n2 * N1 + k1];
      __builtin_amdgcn_sched_barrier(0);
      dft_inplace<N1>(v);
#pragma unroll
      for (int k1 = 1; k1 < N1; ++k1) v[k1] = cmul(v[k1], twv[k1]);
#pragma unroll
      for (int k1 = 0; k1 < N1; ++k1) xa[k1 * KROW + n2 * W + px] = v[k1];
      __syncthreads();  // (1) forward tile written; the inverse tile's reads of the previous chunk are done
      float2 X[N1];
      if constexpr (G == 1) {
#pragma unroll
        for (int q = 0; q < R; ++q) {
          float2 Y[N2];
          const float2* col = xa + (j + N2 * q) * KROW + px;
#pragma unroll
          for (int r = 0; r < N2; ++r) Y[r] = col[r * W];
          dft_inplace<N2>(Y);
#pragma unroll
          for (int k2 = 0; k2 < N2; ++k2) X[q * N2 + k2] = Y[k2];
        }
      } else {
        const float2* col = xa + k1g * KROW + px;
        auto cl = [&](int n) { return col[n * W]; };
        if constexpr (G == 2) {
          if (gg == 0) dif_combine<N1, 2, 0>(cl, X);
          else dif_combine<N1, 2, 1>(cl, X);
        } else {
          if (gg == 0) dif_combine<N1, 4, 0>(cl, X);
          else if (gg == 1) dif_combine<N1, 4, 1>(cl, X);
          else if (gg == 2) dif_combine<N1, 4, 2>(cl, X);
          else dif_combine<N1, 4, 3>(cl, X);
        }
        dft_inplace<N1>(X);
      }
      if constexpr (MT == 3) {  // this thread's share of M_s (bins 0, 1, L - 1)
#pragma unroll
        for (int t = 0; t < N1; ++t) {
          const int m = bin(t);
          const int b = m == 0 ? 0 : (m == 1 ? 1 : (m == L - 1 ? 2 : -1));
          if (b >= 0 && b < a.n_corr) {
            const double g = 2.0 * (double)Gt[t];
            const double2 wb = a.wbin[b];
            const double xx = X[t].x, xy = X[t].y;
            s_mt[b * W + px] = make_double2(g * (wb.x * xx + wb.y * xy), g * (wb.x * xy - wb.y * xx));
          }
        }
      }
      // ---- weight by G: loss value; conj(Z) = conj(G X)
#pragma unroll
      for (int t = 0; t < N1; ++t) {
        const float pw = X[t].x * X[t].x + X[t].y * X[t].y;
        dLval += (double)Gt[t] * (double)pw;
        X[t] = make_float2(Gt[t] * X[t].x, -Gt[t] * X[t].y);
      }
      // ---- inverse, bin side: conj(U(k1, n2)) (or its G partial sums) into the inverse tile
      if constexpr (G == 1) {
#pragma unroll
        for (int q = 0; q < R; ++q) {
          float2 Y[N2];
#pragma unroll
          for (int k2 = 0; k2 < N2; ++k2) Y[k2] = X[q * N2 + k2];
          dft_inplace<N2>(Y);
#pragma unroll
          for (int r = 0; r < N2; ++r) xi[(j + N2 * q) * KROW + r * W + px] = Y[r];
        }
      } else {
        dft_inplace<N1>(X);
        if (gg == 1) TwiddleRow<N1, N2, 1>::apply(X);
        if constexpr (G == 4) {
          if (gg == 2) TwiddleRow<N1, N2, 2>::apply(X);
          else if (gg == 3) TwiddleRow<N1, N2, 3>::apply(X);
        }
#pragma unroll
        for (int n = 0; n < N1; ++n) xi[k1g * KROW + (gg * N1 + n) * W + px] = X[n];
      }
      __syncthreads();  // (2) inverse tile written; the forward tile's reads are done
      // ---- inverse, time side: conj(U(k1, n2)) for every k1, twiddle, N1-point DFT
      if constexpr (G == 1) {
#pragma unroll
        for (int k1 = 0; k1 < N1; ++k1) v[k1] = xi[k1 * KROW + n2 * W + px];
      } else {
        const int n = n2 % N1, jj = n2 / N1;  // jj is uniform per wave
#pragma unroll
        for (int k1 = 0; k1 < N1; ++k1) {
          float2 sum = xi[k1 * KROW + n * W + px];
#pragma unroll
          for (int g = 1; g < G; ++g) {
            const float2 c = rot_g<G>(xi[k1 * KROW + (g * N1 + n) * W + px], g * jj);
            sum.x += c.x;
            sum.y += c.y;
          }
          v[k1] = sum;
        }
      }
#pragma unroll
      for (int k1 = 1; k1 < N1; ++k1) v[k1] = cmul(v[k1], twv[k1]);
      dft_inplace<N1>(v);  // v[n1] = conj(g_y(N2 n1 + n2)) / 2
      float2 msub = make_float2(0.f, 0.f);  // MT 3: M_s / L
      if constexpr (MT == 3) {
        double2 M = make_double2(0.0, 0.0);
        for (int b = 0; b < a.n_corr; ++b) {
          const double2 e = s_mt[b * W + px];
          M.x += e.x;
          M.y += e.y;
        }
        msub = make_float2((float)(M.x / L), (float)(M.y / L));
      }
      // g_z = w g_y; r-derivative term; mean-term sum; overlap carry and stores
#pragma unroll
      for (int n1 = 0; n1 < N1; ++n1) {
        const float w = s_win[n2 * N1 + n1];
        const float2 gy = make_float2(2.f * v[n1].x, -2.f * v[n1].y);
        if constexpr (DW) {  // kept, or (complex128) read again
          float2 z;
          if constexpr (KEEP_Z) z = zk[n1];
          else z = centre(buffer_load<InT>(group(a.in, i, s, n1), group_bytes, lane_off));
          const float dw = s_dwin[n2 * N1 + n1];
          dA += (double)dw * ((double)gy.x * z.x + (double)gy.y * z.y);
        }
        v[n1] = make_float2(w * gy.x - msub.x, w * gy.y - msub.y);
        if constexpr (MT == 1) {
          gsum.x += (double)v[n1].x;
          gsum.y += (double)v[n1].y;
        }
      }
      const bool last = (s == a.n_seg - 1);
#pragma unroll
      for (int n1 = 0; n1 < N1; ++n1) {
        float2 o = v[n1];
        bool store = true;
        if (half_hop) {
          if (n1 < HALF) {
            o.x += carry[n1].x;
            o.y += carry[n1].y;
          } else {
            carry[n1 - HALF] = o;
            store = last;
          }
        }
        if (store && kvalid) {
          InT outv;
          if constexpr (MT == 2 && sizeof(outv.x) == 8) {
            outv.x = (double)o.x - fixd.x;
            outv.y = (double)o.y - fixd.y;
          } else if constexpr (MT == 2) {
            outv.x = o.x - fix.x;
            outv.y = o.y - fix.y;
          } else {
            outv.x = o.x;
            outv.y = o.y;
          }
          buffer_store<InT>(outv, group(a.grad, i, s, n1), group_bytes, lane_off);
        }
      }
    }
    if constexpr (MT == 1) {  // mean-term sum of this probe and pixel
      __syncthreads();        // the last chunk's reads of the forward tile are done
      double2* rr = reinterpret_cast<double2*>(xa);
      rr[tid] = gsum;
      __syncthreads();
      if (n2 == 0 && kvalid) {
        double2 t = make_double2(0.0, 0.0);
#pragma unroll
        for (int r = 0; r < N2; ++r) {
          t.x += rr[r * W + px].x;
          t.y += rr[r * W + px].y;
        }
        a.gmean[(int64_t)i * n_k + k] = t;
      }
      __syncthreads();  // before the next probe's forward tile writes
    }
  }
  // workgroup partials of the r-derivative and the loss value
  red[tid] = kvalid ? dA : 0.0;
  red[NT + tid] = kvalid ? dLval : 0.0;
  __syncthreads();
  // fold onto the largest power of two P2 <= NT (NT = 640 at L = 200), then halve
  constexpr int P2 = (NT & (NT - 1)) == 0 ? NT : 1 << (31 - __builtin_clz(NT));
  if constexpr (P2 != NT) {
    if (tid < NT - P2) {
      red[tid] += red[tid + P2];
      red[NT + tid] += red[NT + tid + P2];
    }
    __syncthreads();
  }
  for (int w = P2 / 2; w > 0; w >>= 1) {
    if (tid < w) {
      red[tid] += red[tid + w];
      red[NT + tid] += red[NT + tid + w];
    }
    __syncthreads();
  }
  if (tid == 0) {
    a.dwpart[2 * tile] = red[0];
    a.dwpart[2 * tile + 1] = red[NT];
  }
}

// grad[i][n][k] -= gmean[i][k] / N_used for n < N_used
template <typename InT>
__global__ void bwd_mean_fix_kernel(const BwdArgs a) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.z;
  if (k >= a.n_k) return;
  const double2 g = a.gmean[(int64_t)i * a.n_k + k];
  const double sx = g.x * a.inv_nused, sy = g.y * a.inv_nused;
  InT* gp = (InT*)a.grad + (int64_t)i * a.pstride + pix_off(k, a.nx, a.row_stride);
  for (int64_t n = blockIdx.y; n < a.n_used; n += gridDim.y) {
    InT v = gp[n * a.fstride];
    v.x = (decltype(v.x))((double)v.x - sx);
    v.y = (decltype(v.y))((double)v.y - sy);
    gp[n * a.fstride] = v;
  }
}

// out[0] += sum_t part[2t] - 2 c sum_t part[2t+1]
__global__ void bwd_wparam_kernel(const double* part, int n, double c, double* out) {
  __shared__ double ra[256], rl[256];
  double sa = 0.0, sl = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    sa += part[2 * i];
    sl += part[2 * i + 1];
  }
  ra[threadIdx.x] = sa;
  rl[threadIdx.x] = sl;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      ra[threadIdx.x] += ra[threadIdx.x + w];
      rl[threadIdx.x] += rl[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] += ra[0] - 2.0 * c * rl[0];
}

template <int L>
static hipError_t launch_bl(int in_dtype, const BwdArgs& a, int n_tiles, hipStream_t st) {
  constexpr int NT = BwdShape<L>::W * (L / BwdShape<L>::N1);
  const bool dw = a.dwin_t != nullptr;
  const int mt = a.per_chunk ? 3 : (a.mean_global ? (a.n_corr > 0 ? 2 : 1) : 0);
  auto go = [&](auto in_t, auto dw_c, auto mt_c) {
    hipLaunchKernelGGL((bwd_kernel<L, decltype(in_t), decltype(dw_c)::value, decltype(mt_c)::value>),
                       dim3(n_tiles), dim3(NT), 0, st, a);
  };
  using T0 = std::false_type;
  using T1 = std::true_type;
  using M0 = std::integral_constant<int, 0>;
  using M1 = std::integral_constant<int, 1>;
  using M2 = std::integral_constant<int, 2>;
  using M3 = std::integral_constant<int, 3>;
  auto by_mt = [&](auto in_t, auto dw_c) {
    if (mt == 3) go(in_t, dw_c, M3{});
    else if (mt == 2) go(in_t, dw_c, M2{});
    else if (mt == 1) go(in_t, dw_c, M1{});
    else go(in_t, dw_c, M0{});
  };
  auto by_dw = [&](auto in_t) {
    if (dw) by_mt(in_t, T1{});
    else by_mt(in_t, T0{});
  };
  if (in_dtype == 1) by_dw(double2{});
  else by_dw(float2{});
  return hipGetLastError();
}

int bwd_tile_pixels(int L) {
  switch (L) {
    case 64: return BwdShape<64>::W;
    case 128: return BwdShape<128>::W;
    case 256: return BwdShape<256>::W;
    case 512: return BwdShape<512>::W;
    case 1024: return BwdShape<1024>::W;
    case 200: return BwdShape<200>::W;
  }
  return 0;
}

// pass-1 DFT size of the adjoint's split; it reads the plan's window and twiddle
// tables, which are laid out for the forward split, so the two must agree
int bwd_pass1_size(int L) {
  switch (L) {
    case 64: return BwdShape<64>::N1;
    case 128: return BwdShape<128>::N1;
    case 256: return BwdShape<256>::N1;
    case 512: return BwdShape<512>::N1;
    case 1024: return BwdShape<1024>::N1;
    case 200: return BwdShape<200>::N1;
  }
  return 0;
}

hipError_t launch_bwd(int L, int in_dtype, const BwdArgs& a, int n_tiles, hipStream_t st) {
  switch (L) {
    case 64: return launch_bl<64>(in_dtype, a, n_tiles, st);
    case 128: return launch_bl<128>(in_dtype, a, n_tiles, st);
    case 256: return launch_bl<256>(in_dtype, a, n_tiles, st);
    case 512: return launch_bl<512>(in_dtype, a, n_tiles, st);
    case 1024: return launch_bl<1024>(in_dtype, a, n_tiles, st);
    case 200: return launch_bl<200>(in_dtype, a, n_tiles, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_bwd_mean_fix(const BwdArgs& a, int in_dtype, hipStream_t st) {
  const int gy = (int)(a.n_used < 64 ? a.n_used : 64);
  dim3 g((a.n_k + 255) / 256, gy, a.n_probes);
  if (in_dtype == 1)
    hipLaunchKernelGGL(bwd_mean_fix_kernel<double2>, g, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(bwd_mean_fix_kernel<float2>, g, dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_bwd_wparam(const double* part, int n, double c, double* out, hipStream_t st) {
  hipLaunchKernelGGL(bwd_wparam_kernel, dim3(1), dim3(256), 0, st, part, n, c, out);
  return hipGetLastError();
}

}  // namespace tacaw
