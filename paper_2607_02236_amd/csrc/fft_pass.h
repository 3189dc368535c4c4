// Two-pass L-point FFT over a tile of W pixels held by W * N2 threads
// (thread (px, n2)); shared by the adjoint kernels.
//
// Input : v[n1] = x(t = N2 n1 + n2) for the thread's pixel (pass-1 layout).
// Output: out[t] = X(bin(t, j)), j = n2 (pass-2 layout), with
//   N2 <= N1: k1 = j + N2 (t / N2), k2 = t % N2
//   N2 >  N1: k1 = j % N1, k2 = G t + j / N1 (G = N2 / N1 threads per k1)
// and bin = k1 + N1 k2. Forward sign exp(-2 pi i m t / L). Uses one LDS
// exchange (tile [k1][n2][px], padded rows) and the inter-pass twiddles
// tw[n2 * N1 + k1] = exp(-2 pi i n2 k1 / L) staged in LDS.
#pragma once

#include "regfft.h"

namespace tacaw {

template <int N1, int G, int g>
__device__ __forceinline__ void dif_fold(const float2* __restrict__ col, int stride,
                                         float2 (&y)[N1]) {
  constexpr int N2 = N1 * G;
#pragma unroll
  for (int n = 0; n < N1; ++n) {
    float2 s = col[n * stride];
#pragma unroll
    for (int j = 1; j < G; ++j) {
      const float2 x = col[(n + N1 * j) * stride];
      const int e = (j * g) % G;  // rotation by exp(-2 pi i j g / G)
      float2 t;
      if (G == 2) {
        t = e == 0 ? x : make_float2(-x.x, -x.y);
      } else {
        t = e == 0 ? x : e == 1 ? make_float2(x.y, -x.x) : e == 2 ? make_float2(-x.x, -x.y)
                                                           : make_float2(-x.y, x.x);
      }
      s.x += t.x;
      s.y += t.y;
    }
    y[n] = s;
  }
  if constexpr (g != 0) TwiddleRow<N1, N2, g>::apply(y);
}

template <int L, int N1, int W>
struct Fft2 {
  static constexpr int N2 = L / N1;
  static constexpr int R = N2 <= N1 ? N1 / N2 : 1;
  static constexpr int G = N2 > N1 ? N2 / N1 : 1;
  static constexpr int KROW = N2 * W + W;
  static constexpr int LDS = N1 * KROW;  // float2 elements of the exchange tile
  static_assert(G == 1 || G == 2 || G == 4, "pass-2 split");

  __device__ static __forceinline__ int bin(int t, int j) {
    if constexpr (G == 1) {
      return (j + N2 * (t / N2)) + N1 * (t % N2);
    } else {
      return (j % N1) + N1 * (G * t + j / N1);
    }
  }

  // v is destroyed. Both __syncthreads() are inside; xbuf is free on return.
  __device__ static __forceinline__ void run(float2 (&v)[N1], float2 (&out)[N1], float2* xbuf,
                                             const float2* s_tw, int px, int n2) {
    dft_inplace<N1>(v);
#pragma unroll
    for (int k1 = 1; k1 < N1; ++k1) v[k1] = cmul(v[k1], s_tw[n2 * N1 + k1]);
    __syncthreads();
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) xbuf[k1 * KROW + n2 * W + px] = v[k1];
    __syncthreads();
    const int j = n2;
    if constexpr (G == 1) {
#pragma unroll
      for (int q = 0; q < R; ++q) {
        float2 X[N2];
        const float2* col = xbuf + (j + N2 * q) * KROW + px;
#pragma unroll
        for (int r = 0; r < N2; ++r) X[r] = col[r * W];
        dft_inplace<N2>(X);
#pragma unroll
        for (int r = 0; r < N2; ++r) out[q * N2 + r] = X[r];
      }
    } else {
      const float2* col = xbuf + (j % N1) * KROW + px;
      const int gg = j / N1;
      if constexpr (G == 2) {
        if (gg == 0) dif_fold<N1, 2, 0>(col, W, out);
        else dif_fold<N1, 2, 1>(col, W, out);
      } else {
        if (gg == 0) dif_fold<N1, 4, 0>(col, W, out);
        else if (gg == 1) dif_fold<N1, 4, 1>(col, W, out);
        else if (gg == 2) dif_fold<N1, 4, 2>(col, W, out);
        else dif_fold<N1, 4, 3>(col, W, out);
      }
      dft_inplace<N1>(out);
    }
    __syncthreads();
  }
};

}  // namespace tacaw
