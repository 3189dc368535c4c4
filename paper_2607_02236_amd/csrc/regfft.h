// In-register complex DFTs of size 8, 16 and 32 for one thread, FP32.
//
// Radix-2 decimation in time on a fully unrolled register array: the input is
// read in bit-reversed order (free: register renaming), every butterfly's
// twiddle exp(-2 pi i K / (2 SPAN)) is a compile-time constant, and twiddles
// of 1, -i and (+-1 - i)/sqrt(2) are applied without a general complex
// multiply. The sign is the forward one, X(m) = sum_t x(t) exp(-2 pi i m t / N);
// the inverse (exp(+...)) is obtained by conjugating input and output.
#pragma once

#include <hip/hip_runtime.h>

namespace tacaw {

// ---- compile-time trigonometry (Taylor series after octant reduction) ----
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double ct_sin_small(double x) {  // |x| <= pi/4
  double x2 = x * x, term = x, sum = x;
  for (int n = 1; n < 14; ++n) {
    term *= -x2 / double((2 * n) * (2 * n + 1));
    sum += term;
  }
  return sum;
}
constexpr double ct_cos_small(double x) {  // |x| <= pi/4
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int n = 1; n < 14; ++n) {
    term *= -x2 / double((2 * n - 1) * (2 * n));
    sum += term;
  }
  return sum;
}
// cos and sin of 2 pi k / n for integers k, n > 0
constexpr double ct_cos2pi(long k, long n) {
  k %= n;
  if (k < 0) k += n;
  long q = (4 * k) / n;       // quadrant
  long r = 4 * k - q * n;     // angle within quadrant = (pi/2) r / n
  double c = 0.0, s = 0.0;
  if (2 * r <= n) {
    double a = (kPi / 2.0) * double(r) / double(n);
    c = ct_cos_small(a);
    s = ct_sin_small(a);
  } else {
    double b = (kPi / 2.0) * double(n - r) / double(n);
    c = ct_sin_small(b);
    s = ct_cos_small(b);
  }
  return q == 0 ? c : q == 1 ? -s : q == 2 ? -c : s;
}
// sin(2 pi k / n) = cos(2 pi (4k - n) / (4n))
constexpr double ct_sin2pi(long k, long n) { return ct_cos2pi(4 * k - n, 4 * n); }

// ---- butterflies ---------------------------------------------------------
__host__ __device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// (a, b) <- (a + w b, a - w b) with w = exp(-2 pi i K / M) (compile-time).
// A general twiddle is applied in factored form, w b = f u with f = cos (or sin)
// and u = b rotated by the tangent (or cotangent) of the angle, so the butterfly
// is 2 + 4 fused multiply-adds instead of 4 + 4 operations; |tan| <= 1 keeps the
// rounding of u at one unit of u.
template <int K, int M>
__host__ __device__ __forceinline__ void bfly(float2& a, float2& b) {
  constexpr int Kr = K % M;
  const float2 v = a;
  if constexpr (Kr == 0) {
    a = make_float2(v.x + b.x, v.y + b.y);
    b = make_float2(v.x - b.x, v.y - b.y);
  } else if constexpr (4 * Kr == M) {  // w = -i: w b = (b.y, -b.x)
    a = make_float2(v.x + b.y, v.y - b.x);
    b = make_float2(v.x - b.y, v.y + b.x);
  } else {
    constexpr double cd = ct_cos2pi(Kr, M);
    constexpr double sd = -ct_sin2pi(Kr, M);  // w = cd + i sd
    constexpr bool by_cos = (cd < 0 ? -cd : cd) >= (sd < 0 ? -sd : sd);
    float2 u;
    float f;
    if constexpr (by_cos) {  // w b = cd (b + i (sd/cd) b)
      constexpr float r = (float)(sd / cd);
      f = (float)cd;
      u = make_float2(__builtin_fmaf(-r, b.y, b.x), __builtin_fmaf(r, b.x, b.y));
    } else {  // w b = sd ((cd/sd) b + i b)
      constexpr float r = (float)(cd / sd);
      f = (float)sd;
      u = make_float2(__builtin_fmaf(r, b.x, -b.y), __builtin_fmaf(r, b.y, b.x));
    }
    a = make_float2(__builtin_fmaf(f, u.x, v.x), __builtin_fmaf(f, u.y, v.y));
    b = make_float2(__builtin_fmaf(-f, u.x, v.x), __builtin_fmaf(-f, u.y, v.y));
  }
}

// x <- x * exp(-2 pi i K / M) with K, M compile-time
template <int K, int M>
__host__ __device__ __forceinline__ void rot(float2& x) {
  constexpr int Kr = K % M;
  if constexpr (Kr == 0) {
  } else if constexpr (4 * Kr == M) {
    x = make_float2(x.y, -x.x);
  } else if constexpr (2 * Kr == M) {
    x = make_float2(-x.x, -x.y);
  } else if constexpr (4 * Kr == 3 * M) {
    x = make_float2(-x.y, x.x);
  } else {
    constexpr float c = (float)ct_cos2pi(Kr, M);
    constexpr float s = -(float)ct_sin2pi(Kr, M);
    x = make_float2(c * x.x - s * x.y, c * x.y + s * x.x);
  }
}

// y[n] <- y[n] * exp(-2 pi i n G / M) for n < N (compile-time twiddles)
template <int N, int M, int G, int n = 1>
struct TwiddleRow {
  static __host__ __device__ __forceinline__ void apply(float2 (&y)[N]) {
    if constexpr (n < N) {
      rot<(n * G) % M, M>(y[n]);
      TwiddleRow<N, M, G, n + 1>::apply(y);
    }
  }
};

template <int N>
constexpr int bitrev(int i) {
  int r = 0;
  for (int b = 1; b < N; b <<= 1) {
    r = (r << 1) | (i & 1);
    i >>= 1;
  }
  return r;
}

template <int N, int SPAN, int K>
struct FftStage {
  static __host__ __device__ __forceinline__ void run(float2 (&a)[N]) {
    if constexpr (K < SPAN) {
#pragma unroll
      for (int g = 0; g < N; g += 2 * SPAN) bfly<K, 2 * SPAN>(a[g + K], a[g + K + SPAN]);
      FftStage<N, SPAN, K + 1>::run(a);
    }
  }
};

template <int N, int SPAN>
struct FftStages {
  static __host__ __device__ __forceinline__ void run(float2 (&a)[N]) {
    if constexpr (SPAN < N) {
      FftStage<N, SPAN, 0>::run(a);
      FftStages<N, 2 * SPAN>::run(a);
    }
  }
};

// In-place forward DFT of N values in natural order (input and output).
template <int N>
__host__ __device__ __forceinline__ void dft_inplace(float2 (&a)[N]) {
  static_assert((N & (N - 1)) == 0 && N >= 2, "power of two");
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const int j = bitrev<N>(i);
    if (j > i) {
      float2 t = a[i];
      a[i] = a[j];
      a[j] = t;
    }
  }
  FftStages<N, 1>::run(a);
}

}  // namespace tacaw
