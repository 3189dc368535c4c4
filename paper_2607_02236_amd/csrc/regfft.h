// In-register complex DFTs for one thread, FP32: sizes 2^k (radix 2) and
// 5 * 2^k (prime-factor split into 2^k- and 5-point DFTs).
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

// 5-point DFT X(k) = sum_n x(n) exp(-2 pi i n k / 5): with a1 = x1 + x4, a2 = x2 + x3,
// b1 = x1 - x4, b2 = x2 - x3, the pairs X(1), X(4) and X(2), X(3) share their real
// combinations x0 + c a1 + c' a2 and differ in the sign of i (s b1 +- s' b2).
__host__ __device__ __forceinline__ void dft5(float2& x0, float2& x1, float2& x2, float2& x3,
                                              float2& x4) {
  constexpr float c1 = (float)ct_cos2pi(1, 5), c2 = (float)ct_cos2pi(2, 5);
  constexpr float s1 = (float)ct_sin2pi(1, 5), s2 = (float)ct_sin2pi(2, 5);
  const float2 a1 = make_float2(x1.x + x4.x, x1.y + x4.y);
  const float2 a2 = make_float2(x2.x + x3.x, x2.y + x3.y);
  const float2 b1 = make_float2(x1.x - x4.x, x1.y - x4.y);
  const float2 b2 = make_float2(x2.x - x3.x, x2.y - x3.y);
  const float2 m1 = make_float2(__builtin_fmaf(c2, a2.x, __builtin_fmaf(c1, a1.x, x0.x)),
                                __builtin_fmaf(c2, a2.y, __builtin_fmaf(c1, a1.y, x0.y)));
  const float2 m2 = make_float2(__builtin_fmaf(c1, a2.x, __builtin_fmaf(c2, a1.x, x0.x)),
                                __builtin_fmaf(c1, a2.y, __builtin_fmaf(c2, a1.y, x0.y)));
  const float2 n1 = make_float2(__builtin_fmaf(s2, b2.x, s1 * b1.x), __builtin_fmaf(s2, b2.y, s1 * b1.y));
  const float2 n2 = make_float2(__builtin_fmaf(-s1, b2.x, s2 * b1.x), __builtin_fmaf(-s1, b2.y, s2 * b1.y));
  x0 = make_float2(x0.x + a1.x + a2.x, x0.y + a1.y + a2.y);
  // X(1) = m1 - i n1, X(4) = m1 + i n1, X(2) = m2 - i n2, X(3) = m2 + i n2
  x1 = make_float2(m1.x + n1.y, m1.y - n1.x);
  x4 = make_float2(m1.x - n1.y, m1.y + n1.x);
  x2 = make_float2(m2.x + n2.y, m2.y - n2.x);
  x3 = make_float2(m2.x - n2.y, m2.y + n2.x);
}

constexpr int inv_mod(int a, int m) {
  for (int x = 1; x < m; ++x)
    if ((a * x) % m == 1) return x;
  return 1;
}

// In-place forward DFT of N values in natural order (input and output): radix-2
// for powers of two; for N = 5 P (P a power of two, coprime to 5) the
// prime-factor (Good-Thomas) split needs no twiddles: x(n) with
// n = (5 n_p + P n_q) mod N goes through P-point DFTs over n_p and 5-point DFTs
// over n_q, and lands at k = (5 (5^-1 mod P) k_p + P (P^-1 mod 5) k_q) mod N.
template <int N>
__host__ __device__ __forceinline__ void dft_inplace(float2 (&a)[N]) {
  if constexpr ((N & (N - 1)) == 0) {
    static_assert(N >= 2, "size");
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
  } else {
    constexpr int Q = 5, P = N / Q;
    static_assert(N % Q == 0 && (P & (P - 1)) == 0 && P >= 1, "N = 5 * 2^k");
    float2 b[Q][P];  // b[n_q][n_p]
#pragma unroll
    for (int nq = 0; nq < Q; ++nq)
#pragma unroll
      for (int np = 0; np < P; ++np) b[nq][np] = a[(Q * np + P * nq) % N];
    if constexpr (P > 1) {
#pragma unroll
      for (int nq = 0; nq < Q; ++nq) dft_inplace<P>(b[nq]);
    }
#pragma unroll
    for (int kp = 0; kp < P; ++kp) dft5(b[0][kp], b[1][kp], b[2][kp], b[3][kp], b[4][kp]);
    constexpr int ep = Q * (P > 1 ? inv_mod(Q % P, P) : 0), eq = P * inv_mod(P % Q, Q);
#pragma unroll
    for (int kq = 0; kq < Q; ++kq)
#pragma unroll
      for (int kp = 0; kp < P; ++kp) a[(ep * kp + eq * kq) % N] = b[kq][kp];
  }
}

// Pass 2 for N2 > N1: the N2-point DFT of one k1 is shared by G = N2 / N1
// threads. Thread g computes the outputs k2 = G r + g (r < N1) from
//   y[n] = W_{N2}^{n g} sum_{j < G} A[n + N1 j] W_G^{j g},  X = DFT_{N1}(y),
// i.e. one decimation-in-frequency stage folded into the loads, so no second
// exchange is needed. G and g are compile-time here (g is uniform per wave).
// c(n) = A[n] (an accessor: registers or LDS). dif_fold_part computes the
// folded sums y[n] for N0 <= n < NE without the final twiddles.
template <int N1, int G, int g, int N0, int NE, typename Col>
__device__ __forceinline__ void dif_fold_part(const Col& c, float2 (&y)[N1]) {
#pragma unroll
  for (int n = N0; n < NE; ++n) {
    float2 s = c(n);
#pragma unroll
    for (int j = 1; j < G; ++j) {
      const float2 x = c(n + N1 * j);
      // rotate by W_G^{j g} = exp(-2 pi i j g / G)
      const int e = (j * g) % G;
      float2 t;
      if (G == 2) {
        t = e == 0 ? x : make_float2(-x.x, -x.y);
      } else {  // G == 4
        t = e == 0 ? x : e == 1 ? make_float2(x.y, -x.x) : e == 2 ? make_float2(-x.x, -x.y)
                                                           : make_float2(-x.y, x.x);
      }
      s.x += t.x;
      s.y += t.y;
    }
    y[n] = s;
  }
}
template <int N1, int G, int g, typename Col>
__device__ __forceinline__ void dif_combine(const Col& c, float2 (&y)[N1]) {
  dif_fold_part<N1, G, g, 0, N1>(c, y);
  if constexpr (g != 0) TwiddleRow<N1, N1 * G, g>::apply(y);
}

}  // namespace tacaw
