// exx_fft.hpp -- register-level DFT building blocks for gfx950.
//
// The Poisson solves of the exchange operator are FFT convolutions
// (arXiv:1712.07973, Section 2.1.2).  Every transform in this library is a
// batch of 1-D lines of length L = L1 * L2 with L1, L2 <= 16, done in two
// register steps with one LDS exchange between them (a two-level
// Cooley-Tukey split):
//
//   X[q1 + L1 q2] = sum_t w_L2^{t q2} [ w_L^{t q1} sum_k1 x[t + L2 k1] w_L1^{k1 q1} ]
//
// Step 1 (per t): DFT_L1 over k1, twiddle w_L^{t q1}.  Step 2 (per q1): DFT_L2
// over t.  The inverse runs the two steps in reverse order with conjugate
// roots, so it can start from the natural-order spectrum a thread holds.
//
// The small DFTs are fully unrolled at compile time by a mixed-radix
// recursion (smallest prime first); their roots of unity are compile-time
// constants computed by a constexpr Taylor series after exact integer
// range reduction.  Twiddles between the two steps come from tables built in
// FP64 on the host and rounded once.
#pragma once

#include <hip/hip_runtime.h>

namespace exx {

template <typename T>
struct cpx {
  T x, y;
};

template <typename T>
__host__ __device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> cmulc(cpx<T> a, cpx<T> b) {  // a * conj(b)
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) {
  return {a.x + b.x, a.y + b.y};
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) {
  return {a.x - b.x, a.y - b.y};
}

// ---------------------------------------------------------------------------
// compile-time roots of unity
// ---------------------------------------------------------------------------
constexpr double kHalfPi = 1.57079632679489661923132169163975144;

constexpr double taylor_sin(double x) {  // |x| <= pi/4
  double term = x, sum = x, x2 = x * x;
  for (int k = 1; k < 14; ++k) {
    term *= -x2 / double((2 * k) * (2 * k + 1));
    sum += term;
  }
  return sum;
}
constexpr double taylor_cos(double x) {  // |x| <= pi/4
  double term = 1.0, sum = 1.0, x2 = x * x;
  for (int k = 1; k < 14; ++k) {
    term *= -x2 / double((2 * k - 1) * (2 * k));
    sum += term;
  }
  return sum;
}
// cos and sin of 2 pi num / den, num >= 0, den > 0
constexpr double cos_2pi(long num, long den) {
  long a = (4 * (num % den));  // angle in quarter turns = a / den
  long q = a / den;            // quadrant 0..3
  long r = a - q * den;        // remainder: phi = (pi/2) r / den in [0, pi/2)
  double c = 0, s = 0;
  if (2 * r <= den) {
    double phi = kHalfPi * double(r) / double(den);
    c = taylor_cos(phi);
    s = taylor_sin(phi);
  } else {
    double phi = kHalfPi * double(den - r) / double(den);
    c = taylor_sin(phi);
    s = taylor_cos(phi);
  }
  return q == 0 ? c : q == 1 ? -s : q == 2 ? -c : s;
}
constexpr double sin_2pi(long num, long den) {
  long a = (4 * (num % den));
  long q = a / den;
  long r = a - q * den;
  double c = 0, s = 0;
  if (2 * r <= den) {
    double phi = kHalfPi * double(r) / double(den);
    c = taylor_cos(phi);
    s = taylor_sin(phi);
  } else {
    double phi = kHalfPi * double(den - r) / double(den);
    c = taylor_sin(phi);
    s = taylor_cos(phi);
  }
  return q == 0 ? s : q == 1 ? c : q == 2 ? -s : -c;
}

constexpr int smallest_prime_factor(int r) {
  for (int p = 2; p * p <= r; ++p)
    if (r % p == 0) return p;
  return r;
}

// w_R^k = exp(DIR * 2 pi i k / R), DIR = -1 forward, +1 inverse.
template <int R, int K, int DIR, typename T>
__host__ __device__ __forceinline__ cpx<T> twiddle_const(cpx<T> v) {
  constexpr int k = ((K % R) + R) % R;
  if constexpr (k == 0) {
    return v;
  } else if constexpr (2 * k == R) {
    return {-v.x, -v.y};
  } else if constexpr (4 * k == R) {  // DIR * i
    return DIR < 0 ? cpx<T>{v.y, -v.x} : cpx<T>{-v.y, v.x};
  } else if constexpr (4 * k == 3 * R) {  // -DIR * i
    return DIR < 0 ? cpx<T>{-v.y, v.x} : cpx<T>{v.y, -v.x};
  } else if constexpr (8 * k == R || 8 * k == 3 * R || 8 * k == 5 * R || 8 * k == 7 * R) {
    // (+-1 +- i)/sqrt2: two adds and two multiplies
    constexpr T c = T(cos_2pi(k, R));
    constexpr T s = T(DIR * sin_2pi(k, R));
    constexpr T a = c;  // |c| == |s|
    constexpr T sg = (c > 0) == (s > 0) ? T(1) : T(-1);
    // (x + i y)(c + i s) with s = sg * c: re = c (x - sg y), im = c (sg x + y)
    return {a * (v.x - sg * v.y), a * (sg * v.x + v.y)};
  } else {
    constexpr T c = T(cos_2pi(k, R));
    constexpr T s = T(DIR * sin_2pi(k, R));
    return {v.x * c - v.y * s, v.x * s + v.y * c};
  }
}

// ---------------------------------------------------------------------------
// prime-size DFTs
// ---------------------------------------------------------------------------
template <int P, int DIR, typename T>
struct PrimeDft;

template <int DIR, typename T>
struct PrimeDft<2, DIR, T> {
  __host__ __device__ __forceinline__ static void run(cpx<T>* v) {
    cpx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

// odd prime: y_k = x0 + sum_m [a_m cos(2pi mk/P) + i DIR b_m sin(2pi mk/P)],
// a_m = x_m + x_{P-m}, b_m = x_m - x_{P-m}
template <int P, int DIR, typename T>
struct PrimeDft {
  static_assert(P % 2 == 1, "odd prime expected");
  __host__ __device__ __forceinline__ static void run(cpx<T>* v) {
    constexpr int H = (P - 1) / 2;
    cpx<T> a[H], b[H];
    cpx<T> x0 = v[0];
    cpx<T> y0 = x0;
#pragma unroll
    for (int m = 1; m <= H; ++m) {
      a[m - 1] = cadd(v[m], v[P - m]);
      b[m - 1] = csub(v[m], v[P - m]);
      y0 = cadd(y0, a[m - 1]);
    }
    cpx<T> out[P];
    out[0] = y0;
    run_k<1>(x0, a, b, out);
#pragma unroll
    for (int k = 0; k < P; ++k) v[k] = out[k];
  }
  template <int K>
  __host__ __device__ __forceinline__ static void run_k(cpx<T> x0, const cpx<T>* a, const cpx<T>* b,
                                               cpx<T>* out) {
    if constexpr (K <= (P - 1) / 2) {
      cpx<T> A = x0, B = {T(0), T(0)};
      accumulate<K, 1>(A, B, a, b);
      // i * DIR * B
      cpx<T> iB = DIR < 0 ? cpx<T>{B.y, -B.x} : cpx<T>{-B.y, B.x};
      out[K] = cadd(A, iB);
      out[P - K] = csub(A, iB);
      run_k<K + 1>(x0, a, b, out);
    }
  }
  template <int K, int M>
  __host__ __device__ __forceinline__ static void accumulate(cpx<T>& A, cpx<T>& B, const cpx<T>* a,
                                                    const cpx<T>* b) {
    if constexpr (M <= (P - 1) / 2) {
      constexpr T c = T(cos_2pi(long(M) * K, P));
      constexpr T s = T(sin_2pi(long(M) * K, P));
      A.x += a[M - 1].x * c;
      A.y += a[M - 1].y * c;
      B.x += b[M - 1].x * s;
      B.y += b[M - 1].y * s;
      accumulate<K, M + 1>(A, B, a, b);
    }
  }
};

// ---------------------------------------------------------------------------
// mixed-radix DFT of size R in registers, natural order in and out (in place)
// ---------------------------------------------------------------------------
template <int R, int DIR, typename T>
struct Dft {
  static constexpr int P = smallest_prime_factor(R);
  static constexpr int Q = R / P;

  __host__ __device__ __forceinline__ static void run(cpx<T>* v) {
    if constexpr (R == 1) {
      return;
    } else if constexpr (Q == 1) {
      PrimeDft<P, DIR, T>::run(v);
    } else {
      cpx<T> sub[P][Q];
#pragma unroll
      for (int p = 0; p < P; ++p) {
#pragma unroll
        for (int q = 0; q < Q; ++q) sub[p][q] = v[p + P * q];
        Dft<Q, DIR, T>::run(sub[p]);
      }
      twiddle_rows<1>(sub);
#pragma unroll
      for (int k1 = 0; k1 < Q; ++k1) {
        cpx<T> t[P];
#pragma unroll
        for (int p = 0; p < P; ++p) t[p] = sub[p][k1];
        Dft<P, DIR, T>::run(t);
#pragma unroll
        for (int k2 = 0; k2 < P; ++k2) v[k1 + Q * k2] = t[k2];
      }
    }
  }
  template <int p>
  __host__ __device__ __forceinline__ static void twiddle_rows(cpx<T> (&sub)[P][Q]) {
    if constexpr (p < P) {
      twiddle_cols<p, 1>(sub);
      twiddle_rows<p + 1>(sub);
    }
  }
  template <int p, int k1>
  __host__ __device__ __forceinline__ static void twiddle_cols(cpx<T> (&sub)[P][Q]) {
    if constexpr (k1 < Q) {
      sub[p][k1] = twiddle_const<R, p * k1, DIR, T>(sub[p][k1]);
      twiddle_cols<p, k1 + 1>(sub);
    }
  }
};

// ---------------------------------------------------------------------------
// line-length factorisation L = L1 * L2 used by every transform
// ---------------------------------------------------------------------------
template <int L>
struct Split {
  static constexpr int L2 = (L > 128) ? 16 : (L >= 16 ? 8 : L);
  static constexpr int L1 = L / L2;
  static_assert(L1 * L2 == L, "unsupported line length");
  static_assert(L1 <= 16 && L2 <= 16, "unsupported line length");
};

}  // namespace exx
