// Complex helpers and register-resident DFTs for gfx950 kernels.
//
// A length-R DFT (R = 2^k <= 64) runs entirely in VGPRs: radix-4
// decimation-in-time steps with radix-2 for the odd power, twiddles folded
// to compile-time constants (trivial ones become sign swaps).  The kernels
// build their N-point transforms from two such register DFTs and one LDS
// exchange (four-step decomposition).
#pragma once
#include <hip/hip_runtime.h>
#include <type_traits>
#include <utility>

#define CPRA_INLINE __attribute__((always_inline))

namespace cpra {

template <typename R> struct vec2;
template <> struct vec2<float> { using type = float2; };
template <> struct vec2<double> { using type = double2; };
template <typename R> using cx = typename vec2<R>::type;

template <typename C> __device__ __forceinline__ C mk(decltype(C{}.x) a, decltype(C{}.x) b) {
  C r; r.x = a; r.y = b; return r;
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return mk<C>(a.x + b.x, a.y + b.y); }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return mk<C>(a.x - b.x, a.y - b.y); }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  return mk<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename C> __device__ __forceinline__ C cmulc(C a, C b) {  // a * conj(b)
  return mk<C>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename C> __device__ __forceinline__ C conj(C a) { return mk<C>(a.x, -a.y); }
template <typename C> __device__ __forceinline__ C cscale(C a, decltype(C{}.x) s) { return mk<C>(a.x * s, a.y * s); }
// multiply by i^(-1) (SIGN<0: -i) or i (SIGN>0)
template <int SIGN, typename C> __device__ __forceinline__ C mul_i(C a) {
  if constexpr (SIGN < 0) return mk<C>(a.y, -a.x);
  else return mk<C>(-a.y, a.x);
}

// ---- compile-time cos/sin of 2*pi*k/R (Taylor series after octant reduction)
constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double taylor_sin(double x) {
  double term = x, sum = x;
  for (int i = 1; i < 14; ++i) { term *= -x * x / ((2 * i) * (2 * i + 1)); sum += term; }
  return sum;
}
constexpr double taylor_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int i = 1; i < 14; ++i) { term *= -x * x / ((2 * i - 1) * (2 * i)); sum += term; }
  return sum;
}
// cos and sin of 2*pi*k/R with exact symmetry reduction (k, R integers)
constexpr double cos2pi(long k, long R) {
  k %= R; if (k < 0) k += R;
  if (8 * k > 4 * R) return cos2pi(R - k, R);               // cos(2pi - x) = cos x
  if (8 * k > 2 * R) return -cos2pi(R / 2 - k, R) * ((R % 2) ? 1 : 1);  // cos(pi - x) = -cos x
  if (8 * k > R) return taylor_sin(2 * kPi * (double)(R - 4 * k) / (4.0 * R));  // cos(pi/2 - y) = sin y
  return taylor_cos(2 * kPi * (double)k / (double)R);
}
constexpr double sin2pi(long k, long R) { return cos2pi(4 * k - R, 4 * R); }   // sin x = cos(x - pi/2)

// x * exp(SIGN * 2*pi*i * K / R) with K, R compile-time
template <int SIGN, int K, int R, typename C>
__device__ __forceinline__ C twc(C x) {
  constexpr int k = ((K % R) + R) % R;
  using T = decltype(C{}.x);
  if constexpr (k == 0) return x;
  else if constexpr (4 * k == R) return mul_i<SIGN>(x);
  else if constexpr (2 * k == R) return mk<C>(-x.x, -x.y);
  else if constexpr (4 * k == 3 * R) return mul_i<-SIGN>(x);
  else if constexpr (8 * k == R || 8 * k == 3 * R || 8 * k == 5 * R || 8 * k == 7 * R) {
    constexpr T h = (T)0.70710678118654752440084436210484904;
    constexpr T c = (T)cos2pi(k, R) > 0 ? h : -h;
    constexpr T s = (T)(SIGN * sin2pi(k, R)) > 0 ? h : -h;
    // (x.x + i x.y)(c + i s) with |c| = |s| = h: h * ((+-x.x -+ x.y) + i(...))
    T re = (c > 0 ? x.x : -x.x) - (s > 0 ? x.y : -x.y);
    T im = (s > 0 ? x.x : -x.x) + (c > 0 ? x.y : -x.y);
    return mk<C>(re * h, im * h);
  } else {
    constexpr T c = (T)cos2pi(k, R);
    constexpr T s = (T)(SIGN * sin2pi(k, R));
    return mk<C>(x.x * c - x.y * s, x.x * s + x.y * c);
  }
}

template <int I, int N, typename F>
__device__ __forceinline__ void sfor(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    sfor<I + 1, N>(f);
  }
}

// In-register DFT of R points, natural order in and out:
//   x[k] <- sum_j x[j] exp(SIGN*2*pi*i*j*k/R)
template <int R, int SIGN, typename C>
__device__ __forceinline__ void dft(C* x) {
  if constexpr (R == 1) {
    return;
  } else if constexpr (R == 2) {
    C a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  } else if constexpr (R == 3) {
    // w = exp(SIGN 2 pi i / 3) = -1/2 + SIGN i sqrt(3)/2
    using T = decltype(C{}.x);
    constexpr T h = (T)0.86602540378443864676372317075293618;   // sqrt(3)/2
    const C a = x[0], b = x[1], c = x[2];
    const C s = cadd(b, c);
    const C m = mk<C>(a.x - (T)0.5 * s.x, a.y - (T)0.5 * s.y);
    const C d = mul_i<SIGN>(csub(b, c));
    x[0] = cadd(a, s);
    x[1] = mk<C>(m.x + h * d.x, m.y + h * d.y);
    x[2] = mk<C>(m.x - h * d.x, m.y - h * d.y);
  } else if constexpr (R % 4 == 0 && R >= 4 && (R == 4 || R >= 16)) {
    constexpr int Q = R / 4;
    C s0[Q], s1[Q], s2[Q], s3[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      s0[i] = x[4 * i]; s1[i] = x[4 * i + 1]; s2[i] = x[4 * i + 2]; s3[i] = x[4 * i + 3];
    }
    dft<Q, SIGN>(s0); dft<Q, SIGN>(s1); dft<Q, SIGN>(s2); dft<Q, SIGN>(s3);
    sfor<0, Q>([&](auto kk) CPRA_INLINE {
      constexpr int k = decltype(kk)::value;
      C t0 = s0[k];
      C t1 = twc<SIGN, k, R>(s1[k]);
      C t2 = twc<SIGN, 2 * k, R>(s2[k]);
      C t3 = twc<SIGN, 3 * k, R>(s3[k]);
      C a = cadd(t0, t2), b = csub(t0, t2);
      C c = cadd(t1, t3), d = mul_i<SIGN>(csub(t1, t3));
      x[k] = cadd(a, c);
      x[k + Q] = cadd(b, d);
      x[k + 2 * Q] = csub(a, c);
      x[k + 3 * Q] = csub(b, d);
    });
  } else {
    constexpr int H = R / 2;
    C e[H], o[H];
#pragma unroll
    for (int i = 0; i < H; ++i) { e[i] = x[2 * i]; o[i] = x[2 * i + 1]; }
    dft<H, SIGN>(e); dft<H, SIGN>(o);
    sfor<0, H>([&](auto kk) CPRA_INLINE {
      constexpr int k = decltype(kk)::value;
      C t = twc<SIGN, k, R>(o[k]);
      x[k] = cadd(e[k], t);
      x[k + H] = csub(e[k], t);
    });
  }
}

}  // namespace cpra
