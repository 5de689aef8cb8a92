// Device kernels of the CPRA hot path (gfx950).
//
// State per angle n (all in HBM, laid out by the host plan):
//   P    [N][N/2] complex  row spectrum S[z][u] = sum_t g[z][t] e^{-2 pi i u t/N}
//                          of the current real iterate, half spectrum:
//                          P[z][0] = S[z][0] + i S[z][N/2] (both real),
//                          P[z][j] = S[z][j] for 1 <= j < N/2
//   Pmid [N][N/2] complex  same packing, after column FFT / modulus / column IFFT
//   g    [N][N] real       real-space iterate, centred (two copies, ping-pong at
//                          episode boundaries)
//   A2   [N][N/2] pairs    (A(q), A(-q)) in native frequency order; for column 0
//                          the pair is (A(w,0), A(w,N/2))
//   mask [N][T][MW] u32    support bits in the row pass's thread order
//
// One iteration = column pass + row pass.  Because g is real, F2(g) is
// Hermitian and Re F2^-1 of the projected spectrum equals F2^-1 of its
// Hermitian part, which is pointwise: G''(q) = (P_q(G) + P_-q(G))/2 with
// P_p(G) = A(p) G/|G| (A(p) >= 0) or G (unmeasured).  So only N/2 packed
// columns are transformed and stored, and no real-space shift is needed:
// the modulus projection commutes with the (-1)^(w+u) factor of a centred
// origin except at G = 0, where the zero-phase value takes that sign.
#pragma once
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "cx.hpp"

namespace cpra {

// ---------------------------------------------------------------- configs
// Column transform of length N = R1 * R2: R1 threads per column, R2 values each.
// S > 1: the R1-point step-2 DFT is shared by S = 2 neighbouring threads
// (an R1/2-point DFT in registers + one radix-2 butterfly across lanes).
template <int N> struct ColCfg;
template <> struct ColCfg<64> { static constexpr int R1 = 8, R2 = 8, C = 16, S = 1; };
template <> struct ColCfg<128> { static constexpr int R1 = 8, R2 = 16, C = 16, S = 1; };
template <> struct ColCfg<256> { static constexpr int R1 = 16, R2 = 16, C = 16, S = 1; };
template <> struct ColCfg<192> { static constexpr int R1 = 8, R2 = 24, C = 16, S = 1; };
template <> struct ColCfg<384> { static constexpr int R1 = 8, R2 = 48, C = 16, S = 1; };
template <> struct ColCfg<512> { static constexpr int R1 = 32, R2 = 16, C = 8, S = 2; };
#ifndef CPRA_C1024
#define CPRA_C1024 8
#endif
template <> struct ColCfg<1024> { static constexpr int R1 = 64, R2 = 16, C = CPRA_C1024, S = 4; };

// Row half-spectrum transform of length L = N/2 = F1 * F2 (F1: frequency
// residue modulus, F2: space residue modulus).  T = F1 threads per row:
// thread t owns frequency class k1 = t (F2 values) and the space classes
// m2 = t + F1 jj (F2 values in all).  The real/complex pairing k <-> L-k
// pairs class t with class (F1 - t) mod F1, i.e. lane (F1 - t) mod F1 of the
// row group, reached with DPP lane moves.
template <int N> struct RowCfg;
template <> struct RowCfg<64> { static constexpr int F1 = 4, F2 = 8, RPB = 32; };
template <> struct RowCfg<128> { static constexpr int F1 = 8, F2 = 8, RPB = 8; };
template <> struct RowCfg<256> { static constexpr int F1 = 8, F2 = 16, RPB = 8; };
template <> struct RowCfg<192> { static constexpr int F1 = 4, F2 = 24, RPB = 32; };
template <> struct RowCfg<384> { static constexpr int F1 = 8, F2 = 24, RPB = 8; };
template <> struct RowCfg<512> { static constexpr int F1 = 16, F2 = 16, RPB = 8; };
template <> struct RowCfg<1024> { static constexpr int F1 = 16, F2 = 32, RPB = 8; };
// The row pass is compiled for two tile heights (rows per workgroup): RowCfg's and twice it; the
// autotuner measures both per shape.  RowRows<N, 0> is the default, RowRows<N, 1> the other.
template <int N, int V> struct RowRows {
  static constexpr int RPB = V == 0 ? RowCfg<N>::RPB : 2 * RowCfg<N>::RPB;
  static_assert(RowCfg<N>::F1 * RPB <= 256, "row workgroup size");
};

template <int N> struct RowGeom {
  static constexpr int L = N / 2;
  static constexpr int F1 = RowCfg<N>::F1, F2 = RowCfg<N>::F2, RPB = RowCfg<N>::RPB;
  static constexpr int T = F1;              // threads per row
  static constexpr int SPT = F2 / T;        // space classes per thread
  static constexpr int BITS = 2 * F2;       // support bits per thread per row
  static constexpr int MW = (BITS + 31) / 32;   // mask words per thread per row
  static constexpr int PADR = 1;
  // row stride of the LDS exchange (complex slots): >= F2 (F1 + 1) and = T mod 32,
  // so that both access patterns of a wave touch distinct 8-byte bank pairs
  static constexpr int RSTRIDE = F2 * (F1 + PADR) + ((T - (F2 * (F1 + PADR)) % 32) + 32) % 32;
  static_assert(F1 * F2 == L, "row decomposition");
  static_assert(F1 <= F2 && F2 % T == 0 && (F1 == 4 || F1 == 8 || F1 == 16), "row ownership");
};

template <int N> struct ColGeom {
  static constexpr int R1 = ColCfg<N>::R1, R2 = ColCfg<N>::R2, C = ColCfg<N>::C, S = ColCfg<N>::S;
  static constexpr int Q = (S == 1) ? R2 / R1 : 1;
  static constexpr int PADC = (S == 1) ? 1 : 16;   // paired layout: slab stride = 16 mod 32 slots
  static constexpr int TILES = (N / 2) / C;
  static_assert(R1 * R2 == N && (N / 2) % C == 0, "column decomposition");
  static_assert(S == 1 ? (R2 % R1 == 0) : ((S == 2 || S == 4) && R1 == S * R2), "step-2 ownership");
};

// x mod N into [0, N) (a mask for powers of two; sizes with a factor 3 take the remainder)
template <int N> __host__ __device__ __forceinline__ int wrapN(int x) {
  if constexpr ((N & (N - 1)) == 0) {
    return x & (N - 1);
  } else {
    const int r = x % N;
    return r < 0 ? r + N : r;
  }
}

// Storage of an angle's N x N/2 complex planes (P, Pmid) and of its amplitude
// pairs: chunks of CB packed columns, each chunk stored [z][CB] contiguously,
// so that a column-pass tile is one contiguous run of N*CB values (or, when
// the column pass takes half a chunk per workgroup, runs of CB/2) and a row
// pass block of rows reads CB-wide runs of consecutive rows.
#ifndef CPRA_PIX512
#define CPRA_PIX512 16
#endif
template <int N> struct PixCfg { static constexpr int CB = ColCfg<N>::C; };
template <> struct PixCfg<512> { static constexpr int CB = CPRA_PIX512; };
#ifndef CPRA_PIX1024
#define CPRA_PIX1024 8
#endif
template <> struct PixCfg<1024> { static constexpr int CB = CPRA_PIX1024; };
template <int N> __host__ __device__ __forceinline__ size_t pix(int z, int j) {
  constexpr int CB = PixCfg<N>::CB;
  return ((size_t)(j / CB) * N + z) * CB + (j % CB);
}

// First packed column of column-pass workgroup bx.  With CB = C one tile is
// one chunk.  With CB = 2C, the two halves of a chunk go to workgroups bx and
// bx + 8: the dispatcher deals consecutive workgroups round-robin to the 8
// XCDs, so both halves land on one XCD (one L2) and close together in time,
// and each 128-byte line of the chunk is fetched from HBM once.
template <int N> __device__ __forceinline__ int col_tile_start(int bx) {
  constexpr int C = ColCfg<N>::C, CB = PixCfg<N>::CB;
  if constexpr (CB == C) {
    return bx * C;
  } else {
    static_assert(CB == 2 * C && ((N / 2) / CB) % 8 == 0, "half-chunk tiles");
    const int g = bx >> 4, r = bx & 15;
    return (g * 8 + (r & 7)) * CB + (r >> 3) * C;
  }
}

// Space position (t index) of support bit b of thread tau in a row; -1 past the last bit.
template <int N> __host__ __device__ inline int mask_bit_t(int tau, int b) {
  using G = RowGeom<N>;
  if (b >= G::BITS) return -1;
  int e = b & 1, q = b >> 1;
  int j = q / G::F1, m1 = q % G::F1;
  int m = tau + G::T * j + G::F2 * m1;
  return 2 * m + e;
}

struct Coupling {   // per angle, used at episode boundaries
  int left, right;
  int mirror_left, mirror_right;
  double wl, w0, wr;
};

struct Tap {        // one term of Eq. 4 with 2K+1 taps: weight w on slot nb, t-mirrored or not
  int nb, mirror;
  double w;
};

// Eq. 4 with 2K+1 taps as a pass of its own at an episode boundary: for every listed slot,
// Pc = sum_k w_k M_k(P_nb_k) into Pout (packed half spectra, layout pix<N>; the mirror
// conjugates every entry but the packed DC/Nyquist column) and gc = sum_k w_k M_k(g_nb_k) into
// gout (M: t -> N - t).  grid (N rows, count); the neighbours of a listed slot are not listed
// when gin == gout.
template <int N, typename T>
__global__ void __launch_bounds__(256) k_couple_taps(const cx<T>* __restrict__ P, cx<T>* __restrict__ Pout,
                                                     const T* gin, T* gout, const int* __restrict__ alist,
                                                     const Tap* __restrict__ taps, int ntap) {
  using C = cx<T>;
  constexpr int H = N / 2, CB = PixCfg<N>::CB;
  const int z = blockIdx.x, ai = blockIdx.y;
  const int n = alist[ai];
  const Tap* tp = taps + (size_t)n * ntap;
  // spectra: row z holds H packed values; element j sits at pix(z, j)
  for (int j = threadIdx.x; j < H; j += blockDim.x) {
    const size_t e = pix<N>(z, j);
    C acc = mk<C>((T)0, (T)0);
    for (int q = 0; q < ntap; ++q) {
      const Tap t = tp[q];
      const C v = P[(size_t)t.nb * N * H + e];
      const T sy = (t.mirror && j != 0) ? (T)-t.w : (T)t.w;
      acc = mk<C>(acc.x + (T)t.w * v.x, acc.y + sy * v.y);
    }
    Pout[(size_t)n * N * H + e] = acc;
  }
  // objects: row z of the centred [z][t] plane
  for (int t = threadIdx.x; t < N; t += blockDim.x) {
    T acc = (T)0;
    for (int q = 0; q < ntap; ++q) {
      const Tap tq = tp[q];
      const T* x = gin + ((size_t)tq.nb * N + z) * N;
      acc += (T)tq.w * x[tq.mirror ? (wrapN<N>(N - t)) : t];
    }
    gout[((size_t)n * N + z) * N + t] = acc;
  }
  (void)CB;
}

// ---------------------------------------------------------------- amplitudes
// Plane stores and loads with an optional non-temporal cache hint.  Per size, which plane
// traffic takes the hint: the planes are streamed once per pass, and whether the hint pays was
// measured per size at 360 angles (it depends on how much of a pass's planes the last-level
// cache holds, and on the store pattern: at N = 192 hinted row stores double the row pass).
// Loads of the column pass's P and amplitudes and of the row pass's Pmid take no hint: the two
// workgroups that share each cache line find the second half in L2.
template <int N> struct NtPolicy {
  static constexpr bool col_store = (N == 384 || N >= 512);   // column pass: Pmid stores
  static constexpr bool row_store = (N == 256 || N >= 512);   // row pass: g and P stores
  static constexpr bool row_gload = (N == 256 || N >= 512);   // row pass: loads of the iterate g
};
typedef float cpra_f2v __attribute__((ext_vector_type(2)));
typedef double cpra_d2v __attribute__((ext_vector_type(2)));
template <bool NT>
__device__ __forceinline__ void st_plane(float2* p, float2 v) {
  if constexpr (NT) {
    cpra_f2v w = {v.x, v.y};
    __builtin_nontemporal_store(w, reinterpret_cast<cpra_f2v*>(p));
  } else {
    *p = v;
  }
}
template <bool NT>
__device__ __forceinline__ void st_plane(double2* p, double2 v) {
  if constexpr (NT) {
    cpra_d2v w = {v.x, v.y};
    __builtin_nontemporal_store(w, reinterpret_cast<cpra_d2v*>(p));
  } else {
    *p = v;
  }
}
template <bool NT>
__device__ __forceinline__ float2 ld_plane(const float2* p) {
  if constexpr (NT) {
    const cpra_f2v w = __builtin_nontemporal_load(reinterpret_cast<const cpra_f2v*>(p));
    return make_float2(w.x, w.y);
  } else {
    return *p;
  }
}
template <bool NT>
__device__ __forceinline__ double2 ld_plane(const double2* p) {
  if constexpr (NT) {
    const cpra_d2v w = __builtin_nontemporal_load(reinterpret_cast<const cpra_d2v*>(p));
    return make_double2(w.x, w.y);
  } else {
    return *p;
  }
}

template <typename AP> struct AmpIO;
template <> struct AmpIO<float2> {
  using real = float;
  using pair_t = float2;
  __device__ static pair_t raw(const float2* p) { return *p; }
  __device__ static float2 decode(pair_t v, float) { return v; }
  __device__ static float2 load(const float2* p, float) { return *p; }
};
template <> struct AmpIO<double2> {
  using real = double;
  using pair_t = double2;
  __device__ static pair_t raw(const double2* p) { return *p; }
  __device__ static double2 decode(pair_t v, double) { return v; }
  __device__ static double2 load(const double2* p, double) { return *p; }
};
template <> struct AmpIO<__half2> {
  using real = float;
  using pair_t = __half2;
  __device__ static pair_t raw(const __half2* p) { return *p; }
  __device__ static float2 decode(pair_t h, float s) {
    float2 v = __half22float2(h);
    v.x *= s; v.y *= s;
    return v;
  }
  __device__ static float2 load(const __half2* p, float s) { return decode(*p, s); }
};

__host__ __device__ inline uint64_t splitmix64_at(uint64_t seed, uint64_t c) {
  uint64_t z = seed + (c + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// ---------------------------------------------------------------- twiddles
// One FP64-generated table per plan, rounded to the working precision, laid
// out so that every thread reads its twiddles as consecutive pairs:
//   [0, N)            W_N^j
//   colf [a][c]       W_N^{a c}            (column pass, forward, R1 x R2)
//   coli [c][a]       conj W_N^{a c}       (column pass, inverse, R2 x R1)
//   rc2r [k1][m2]     conj W_L^{k1 m2}     (row pass C2R, F1 x F2, L = N/2)
//   rr2c [m2][k1]     W_L^{m2 k1}          (row pass R2C, F2 x F1)
//   rpp  [k1][k2]     W_N^{k1 + F1 k2}     (row pass real/complex pre/post-processing)
template <int N> struct TwLayout {
  static constexpr int L = N / 2;
  static constexpr int COLF = N, COLI = 2 * N, RC2R = 3 * N, RR2C = 3 * N + L, RPP = 3 * N + 2 * L;
  static constexpr int SIZE = 3 * N + 3 * L;
};

template <int N, typename T>
__global__ void k_twiddles(cx<T>* tw) {
  using TL = TwLayout<N>;
  constexpr int R1 = ColCfg<N>::R1, R2 = ColCfg<N>::R2, F1 = RowCfg<N>::F1, F2 = RowCfg<N>::F2;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= TL::SIZE) return;
  long e;          // exponent of W_N (exp(-2 pi i e / N))
  bool cj = false;
  if (i < TL::COLF) {
    e = i;
  } else if (i < TL::COLI) {
    const int r = i - TL::COLF; e = (long)(r / R2) * (r % R2);
  } else if (i < TL::RC2R) {
    // coli [c][a-slot]: a = slot (S = 1) or a = s + S a' with slot = s R1/S + a' (S = 2, 4)
    constexpr int S = ColCfg<N>::S;
    const int r = i - TL::COLI, c = r / R1, slot = r % R1;
    const int aa = (S == 1) ? slot : (slot / (R1 / S)) + S * (slot % (R1 / S));
    e = (long)c * aa; cj = true;
  } else if (i < TL::RR2C) {
    const int r = i - TL::RC2R; e = 2L * (r / F2) * (r % F2); cj = true;
  } else if (i < TL::RPP) {
    const int r = i - TL::RR2C; e = 2L * (r / F1) * (r % F1);
  } else {
    const int r = i - TL::RPP; e = (r / F2) + (long)F1 * (r % F2);
  }
  e %= N;
  double s, c;
  sincospi(-2.0 * (double)e / (double)N, &s, &c);
  tw[i] = mk<cx<T>>((T)c, (T)(cj ? -s : s));
}

// two consecutive complex values (16-byte load for FP32)
__device__ __forceinline__ void load_pair(const float2* p, float2& a, float2& b) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  a = make_float2(v.x, v.y);
  b = make_float2(v.z, v.w);
}
__device__ __forceinline__ void load_pair(const double2* p, double2& a, double2& b) {
  a = p[0];
  b = p[1];
}

// ---------------------------------------------------------------- prep
// Input preparation in three launches over all submitted angles:
//   k_prep_stats  : per (angle, 1/16 of the map) partial sum of I >= 0 (FP64),
//                   max sqrt(I), NaN/Inf flag
//   k_prep_final  : per angle, fixed-order sum -> den = sum A^2, binary16 scale
//   k_prep_encode : amplitude pairs (A(q), A(-q)) in native order and the
//                   support bits in the row pass's thread order
constexpr int kPrepBlocks = 16;

template <int N>
__global__ void __launch_bounds__(256) k_prep_stats(const float* __restrict__ I, int first, double* __restrict__ psum,
                                                    float* __restrict__ pmax, int* __restrict__ flags) {
  __shared__ double red[256];
  __shared__ float redm[256];
  __shared__ int redb[256];
  const int b = blockIdx.x, idx = blockIdx.y;
  const float* In = I + (size_t)idx * N * N;
  constexpr int per = N * N / kPrepBlocks;
  double acc = 0.0;
  float amax = 0.f;
  int bad = 0;
  for (int i = b * per + threadIdx.x; i < (b + 1) * per; i += blockDim.x) {
    const float v = In[i];
    if (!isfinite(v)) bad = 1;
    if (v >= 0.f) { acc += (double)v; amax = fmaxf(amax, sqrtf(v)); }
  }
  red[threadIdx.x] = acc;
  redm[threadIdx.x] = amax;
  redb[threadIdx.x] = bad;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      red[threadIdx.x] += red[threadIdx.x + s];
      redm[threadIdx.x] = fmaxf(redm[threadIdx.x], redm[threadIdx.x + s]);
      redb[threadIdx.x] |= redb[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int n = first + idx;
    psum[(size_t)n * kPrepBlocks + b] = red[0];
    pmax[(size_t)n * kPrepBlocks + b] = redm[0];
    if (redb[0]) atomicOr(flags, 1);
  }
}

template <typename T, typename AP>
__global__ void k_prep_final(int first, int count, const double* __restrict__ psum, const float* __restrict__ pmax,
                             double* __restrict__ den, T* __restrict__ ampscale) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int n = first + i;
  double s = 0.0;
  float m = 0.f;
  for (int b = 0; b < kPrepBlocks; ++b) {
    s += psum[(size_t)n * kPrepBlocks + b];
    m = fmaxf(m, pmax[(size_t)n * kPrepBlocks + b]);
  }
  den[n] = s;
  if constexpr (std::is_same<AP, __half2>::value) {
    int e = 0;
    frexpf(m > 0.f ? m : 1.f, &e);   // max A < 2^e
    ampscale[n] = ldexpf(1.f, e - 14);   // stored values < 2^14
  } else {
    ampscale[n] = (T)1;
  }
}

template <int N, typename T, typename AP>
__global__ void __launch_bounds__(256) k_prep_encode(const float* __restrict__ I, const uint8_t* __restrict__ sup,
                                                     int first, AP* __restrict__ A2, const T* __restrict__ ampscale,
                                                     uint32_t* __restrict__ maskw) {
  using G = RowGeom<N>;
  constexpr int H = N / 2, ROWS = 8;
  const int idx = blockIdx.y;
  const int n = first + idx;
  const int r0 = blockIdx.x * ROWS;
  const float* In = I + (size_t)idx * N * N;
  const uint8_t* Sn = sup + (size_t)idx * N * N;
  auto ampf = [&](int wn, int un) -> float {       // native (w, u) -> A, -1 if unmeasured
    const float v = In[((wn + H) % N) * N + ((un + H) % N)];
    return v >= 0.f ? sqrtf(v) : -1.f;
  };
  auto ampd = [&](int wn, int un) -> double {
    const float v = In[((wn + H) % N) * N + ((un + H) % N)];
    return v >= 0.f ? sqrt((double)v) : -1.0;
  };
  AP* An = A2 + (size_t)n * N * H;
  for (int i = threadIdx.x; i < ROWS * H; i += blockDim.x) {
    const int w = r0 + i / H, j = i % H;
    const int wm = (N - w) % N;
    if constexpr (std::is_same<AP, double2>::value) {
      double a, b;
      if (j == 0) { a = ampd(w, 0); b = ampd(w, H); }
      else { a = ampd(w, j); b = ampd(wm, N - j); }
      An[pix<N>(w, j)] = make_double2(a, b);
    } else {
      float a, b;
      if (j == 0) { a = ampf(w, 0); b = ampf(w, H); }
      else { a = ampf(w, j); b = ampf(wm, N - j); }
      if constexpr (std::is_same<AP, __half2>::value) {
        const float inv = 1.f / (float)ampscale[n];    // power of two: exact
        An[pix<N>(w, j)] = __floats2half2_rn(a >= 0.f ? a * inv : -1.f, b >= 0.f ? b * inv : -1.f);
      } else {
        An[pix<N>(w, j)] = make_float2(a, b);
      }
    }
  }
  uint32_t* Mn = maskw + (size_t)n * N * G::T * G::MW;
  for (int i = threadIdx.x; i < ROWS * G::T * G::MW; i += blockDim.x) {
    const int z = r0 + i / (G::T * G::MW);
    const int r = i % (G::T * G::MW);
    const int tau = r / G::MW, wd = r % G::MW;
    uint32_t word = 0;
    for (int b = 0; b < 32; ++b) {
      const int t = mask_bit_t<N>(tau, wd * 32 + b);
      if (t >= 0 && Sn[z * N + t]) word |= (1u << b);
    }
    Mn[(size_t)z * G::T * G::MW + r] = word;
  }
}

// ---------------------------------------------------------------- column pass
// Modulus projection of one Fourier value G with the amplitudes of q and -q
// (Hermitian part of the projected spectrum), scaled by `scale` (1/(2N^2)).
// a < 0 marks an unmeasured pixel (G kept); G = 0 takes the zero-phase value
// with the sign (-1)^(w+u) of the centred origin (`neg`).  `ew` weights the
// error terms (1/2 for the self-paired columns, whose -q is also in the column).
template <typename T> struct Proj;

template <> struct Proj<float> {
  template <bool ERR>
  static __device__ __forceinline__ float2 two(float2 G, float a1, float a2, bool neg, float scale, double& err,
                                               double ew) {
    const float m2 = fmaf(G.x, G.x, G.y * G.y);
    const bool nz = m2 >= 1.17549435e-38f;          // |G|^2 normal: rsq is exact to ~1 ulp there
    const float r = __builtin_amdgcn_rsqf(m2);       // 1/|G|
    const bool u1 = a1 >= 0.f, u2 = a2 >= 0.f;
    const float s = ((u1 ? a1 * r : 1.f) + (u2 ? a2 * r : 1.f)) * scale;
    const float z = ((u1 ? a1 : 0.f) + (u2 ? a2 : 0.f)) * (neg ? -scale : scale);
    if constexpr (ERR) {
      const double mag = nz ? (double)(m2 * r) : 0.0;
      const double d1 = mag - (double)a1, d2 = mag - (double)a2;
      err += ew * ((u1 ? d1 * d1 : 0.0) + (u2 ? d2 * d2 : 0.0));
    }
    return make_float2(nz ? G.x * s : z, nz ? G.y * s : 0.f);
  }
};

template <> struct Proj<double> {
  template <bool ERR>
  static __device__ __forceinline__ double2 two(double2 G, double a1, double a2, bool neg, double scale, double& err,
                                                double ew) {
    const double mag = sqrt(G.x * G.x + G.y * G.y);
    const bool nz = mag > 0.0;
    const double inv = nz ? 1.0 / mag : 0.0;
    const bool u1 = a1 >= 0.0, u2 = a2 >= 0.0;
    const double s = ((u1 ? a1 * inv : 1.0) + (u2 ? a2 * inv : 1.0)) * scale;
    const double z = ((u1 ? a1 : 0.0) + (u2 ? a2 : 0.0)) * (neg ? -scale : scale);
    if constexpr (ERR) {
      const double d1 = mag - a1, d2 = mag - a2;
      err += ew * ((u1 ? d1 * d1 : 0.0) + (u2 ? d2 * d2 : 0.0));
    }
    return make_double2(nz ? G.x * s : z, nz ? G.y * s : 0.0);
  }
};

template <int N, typename T, int NT = 256>
__device__ __forceinline__ void block_reduce_store(double v, double* out) {
  __shared__ double red[NT];
  const int nt = blockDim.x;
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = nt / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// Column pass.  One workgroup = C packed columns x N rows of one angle;
// R1 threads per column, R2 values each (four-step FFT along z).
// MODE 0: iteration (read P, optionally coupled; FFT_z; error; modulus
// projection; IFFT_z; write Pmid).  MODE 1: initial guess (generate the
// Hermitian part of (-1)^(w+u) A e^{i phi} / N^2, IFFT_z, write Pmid).
// The body runs slot n's tile blockIdx.x; errout receives the tile's FP64 error partial (ERR).
template <int N, typename T, typename AP, int MODE, bool ERR, bool CPL>
__device__ __forceinline__ void col_body(const cx<T>* __restrict__ P, cx<T>* __restrict__ Pmid,
                                         const AP* __restrict__ A2, const T* __restrict__ ampscale,
                                         const cx<T>* __restrict__ tw, int n, const Coupling* __restrict__ coup,
                                         int npd, double* __restrict__ errout, uint64_t seed) {
  using Gm = ColGeom<N>;
  using TL = TwLayout<N>;
  using C = cx<T>;
  constexpr int R1 = Gm::R1, R2 = Gm::R2, CC = Gm::C, Q = Gm::Q, H = N / 2;
  constexpr int LSTRIDE = R1 * CC + Gm::PADC;     // per c-slab
  __shared__ C lds[R2 * LSTRIDE];
  __shared__ C zl[(MODE == 0) ? N : 1];
  const int col = threadIdx.x % CC;
  const int a = threadIdx.x / CC;
  const int tile = blockIdx.x;
  static_assert(PixCfg<N>::CB == CC, "one chunk per tile");
  const int j0 = tile * CC;
  const int j = j0 + col;
  const size_t plane = (size_t)N * H;
  const T scale = (T)0.5 / ((T)N * (T)N);
  const int dn = n % npd;                  // data angle of slot n (slots r * npd + dn)
  const AP* An = A2 + (size_t)dn * plane;
  const T as = ampscale[dn];
  double err = 0.0;
  C g[R2];   // [q][d] after the forward transform (Q * R1 == R2)

  if constexpr (MODE == 0) {
    C v[R2];
    const C* Pn = P + (size_t)n * plane;
    sfor<0, R2>([&](auto bv) CPRA_INLINE {
      constexpr int b = decltype(bv)::value;
      v[b] = Pn[pix<N>(a + R1 * b, j)];
    });
    // amplitude pairs of the values this thread will hold after the forward
    // transform (w = a + R1 q + R2 d), fetched now so both HBM streams overlap
    constexpr bool PREFETCH = R2 <= 16;
    typename AmpIO<AP>::pair_t amp[PREFETCH ? R2 : 1];
    if (PREFETCH && j0 != 0) {
      sfor<0, R2>([&](auto iv) CPRA_INLINE {
        constexpr int i = decltype(iv)::value;
        constexpr int q = i / R1, d = i % R1;
        if constexpr (PREFETCH) amp[i] = AmpIO<AP>::raw(An + pix<N>(a + R1 * q + R2 * d, j));
      });
    }
    if (CPL) {
      const Coupling cp = coup[n];
      const T wl = (T)cp.wl, w0 = (T)cp.w0, wr = (T)cp.wr;
      const C* Pl = P + (size_t)cp.left * plane;
      const C* Pr = P + (size_t)cp.right * plane;
      // the seam mirror t -> -t conjugates a real row's spectrum; the packed
      // DC/Nyquist column (both real) is unchanged
      const T sl = (cp.mirror_left && j != 0) ? (T)-1 : (T)1;
      const T sr = (cp.mirror_right && j != 0) ? (T)-1 : (T)1;
      sfor<0, R2>([&](auto bv) CPRA_INLINE {
        constexpr int b = decltype(bv)::value;
        const C l = Pl[pix<N>(a + R1 * b, j)];
        const C r = Pr[pix<N>(a + R1 * b, j)];
        v[b] = mk<C>(w0 * v[b].x + wl * l.x + wr * r.x, w0 * v[b].y + (wl * sl) * l.y + (wr * sr) * r.y);
      });
    }
    // forward step 1: R2-point DFT over b, twiddle W_N^{a c}
    dft<R2, -1>(v);
    const C* tf = tw + TL::COLF + a * R2;
    sfor<0, R2 / 2>([&](auto iv) CPRA_INLINE {
      constexpr int c = 2 * decltype(iv)::value;
      C t0, t1;
      load_pair(tf + c, t0, t1);
      if (c != 0) v[c] = cmul(v[c], t0);
      v[c + 1] = cmul(v[c + 1], t1);
    });
    sfor<0, R2>([&](auto cv) CPRA_INLINE {
      constexpr int c = decltype(cv)::value;
      lds[c * LSTRIDE + a * CC + col] = v[c];
    });
    __syncthreads();
    // forward step 2: for c = a + R1 q, R1-point DFT over a' -> G[c + R2 d]
    sfor<0, Q>([&](auto qv) CPRA_INLINE {
      constexpr int q = decltype(qv)::value;
      const int c = a + R1 * q;
      sfor<0, R1>([&](auto av) CPRA_INLINE {
        constexpr int ap = decltype(av)::value;
        g[q * R1 + ap] = lds[c * LSTRIDE + ap * CC + col];
      });
      dft<R1, -1>(g + q * R1);
    });
    // modulus projection
    if (j0 != 0) {
      sfor<0, R2>([&](auto iv) CPRA_INLINE {
        constexpr int i = decltype(iv)::value;
        constexpr int q = i / R1, d = i % R1;
        const int w = a + R1 * q + R2 * d;
        typename AmpIO<AP>::pair_t raw;
        if constexpr (PREFETCH) raw = amp[i];
        else raw = AmpIO<AP>::raw(An + pix<N>(w, j));
        const auto pa = AmpIO<AP>::decode(raw, as);
        g[i] = Proj<T>::template two<ERR>(g[i], (T)pa.x, (T)pa.y, ((w + j) & 1) != 0, scale, err, 1.0);
      });
    } else {
      // tile 0 holds the packed column 0 = DC + i * Nyquist column: split
      // Z[w] into Ga = (Z[w] + conj Z[-w])/2 and Gb = (Z[w] - conj Z[-w])/(2i)
      // (pairing w with -w through LDS), project each, and pack again
      __syncthreads();
      if (col == 0) {
        sfor<0, R2>([&](auto iv) CPRA_INLINE {
          constexpr int i = decltype(iv)::value;
          constexpr int q = i / R1, d = i % R1;
          zl[a + R1 * q + R2 * d] = g[i];
        });
      }
      __syncthreads();
      sfor<0, R2>([&](auto iv) CPRA_INLINE {
        constexpr int i = decltype(iv)::value;
        constexpr int q = i / R1, d = i % R1;
        const int w = a + R1 * q + R2 * d;
        if (j != 0) {
          const auto pa = AmpIO<AP>::load(An + pix<N>(w, j), as);
          g[i] = Proj<T>::template two<ERR>(g[i], (T)pa.x, (T)pa.y, ((w + j) & 1) != 0, scale, err, 1.0);
        } else {
          const int wm = wrapN<N>(N - w);
          const C Z = g[i], Zm = zl[wm];
          const C Ga = mk<C>((T)0.5 * (Z.x + Zm.x), (T)0.5 * (Z.y - Zm.y));
          const C Gb = mk<C>((T)0.5 * (Z.y + Zm.y), (T)0.5 * (Zm.x - Z.x));
          const auto p0 = AmpIO<AP>::load(An + pix<N>(w, 0), as);     // (A(w,0), A(w,N/2))
          const auto pm = AmpIO<AP>::load(An + pix<N>(wm, 0), as);    // (A(-w,0), A(-w,N/2))
          // each of w, -w is visited once per column: half weight on the paired error terms
          const C Pa = Proj<T>::template two<ERR>(Ga, (T)p0.x, (T)pm.x, (w & 1) != 0, scale, err, 0.5);
          const C Pb = Proj<T>::template two<ERR>(Gb, (T)p0.y, (T)pm.y, ((w + H) & 1) != 0, scale, err, 0.5);
          g[i] = mk<C>(Pa.x - Pb.y, Pa.y + Pb.x);   // Ga'' + i Gb''
        }
      });
    }
  } else {
    // initial guess: Hermitian part of (-1)^{w+u} A e^{i phi}, scaled by 1/N^2
    auto phase = [&](int w, int u) CPRA_INLINE -> C {
      const uint64_t cnt = ((uint64_t)n * N + (uint64_t)w) * N + (uint64_t)u;
      const uint64_t r = splitmix64_at(seed, cnt) >> 40;
      double s, c;
      sincospi(2.0 * (double)r / 16777216.0, &s, &c);
      return mk<C>((T)c, (T)s);
    };
    sfor<0, R2>([&](auto iv) CPRA_INLINE {
      constexpr int i = decltype(iv)::value;
      constexpr int q = i / R1, d = i % R1;
      const int w = a + R1 * q + R2 * d;
      const int wm = wrapN<N>(N - w);
      C out;
      if (j != 0) {
        const auto pa = AmpIO<AP>::load(An + pix<N>(w, j), as);
        const T a1 = pa.x > (T)0 ? (T)pa.x : (T)0, a2 = pa.y > (T)0 ? (T)pa.y : (T)0;
        const C e1 = phase(w, j), e2 = conj(phase(wm, N - j));
        const T sg = ((w + j) & 1) ? -scale : scale;
        out = mk<C>(sg * (a1 * e1.x + a2 * e2.x), sg * (a1 * e1.y + a2 * e2.y));
      } else {
        const auto p0 = AmpIO<AP>::load(An + pix<N>(w, 0), as);
        const auto pm = AmpIO<AP>::load(An + pix<N>(wm, 0), as);
        const T a0 = p0.x > 0 ? (T)p0.x : (T)0, am0 = pm.x > 0 ? (T)pm.x : (T)0;
        const T aH = p0.y > 0 ? (T)p0.y : (T)0, amH = pm.y > 0 ? (T)pm.y : (T)0;
        const C e1 = phase(w, 0), e2 = conj(phase(wm, 0));
        const C f1 = phase(w, H), f2 = conj(phase(wm, H));
        const T sa = (w & 1) ? -scale : scale, sb = ((w + H) & 1) ? -scale : scale;
        const C Ga = mk<C>(sa * (a0 * e1.x + am0 * e2.x), sa * (a0 * e1.y + am0 * e2.y));
        const C Gb = mk<C>(sb * (aH * f1.x + amH * f2.x), sb * (aH * f1.y + amH * f2.y));
        out = mk<C>(Ga.x - Gb.y, Ga.y + Gb.x);
      }
      g[i] = out;
    });
  }

  // inverse step 1: for each owned c, R1-point IDFT over d, twiddle W_N^{-a' c}
  if constexpr (MODE == 0) __syncthreads();   // all forward reads of lds are done
  sfor<0, Q>([&](auto qv) CPRA_INLINE {
    constexpr int q = decltype(qv)::value;
    const int c = a + R1 * q;
    dft<R1, +1>(g + q * R1);
    const C* ti = tw + TL::COLI + c * R1;
    sfor<0, R1 / 2>([&](auto iv) CPRA_INLINE {
      constexpr int ap = 2 * decltype(iv)::value;
      C t0, t1;
      load_pair(ti + ap, t0, t1);
      C x0 = g[q * R1 + ap], x1 = cmul(g[q * R1 + ap + 1], t1);
      if (ap != 0) x0 = cmul(x0, t0);
      lds[c * LSTRIDE + ap * CC + col] = x0;
      lds[c * LSTRIDE + (ap + 1) * CC + col] = x1;
    });
  });
  __syncthreads();
  // inverse step 2: thread a gathers all c, R2-point IDFT -> s[a + R1 b]
  {
    C v[R2];
    sfor<0, R2>([&](auto cv) CPRA_INLINE {
      constexpr int c = decltype(cv)::value;
      v[c] = lds[c * LSTRIDE + a * CC + col];
    });
    dft<R2, +1>(v);
    C* Mn = Pmid + (size_t)n * plane;
    sfor<0, R2>([&](auto bv) CPRA_INLINE {
      constexpr int b = decltype(bv)::value;
      st_plane<NtPolicy<N>::col_store>(Mn + pix<N>(a + R1 * b, j), v[b]);
    });
  }
  if constexpr (MODE == 0 && ERR) {
    block_reduce_store<N, T>(err, errout);
  }
}

template <int N, typename T, typename AP, int MODE, bool ERR, bool CPL = false>
__global__ void __launch_bounds__(ColCfg<N>::R1* ColCfg<N>::C)
    k_col(const cx<T>* __restrict__ P, cx<T>* __restrict__ Pmid, const AP* __restrict__ A2,
          const T* __restrict__ ampscale, const cx<T>* __restrict__ tw, const int* __restrict__ alist,
          const Coupling* __restrict__ coup, int npd, double* __restrict__ errpart, int ntiles,
          uint64_t seed) {
  const int ai = blockIdx.y;
  col_body<N, T, AP, MODE, ERR, CPL>(P, Pmid, A2, ampscale, tw, alist[ai], coup, npd,
                                     ERR ? errpart + (size_t)ai * ntiles + blockIdx.x : nullptr, seed);
}

// Column pass with step-2 DFTs shared by S = 2 or 4 lanes: R1 = S R2 threads per
// column, R2 values each.  Step 1 as in k_col; in step 2 thread a owns c = a/S and
// part s = a%S of the R1-point DFT over a: an R2-point DFT over the a = s (mod S),
// a W_R1^{s k'} twiddle and an S-point DFT across the S lanes of c.  S = 2: one
// radix-2 butterfly with lane a ^ 1 (lane ^ C); it then holds G[w] for
// w = c + R2 (k' + R2 s).  S = 4: a radix-2 butterfly across s1 (lane ^ 2C), then
// one across s0 (lane ^ C) with W_4^{s1} on the odd half, s = s0 + 2 s1; it then
// holds G[w] for w = c + R2 (k' + R2 m), m = s1 + 2 s0.  The inverse mirrors it.
// Same modes and outputs as k_col.
// value of lane ^ PM (the step-2 partner)
template <int PM, typename T>
__device__ __forceinline__ cx<T> pair_lane(cx<T> v) {
  return mk<cx<T>>(__shfl_xor(v.x, PM), __shfl_xor(v.y, PM));
}

template <int N, typename T, typename AP, int MODE, bool ERR, bool CPL>
__device__ __forceinline__ void col_pair_body(const cx<T>* __restrict__ P, cx<T>* __restrict__ Pmid,
                                              const AP* __restrict__ A2, const T* __restrict__ ampscale,
                                              const cx<T>* __restrict__ tw, int n,
                                              const Coupling* __restrict__ coup, int npd,
                                              double* __restrict__ errout, uint64_t seed) {
  using Gm = ColGeom<N>;
  using TL = TwLayout<N>;
  using C = cx<T>;
  constexpr int R1 = Gm::R1, R2 = Gm::R2, CC = Gm::C, H = N / 2, NT = R1 * CC, SS = Gm::S;
  constexpr int LSTRIDE = R1 * CC + Gm::PADC;
  static_assert(SS == 2 || SS == 4, "step 2 shared by 2 or 4 lanes");
  __shared__ C lds[R2 * LSTRIDE];
  // tile 0's column exchange: its own array (S = 2), or lds (S = 4, so that four workgroups fit a
  // CU): written after every step-2 read of lds (barrier), read before the inverse writes to lds
  // (barrier)
  __shared__ C zl_own[(MODE == 0 && SS == 2) ? N : 1];
  static_assert(R2 * LSTRIDE >= N, "column exchange fits in lds");
  C* const zl = SS == 2 ? zl_own : lds;
  // lane = a * CC + col: the lanes of one row of a tile are neighbours, and the
  // step-2 partners (a ^ 1, a ^ 2) are lane ^ CC, lane ^ 2 CC
  constexpr int PM = CC;
  const int col = threadIdx.x % CC;
  const int a = threadIdx.x / CC;          // row residue in step 1
  const int sh = a & (SS - 1);             // step 2: part s of the DFT over a ...
  const int c = a / SS;                    // ... for the owned c
  const int s0 = sh & 1, s1 = sh >> 1;
  const int mo = SS == 2 ? sh : s1 + 2 * s0;   // output quarter / half: G[c + R2 (k' + R2 mo)]
  const int tile = blockIdx.x;
  const int j0 = col_tile_start<N>(tile);
  const int j = j0 + col;
  const size_t plane = (size_t)N * H;
  const T scale = (T)0.5 / ((T)N * (T)N);
  const int dn = n % npd;                  // data angle of slot n (slots r * npd + dn)
  const AP* An = A2 + (size_t)dn * plane;
  const T as = ampscale[dn];
  double err = 0.0;
  C g[R2];   // after the forward transform: G[c + R2 (k' + R2 sh)] at index k'

  if constexpr (MODE == 0) {
    C v[R2];
    const C* Pn = P + (size_t)n * plane;
    sfor<0, R2>([&](auto bv) CPRA_INLINE {
      constexpr int b = decltype(bv)::value;
      v[b] = Pn[pix<N>(a + R1 * b, j)];
    });
    typename AmpIO<AP>::pair_t amp[R2];
    if (CPL) {
      const Coupling cp = coup[n];
      const T wl = (T)cp.wl, w0 = (T)cp.w0, wr = (T)cp.wr;
      const C* Pl = P + (size_t)cp.left * plane;
      const C* Pr = P + (size_t)cp.right * plane;
      const T sl = (cp.mirror_left && j != 0) ? (T)-1 : (T)1;
      const T sr = (cp.mirror_right && j != 0) ? (T)-1 : (T)1;
      sfor<0, R2>([&](auto bv) CPRA_INLINE {
        constexpr int b = decltype(bv)::value;
        const C l = Pl[pix<N>(a + R1 * b, j)];
        const C r = Pr[pix<N>(a + R1 * b, j)];
        v[b] = mk<C>(w0 * v[b].x + wl * l.x + wr * r.x, w0 * v[b].y + (wl * sl) * l.y + (wr * sr) * r.y);
      });
    }
    // forward step 1: R2-point DFT over b, twiddle W_N^{a c'}
    dft<R2, -1>(v);
    const C* tf = tw + TL::COLF + a * R2;
    sfor<0, R2 / 2>([&](auto iv) CPRA_INLINE {
      constexpr int cc = 2 * decltype(iv)::value;
      C t0, t1;
      load_pair(tf + cc, t0, t1);
      if (cc != 0) v[cc] = cmul(v[cc], t0);
      v[cc + 1] = cmul(v[cc + 1], t1);
    });
    sfor<0, R2>([&](auto cv) CPRA_INLINE {
      constexpr int cc = decltype(cv)::value;
      lds[cc * LSTRIDE + a * CC + col] = v[cc];
    });
    __syncthreads();
    // the amplitude pairs, fetched here so that their latency overlaps step 2 without holding
    // registers through step 1
    if (j0 != 0) {
      sfor<0, R2>([&](auto kv) CPRA_INLINE {
        constexpr int k = decltype(kv)::value;
        amp[k] = AmpIO<AP>::raw(An + pix<N>(c + R2 * (k + R2 * mo), j));
      });
    }
    // forward step 2: part sh of the R1-point DFT over a for this c
    sfor<0, R2>([&](auto kv) CPRA_INLINE {
      constexpr int k = decltype(kv)::value;
      g[k] = lds[c * LSTRIDE + (sh + SS * k) * CC + col];
    });
    dft<R2, -1>(g);
    if constexpr (SS == 2) {
      const T sgn = sh ? (T)-1 : (T)1;
      sfor<0, R2>([&](auto kv) CPRA_INLINE {
        constexpr int k = decltype(kv)::value;
        const C t = sh ? twc<-1, k, R1>(g[k]) : g[k];
        const C o = pair_lane<PM, T>(t);
        g[k] = mk<C>(o.x + sgn * t.x, o.y + sgn * t.y);    // sh = 0: t + o; sh = 1: o - t
      });
    } else {
      sfor<0, R2>([&](auto kv) CPRA_INLINE {
        constexpr int k = decltype(kv)::value;
        C t = s0 ? twc<-1, k, R1>(g[k]) : g[k];              // W_R1^{s k}, s = s0 + 2 s1
        t = s1 ? twc<-1, 2 * k, R1>(t) : t;
        const C o1 = pair_lane<2 * PM, T>(t);                // across s1
        const C u = s1 ? mk<C>(o1.x - t.x, o1.y - t.y) : mk<C>(t.x + o1.x, t.y + o1.y);
        const C o0 = pair_lane<PM, T>(u);                    // across s0, W_4^{s1} on the odd half
        const C wu = s1 ? mk<C>(u.y, -u.x) : u;              // W_4 = -i
        const C wo = s1 ? mk<C>(o0.y, -o0.x) : o0;
        g[k] = s0 ? mk<C>(o0.x - wu.x, o0.y - wu.y) : mk<C>(u.x + wo.x, u.y + wo.y);
      });
    }
    // modulus projection
    if (j0 != 0) {
      const bool neg = ((c + j) & 1) != 0;   // (-1)^(w + j), w = c + R2 (k + R2 sh), R2 even
      sfor<0, R2>([&](auto kv) CPRA_INLINE {
        constexpr int k = decltype(kv)::value;
        const auto pa = AmpIO<AP>::decode(amp[k], as);
        g[k] = Proj<T>::template two<ERR>(g[k], (T)pa.x, (T)pa.y, neg, scale, err, 1.0);
      });
    } else {
      __syncthreads();
      if (col == 0) {
        sfor<0, R2>([&](auto kv) CPRA_INLINE {
          constexpr int k = decltype(kv)::value;
          zl[c + R2 * (k + R2 * mo)] = g[k];
        });
      }
      __syncthreads();
      sfor<0, R2>([&](auto kv) CPRA_INLINE {
        constexpr int k = decltype(kv)::value;
        const int w = c + R2 * (k + R2 * mo);
        if (j != 0) {
          const auto pa = AmpIO<AP>::load(An + pix<N>(w, j), as);
          g[k] = Proj<T>::template two<ERR>(g[k], (T)pa.x, (T)pa.y, ((w + j) & 1) != 0, scale, err, 1.0);
        } else {
          const int wm = wrapN<N>(N - w);
          const C Z = g[k], Zm = zl[wm];
          const C Ga = mk<C>((T)0.5 * (Z.x + Zm.x), (T)0.5 * (Z.y - Zm.y));
          const C Gb = mk<C>((T)0.5 * (Z.y + Zm.y), (T)0.5 * (Zm.x - Z.x));
          const auto p0 = AmpIO<AP>::load(An + pix<N>(w, 0), as);
          const auto pm = AmpIO<AP>::load(An + pix<N>(wm, 0), as);
          const C Pa = Proj<T>::template two<ERR>(Ga, (T)p0.x, (T)pm.x, (w & 1) != 0, scale, err, 0.5);
          const C Pb = Proj<T>::template two<ERR>(Gb, (T)p0.y, (T)pm.y, ((w + H) & 1) != 0, scale, err, 0.5);
          g[k] = mk<C>(Pa.x - Pb.y, Pa.y + Pb.x);
        }
      });
    }
  } else {
    auto phase = [&](int w, int u) CPRA_INLINE -> C {
      const uint64_t cnt = ((uint64_t)n * N + (uint64_t)w) * N + (uint64_t)u;
      const uint64_t r = splitmix64_at(seed, cnt) >> 40;
      double s, co;
      sincospi(2.0 * (double)r / 16777216.0, &s, &co);
      return mk<C>((T)co, (T)s);
    };
    sfor<0, R2>([&](auto kv) CPRA_INLINE {
      constexpr int k = decltype(kv)::value;
      const int w = c + R2 * (k + R2 * mo);
      const int wm = wrapN<N>(N - w);
      C out;
      if (j != 0) {
        const auto pa = AmpIO<AP>::load(An + pix<N>(w, j), as);
        const T a1 = pa.x > (T)0 ? (T)pa.x : (T)0, a2 = pa.y > (T)0 ? (T)pa.y : (T)0;
        const C e1 = phase(w, j), e2 = conj(phase(wm, N - j));
        const T sg = ((w + j) & 1) ? -scale : scale;
        out = mk<C>(sg * (a1 * e1.x + a2 * e2.x), sg * (a1 * e1.y + a2 * e2.y));
      } else {
        const auto p0 = AmpIO<AP>::load(An + pix<N>(w, 0), as);
        const auto pm = AmpIO<AP>::load(An + pix<N>(wm, 0), as);
        const T a0 = p0.x > 0 ? (T)p0.x : (T)0, am0 = pm.x > 0 ? (T)pm.x : (T)0;
        const T aH = p0.y > 0 ? (T)p0.y : (T)0, amH = pm.y > 0 ? (T)pm.y : (T)0;
        const C e1 = phase(w, 0), e2 = conj(phase(wm, 0));
        const C f1 = phase(w, H), f2 = conj(phase(wm, H));
        const T sa = (w & 1) ? -scale : scale, sb = ((w + H) & 1) ? -scale : scale;
        const C Ga = mk<C>(sa * (a0 * e1.x + am0 * e2.x), sa * (a0 * e1.y + am0 * e2.y));
        const C Gb = mk<C>(sb * (aH * f1.x + amH * f2.x), sb * (aH * f1.y + amH * f2.y));
        out = mk<C>(Ga.x - Gb.y, Ga.y + Gb.x);
      }
      g[k] = out;
    });
  }

  // inverse: the S-point IDFT across the lanes, W_R1^{-sh k'}, R2-point IDFT over k'
  if constexpr (MODE == 0) __syncthreads();   // all forward reads of lds are done
  if constexpr (SS == 2) {
    const T sgn = sh ? (T)-1 : (T)1;
    sfor<0, R2>([&](auto kv) CPRA_INLINE {
      constexpr int k = decltype(kv)::value;
      const C o = pair_lane<PM, T>(g[k]);
      const C u = mk<C>(o.x + sgn * g[k].x, o.y + sgn * g[k].y);
      g[k] = sh ? twc<+1, k, R1>(u) : u;
    });
  } else {
    sfor<0, R2>([&](auto kv) CPRA_INLINE {
      constexpr int k = decltype(kv)::value;
      const C o0 = pair_lane<PM, T>(g[k]);                // across s0 (the lane holds m = s1 + 2 s0)
      C u = s0 ? mk<C>(o0.x - g[k].x, o0.y - g[k].y) : mk<C>(g[k].x + o0.x, g[k].y + o0.y);
      u = (s0 & s1) ? mk<C>(-u.y, u.x) : u;                 // W_4^{-s0 s1}: +i
      const C o1 = pair_lane<2 * PM, T>(u);                 // across s1
      C z = s1 ? mk<C>(o1.x - u.x, o1.y - u.y) : mk<C>(u.x + o1.x, u.y + o1.y);
      z = s0 ? twc<+1, k, R1>(z) : z;                       // W_R1^{-s k'}, s = s0 + 2 s1
      g[k] = s1 ? twc<+1, 2 * k, R1>(z) : z;
    });
  }
  dft<R2, +1>(g);   // g[a'] = Y'[c][sh + S a']
  {
    const C* ti = tw + TL::COLI + c * R1 + sh * R2;   // conj W_N^{(sh + S a') c}
    sfor<0, R2 / 2>([&](auto iv) CPRA_INLINE {
      constexpr int k = 2 * decltype(iv)::value;
      C t0, t1;
      load_pair(ti + k, t0, t1);
      lds[c * LSTRIDE + (sh + SS * k) * CC + col] = cmul(g[k], t0);
      lds[c * LSTRIDE + (sh + SS * (k + 1)) * CC + col] = cmul(g[k + 1], t1);
    });
  }
  __syncthreads();
  {
    C v[R2];
    sfor<0, R2>([&](auto cv) CPRA_INLINE {
      constexpr int cc = decltype(cv)::value;
      v[cc] = lds[cc * LSTRIDE + a * CC + col];
    });
    dft<R2, +1>(v);
    C* Mn = Pmid + (size_t)n * plane;
    sfor<0, R2>([&](auto bv) CPRA_INLINE {
      constexpr int b = decltype(bv)::value;
      st_plane<NtPolicy<N>::col_store>(Mn + pix<N>(a + R1 * b, j), v[b]);
    });
  }
  if constexpr (MODE == 0 && ERR) {
    block_reduce_store<N, T, NT>(err, errout);
  }
}

template <int N, typename T, typename AP, int MODE, bool ERR, bool CPL = false>
__global__ void __launch_bounds__(ColCfg<N>::R1* ColCfg<N>::C) __attribute__((amdgpu_waves_per_eu(4)))
    k_col_pair(const cx<T>* __restrict__ P, cx<T>* __restrict__ Pmid, const AP* __restrict__ A2,
               const T* __restrict__ ampscale, const cx<T>* __restrict__ tw, const int* __restrict__ alist,
               const Coupling* __restrict__ coup, int npd, double* __restrict__ errpart, int ntiles,
               uint64_t seed) {
  const int ai = blockIdx.y;
  col_pair_body<N, T, AP, MODE, ERR, CPL>(P, Pmid, A2, ampscale, tw, alist[ai], coup, npd,
                                          ERR ? errpart + (size_t)ai * ntiles + blockIdx.x : nullptr, seed);
}

// ---------------------------------------------------------------- row pass
// Value of lane (F1 - t) mod F1 of this lane's group of F1 lanes (t = lane
// mod F1); lanes t = 0 and t = F1/2 get an unspecified value (they pair with
// themselves and never use it).
template <int F1>
__device__ __forceinline__ float partner_lane(float v) {
  const int x = __float_as_int(v);
  int y;
  if constexpr (F1 == 16) {
    y = __builtin_amdgcn_update_dpp(0, x, 0x140, 0xF, 0xF, false);   // row_mirror: 15 - t
    y = __builtin_amdgcn_update_dpp(0, y, 0x111, 0xF, 0xF, false);   // row_shr:1 -> 16 - t
  } else if constexpr (F1 == 8) {
    y = __builtin_amdgcn_update_dpp(0, x, 0x141, 0xF, 0xF, false);   // row_half_mirror: 7 - t
    y = __builtin_amdgcn_update_dpp(0, y, 0x111, 0xF, 0xF, false);   // row_shr:1 -> 8 - t
  } else {
    static_assert(F1 == 4, "partner_lane");
    y = __builtin_amdgcn_update_dpp(0, x, 0x6C, 0xF, 0xF, false);    // quad_perm [0,3,2,1]
  }
  return __int_as_float(y);
}
__device__ __forceinline__ double partner_lane_d(double v, int lane_src) {
  return __shfl(v, lane_src);
}
template <int F1, typename C>
__device__ __forceinline__ C partner_c(C v, int partner_lane_idx) {
  if constexpr (std::is_same<C, float2>::value) {
    return make_float2(partner_lane<F1>(v.x), partner_lane<F1>(v.y));
  } else {
    return make_double2(partner_lane_d(v.x, partner_lane_idx), partner_lane_d(v.y, partner_lane_idx));
  }
}

// Row pass over RPB rows of one angle, F1 threads per row.
// MODE 0: initial guess (g <- g'); 1: HIO; 2: ER / episode estimate;
// 3: reload (P <- F_t(g) from the iterate in gin; Pmid unused, g unchanged);
// 4: RAAR.
// Per row: C2R of Pmid (pre-processing, F2-point IDFT, twiddle, LDS
// exchange, F1-point IDFT) -> g' in the space layout; real-space update with
// the support bits and g; R2C back (F1-point DFT, twiddle, LDS exchange,
// F2-point DFT, post-processing) -> P.
template <int N, typename T, bool CPL, int RPB>
__device__ __forceinline__ void row_body(const cx<T>* __restrict__ Pmid, cx<T>* __restrict__ P, const T* gin,
                                         T* gout, const uint32_t* __restrict__ maskw,
                                         const cx<T>* __restrict__ tw, int n, const Coupling* __restrict__ coup,
                                         int npd, int mode, T beta, int positivity) {
  using Gm = RowGeom<N>;
  using TL = TwLayout<N>;
  using C = cx<T>;
  constexpr int F1 = Gm::F1, F2 = Gm::F2, TT = Gm::T, SPT = Gm::SPT, H = N / 2;
  constexpr int MW = Gm::MW;
  constexpr int LS = F1 + Gm::PADR;       // lds stride per m2
  __shared__ C lds[RPB * Gm::RSTRIDE];
  const int tau = threadIdx.x % TT;       // owned frequency class k1 = tau
  const int r = threadIdx.x / TT;
  const int z = blockIdx.x * RPB + r;
  C* L0 = lds + r * Gm::RSTRIDE;
  const size_t pbase = (size_t)n * N * H;           // the angle's complex planes
  const size_t rowr = ((size_t)n * N + z) * N;     // real row base
  const bool t0 = (tau == 0);
  const int plane_lane = (threadIdx.x & ~(TT - 1)) + ((TT - tau) & (TT - 1));   // partner, for __shfl

  // the current iterate of this thread's pixels (HIO and RAAR need it), fetched after the first
  // LDS exchange of the C2R so that its latency overlaps the second half of the transform
  C gk[SPT][F1];
  auto load_gk = [&]() CPRA_INLINE {
    if (mode == 1 || mode == 4) {
      sfor<0, SPT>([&](auto jv) CPRA_INLINE {
        constexpr int jj = decltype(jv)::value;
        sfor<0, F1>([&](auto mv) CPRA_INLINE {
          constexpr int m1 = decltype(mv)::value;
          gk[jj][m1] = ld_plane<NtPolicy<N>::row_gload>(reinterpret_cast<const C*>(gin + rowr + 2 * (tau + TT * jj + F2 * m1)));
        });
      });
    }
  };
  C sp[SPT][F1];
  C x[F2];
  if (mode == 3) {
    sfor<0, SPT>([&](auto jv) CPRA_INLINE {
      constexpr int jj = decltype(jv)::value;
      sfor<0, F1>([&](auto mv) CPRA_INLINE {
        constexpr int m1 = decltype(mv)::value;
        sp[jj][m1] = *reinterpret_cast<const C*>(gin + rowr + 2 * (tau + TT * jj + F2 * m1));
      });
    });
  } else {
    // ---- load Pmid class tau, C2R pre-processing:
    //   X'[k] = (a + b) + i (a - b) e^{+2 pi i k/N},  a = T[k], b = conj T[L-k]
    // (k = 0: a, b = the packed real DC and Nyquist values)
    // the partner T[L-k] of k = tau + F1 k2 is class (F1 - tau)'s value at index
    // F2-1-k2, taken from that lane by DPP, or for class 0 its own value at index
    // (F2 - k2) mod F2
    C pv[F2];
    sfor<0, F2>([&](auto kk) CPRA_INLINE {
      constexpr int k2 = decltype(kk)::value;
      x[k2] = Pmid[pbase + pix<N>(z, tau + F1 * k2)];
    });
    sfor<0, F2>([&](auto kk) CPRA_INLINE {
      constexpr int k2 = decltype(kk)::value;
      const C other = partner_c<F1>(x[F2 - 1 - k2], plane_lane);
      pv[k2] = t0 ? x[(F2 - k2) % F2] : other;
    });
    const C* tp = tw + TL::RPP + tau * F2;             // W_N^{k1 + F1 k2}
    sfor<0, F2 / 2>([&](auto kk) CPRA_INLINE {
      C tpair[2];
      load_pair(tp + 2 * decltype(kk)::value, tpair[0], tpair[1]);
      sfor<0, 2>([&](auto hh) CPRA_INLINE {
        constexpr int k2 = 2 * decltype(kk)::value + decltype(hh)::value;
        const C a = x[k2];
        const C b = conj(pv[k2]);
        const C sum = cadd(a, b), dif = csub(a, b);
        const C t = cmulc(dif, tpair[decltype(hh)::value]);   // (a - b) e^{+2 pi i k/N}
        const bool k0 = (k2 == 0) && t0;
        x[k2] = k0 ? mk<C>(a.x + a.y, a.x - a.y) : mk<C>(sum.x - t.y, sum.y + t.x);
      });
    });
    // ---- C2R step 1: F2-point IDFT over k2, twiddle e^{+2 pi i k1 m2 / L}, to LDS
    dft<F2, +1>(x);
    {
      const C* tq = tw + TL::RC2R + tau * F2;
      sfor<0, F2 / 2>([&](auto mm) CPRA_INLINE {
        constexpr int m2 = 2 * decltype(mm)::value;
        C t0w, t1w;
        load_pair(tq + m2, t0w, t1w);
        C v0 = x[m2];
        if (m2 != 0) v0 = cmul(v0, t0w);
        L0[m2 * LS + tau] = v0;
        L0[(m2 + 1) * LS + tau] = cmul(x[m2 + 1], t1w);
      });
    }
    __syncthreads();
    load_gk();
    // ---- C2R step 2: for owned m2, F1-point IDFT over k1 -> x[m2 + F2 m1]
    sfor<0, SPT>([&](auto jv) CPRA_INLINE {
      constexpr int jj = decltype(jv)::value;
      const int m2 = tau + TT * jj;
      sfor<0, F1>([&](auto kv) CPRA_INLINE {
        constexpr int k1 = decltype(kv)::value;
        sp[jj][k1] = L0[m2 * LS + k1];
      });
      dft<F1, +1>(sp[jj]);
    });
    // ---- real-space update (pixels t = 2m and 2m+1 of x[m])
    uint32_t mwd[MW];
    const uint32_t* Mrow = maskw + (((size_t)(n % npd) * N + z) * TT + tau) * MW;
    sfor<0, MW>([&](auto iv) CPRA_INLINE { mwd[decltype(iv)::value] = Mrow[decltype(iv)::value]; });
    Coupling cp{};
    if constexpr (CPL) cp = coup[n];
    const T* gl = gin + ((size_t)cp.left * N + z) * N;
    const T* gr = gin + ((size_t)cp.right * N + z) * N;
    const T wl = (T)cp.wl, w0 = (T)cp.w0, wr = (T)cp.wr;
    sfor<0, SPT>([&](auto jv) CPRA_INLINE {
      constexpr int jj = decltype(jv)::value;
      sfor<0, F1>([&](auto mv) CPRA_INLINE {
        constexpr int m1 = decltype(mv)::value;
        const int m = tau + TT * jj + F2 * m1;
        const C gp = sp[jj][m1];                      // (g'[2m], g'[2m+1])
        C out = gp;
        if (mode != 0) {
          constexpr int b0 = (jj * F1 + m1) * 2;
          const bool s0 = (mwd[b0 >> 5] >> (b0 & 31)) & 1u;
          const bool s1 = (mwd[(b0 + 1) >> 5] >> ((b0 + 1) & 31)) & 1u;
          const bool g0 = s0 && (!positivity || gp.x >= (T)0);
          const bool g1 = s1 && (!positivity || gp.y >= (T)0);
          if (mode == 2) {
            out = mk<C>(g0 ? gp.x : (T)0, g1 ? gp.y : (T)0);
          } else {
            C gkv = gk[jj][m1];
            if constexpr (CPL) {
              C lv, rv;
              if (cp.mirror_left) lv = mk<C>(gl[wrapN<N>(N - 2 * m)], gl[N - 1 - 2 * m]);
              else lv = *reinterpret_cast<const C*>(gl + 2 * m);
              if (cp.mirror_right) rv = mk<C>(gr[wrapN<N>(N - 2 * m)], gr[N - 1 - 2 * m]);
              else rv = *reinterpret_cast<const C*>(gr + 2 * m);
              gkv = mk<C>(w0 * gkv.x + wl * lv.x + wr * rv.x, w0 * gkv.y + wl * lv.y + wr * rv.y);
            }
            if (mode == 4) {
              // RAAR, pixel form of beta/2 (R_S R_M + I) + (1 - beta) P_M: g' where the
              // reflection 2g' - g meets the constraints, beta g + (1 - 2 beta) g' elsewhere
              const bool r0 = s0 && (!positivity || (T)2 * gp.x - gkv.x >= (T)0);
              const bool r1 = s1 && (!positivity || (T)2 * gp.y - gkv.y >= (T)0);
              const T c1 = (T)1 - (T)2 * beta;
              out = mk<C>(r0 ? gp.x : beta * gkv.x + c1 * gp.x, r1 ? gp.y : beta * gkv.y + c1 * gp.y);
            } else {
              out = mk<C>(g0 ? gp.x : gkv.x - beta * gp.x, g1 ? gp.y : gkv.y - beta * gp.y);
            }
          }
        }
        st_plane<NtPolicy<N>::row_store>(reinterpret_cast<C*>(gout + rowr + 2 * m), out);
        sp[jj][m1] = out;
      });
    });
    __syncthreads();   // everyone has read the C2R exchange
  }
  // ---- R2C step 1: for owned m2, F1-point DFT over m1, twiddle e^{-2 pi i m2 k1 / L}
  sfor<0, SPT>([&](auto jv) CPRA_INLINE {
    constexpr int jj = decltype(jv)::value;
    const int m2 = tau + TT * jj;
    dft<F1, -1>(sp[jj]);
    const C* tq = tw + TL::RR2C + m2 * F1;
    sfor<0, F1 / 2>([&](auto kv) CPRA_INLINE {
      constexpr int k1 = 2 * decltype(kv)::value;
      C t0w, t1w;
      load_pair(tq + k1, t0w, t1w);
      C v0 = sp[jj][k1];
      if (k1 != 0) v0 = cmul(v0, t0w);
      L0[m2 * LS + k1] = v0;
      L0[m2 * LS + k1 + 1] = cmul(sp[jj][k1 + 1], t1w);
    });
  });
  __syncthreads();
  // ---- R2C step 2: class tau, F2-point DFT over m2 -> Z[tau + F1 k2]
  sfor<0, F2>([&](auto mm) CPRA_INLINE {
    constexpr int m2 = decltype(mm)::value;
    x[m2] = L0[m2 * LS + tau];
  });
  dft<F2, -1>(x);
  // ---- post-processing to the packed half spectrum:
  //   Fe = (Z[k] + conj Z[L-k])/2, Fo = (Z[k] - conj Z[L-k])/(2i), S[k] = Fe + W_N^k Fo
  {
    const C* tp = tw + TL::RPP + tau * F2;
    sfor<0, F2 / 2>([&](auto kk) CPRA_INLINE {
      C tpair[2];
      load_pair(tp + 2 * decltype(kk)::value, tpair[0], tpair[1]);
      sfor<0, 2>([&](auto hh) CPRA_INLINE {
        constexpr int k2 = 2 * decltype(kk)::value + decltype(hh)::value;
        const C other = partner_c<F1>(x[F2 - 1 - k2], plane_lane);   // Z[L-k] from the partner lane
        const C self0 = x[(F2 - k2) % F2];                            // class 0 pairs with itself
        const C Z = x[k2];
        const C Zp = t0 ? self0 : other;
        const bool k0 = (k2 == 0) && t0;
        const C Fe = mk<C>((T)0.5 * (Z.x + Zp.x), (T)0.5 * (Z.y - Zp.y));
        const C Fo = mk<C>((T)0.5 * (Z.y + Zp.y), (T)0.5 * (Zp.x - Z.x));
        const C o = cadd(Fe, cmul(Fo, tpair[decltype(hh)::value]));
        st_plane<NtPolicy<N>::row_store>(P + pbase + pix<N>(z, tau + F1 * k2), k0 ? mk<C>(Z.x + Z.y, Z.x - Z.y) : o);
      });
    });
  }
}

template <int N, typename T, bool CPL = false, int RPB = RowCfg<N>::RPB>
__global__ void __launch_bounds__(RowCfg<N>::F1* RPB) __attribute__((amdgpu_waves_per_eu(4)))
    k_row(const cx<T>* __restrict__ Pmid, cx<T>* __restrict__ P, const T* gin, T* gout,
          const uint32_t* __restrict__ maskw, const cx<T>* __restrict__ tw, const int* __restrict__ alist,
          const Coupling* __restrict__ coup, int npd, int mode, T beta, int positivity) {
  row_body<N, T, CPL, RPB>(Pmid, P, gin, gout, maskw, tw, alist[blockIdx.y], coup, npd, mode, beta, positivity);
}

// ---------------------------------------------------------------- fused launches
// One launch of a pass over the listed slots of up to kFuseMax plans of the same N and precision
// (several scans iterated together): work item i (blockIdx.y) belongs to plan p with
// start[p] <= i < start[p + 1] and is that plan's slot alist[i - start[p]].  Every plan brings its
// own planes, data, coupling table and current iterate buffers; the arithmetic per slot is that
// of the single-plan launch.
constexpr int kFuseMax = 16;
template <typename T, typename AP> struct FusePlan {
  cx<T>* P;
  cx<T>* Pmid;
  const AP* A2;
  const T* ampscale;
  const cx<T>* tw;
  const int* alist;
  const Coupling* coup;
  const T* gin;
  T* gout;
  const uint32_t* maskw;
  int npd, positivity;
};
template <typename T, typename AP> struct FuseTab {
  int count;
  int start[kFuseMax + 1];
  FusePlan<T, AP> p[kFuseMax];
};

__device__ __forceinline__ int fuse_plan_of(const int* start, int count, int i) {
  int p = 0;
  for (int q = 1; q < count; ++q) p = i >= start[q] ? q : p;
  return p;
}

template <int N, typename T, typename AP, bool CPL>
__global__ void __launch_bounds__(ColCfg<N>::R1* ColCfg<N>::C) __attribute__((amdgpu_waves_per_eu(4)))
    k_colpair_fused(const FuseTab<T, AP> ft) {
  const int i = blockIdx.y;
  const int p = fuse_plan_of(ft.start, ft.count, i);
  const FusePlan<T, AP>& q = ft.p[p];
  col_pair_body<N, T, AP, 0, false, CPL>(q.P, q.Pmid, q.A2, q.ampscale, q.tw, q.alist[i - ft.start[p]], q.coup,
                                         q.npd, nullptr, 0);
}

template <int N, typename T, typename AP, bool CPL>
__global__ void __launch_bounds__(ColCfg<N>::R1* ColCfg<N>::C) k_col_fused(const FuseTab<T, AP> ft) {
  const int i = blockIdx.y;
  const int p = fuse_plan_of(ft.start, ft.count, i);
  const FusePlan<T, AP>& q = ft.p[p];
  col_body<N, T, AP, 0, false, CPL>(q.P, q.Pmid, q.A2, q.ampscale, q.tw, q.alist[i - ft.start[p]], q.coup, q.npd,
                                    nullptr, 0);
}

template <int N, typename T, typename AP, bool CPL, int RPB = RowCfg<N>::RPB>
__global__ void __launch_bounds__(RowCfg<N>::F1* RPB) __attribute__((amdgpu_waves_per_eu(4)))
    k_row_fused(const FuseTab<T, AP> ft, int mode, T beta) {
  const int i = blockIdx.y;
  const int p = fuse_plan_of(ft.start, ft.count, i);
  const FusePlan<T, AP>& q = ft.p[p];
  row_body<N, T, CPL, RPB>(q.Pmid, q.P, q.gin, q.gout, q.maskw, q.tw, q.alist[i - ft.start[p]],
                      q.coup, q.npd, mode, beta, q.positivity);
}

// ---------------------------------------------------------------- autotuning input
// A synthetic scan for timing the passes: intensities (u24 / 2^24)^4 * 1e4 from SplitMix64 at
// counter (n * N + w) * N + u, and a centred disc support of radius 0.3 N.  count angles from
// `first`, written [i][w][u] and [i][z][t].  The values only need to be finite and non-trivial.
template <int N>
__global__ void __launch_bounds__(256) k_synth_scan(float* __restrict__ I, uint8_t* __restrict__ S, int first,
                                                    uint64_t seed) {
  const int i = blockIdx.y, w = blockIdx.x;
  const float r2 = 0.09f * (float)N * (float)N;
  for (int u = threadIdx.x; u < N; u += blockDim.x) {
    const uint64_t cnt = ((uint64_t)(first + i) * N + (uint64_t)w) * N + (uint64_t)u;
    const float x = (float)(splitmix64_at(seed, cnt) >> 40) * (1.0f / 16777216.0f);
    I[((size_t)i * N + w) * N + u] = 1e4f * (x * x) * (x * x);
    const float dz = (float)(w - N / 2), dt = (float)(u - N / 2);
    S[((size_t)i * N + w) * N + u] = (dz * dz + dt * dt) < r2 ? 1 : 0;
  }
}

// ---------------------------------------------------------------- error reduce
static __global__ void k_err_reduce(const double* __restrict__ errpart, const double* __restrict__ den,
                             const int* __restrict__ alist, int nact, int ntiles, int nslots, int npd,
                             double* __restrict__ hist) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nslots * nact) return;
  int slot = i / nact, ai = i % nact;
  const double* p = errpart + ((size_t)slot * nact + ai) * ntiles;
  double s = 0.0;
  for (int t = 0; t < ntiles; ++t) s += p[t];
  double d = den[alist[ai] % npd];
  hist[i] = d > 0.0 ? sqrt(s / d) : sqrt(s);
}

}  // namespace cpra
