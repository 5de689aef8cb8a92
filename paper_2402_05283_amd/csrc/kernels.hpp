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
template <int N> struct ColCfg;
template <> struct ColCfg<64> { static constexpr int R1 = 8, R2 = 8, C = 16; };
template <> struct ColCfg<128> { static constexpr int R1 = 8, R2 = 16, C = 16; };
template <> struct ColCfg<256> { static constexpr int R1 = 16, R2 = 16, C = 16; };
template <> struct ColCfg<512> { static constexpr int R1 = 16, R2 = 32, C = 16; };
template <> struct ColCfg<1024> { static constexpr int R1 = 32, R2 = 32, C = 8; };

// Row half-spectrum transform of length L = N/2 = F1 * F2 (F1: frequency
// residue modulus, F2: space residue modulus), T = F1/2 threads per row,
// each owning the frequency classes {t, F1-t} ({0, F1/2} for t = 0), so that
// the real-to-complex pairing k <-> L-k stays inside a thread.
template <int N> struct RowCfg;
template <> struct RowCfg<64> { static constexpr int F1 = 4, F2 = 8, RPB = 64; };
template <> struct RowCfg<128> { static constexpr int F1 = 8, F2 = 8, RPB = 32; };
template <> struct RowCfg<256> { static constexpr int F1 = 8, F2 = 16, RPB = 32; };
template <> struct RowCfg<512> { static constexpr int F1 = 16, F2 = 16, RPB = 16; };
template <> struct RowCfg<1024> { static constexpr int F1 = 16, F2 = 32, RPB = 16; };

template <int N> struct RowGeom {
  static constexpr int L = N / 2;
  static constexpr int F1 = RowCfg<N>::F1, F2 = RowCfg<N>::F2, RPB = RowCfg<N>::RPB;
  static constexpr int T = F1 / 2;          // threads per row
  static constexpr int SPT = F2 / T;        // space classes per thread
  static constexpr int E = 2 * F2;          // complex values per thread
  static constexpr int MW = N / (32 * T);   // mask words per thread per row
  static constexpr int PADR = 1;
  static_assert(F1 * F2 == L, "row decomposition");
  static_assert(F1 <= F2 && F2 % T == 0, "row ownership");
  static_assert(MW >= 1 && (N % (32 * T)) == 0, "mask words");
};

template <int N> struct ColGeom {
  static constexpr int R1 = ColCfg<N>::R1, R2 = ColCfg<N>::R2, C = ColCfg<N>::C;
  static constexpr int Q = R2 / R1;
  static constexpr int PADC = 1;
  static constexpr int TILES = (N / 2) / C;
  static_assert(R1 * R2 == N && R2 % R1 == 0 && (N / 2) % C == 0, "column decomposition");
};

// Space position of bit b of thread tau's mask words in a row: t index.
template <int N> __host__ __device__ inline int mask_bit_t(int tau, int b) {
  using G = RowGeom<N>;
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

// ---------------------------------------------------------------- amplitudes
template <typename AP> struct AmpIO;
template <> struct AmpIO<float2> {
  using real = float;
  __device__ static float2 load(const float2* p, float) { return *p; }
};
template <> struct AmpIO<double2> {
  using real = double;
  __device__ static double2 load(const double2* p, double) { return *p; }
};
template <> struct AmpIO<__half2> {
  using real = float;
  __device__ static float2 load(const __half2* p, float s) {
    float2 v = __half22float2(*p);
    v.x *= s; v.y *= s;
    return v;
  }
};

__host__ __device__ inline uint64_t splitmix64_at(uint64_t seed, uint64_t c) {
  uint64_t z = seed + (c + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// ---------------------------------------------------------------- twiddles
template <typename T>
__global__ void k_twiddles(cx<T>* tw, int N) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < N) {
    double s, c;
    sincospi(-2.0 * (double)j / (double)N, &s, &c);
    tw[j] = mk<cx<T>>((T)c, (T)s);
  }
}

// ---------------------------------------------------------------- prep
// One block per submitted angle: amplitude pairs, support bits, sum A^2.
template <int N, typename T, typename AP>
__global__ void __launch_bounds__(256) k_prep(const float* __restrict__ I, const uint8_t* __restrict__ sup,
                                              int first, AP* __restrict__ A2, T* __restrict__ ampscale,
                                              uint32_t* __restrict__ maskw, double* __restrict__ den,
                                              int* __restrict__ flags) {
  using G = RowGeom<N>;
  constexpr int H = N / 2;
  const int n = first + blockIdx.x;
  const float* In = I + (size_t)blockIdx.x * N * N;
  const uint8_t* Sn = sup + (size_t)blockIdx.x * N * N;
  __shared__ double red[256];
  __shared__ float redm[256];
  double acc = 0.0;
  float amax = 0.f;
  int bad = 0;
  for (int i = threadIdx.x; i < N * N; i += blockDim.x) {
    float v = In[i];
    if (!isfinite(v)) bad = 1;
    if (v >= 0.f) { acc += (double)v; amax = fmaxf(amax, sqrtf(v)); }
  }
  red[threadIdx.x] = acc;
  redm[threadIdx.x] = amax;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      red[threadIdx.x] += red[threadIdx.x + s];
      redm[threadIdx.x] = fmaxf(redm[threadIdx.x], redm[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (bad) atomicOr(flags, 1);
  if (threadIdx.x == 0) den[n] = red[0];
  float scale = 1.f;
  if constexpr (std::is_same<AP, __half2>::value) {
    int e = 0;
    frexpf(redm[0] > 0.f ? redm[0] : 1.f, &e);   // max A < 2^e
    scale = ldexpf(1.f, e - 14);                  // stored values < 2^14
    if (threadIdx.x == 0) ampscale[n] = scale;
  } else {
    if (threadIdx.x == 0) ampscale[n] = (T)1;
  }
  const float inv = 1.f / scale;
  auto amp = [&](int wn, int un) -> float {       // native (w, u) -> A, -1 if unmeasured
    float v = In[((wn + H) % N) * N + ((un + H) % N)];
    return v >= 0.f ? sqrtf(v) : -1.f;
  };
  auto ampd = [&](int wn, int un) -> double {
    float v = In[((wn + H) % N) * N + ((un + H) % N)];
    return v >= 0.f ? sqrt((double)v) : -1.0;
  };
  AP* An = A2 + (size_t)n * N * H;
  for (int i = threadIdx.x; i < N * H; i += blockDim.x) {
    int w = i / H, j = i % H;
    int wm = (N - w) % N;
    if constexpr (std::is_same<AP, double2>::value) {
      double a, b;
      if (j == 0) { a = ampd(w, 0); b = ampd(w, H); }
      else { a = ampd(w, j); b = ampd(wm, N - j); }
      An[i] = make_double2(a, b);
    } else {
      float a, b;
      if (j == 0) { a = amp(w, 0); b = amp(w, H); }
      else { a = amp(w, j); b = amp(wm, N - j); }
      if constexpr (std::is_same<AP, __half2>::value) {
        An[i] = __floats2half2_rn(a >= 0.f ? a * inv : -1.f, b >= 0.f ? b * inv : -1.f);
      } else {
        An[i] = make_float2(a, b);
      }
    }
  }
  uint32_t* Mn = maskw + (size_t)n * N * G::T * G::MW;
  for (int i = threadIdx.x; i < N * G::T * G::MW; i += blockDim.x) {
    int z = i / (G::T * G::MW);
    int r = i % (G::T * G::MW);
    int tau = r / G::MW, wd = r % G::MW;
    uint32_t word = 0;
    for (int b = 0; b < 32; ++b) {
      int t = mask_bit_t<N>(tau, wd * 32 + b);
      if (Sn[z * N + t]) word |= (1u << b);
    }
    Mn[i] = word;
  }
}

// ---------------------------------------------------------------- column pass
// Modulus projection of one value with its two amplitudes (q and -q).
template <typename T, bool ERR>
__device__ __forceinline__ cx<T> project2(cx<T> G, T a1, T a2, bool neg, T scale, double& err) {
  T mag2 = G.x * G.x + G.y * G.y;
  T mag = sqrt(mag2);
  T inv = mag > (T)0 ? (T)1 / mag : (T)0;
  T sg = neg ? (T)-1 : (T)1;
  cx<T> p1 = a1 >= (T)0 ? (mag > (T)0 ? cscale(G, a1 * inv) : mk<cx<T>>(a1 * sg, (T)0)) : G;
  cx<T> p2 = a2 >= (T)0 ? (mag > (T)0 ? cscale(G, a2 * inv) : mk<cx<T>>(a2 * sg, (T)0)) : G;
  if constexpr (ERR) {
    if (a1 >= (T)0) { double d = (double)mag - (double)a1; err += d * d; }
    if (a2 >= (T)0) { double d = (double)mag - (double)a2; err += d * d; }
  }
  return cscale(cadd(p1, p2), scale);
}

// Single-amplitude version (used for the self-paired columns 0 and N/2).
template <typename T, bool ERR>
__device__ __forceinline__ cx<T> project1(cx<T> G, T a, bool neg, double& err) {
  T mag = sqrt(G.x * G.x + G.y * G.y);
  T sg = neg ? (T)-1 : (T)1;
  if constexpr (ERR) {
    if (a >= (T)0) { double d = (double)mag - (double)a; err += d * d; }
  }
  if (a < (T)0) return G;
  return mag > (T)0 ? cscale(G, a / mag) : mk<cx<T>>(a * sg, (T)0);
}

template <int N, typename T>
__device__ __forceinline__ void block_reduce_store(double v, double* out) {
  __shared__ double red[256];
  const int nt = blockDim.x;
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = nt / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// Column pass.  MODE 0: iteration (read P, optionally coupled; FFT_z;
// error; modulus projection; IFFT_z; write Pmid).  MODE 1: initial guess
// (generate the Hermitian part of A e^{i phi}, IFFT_z, write Pmid).
template <int N, typename T, typename AP, int MODE, bool ERR>
__global__ void __launch_bounds__(ColCfg<N>::R1* ColCfg<N>::C)
    k_col(const cx<T>* __restrict__ P, cx<T>* __restrict__ Pmid, const AP* __restrict__ A2,
          const T* __restrict__ ampscale, const cx<T>* __restrict__ tw, const int* __restrict__ alist,
          const Coupling* __restrict__ coup, int couple, double* __restrict__ errpart, int ntiles,
          uint64_t seed) {
  using Gm = ColGeom<N>;
  using C = cx<T>;
  constexpr int R1 = Gm::R1, R2 = Gm::R2, CC = Gm::C, Q = Gm::Q, H = N / 2;
  constexpr int LSTRIDE = R1 * CC + Gm::PADC;     // per c-slab
  __shared__ C lds[R2 * LSTRIDE];
  __shared__ C zl[(MODE == 0) ? N : 1];
  const int col = threadIdx.x % CC;
  const int a = threadIdx.x / CC;
  const int tile = blockIdx.x;
  const int ai = blockIdx.y;
  const int n = alist[ai];
  const int j0 = tile * CC;
  const int j = j0 + col;
  const size_t plane = (size_t)N * H;
  const T scale = (T)0.5 / ((T)N * (T)N);
  double err = 0.0;
  C g[R2];   // holds [q][d] after the forward transform (Q*R1 == R2)

  if constexpr (MODE == 0) {
    C v[R2];
    const C* Pn = P + (size_t)n * plane;
#pragma unroll
    for (int b = 0; b < R2; ++b) v[b] = Pn[(size_t)(a + R1 * b) * H + j];
    if (couple) {
      const Coupling cp = coup[n];
      const T wl = (T)cp.wl, w0 = (T)cp.w0, wr = (T)cp.wr;
      const C* Pl = P + (size_t)cp.left * plane;
      const C* Pr = P + (size_t)cp.right * plane;
      const bool ml = cp.mirror_left && j != 0, mr = cp.mirror_right && j != 0;
#pragma unroll
      for (int b = 0; b < R2; ++b) {
        C l = Pl[(size_t)(a + R1 * b) * H + j];
        C r = Pr[(size_t)(a + R1 * b) * H + j];
        if (ml) l.y = -l.y;
        if (mr) r.y = -r.y;
        v[b] = mk<C>(w0 * v[b].x + wl * l.x + wr * r.x, w0 * v[b].y + wl * l.y + wr * r.y);
      }
    }
    // forward step 1: R2-point DFT over b, twiddle W_N^{a c}
    dft<R2, -1>(v);
#pragma unroll
    for (int c = 1; c < R2; ++c) v[c] = cmul(v[c], tw[(a * c) & (N - 1)]);
#pragma unroll
    for (int c = 0; c < R2; ++c) lds[c * LSTRIDE + a * CC + col] = v[c];
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
    const AP* An = A2 + (size_t)n * plane;
    const T as = ampscale[n];
    if (j0 == 0) {
      // packed column 0 (DC and Nyquist columns): pair Z[w] with Z[-w]
      __syncthreads();
      if (col == 0) {
        sfor<0, R2>([&](auto iv) CPRA_INLINE {
          constexpr int i = decltype(iv)::value;
          constexpr int q = i / R1, d = i % R1;
          zl[a + R1 * q + R2 * d] = g[i];
        });
      }
      __syncthreads();
    }
    sfor<0, R2>([&](auto iv) CPRA_INLINE {
      constexpr int i = decltype(iv)::value;
      constexpr int q = i / R1, d = i % R1;
      {
        const int c = a + R1 * q;
        const int w = c + R2 * d;
        C Gv = g[i];
        if (j != 0) {
          auto pa = AmpIO<AP>::load(An + (size_t)w * H + j, as);
          g[i] = project2<T, ERR>(Gv, (T)pa.x, (T)pa.y, ((w + j) & 1) != 0, scale, err);
        } else {
          const int wm = (N - w) & (N - 1);
          C Zm = zl[wm];
          // Ga = (Z + conj Zm)/2, Gb = (Z - conj Zm)/(2i)
          C Ga = mk<C>((T)0.5 * (Gv.x + Zm.x), (T)0.5 * (Gv.y - Zm.y));
          C Gb = mk<C>((T)0.5 * (Gv.y + Zm.y), (T)0.5 * (Zm.x - Gv.x));
          auto p0 = AmpIO<AP>::load(An + (size_t)w * H, as);     // (A(w,0), A(w,N/2))
          auto pm = AmpIO<AP>::load(An + (size_t)wm * H, as);    // (A(-w,0), A(-w,N/2))
          double e1 = 0.0, e2 = 0.0;
          C a1 = project1<T, ERR>(Ga, (T)p0.x, (w & 1) != 0, e1);
          C a2 = project1<T, false>(Ga, (T)pm.x, (w & 1) != 0, e2);
          C b1 = project1<T, ERR>(Gb, (T)p0.y, ((w + H) & 1) != 0, e1);
          C b2 = project1<T, false>(Gb, (T)pm.y, ((w + H) & 1) != 0, e2);
          if constexpr (ERR) err += e1;
          C Gah = cscale(cadd(a1, a2), scale);
          C Gbh = cscale(cadd(b1, b2), scale);
          g[i] = mk<C>(Gah.x - Gbh.y, Gah.y + Gbh.x);   // Ga + i Gb
        }
      }
    });
  } else {
    // initial guess: Hermitian part of (-1)^{w+u} A e^{i phi}, scaled by 1/N^2
    const AP* An = A2 + (size_t)n * plane;
    const T as = ampscale[n];
    auto phase = [&](int w, int u) -> C {
      uint64_t cnt = ((uint64_t)n * N + (uint64_t)w) * N + (uint64_t)u;
      uint64_t r = splitmix64_at(seed, cnt) >> 40;
      double s, c;
      sincospi(2.0 * (double)r / 16777216.0, &s, &c);
      return mk<C>((T)c, (T)s);
    };
    sfor<0, R2>([&](auto iv) CPRA_INLINE {
      constexpr int i = decltype(iv)::value;
      constexpr int q = i / R1, d = i % R1;
      {
        const int c = a + R1 * q;
        const int w = c + R2 * d;
        const int wm = (N - w) & (N - 1);
        C out;
        if (j != 0) {
          auto pa = AmpIO<AP>::load(An + (size_t)w * H + j, as);
          T a1 = pa.x > (T)0 ? (T)pa.x : (T)0, a2 = pa.y > (T)0 ? (T)pa.y : (T)0;
          C e1 = phase(w, j), e2 = conj(phase(wm, N - j));
          T sg = ((w + j) & 1) ? -scale : scale;
          out = mk<C>(sg * (a1 * e1.x + a2 * e2.x), sg * (a1 * e1.y + a2 * e2.y));
        } else {
          auto p0 = AmpIO<AP>::load(An + (size_t)w * H, as);
          auto pm = AmpIO<AP>::load(An + (size_t)wm * H, as);
          T a0 = p0.x > 0 ? (T)p0.x : (T)0, am0 = pm.x > 0 ? (T)pm.x : (T)0;
          T aH = p0.y > 0 ? (T)p0.y : (T)0, amH = pm.y > 0 ? (T)pm.y : (T)0;
          C e1 = phase(w, 0), e2 = conj(phase(wm, 0));
          C f1 = phase(w, H), f2 = conj(phase(wm, H));
          T sa = (w & 1) ? -scale : scale, sb = ((w + H) & 1) ? -scale : scale;
          C Ga = mk<C>(sa * (a0 * e1.x + am0 * e2.x), sa * (a0 * e1.y + am0 * e2.y));
          C Gb = mk<C>(sb * (aH * f1.x + amH * f2.x), sb * (aH * f1.y + amH * f2.y));
          out = mk<C>(Ga.x - Gb.y, Ga.y + Gb.x);
        }
        g[i] = out;
      }
    });
  }

  // inverse step 1: for each owned c, R1-point IDFT over d, twiddle W_N^{-a' c}
  if constexpr (MODE == 0) __syncthreads();   // all forward reads of lds are done
  sfor<0, Q>([&](auto qv) CPRA_INLINE {
    constexpr int q = decltype(qv)::value;
    const int c = a + R1 * q;
    dft<R1, +1>(g + q * R1);
    sfor<0, R1>([&](auto av) CPRA_INLINE {
      constexpr int ap = decltype(av)::value;
      C t = g[q * R1 + ap];
      if (ap != 0) t = cmulc(t, tw[(ap * c) & (N - 1)]);
      lds[c * LSTRIDE + ap * CC + col] = t;
    });
  });
  __syncthreads();
  // inverse step 2: thread a gathers all c, R2-point IDFT -> s[a + R1 b]
  {
    C v[R2];
#pragma unroll
    for (int c = 0; c < R2; ++c) v[c] = lds[c * LSTRIDE + a * CC + col];
    dft<R2, +1>(v);
    C* Mn = Pmid + (size_t)n * plane;
#pragma unroll
    for (int b = 0; b < R2; ++b) Mn[(size_t)(a + R1 * b) * H + j] = v[b];
  }
  if constexpr (MODE == 0 && ERR) {
    block_reduce_store<N, T>(err, errpart + (size_t)ai * ntiles + tile);
  }
}

// ---------------------------------------------------------------- row pass
// MODE 0: initial guess (g <- g'); 1: HIO; 2: ER / episode estimate;
// 3: reload (P <- F_t(g) from the iterate in gin; Pmid unused, g unchanged).
// All register-array loops are compile-time (sfor) so the arrays stay in VGPRs.
template <int N, typename T>
__global__ void __launch_bounds__(RowCfg<N>::F1 / 2 * RowCfg<N>::RPB)
    k_row(const cx<T>* __restrict__ Pmid, cx<T>* __restrict__ P, const T* gin, T* gout,
          const uint32_t* __restrict__ maskw, const cx<T>* __restrict__ tw, const int* __restrict__ alist,
          const Coupling* __restrict__ coup, int couple, int mode, T beta, int positivity) {
  using Gm = RowGeom<N>;
  using C = cx<T>;
  constexpr int F1 = Gm::F1, F2 = Gm::F2, TT = Gm::T, SPT = Gm::SPT, H = N / 2;
  constexpr int RPB = Gm::RPB, MW = Gm::MW;
  constexpr int LS = F1 + Gm::PADR;       // lds stride per m2
  __shared__ C lds[RPB * F2 * LS];
  const int tau = threadIdx.x % TT;
  const int r = threadIdx.x / TT;
  const int n = alist[blockIdx.y];
  const int z = blockIdx.x * RPB + r;
  C* L0 = lds + r * F2 * LS;
  const size_t rowc = ((size_t)n * N + z) * H;     // complex row base
  const size_t rowr = ((size_t)n * N + z) * N;     // real row base
  const bool t0 = (tau == 0);
  // owned frequency classes: {tau, F1 - tau}, or {0, F1/2} for tau = 0
  const int k1v[2] = {t0 ? 0 : tau, t0 ? F1 / 2 : F1 - tau};

  C sp[SPT][F1];
  C x[2][F2];
  if (mode == 3) {
    sfor<0, SPT>([&](auto jv) CPRA_INLINE {
      constexpr int jj = decltype(jv)::value;
      sfor<0, F1>([&](auto mv) CPRA_INLINE {
        constexpr int m1 = decltype(mv)::value;
        const int m = tau + TT * jj + F2 * m1;
        sp[jj][m1] = *reinterpret_cast<const C*>(gin + rowr + 2 * m);
      });
    });
  } else {
  // ---- load Pmid row (frequency layout) and C2R pre-processing
  C f[2][F2];
  sfor<0, 2>([&](auto ss) CPRA_INLINE {
    constexpr int s = decltype(ss)::value;
    sfor<0, F2>([&](auto kk) CPRA_INLINE {
      constexpr int k2 = decltype(kk)::value;
      f[s][k2] = Pmid[rowc + k1v[s] + F1 * k2];
    });
  });
  sfor<0, 2>([&](auto ss) CPRA_INLINE {
    constexpr int s = decltype(ss)::value;
    sfor<0, F2>([&](auto kk) CPRA_INLINE {
      constexpr int k2 = decltype(kk)::value;
      // partner L - k of k = k1 + F1 k2 lives in this thread
      constexpr int pk_t0 = (s == 0) ? ((F2 - k2) % F2) : (F2 - 1 - k2);
      const C a = f[s][k2];
      const C pa = f[s][pk_t0], pb = f[1 - s][F2 - 1 - k2];
      const C pv = mk<C>(t0 ? pa.x : pb.x, t0 ? pa.y : pb.y);
      const int k = k1v[s] + F1 * k2;
      if (k == 0) {
        x[s][k2] = mk<C>(a.x + a.y, a.x - a.y);
      } else {
        const C b = conj(pv);
        const C sum = cadd(a, b), dif = csub(a, b);
        const C t = cmulc(dif, tw[k]);                 // (a - b) e^{+2 pi i k/N}
        x[s][k2] = mk<C>(sum.x - t.y, sum.y + t.x);    // sum + i t
      }
    });
  });
  // ---- C2R step 1: F2-point IDFT over k2, twiddle e^{+2 pi i k1 m2 / L}, to LDS
  sfor<0, 2>([&](auto ss) CPRA_INLINE {
    constexpr int s = decltype(ss)::value;
    dft<F2, +1>(x[s]);
    const int k1 = k1v[s];
    sfor<0, F2>([&](auto mm) CPRA_INLINE {
      constexpr int m2 = decltype(mm)::value;
      C v = x[s][m2];
      if (m2 != 0) v = cmulc(v, tw[(2 * k1 * m2) & (N - 1)]);
      L0[m2 * LS + k1] = v;
    });
  });
  __syncthreads();
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
  if (mode != 3) {
  uint32_t mwd[MW];
  const uint32_t* Mrow = maskw + (((size_t)n * N + z) * TT + tau) * MW;
  sfor<0, MW>([&](auto iv) CPRA_INLINE { mwd[decltype(iv)::value] = Mrow[decltype(iv)::value]; });
  Coupling cp{};
  if (couple) cp = coup[n];
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
          C gk = *reinterpret_cast<const C*>(gin + rowr + 2 * m);
          if (couple) {
            C lv, rv;
            if (cp.mirror_left) lv = mk<C>(gl[(N - 2 * m) & (N - 1)], gl[N - 1 - 2 * m]);
            else lv = *reinterpret_cast<const C*>(gl + 2 * m);
            if (cp.mirror_right) rv = mk<C>(gr[(N - 2 * m) & (N - 1)], gr[N - 1 - 2 * m]);
            else rv = *reinterpret_cast<const C*>(gr + 2 * m);
            gk = mk<C>(w0 * gk.x + wl * lv.x + wr * rv.x, w0 * gk.y + wl * lv.y + wr * rv.y);
          }
          out = mk<C>(g0 ? gp.x : gk.x - beta * gp.x, g1 ? gp.y : gk.y - beta * gp.y);
        }
      }
      *reinterpret_cast<C*>(gout + rowr + 2 * m) = out;
      sp[jj][m1] = out;
    });
  });
  }
  }   // mode != 3
  // ---- R2C step 1: for owned m2, F1-point DFT over m1, twiddle e^{-2 pi i m2 k1 / L}
  __syncthreads();   // everyone has read the C2R exchange
  sfor<0, SPT>([&](auto jv) CPRA_INLINE {
    constexpr int jj = decltype(jv)::value;
    const int m2 = tau + TT * jj;
    dft<F1, -1>(sp[jj]);
    sfor<0, F1>([&](auto kv) CPRA_INLINE {
      constexpr int k1 = decltype(kv)::value;
      C v = sp[jj][k1];
      if (k1 != 0) v = cmul(v, tw[(2 * k1 * m2) & (N - 1)]);
      L0[m2 * LS + k1] = v;
    });
  });
  __syncthreads();
  // ---- R2C step 2: for owned classes, F2-point DFT over m2 -> Z[k1 + F1 k2]
  sfor<0, 2>([&](auto ss) CPRA_INLINE {
    constexpr int s = decltype(ss)::value;
    const int k1 = k1v[s];
    sfor<0, F2>([&](auto mm) CPRA_INLINE {
      constexpr int m2 = decltype(mm)::value;
      x[s][m2] = L0[m2 * LS + k1];
    });
    dft<F2, -1>(x[s]);
  });
  // ---- post-processing to the packed half spectrum, store
  sfor<0, 2>([&](auto ss) CPRA_INLINE {
    constexpr int s = decltype(ss)::value;
    sfor<0, F2>([&](auto kk) CPRA_INLINE {
      constexpr int k2 = decltype(kk)::value;
      constexpr int pk_t0 = (s == 0) ? ((F2 - k2) % F2) : (F2 - 1 - k2);
      const C Z = x[s][k2];
      const C za = x[s][pk_t0], zb = x[1 - s][F2 - 1 - k2];
      const C Zp = mk<C>(t0 ? za.x : zb.x, t0 ? za.y : zb.y);
      const int k = k1v[s] + F1 * k2;
      C o;
      if (k == 0) {
        o = mk<C>(Z.x + Z.y, Z.x - Z.y);
      } else {
        const C Fe = mk<C>((T)0.5 * (Z.x + Zp.x), (T)0.5 * (Z.y - Zp.y));
        const C Fo = mk<C>((T)0.5 * (Z.y + Zp.y), (T)0.5 * (Zp.x - Z.x));
        o = cadd(Fe, cmul(Fo, tw[k]));
      }
      P[rowc + k] = o;
    });
  });
}

// ---------------------------------------------------------------- error reduce
static __global__ void k_err_reduce(const double* __restrict__ errpart, const double* __restrict__ den,
                             const int* __restrict__ alist, int nact, int ntiles, int nslots,
                             double* __restrict__ hist) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nslots * nact) return;
  int slot = i / nact, ai = i % nact;
  const double* p = errpart + ((size_t)slot * nact + ai) * ntiles;
  double s = 0.0;
  for (int t = 0; t < ntiles; ++t) s += p[t];
  double d = den[alist[ai]];
  hist[i] = d > 0.0 ? sqrt(s / d) : sqrt(s);
}

}  // namespace cpra
