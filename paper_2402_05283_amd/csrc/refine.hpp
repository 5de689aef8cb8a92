// 3D refinement after step D on the device.  The inserted spectrum fills whole k_z lines, so the
// 3D Fourier constraint separates per z-plane: in the mixed domain (z, k_y, k_x) the measured
// values Q(z, k_y, k_x) are those step D gathers before its (k_y, k_x) inverse transform.  One
// iteration per plane: 2D FFT of the centred real plane, Q imposed on the measured cells, 2D
// inverse, real part, support and positivity (error reduction).  Plain complex line FFTs through
// LDS (four-step StepdCfg decomposition); this runs a few tens of times per reconstruction.
#pragma once
#include <hip/hip_runtime.h>

#include "stepd.hpp"

namespace cpra {

constexpr int kRefLines = 4;   // lines (rows or columns) per workgroup

// In-place FFT of the line held in LDS (natural order in and out), SIGN -1 forward, +1 inverse,
// unnormalised; thread a = 0 .. R1-1 of the line's group; scr: R2 x (R1+1) slots of the group.
// Every thread of the workgroup must call it (it synchronises).
template <int N, typename T, int SIGN>
__device__ __forceinline__ void line_fft(cx<T>* line, cx<T>* scr, const cx<T>* __restrict__ tw, int a) {
  using C = cx<T>;
  constexpr int R1 = StepdCfg<N>::R1, R2 = StepdCfg<N>::R2, Q = R2 / R1, LS = R1 + 1;
  C v[R2];
#pragma unroll
  for (int b = 0; b < R2; ++b) v[b] = line[a + R1 * b];
  dft<R2, SIGN>(v);
#pragma unroll
  for (int c = 0; c < R2; ++c) {
    const C w = tw[wrapN<N>(a * c)];   // W_N^{ac} = exp(-2 pi i a c / N)
    scr[c * LS + a] = (c == 0 || a == 0) ? v[c] : (SIGN < 0 ? cmul(v[c], w) : cmulc(v[c], w));
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int c = a + R1 * q;
    C u[R1];
#pragma unroll
    for (int ap = 0; ap < R1; ++ap) u[ap] = scr[c * LS + ap];
    dft<R1, SIGN>(u);
#pragma unroll
    for (int d = 0; d < R1; ++d) line[c + R2 * d] = u[d];
  }
  __syncthreads();
}

// Step D's gather of cell (ky, kx) at plane z: sum of the inserted samples times 1/count (or
// 1/sum of weights) and the centring sign (-1)^(ky+kx); *hit = whether the cell has samples.
template <int N, typename T>
__device__ __forceinline__ cx<T> gather_cell(const cx<T>* __restrict__ P, const int* __restrict__ ptr,
                                             const int* __restrict__ ent, const T* __restrict__ wts,
                                             const T* __restrict__ cnt_inv, int z, int ky, int kx, bool* hit) {
  using C = cx<T>;
  constexpr int H = N / 2;
  const int cell = ky * N + kx;
  C acc = mk<C>((T)0, (T)0);
  const int e1 = ptr[cell + 1];
  *hit = ptr[cell] < e1;
  for (int e = ptr[cell]; e < e1; ++e) {
    const int code = ent[e];
    const int n = code / N, u = code % N;
    C s = spectrum_at<N, T>(P + (size_t)n * N * H, z, u);
    if (u & 1) { s.x = -s.x; s.y = -s.y; }
    if (wts) s = cscale(s, wts[e]);
    acc = cadd(acc, s);
  }
  T f = cnt_inv[cell];
  if ((ky + kx) & 1) f = -f;
  return cscale(acc, f);
}

// Q_h(z, q) = (Q(z, q) + conj Q(z, -q)) / 2 on the measured cells and their mirrors, NaN (free)
// elsewhere; Qh is [z][ky][kx], native (ky, kx).  grid (N ky, N z), 256 threads over kx.
template <int N, typename T>
__global__ void __launch_bounds__(256) k_ref_gather(const cx<T>* __restrict__ P, const int* __restrict__ ptr,
                                                    const int* __restrict__ ent, const T* __restrict__ wts,
                                                    const T* __restrict__ cnt_inv, cx<T>* __restrict__ Qh) {
  using C = cx<T>;
  const int ky = blockIdx.x, z = blockIdx.y;
  const int mky = wrapN<N>(N - ky);
  for (int kx = threadIdx.x; kx < N; kx += 256) {
    bool h1, h2;
    const C a = gather_cell<N, T>(P, ptr, ent, wts, cnt_inv, z, ky, kx, &h1);
    const C b = gather_cell<N, T>(P, ptr, ent, wts, cnt_inv, z, mky, wrapN<N>(N - kx), &h2);
    C out;
    if (h1 || h2) {
      const C av = h1 ? a : mk<C>((T)0, (T)0), bv = h2 ? b : mk<C>((T)0, (T)0);
      out = mk<C>((T)0.5 * (av.x + bv.x), (T)0.5 * (av.y - bv.y));
    } else {
      out = mk<C>((T)NAN, (T)0);
    }
    Qh[((size_t)z * N + ky) * N + kx] = out;
  }
}

// Bit of support pixel (z, t) of a data angle in the row pass's thread order (inverse of
// mask_bit_t): word index within the angle's mask, and bit.
template <int N>
__device__ __forceinline__ void mask_word_bit(int z, int t, size_t* word, int* bit) {
  using G = RowGeom<N>;
  const int m = t >> 1, e = t & 1;
  const int m1 = m / G::F2, rem = m % G::F2;
  const int tau = rem % G::T, j = rem / G::T;
  const int b = 2 * (j * G::F1 + m1) + e;
  *word = ((size_t)z * G::T + tau) * G::MW + (b >> 5);
  *bit = b & 31;
}

// 3D support: voxel (z, y, x) (centred) is in it when, for every listed angle n, the projected
// coordinate t = floor(y cos - x sin + 1/2) (FP64, no contraction) lands in angle n's 2D support
// at row z.  sc: (sin, cos) per listed angle.  grid (N y, N z), 256 threads over x.
template <int N>
__global__ void __launch_bounds__(256) k_ref_support(const uint32_t* __restrict__ maskw, const int* __restrict__ list,
                                                     const double* __restrict__ sc, int count,
                                                     uint8_t* __restrict__ S3) {
  using G = RowGeom<N>;
  const int y = blockIdx.x, z = blockIdx.y;
  const double yc = (double)(y - N / 2);
  for (int x = threadIdx.x; x < N; x += 256) {
    const double xc = (double)(x - N / 2);
    bool in = true;
    for (int i = 0; i < count && in; ++i) {
      const double t = floor(__dadd_rn(__dsub_rn(__dmul_rn(yc, sc[2 * i + 1]), __dmul_rn(xc, sc[2 * i])), 0.5));
      const int ti = (int)t + N / 2;
      if (ti < 0 || ti >= N) { in = false; break; }
      size_t w;
      int b;
      mask_word_bit<N>(z, ti, &w, &b);
      in = (maskw[(size_t)list[i] * N * G::T * G::MW + w] >> b) & 1u;
    }
    S3[((size_t)z * N + y) * N + x] = in ? 1 : 0;
  }
}

// Rows of all planes (row r = z * N + y), kRefLines per workgroup.  FIRST: C = F_x(V).
// Otherwise: v = Re F_x^-1(C) / N^2, error reduction with the support (and positivity) into V,
// then C = F_x(v).
template <int N, typename T, bool FIRST>
__global__ void __launch_bounds__(StepdCfg<N>::R1* kRefLines)
    k_ref_rows(cx<T>* __restrict__ Cb, T* __restrict__ V, const uint8_t* __restrict__ S3, int positivity,
               const cx<T>* __restrict__ tw) {
  using C = cx<T>;
  constexpr int R1 = StepdCfg<N>::R1, R2 = StepdCfg<N>::R2, SCR = R2 * (R1 + 1);
  __shared__ C lds[kRefLines * (N + SCR)];
  const int l = threadIdx.x / R1, a = threadIdx.x % R1;
  const size_t r = (size_t)blockIdx.x * kRefLines + l;
  C* line = lds + l * (N + SCR);
  C* scr = line + N;
  C* crow = Cb + r * N;
  T* vrow = V + r * N;
  const uint8_t* srow = S3 + r * N;
  if constexpr (FIRST) {
    for (int x = a; x < N; x += R1) line[x] = mk<C>(vrow[x], (T)0);
    __syncthreads();
  } else {
    for (int x = a; x < N; x += R1) line[x] = crow[x];
    __syncthreads();
    line_fft<N, T, +1>(line, scr, tw, a);
    const T norm = (T)1 / ((T)N * (T)N);
    for (int x = a; x < N; x += R1) {
      T v = line[x].x * norm;
      if (!srow[x] || (positivity && v < (T)0)) v = (T)0;
      vrow[x] = v;
      line[x] = mk<C>(v, (T)0);
    }
    __syncthreads();
  }
  line_fft<N, T, -1>(line, scr, tw, a);
  for (int x = a; x < N; x += R1) crow[x] = line[x];
}

// Columns (k_x) of one plane, kRefLines per workgroup: F_y, the measured values imposed where Qh
// is not NaN, F_y^-1.  grid (N / kRefLines, N z).
template <int N, typename T>
__global__ void __launch_bounds__(StepdCfg<N>::R1* kRefLines)
    k_ref_cols(cx<T>* __restrict__ Cb, const cx<T>* __restrict__ Qh, const cx<T>* __restrict__ tw) {
  using C = cx<T>;
  constexpr int R1 = StepdCfg<N>::R1, R2 = StepdCfg<N>::R2, SCR = R2 * (R1 + 1);
  __shared__ C lds[kRefLines * (N + SCR)];
  const int l = threadIdx.x / R1, a = threadIdx.x % R1;
  const int kx = blockIdx.x * kRefLines + l, z = blockIdx.y;
  C* line = lds + l * (N + SCR);
  C* scr = line + N;
  C* plane = Cb + (size_t)z * N * N;
  const C* qp = Qh + (size_t)z * N * N;
  for (int y = a; y < N; y += R1) line[y] = plane[(size_t)y * N + kx];
  __syncthreads();
  line_fft<N, T, -1>(line, scr, tw, a);
  for (int ky = a; ky < N; ky += R1) {
    const C q = qp[(size_t)ky * N + kx];
    if (q.x == q.x) line[ky] = q;       // measured cell (NaN marks a free one)
  }
  __syncthreads();
  line_fft<N, T, +1>(line, scr, tw, a);
  for (int y = a; y < N; y += R1) plane[(size_t)y * N + kx] = line[y];
}

// z-direction blur of the 3D shrinkwrap, in place over CB x-values of one y per workgroup, with the
// workgroup's maximum; grid (N / CB, N y).
template <int N, typename T, int CB>
__global__ void __launch_bounds__(256) k_blur_z(T* __restrict__ buf, const T* __restrict__ k, int W,
                                                double* __restrict__ pmax) {
  __shared__ T col[N * CB];
  __shared__ double red[256];
  const int x0 = blockIdx.x * CB, y = blockIdx.y;
  for (int i = threadIdx.x; i < N * CB; i += 256) col[i] = buf[((size_t)(i / CB) * N + y) * N + x0 + i % CB];
  __syncthreads();
  double m = -HUGE_VAL;
  for (int i = threadIdx.x; i < N * CB; i += 256) {
    const int z = i / CB, c = i % CB;
    T acc = (T)0;
    for (int d = -W; d <= W; ++d) acc += k[d + W] * col[(wrapN<N>(z - d)) * CB + c];
    buf[((size_t)z * N + y) * N + x0 + c] = acc;
    m = fmax(m, (double)acc);
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) pmax[(size_t)y * (N / CB) + blockIdx.x] = red[0];
}

// S3 = blurred >= frac * max (max over the npart partial maxima); one workgroup reduces the
// partials first (grid 1), then the threshold runs over all voxels.
static __global__ void __launch_bounds__(256) k_max_reduce(double* __restrict__ pmax, int npart) {
  __shared__ double red[256];
  double m = -HUGE_VAL;
  for (int i = threadIdx.x; i < npart; i += 256) m = fmax(m, pmax[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) pmax[npart] = red[0];
}

template <typename T>
__global__ void __launch_bounds__(256) k_threshold(const T* __restrict__ buf, size_t n, const double* __restrict__ mx,
                                                   double frac, uint8_t* __restrict__ S3) {
  const double thr = frac * mx[0];
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    S3[i] = (double)buf[i] >= thr ? 1 : 0;
}

}  // namespace cpra
