// Shrinkwrap support update on the device: periodic separable Gaussian blur of the current
// objects, threshold at a fraction of each plane's maximum, support bits rewritten in the row
// pass's thread order.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace cpra {

// c[z][t] = sum_{d=-W..W} k[d + W] g[z][(t - d) mod N] for the listed slots; grid (N rows, count)
template <int N, typename T>
__global__ void __launch_bounds__(256) k_blur_rows(const T* __restrict__ g, const int* __restrict__ list,
                                                   const T* __restrict__ k, int W, T* __restrict__ out) {
  __shared__ T row[N];
  const int z = blockIdx.x, ai = blockIdx.y;
  const T* x = g + ((size_t)list[ai] * N + z) * N;
  for (int t = threadIdx.x; t < N; t += 256) row[t] = x[t];
  __syncthreads();
  T* o = out + ((size_t)ai * N + z) * N;
  for (int t = threadIdx.x; t < N; t += 256) {
    T acc = (T)0;
    for (int d = -W; d <= W; ++d) acc += k[d + W] * row[wrapN<N>(t - d)];
    o[t] = acc;
  }
}

// b[z][t] = sum_d k[d + W] c[(z - d) mod N][t], in place over CB columns per workgroup, with the
// workgroup's maximum of b in pmax[ai * (N / CB) + blockIdx.x]; grid (N / CB, count)
template <int N, typename T, int CB>
__global__ void __launch_bounds__(256) k_blur_cols(T* __restrict__ buf, const T* __restrict__ k, int W,
                                                   double* __restrict__ pmax) {
  __shared__ T col[N * CB];
  __shared__ double red[256];
  const int ai = blockIdx.y, t0 = blockIdx.x * CB;
  T* x = buf + (size_t)ai * N * N;
  for (int i = threadIdx.x; i < N * CB; i += 256) col[i] = x[(size_t)(i / CB) * N + t0 + i % CB];
  __syncthreads();
  double m = -HUGE_VAL;
  for (int i = threadIdx.x; i < N * CB; i += 256) {
    const int z = i / CB, c = i % CB;
    T acc = (T)0;
    for (int d = -W; d <= W; ++d) acc += k[d + W] * col[(wrapN<N>(z - d)) * CB + c];
    x[(size_t)z * N + t0 + c] = acc;
    m = fmax(m, (double)acc);
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) pmax[(size_t)ai * (N / CB) + blockIdx.x] = red[0];
}

// Support bits of data angle list[ai] from its blurred plane: b >= frac * max(b); grid (N, count)
template <int N, typename T, int CB>
__global__ void __launch_bounds__(256) k_shrink_mask(const T* __restrict__ buf, const int* __restrict__ list,
                                                     const double* __restrict__ pmax, double frac,
                                                     uint32_t* __restrict__ maskw) {
  using G = RowGeom<N>;
  __shared__ double thr;
  const int z = blockIdx.x, ai = blockIdx.y;
  if (threadIdx.x == 0) {
    double m = -HUGE_VAL;
    for (int i = 0; i < N / CB; ++i) m = fmax(m, pmax[(size_t)ai * (N / CB) + i]);
    thr = frac * m;
  }
  __syncthreads();
  const T* b = buf + ((size_t)ai * N + z) * N;
  uint32_t* Mz = maskw + ((size_t)list[ai] * N + z) * G::T * G::MW;
  for (int r = threadIdx.x; r < G::T * G::MW; r += 256) {
    const int tau = r / G::MW, wd = r % G::MW;
    uint32_t word = 0;
    for (int bit = 0; bit < 32; ++bit) {
      const int t = mask_bit_t<N>(tau, wd * 32 + bit);
      if (t >= 0 && (double)b[t] >= thr) word |= (1u << bit);
    }
    Mz[r] = word;
  }
}

}  // namespace cpra
