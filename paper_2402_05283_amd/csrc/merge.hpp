// Step C of the paper's schedule on the device: per-PO mass moments, the twin test against the
// reference guess, and the average of the kept guesses after their shifts and inversions.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace cpra {

template <int NT>
__device__ __forceinline__ void block_sum3(double& a, double& b, double& c) {
  __shared__ double red[3][NT];
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  red[2][threadIdx.x] = c;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      red[0][threadIdx.x] += red[0][threadIdx.x + s];
      red[1][threadIdx.x] += red[1][threadIdx.x + s];
      red[2][threadIdx.x] += red[2][threadIdx.x + s];
    }
    __syncthreads();
  }
  a = red[0][0];
  b = red[1][0];
  c = red[2][0];
}

// out[3 b + (0, 1, 2)] = (sum g, sum g (z - N/2), sum g (t - N/2)) over the centred plane of
// slot list[b]; FP64, fixed summation order.  256 threads per block.
template <int N, typename T>
__global__ void __launch_bounds__(256) k_moments(const T* __restrict__ g, const int* __restrict__ list,
                                                 double* __restrict__ out) {
  const T* x = g + (size_t)list[blockIdx.x] * N * N;
  double s0 = 0.0, sz = 0.0, st = 0.0;
  for (int p = threadIdx.x; p < N * N; p += 256) {
    const double v = (double)x[p];
    s0 += v;
    sz += v * (double)(p / N - N / 2);
    st += v * (double)(p % N - N / 2);
  }
  block_sum3<256>(s0, sz, st);
  if (threadIdx.x == 0) {
    out[3 * blockIdx.x + 0] = s0;
    out[3 * blockIdx.x + 1] = sz;
    out[3 * blockIdx.x + 2] = st;
  }
}

// Twin test of one kept guess per block against the reference:
//   same = sum (S_j X_j - S_ref X_ref)^2,  inv = sum (I S_j X_j - S_ref X_ref)^2,
// S = cyclic shift (out[z][t] = x[z - s_z][t - s_t]), I = central inversion (i -> N - i mod N).
// slot[b], shift[2 b..]: the guess's PO and its shift; slot/shift of the reference at index 0.
template <int N, typename T>
__global__ void __launch_bounds__(256) k_twin_dist(const T* __restrict__ g, const int* __restrict__ slot,
                                                   const int* __restrict__ shift, double* __restrict__ out) {
  const int b = blockIdx.x;
  const T* xr = g + (size_t)slot[0] * N * N;
  const T* xj = g + (size_t)slot[b] * N * N;
  const int rz = shift[0], rt = shift[1], jz = shift[2 * b], jt = shift[2 * b + 1];
  double same = 0.0, inv = 0.0, unused = 0.0;
  for (int p = threadIdx.x; p < N * N; p += 256) {
    const int z = p / N, t = p % N;
    const double ref = (double)xr[(wrapN<N>(z - rz)) * N + (wrapN<N>(t - rt))];
    const double a = (double)xj[(wrapN<N>(z - jz)) * N + (wrapN<N>(t - jt))];
    const double c = (double)xj[(wrapN<N>(N - z - jz)) * N + (wrapN<N>(N - t - jt))];
    same += (a - ref) * (a - ref);
    inv += (c - ref) * (c - ref);
  }
  block_sum3<256>(same, inv, unused);
  if (threadIdx.x == 0) {
    out[2 * b] = same;
    out[2 * b + 1] = inv;
  }
}

// Final episode: out[n][z][t] = (1/K) sum_j (I^inv_j S_{j,n} X_{keep_j, n})[z][t] for the K kept
// guesses in rank order; FP64 sum in rank order.  grid (N rows z, Np angles); 256 threads stride
// over the row.
template <int N, typename T>
__global__ void __launch_bounds__(256) k_merge_avg(const T* __restrict__ g, int npd, int K,
                                                   const int* __restrict__ keep, const int* __restrict__ inv,
                                                   const int* __restrict__ shift, T* __restrict__ out) {
  const int z = blockIdx.x, n = blockIdx.y;
  for (int t = threadIdx.x; t < N; t += 256) {
    double acc = 0.0;
    for (int j = 0; j < K; ++j) {
      const T* x = g + ((size_t)keep[j] * npd + n) * N * N;
      const int sz = shift[2 * (j * npd + n)], st = shift[2 * (j * npd + n) + 1];
      const int zz = inv[j] ? N - z : z, tt = inv[j] ? N - t : t;
      acc += (double)x[(wrapN<N>(zz - sz)) * N + (wrapN<N>(tt - st))];
    }
    out[((size_t)n * N + z) * N + t] = (T)(acc / (double)K);
  }
}

}  // namespace cpra
