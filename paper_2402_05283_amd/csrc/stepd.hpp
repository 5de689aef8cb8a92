// Step D on the device: Fourier-slice insertion and the 3D inverse FFT,
// factorised per z-plane.
//
// The insertion weights do not depend on the frequency w along z, so the
// inverse transform along z undoes the forward one exactly:
//   F3^-1[Insert(F2 O'_n)] = F2^-1_xy[Insert_z(F_t O'_n)]   for every z.
// The row spectra F_t O'_n are the packed P rows the iteration keeps, so
// step D needs no N^3 complex grid: per z-plane it gathers
//   Q_z[ky][kx] = (-1)^(ky+kx) / cnt(ky,kx) * sum_{(n,u) in cell} (-1)^u S_n[z][u]
// (the signs move the origin of u, ky, kx to the array centre) and the
// volume slice is Re F2^-1(Q_z) / N^2, written centred [z][y][x].
#pragma once
#include "kernels.hpp"

namespace cpra {

// decomposition of the length-N inverse transforms of step D: N = R1 * R2,
// R1 threads per row / column with R2 values each (R2 a multiple of R1)
template <int N> struct StepdCfg;
template <> struct StepdCfg<64> { static constexpr int R1 = 8, R2 = 8; };
template <> struct StepdCfg<128> { static constexpr int R1 = 8, R2 = 16; };
template <> struct StepdCfg<256> { static constexpr int R1 = 16, R2 = 16; };
template <> struct StepdCfg<192> { static constexpr int R1 = 8, R2 = 24; };
template <> struct StepdCfg<384> { static constexpr int R1 = 8, R2 = 48; };
template <> struct StepdCfg<512> { static constexpr int R1 = 16, R2 = 32; };
template <> struct StepdCfg<1024> { static constexpr int R1 = 32, R2 = 32; };

// largest power-of-two count <= want whose LDS (per_line complex values each) fits 128 KiB
template <int N, typename T> constexpr int stepd_lines(int want, size_t per_line) {
  int k = want;
  while (k > 1 && (size_t)k * per_line * sizeof(cx<T>) > 131072) k /= 2;
  return k;
}

// Staging of a chunk of z-planes: rows z0 .. z0+nz-1 of every angle's packed half spectrum into
// Tz[zi][n][j] (contiguous per plane), so that the gather of one plane reads one contiguous block
// of N_p N/2 values instead of N_p rows scattered over the angles' planes.  grid (nz, Np).
template <int N, typename T>
__global__ void __launch_bounds__(256) k_stepd_stage(const cx<T>* __restrict__ P, cx<T>* __restrict__ Tz, int z0,
                                                     int Np) {
  constexpr int H = N / 2;
  const int zi = blockIdx.x, n = blockIdx.y;
  const cx<T>* Pn = P + (size_t)n * N * H;
  cx<T>* out = Tz + ((size_t)zi * Np + n) * H;
  for (int j = threadIdx.x; j < H; j += blockDim.x) out[j] = Pn[pix<N>(z0 + zi, j)];
}

// S[z][u] of an angle from its packed half spectrum Pn (layout pix<N>)
template <int N, typename T>
__device__ __forceinline__ cx<T> spectrum_at(const cx<T>* Pn, int z, int u) {
  constexpr int H = N / 2;
  using C = cx<T>;
  if (u == 0) return mk<C>(Pn[pix<N>(z, 0)].x, (T)0);
  if (u == H) return mk<C>(Pn[pix<N>(z, 0)].y, (T)0);
  if (u < H) return Pn[pix<N>(z, u)];
  return conj(Pn[pix<N>(z, N - u)]);
}

// Per cell (ky, kx) of the insertion grid, one 16-byte record: the first entry's code n N + u (or
// -1 for an empty cell), the CSR range [begin, end) of all its entries, and the inverse count (or
// inverse weight sum) as FP32 bits.  One load gives what a cell with a single entry needs.
struct CellRec {
  int first, begin, end, inv_bits;
};

// Cells with more than kStepdHeavy entries (the cells near k = 0: the zero-frequency cell holds one
// entry per angle) are left out of the per-cell gather, whose time is set by its longest chain of
// dependent loads, and summed by k_stepd_heavy, one wavefront per (cell, plane).  Their records in
// the gather's table carry first = -2 (the gather skips them); the heavy list holds their real
// records with first = the cell index.
constexpr int kStepdHeavy = 16;

// Gather: Q_z[ky][kx] = (-1)^(ky+kx) / cnt(ky,kx) * sum over the cell's entries (n, u) of
// (-1)^u S_n[z][u] (bilinear: weighted), into the plane buffer.  One thread per (cell, group of
// kStepdZP planes): the cell's record and entry codes are read once for the group, and each entry
// is one load per plane, all independent.  No LDS, so many waves are resident to hide the loads.
// A cell's entries are summed in CSR order for every plane.  Heavy cells (first = -2) are left to
// k_stepd_heavy.  1D grid of (N^2 / 256) * (nz / kStepdZP) workgroups; with 8 or more plane groups,
// XCD x (workgroup L mod 8) takes groups [x G/8, (x+1) G/8) whole, so the staged rows those planes
// read stay in its L2.
constexpr int kStepdZP = 4;
template <int N, typename T>
__global__ void __launch_bounds__(256)
    k_stepd_gather(const cx<T>* __restrict__ Tz, int Np, const CellRec* __restrict__ cells,
                   const int* __restrict__ ent, const T* __restrict__ wts, const T* __restrict__ cnt_inv,
                   cx<T>* __restrict__ plane, int nz) {
  using C = cx<T>;
  constexpr int H = N / 2, CBLK = N * N / 256, ZP = kStepdZP;
  const int G = nz / ZP;
  const int L = blockIdx.x;
  int zg, cb;
  if (G % 8 == 0) {
    const int x = L % 8, k = L / 8;
    zg = x * (G / 8) + k / CBLK;
    cb = k % CBLK;
  } else {
    zg = L / CBLK;
    cb = L % CBLK;
  }
  const int cell = cb * 256 + threadIdx.x;
  const int ky = cell / N, kx = cell % N;
  const CellRec rec = cells[cell];
  if (rec.first == -2) return;          // summed by k_stepd_heavy
  const size_t pstride = (size_t)Np * H;   // one plane's rows of every angle
  const C* Tp = Tz + (size_t)zg * ZP * pstride;
  C v[ZP];
  // v (first) or v + (-1)^u S_n[z][u] for the group's planes, from the packed rows of angle n:
  // S[u] = P[u] (u < N/2), conj P[N-u] (u > N/2), Re P[0] (u = 0), Im P[0] (u = N/2)
  auto take = [&](int e, int code, bool first) CPRA_INLINE {
    const int n = code / N, u = code % N;
    const int j = u <= H ? (u == H ? 0 : u) : N - u;
    const C* src = Tp + (size_t)n * H + j;
    C p[ZP];
#pragma unroll
    for (int z = 0; z < ZP; ++z) p[z] = src[(size_t)z * pstride];
    const T w = wts ? wts[e] : (T)1;
#pragma unroll
    for (int z = 0; z < ZP; ++z) {
      T re = u == H ? p[z].y : p[z].x;
      T im = (u == 0 || u == H) ? (T)0 : (u > H ? -p[z].y : p[z].y);
      if (u & 1) { re = -re; im = -im; }
      C sv = mk<C>(re, im);
      if (wts) sv = cscale(sv, w);      // bilinear insertion weight
      v[z] = first ? sv : cadd(v[z], sv);
    }
  };
  if (rec.first >= 0) {
    take(rec.begin, rec.first, true);
  } else {
#pragma unroll
    for (int z = 0; z < ZP; ++z) v[z] = mk<C>((T)0, (T)0);
  }
  for (int e = rec.begin + 1; e < rec.end; ++e) take(e, ent[e], false);
  T f;
  if constexpr (std::is_same<T, float>::value) f = __int_as_float(rec.inv_bits);
  else f = cnt_inv[cell];
  if ((ky + kx) & 1) f = -f;
#pragma unroll
  for (int z = 0; z < ZP; ++z) plane[(size_t)(zg * ZP + z) * N * N + cell] = cscale(v[z], f);
}

// The heavy cells of the gather: one wavefront per (heavy cell, plane), lane l summing entries
// begin + l, begin + l + 64, ... in order, then a butterfly sum over the 64 lanes.  grid
// (n_heavy / 4 rounded up, nz), 4 wavefronts per workgroup.
template <int N, typename T>
__global__ void __launch_bounds__(256)
    k_stepd_heavy(const cx<T>* __restrict__ Tz, int Np, const CellRec* __restrict__ heavy, int n_heavy,
                  const int* __restrict__ ent, const T* __restrict__ wts, const T* __restrict__ cnt_inv,
                  cx<T>* __restrict__ plane) {
  using C = cx<T>;
  constexpr int H = N / 2;
  const int h = blockIdx.x * 4 + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  const int zi = blockIdx.y;
  if (h >= n_heavy) return;             // whole wavefronts leave together
  const CellRec rec = heavy[h];
  const int cell = rec.first;
  const C* Tp = Tz + (size_t)zi * Np * H;
  T re = 0, im = 0;
  for (int e = rec.begin + lane; e < rec.end; e += 64) {
    const int code = ent[e];
    const int n = code / N, u = code % N;
    const int j = u <= H ? (u == H ? 0 : u) : N - u;
    const C p = Tp[(size_t)n * H + j];
    T sr = u == H ? p.y : p.x;
    T si = (u == 0 || u == H) ? (T)0 : (u > H ? -p.y : p.y);
    if (u & 1) { sr = -sr; si = -si; }
    if (wts) {
      const T w = wts[e];
      sr *= w;
      si *= w;
    }
    re += sr;
    im += si;
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    re += __shfl_xor(re, m);
    im += __shfl_xor(im, m);
  }
  if (lane == 0) {
    const int ky = cell / N, kx = cell % N;
    T f;
    if constexpr (std::is_same<T, float>::value) f = __int_as_float(rec.inv_bits);
    else f = cnt_inv[cell];
    if ((ky + kx) & 1) f = -f;
    plane[(size_t)zi * N * N + cell] = mk<C>(re * f, im * f);
  }
}

// Rows: inverse transform of the gathered Q_z[ky][:] along kx, in place in the plane buffer.
// Block: RB rows x R1 threads; grid: (N / RB) * nz, planes of an XCD as in the gather.
template <int N, typename T, int RB>
__global__ void __launch_bounds__(StepdCfg<N>::R1* RB)
    k_stepd_rows(const cx<T>* __restrict__ tw, cx<T>* __restrict__ plane, int nz) {
  using C = cx<T>;
  constexpr int R1 = StepdCfg<N>::R1, R2 = StepdCfg<N>::R2, Q = R2 / R1;
  static_assert(R1 * R2 == N && Q >= 1 && R2 % R1 == 0, "step D decomposition");
  constexpr int LS = R1 + 1;
  __shared__ C lds[RB * R2 * LS];
  const int a = threadIdx.x % R1;
  const int r = threadIdx.x / R1;
  constexpr int KB = N / RB;
  const int L = blockIdx.x;
  int zi, kyb;
  if (nz % 8 == 0) {
    const int x = L % 8, k = L / 8;
    zi = x * (nz / 8) + k / KB;
    kyb = k % KB;
  } else {
    zi = L / KB;
    kyb = L % KB;
  }
  const int ky = kyb * RB + r;
  C* L0 = lds + r * R2 * LS;
  C* row = plane + ((size_t)zi * N + ky) * N;
  C v[R2];
#pragma unroll
  for (int b = 0; b < R2; ++b) v[b] = row[a + R1 * b];
  // inverse four-step along kx = a + R1 b -> x = c + R2 d
  dft<R2, +1>(v);
#pragma unroll
  for (int c = 0; c < R2; ++c) L0[c * LS + a] = (c == 0 || a == 0) ? v[c] : cmulc(v[c], tw[wrapN<N>(a * c)]);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int c = a + R1 * q;
    C u[R1];
#pragma unroll
    for (int ap = 0; ap < R1; ++ap) u[ap] = L0[c * LS + ap];
    dft<R1, +1>(u);
#pragma unroll
    for (int d = 0; d < R1; ++d) row[c + R2 * d] = u[d];
  }
}

// Columns: inverse transform along ky, real part / N^2 -> volume [z][y][x].
// Block: C columns x R1 threads; grid: (N / C, zc).
template <int N, typename T, int CC>
__global__ void __launch_bounds__(StepdCfg<N>::R1* CC)
    k_stepd_cols(const cx<T>* __restrict__ plane, const cx<T>* __restrict__ tw, T* __restrict__ vol, int z0) {
  using C = cx<T>;
  constexpr int R1 = StepdCfg<N>::R1, R2 = StepdCfg<N>::R2, Q = R2 / R1;
  constexpr int LSTRIDE = R1 * CC + 1;
  __shared__ C lds[R2 * LSTRIDE];
  const int col = threadIdx.x % CC;
  const int a = threadIdx.x / CC;
  const int x = blockIdx.x * CC + col;
  const int zi = blockIdx.y;
  const C* in = plane + (size_t)zi * N * N;
  C v[R2];
#pragma unroll
  for (int b = 0; b < R2; ++b) v[b] = in[(size_t)(a + R1 * b) * N + x];
  dft<R2, +1>(v);
#pragma unroll
  for (int c = 0; c < R2; ++c)
    lds[c * LSTRIDE + a * CC + col] = (c == 0 || a == 0) ? v[c] : cmulc(v[c], tw[wrapN<N>(a * c)]);
  __syncthreads();
  const T norm = (T)1 / ((T)N * (T)N);
  T* out = vol + (size_t)(z0 + zi) * N * N;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int c = a + R1 * q;
    C u[R1];
#pragma unroll
    for (int ap = 0; ap < R1; ++ap) u[ap] = lds[c * LSTRIDE + ap * CC + col];
    dft<R1, +1>(u);
#pragma unroll
    for (int d = 0; d < R1; ++d) out[(size_t)(c + R2 * d) * N + x] = u[d].x * norm;
  }
}

// tw: W_N^j, j < N (the first N entries of the plan's twiddle table)
template <int N, typename T>
void stepd_run(const cx<T>* P, int Np, cx<T>* Tz, const CellRec* cells, const CellRec* heavy, int n_heavy,
               const int* ent, const T* wts, const T* cnt_inv, const cx<T>* tw, cx<T>* plane, int zc, T* vol,
               hipStream_t st) {
  constexpr int R1 = StepdCfg<N>::R1, R2 = StepdCfg<N>::R2;
  // rows / columns per workgroup: up to 256 threads, LDS within 128 KiB
  constexpr int RB = stepd_lines<N, T>(256 / R1 < N ? 256 / R1 : N, (size_t)R2 * (R1 + 1));
  constexpr int CC = stepd_lines<N, T>(256 / R1 < N ? 256 / R1 : N, (size_t)R2 * R1);
  for (int z0 = 0; z0 < N; z0 += zc) {
    const int nz = (N - z0) < zc ? (N - z0) : zc;
    k_stepd_stage<N, T><<<dim3(nz, Np), 256, 0, st>>>(P, Tz, z0, Np);
    k_stepd_gather<N, T><<<(N * N / 256) * (nz / kStepdZP), 256, 0, st>>>(Tz, Np, cells, ent, wts, cnt_inv,
                                                                          plane, nz);
    if (n_heavy > 0)
      k_stepd_heavy<N, T><<<dim3((n_heavy + 3) / 4, nz), 256, 0, st>>>(Tz, Np, heavy, n_heavy, ent, wts, cnt_inv,
                                                                        plane);
    k_stepd_rows<N, T, RB><<<(N / RB) * nz, R1 * RB, 0, st>>>(tw, plane, nz);
    k_stepd_cols<N, T, CC><<<dim3(N / CC, nz), R1 * CC, 0, st>>>(plane, tw, vol, z0);
  }
}

}  // namespace cpra
