// Host-only geometry and bookkeeping of the CPRA library (no GPU calls).
//
// Built with -ffp-contract=off so that the FP64 slice rounding is the plain
// IEEE sequence (product, add 0.5, floor) on every build.
#include <cmath>
#include <cstdint>
#include <vector>

#include "host_geom.hpp"

namespace cpra_host {

double default_theta(int n, int Np) { return M_PI * (double)n / (double)Np; }

// Nearest voxel of the Fourier slice of angle theta (rotation about z):
// centred frequency u maps to (kx, ky) = (-u sin t, u cos t), rounded with
// floor(x + 0.5) and wrapped to native indices mod N.
void slice_cells(int N, int Np, const double* theta, int32_t* kx, int32_t* ky) {
  for (int n = 0; n < Np; ++n) {
    const double t = theta ? theta[n] : default_theta(n, Np);
    const double s = std::sin(t), c = std::cos(t);
    for (int iu = 0; iu < N; ++iu) {
      const double u = (double)(iu - N / 2);
      const double x = -(u * s);
      const double y = u * c;
      long fx = (long)std::floor(x + 0.5), fy = (long)std::floor(y + 0.5);
      kx[(size_t)n * N + iu] = (int32_t)(((fx % N) + N) % N);
      ky[(size_t)n * N + iu] = (int32_t)(((fy % N) + N) % N);
    }
  }
}

// CSR of the insertion: for each native cell ky*N + kx, the entries n*N + u
// (u native frequency index, (u - N/2 + N) % N style wrap of the centred u).
void insertion_csr(int N, int Np, const double* theta, std::vector<int32_t>& row_ptr,
                   std::vector<int32_t>& entries) {
  std::vector<int32_t> kx((size_t)Np * N), ky((size_t)Np * N);
  slice_cells(N, Np, theta, kx.data(), ky.data());
  row_ptr.assign((size_t)N * N + 1, 0);
  for (size_t i = 0; i < kx.size(); ++i) row_ptr[(size_t)ky[i] * N + kx[i] + 1]++;
  for (size_t c = 0; c < (size_t)N * N; ++c) row_ptr[c + 1] += row_ptr[c];
  entries.assign(kx.size(), 0);
  std::vector<int32_t> fill(row_ptr.begin(), row_ptr.end() - 1);
  for (int n = 0; n < Np; ++n) {
    for (int iu = 0; iu < N; ++iu) {
      size_t i = (size_t)n * N + iu;
      size_t cell = (size_t)ky[i] * N + kx[i];
      int un = ((iu - N / 2) % N + N) % N;
      entries[fill[cell]++] = n * N + un;
    }
  }
}

// Bilinear insertion: sample (n, u) at (x, y) = (-u sin t, u cos t) spreads over the four cells
// around it with weights (1-fy)(1-fx), (1-fy)fx, fy(1-fx), fy fx (fx = x - floor x, fy = y -
// floor y); entries with weight exactly 0 are left out.  Same CSR layout as insertion_csr, plus
// the weight of every entry.
void insertion_csr_bilinear(int N, int Np, const double* theta, std::vector<int32_t>& row_ptr,
                            std::vector<int32_t>& entries, std::vector<double>& weights) {
  struct Hit { int32_t cell, code; double w; };
  std::vector<Hit> hits;
  hits.reserve((size_t)Np * N * 4);
  for (int n = 0; n < Np; ++n) {
    const double t = theta ? theta[n] : default_theta(n, Np);
    const double s = std::sin(t), c = std::cos(t);
    for (int iu = 0; iu < N; ++iu) {
      const double u = (double)(iu - N / 2);
      const double x = -(u * s);
      const double y = u * c;
      const double x0 = std::floor(x), y0 = std::floor(y);
      const double fx = x - x0, fy = y - y0;
      const long cx[4] = {(long)x0, (long)x0 + 1, (long)x0, (long)x0 + 1};
      const long cy[4] = {(long)y0, (long)y0, (long)y0 + 1, (long)y0 + 1};
      const double w[4] = {(1.0 - fy) * (1.0 - fx), (1.0 - fy) * fx, fy * (1.0 - fx), fy * fx};
      const int un = ((iu - N / 2) % N + N) % N;
      for (int k = 0; k < 4; ++k) {
        if (w[k] == 0.0) continue;
        const long kx = ((cx[k] % N) + N) % N, ky = ((cy[k] % N) + N) % N;
        hits.push_back(Hit{(int32_t)(ky * N + kx), n * N + un, w[k]});
      }
    }
  }
  row_ptr.assign((size_t)N * N + 1, 0);
  for (const Hit& h : hits) row_ptr[(size_t)h.cell + 1]++;
  for (size_t c = 0; c < (size_t)N * N; ++c) row_ptr[c + 1] += row_ptr[c];
  entries.assign(hits.size(), 0);
  weights.assign(hits.size(), 0.0);
  std::vector<int32_t> fill(row_ptr.begin(), row_ptr.end() - 1);
  for (const Hit& h : hits) {
    const int32_t at = fill[h.cell]++;
    entries[at] = h.code;
    weights[at] = h.w;
  }
}

void coupling_table(int Np, const uint8_t* present, const double alpha[3], int wrap_mirror,
                    std::vector<Coupling>& out) {
  out.assign(Np, Coupling{});
  for (int n = 0; n < Np; ++n) {
    int l = (n - 1 + Np) % Np, r = (n + 1) % Np;
    double wl = (present == nullptr || present[l]) ? alpha[0] : 0.0;
    double wr = (present == nullptr || present[r]) ? alpha[2] : 0.0;
    double w0 = alpha[1];
    double s = wl + w0 + wr;
    Coupling c;
    c.left = l;
    c.right = r;
    c.mirror_left = (wrap_mirror && n == 0) ? 1 : 0;
    c.mirror_right = (wrap_mirror && n == Np - 1) ? 1 : 0;
    c.wl = wl / s;
    c.w0 = w0 / s;
    c.wr = wr / s;
    out[n] = c;
  }
}

// Eq. 4 with 2K+1 taps: per angle n the terms k = -K..K (slot n + k on the periodic ring,
// t-mirrored where it wraps under the mirror rule); absent neighbours get weight 0 (and point at
// n itself), the rest are rescaled to sum to 1.  Needs 2K+1 <= Np.
void tap_table(int Np, const uint8_t* present, const double* taps, int K, int wrap_mirror, std::vector<Tap>& out) {
  const int nt = 2 * K + 1;
  out.assign((size_t)Np * nt, Tap{0, 0, 0.0});
  for (int n = 0; n < Np; ++n) {
    double s = 0.0;
    for (int k = -K; k <= K; ++k) {
      const int m = n + k;
      const bool wrapped = m < 0 || m >= Np;
      const int mm = ((m % Np) + Np) % Np;
      const bool here = k == 0 || present == nullptr || present[mm];
      Tap t{here ? mm : n, (here && wrapped && wrap_mirror) ? 1 : 0, here ? taps[k + K] : 0.0};
      out[(size_t)n * nt + (k + K)] = t;
      s += t.w;
    }
    for (int q = 0; q < nt; ++q) out[(size_t)n * nt + q].w /= s;
  }
}

}  // namespace cpra_host
