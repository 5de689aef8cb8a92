// Host-only helpers shared by the C ABI (no GPU calls).
#pragma once
#include <cstdint>
#include <vector>

namespace cpra_host {

// Same layout as the device-side coupling record.
struct Coupling {
  int left, right;
  int mirror_left, mirror_right;
  double wl, w0, wr;
};

struct Tap {
  int nb, mirror;
  double w;
};

double default_theta(int n, int Np);
void tap_table(int Np, const uint8_t* present, const double* taps, int K, int wrap_mirror, std::vector<Tap>& out);
void slice_cells(int N, int Np, const double* theta, int32_t* kx, int32_t* ky);
void insertion_csr(int N, int Np, const double* theta, std::vector<int32_t>& row_ptr,
                   std::vector<int32_t>& entries);
void insertion_csr_bilinear(int N, int Np, const double* theta, std::vector<int32_t>& row_ptr,
                            std::vector<int32_t>& entries, std::vector<double>& weights);
void coupling_table(int Np, const uint8_t* present, const double alpha[3], int wrap_mirror,
                    std::vector<Coupling>& out);

}  // namespace cpra_host
