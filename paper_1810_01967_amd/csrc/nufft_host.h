// Host-side pieces of the non-uniform FFT plan (pure C++, no HIP): the
// "exponential of semicircle" kernel, the Fourier transform of it used for
// the deapodisation (composite Simpson quadrature in FP64), and the sorting
// of each (slice, frame) pair's samples into bins of the oversampled grid.
#pragma once
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <numeric>
#include <vector>

namespace mrf {
namespace nufft_host {

// phi(z) = exp(beta (sqrt(1 - z^2) - 1)) for |z| < 1, else 0
inline double es(double z, double beta) {
  const double q = 1.0 - z * z;
  return q > 0.0 ? std::exp(beta * (std::sqrt(q) - 1.0)) : 0.0;
}

// phihat(xi) = int_{-W/2}^{W/2} phi(2u/W) exp(-2 pi i u xi) du
//            = 2 int_0^{W/2} phi(2u/W) cos(2 pi u xi) du (phi is even)
inline double phihat(double xi, int W, double beta) {
  const int nq = 4096;
  const double h = 0.5 * W / nq;
  double acc = 0.0;
  for (int i = 0; i <= nq; ++i) {
    const double u = i * h;
    const double f = es(2.0 * u / W, beta) * std::cos(2.0 * M_PI * u * xi);
    acc += f * ((i == 0 || i == nq) ? 1.0 : (i & 1) ? 4.0 : 2.0);
  }
  return 2.0 * acc * h / 3.0;
}

// Bin of a sample: its fine-grid position k N taken modulo N, in bins of
// `bin` cells per dimension, row-major (y, x).
inline int bin_of(float ky, float kx, int Ny, int Nx, int bin) {
  double uy = (double)ky * Ny, ux = (double)kx * Nx;
  uy -= std::floor(uy / Ny) * Ny;
  ux -= std::floor(ux / Nx) * Nx;
  const int nby = Ny / bin, nbx = Nx / bin;
  const int by = std::min(nby - 1, std::max(0, (int)(uy / bin)));
  const int bx = std::min(nbx - 1, std::max(0, (int)(ux / bin)));
  return by * nbx + bx;
}

// For every pair p: bperm[off[p] ..] lists the pair's samples (global
// indices) sorted by bin, ties in sample order; boff[p (nb + 1) + b] is the
// offset of bin b within the pair's range.
inline void bin_samples(const int64_t *off, int64_t npairs, const float *coords, int Ny, int Nx, int bin,
                        std::vector<int32_t> &bperm, std::vector<int32_t> &boff) {
  const int nb = (Ny / bin) * (Nx / bin);
  bperm.assign((size_t)std::max<int64_t>(off[npairs], 1), 0);
  boff.assign((size_t)npairs * (nb + 1), 0);
  std::vector<int32_t> key, ord;
  for (int64_t p = 0; p < npairs; ++p) {
    const int64_t b = off[p], e = off[p + 1];
    key.resize((size_t)(e - b));
    for (int64_t i = b; i < e; ++i) key[(size_t)(i - b)] = bin_of(coords[2 * i], coords[2 * i + 1], Ny, Nx, bin);
    ord.resize((size_t)(e - b));
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t c) { return key[(size_t)a] < key[(size_t)c]; });
    int32_t *bo = boff.data() + (size_t)p * (nb + 1);
    for (int64_t r = 0; r < e - b; ++r) {
      bperm[(size_t)(b + r)] = (int32_t)(b + ord[(size_t)r]);
      ++bo[key[(size_t)ord[(size_t)r]] + 1];
    }
    for (int q = 0; q < nb; ++q) bo[q + 1] += bo[q];
  }
}

}  // namespace nufft_host
}  // namespace mrf
