// Host driver for the non-uniform FFT plan pieces: reads W, Ny, Nx, the
// frequencies to evaluate phihat at, and a trajectory; writes phihat and the
// per-pair bin sorting (bperm, boff) as text.
#include <cstdio>
#include <vector>

#include "../paper_1810_01967_amd/csrc/nufft_host.h"

int main(int argc, char **argv) {
  if (argc != 3) return 2;
  FILE *f = std::fopen(argv[1], "rb");
  if (!f) return 3;
  int64_t hdr[5];  // W, Ny, Nx, nxi, npairs
  if (std::fread(hdr, 8, 5, f) != 5) return 4;
  const int W = (int)hdr[0], Ny = (int)hdr[1], Nx = (int)hdr[2];
  const int64_t nxi = hdr[3], npairs = hdr[4];
  std::vector<double> xi((size_t)nxi);
  std::vector<int64_t> off((size_t)npairs + 1);
  if (std::fread(xi.data(), 8, (size_t)nxi, f) != (size_t)nxi) return 5;
  if (std::fread(off.data(), 8, off.size(), f) != off.size()) return 6;
  std::vector<float> coords((size_t)off[(size_t)npairs] * 2);
  if (std::fread(coords.data(), 4, coords.size(), f) != coords.size()) return 7;
  std::fclose(f);
  std::vector<int32_t> bperm, boff;
  mrf::nufft_host::bin_samples(off.data(), npairs, coords.data(), Ny, Nx, 8, bperm, boff);
  FILE *o = std::fopen(argv[2], "w");
  for (double x : xi) std::fprintf(o, "%.17g\n", mrf::nufft_host::phihat(x, W, 2.30 * W));
  for (size_t i = 0; i < (size_t)off[(size_t)npairs]; ++i) std::fprintf(o, "%d ", bperm[i]);
  std::fprintf(o, "\n");
  for (int32_t v : boff) std::fprintf(o, "%d ", v);
  std::fprintf(o, "\n");
  std::fclose(o);
  return 0;
}
