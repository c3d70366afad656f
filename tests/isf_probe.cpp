// Prints the ISF Fourier table of the library's host code for (n, h) as text,
// one value per line in [fx][fy][fz] order, for the CPU check against the oracle.
#include <cstdio>
#include <cstdlib>

#include "../paper_1712_07973_amd/csrc/exx_isf.hpp"

int main(int argc, char** argv) {
  if (argc < 3) return 2;
  const int n = std::atoi(argv[1]);
  const double h = std::atof(argv[2]);
  const auto t = exx::isf_octant(n, h, h, h);
  for (double v : t) std::printf("%.17g\n", v);
  return 0;
}
