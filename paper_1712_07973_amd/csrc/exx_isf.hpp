// exx_isf.hpp -- Fourier table of the interpolating-scaling-function Green's
// function of the free boundary (host only, no HIP).
#pragma once

#include <vector>

namespace exx {

// K^(f) / (2n)^3 on the 2n grid per axis, octant 0 <= f <= n per axis,
// [fx][fy][fz] with fz fastest, FP64 (exx_isf.cpp).
std::vector<double> isf_octant(int n, double hx, double hy, double hz);

}  // namespace exx
