// exx_isf.cpp -- Green's function of the interpolating-scaling-function
// Poisson solver (free boundary), tabulated in Fourier space on the host in FP64.
//
// The solver the paper uses (Section 2.1.2) treats the density on the grid as
// rho(r) = sum_j rho_j phi(x/hx - j1) phi(y/hy - j2) phi(z/hz - j3), phi the
// order-16 Deslauriers-Dubuc interpolating scaling function, and returns the
// exact Coulomb potential of that density at the grid points:
//
//   V_i = sum_j K(i - j) rho_j,   K(d) = hx hy hz  int phi(u1) phi(u2) phi(u3) / |H (d - u)| du
//
// with H = diag(hx, hy, hz).  On the grid doubled per axis every displacement
// of the n^3 box fits without wrapping, so the convolution is applied by the
// same FFT passes as the other kernels with the table K^(f) = DFT_2n(K) / (2n)^3.
//
// K is built from a sum of Gaussians for 1/r, which makes every term separable:
//   1/r = (2/sqrt(pi)) int exp(s - e^{2s} r^2) ds ~ sum_q w_q exp(-a_q r^2)
//   K(d) = hx hy hz sum_q w_q I(a_q hx^2, d1) I(a_q hy^2, d2) I(a_q hz^2, d3),
//   I(b, d) = int phi(u) exp(-b (d - u)^2) du,
// and the DFT of a separable term is the product of three 1-D cosine sums.
// I(b, d) is the trapezoid sum over phi's dyadic samples at a spacing where
// the Gaussian is wide (phi reproduces polynomials of degree < 16, so the sum
// is exact up to a 16th-moment term), and sqrt(pi/b) (phi(d) + phi''(d)/(4b))
// for Gaussians narrower than the finest sampling.
#include "exx_isf.hpp"

#include <algorithm>
#include <cmath>
#include <vector>

namespace exx {

namespace {

constexpr int kOrder = 16;           // interpolation degree 15
constexpr int kSupport = kOrder - 1; // phi vanishes outside [-15, 15]
constexpr int kFinest = 15;          // dyadic levels of the sampled phi

// phi at u = -kSupport + i 2^-kFinest by interpolating subdivision: each new
// midpoint is the degree-15 Lagrange interpolant of the 16 nearest known values.
std::vector<double> isf_samples() {
  const int half = kOrder / 2;
  double w[kOrder];
  for (int k = 0; k < kOrder; ++k) {  // weight of node t = k - half + 1 at 1/2
    const double t = k - half + 1;
    double p = 1.0;
    for (int j = 0; j < kOrder; ++j) {
      const double u = j - half + 1;
      if (j != k) p *= (0.5 - u) / (t - u);
    }
    w[k] = p;
  }
  std::vector<double> v(2 * kSupport + 1, 0.0);
  v[kSupport] = 1.0;
  for (int level = 0; level < kFinest; ++level) {
    const int np = (int)v.size();
    std::vector<double> out(2 * np - 1);
    for (int i = 0; i < np; ++i) out[2 * i] = v[i];
    for (int i = 0; i + 1 < np; ++i) {
      double m = 0.0;
      for (int k = 0; k < kOrder; ++k) {
        const int j = i + k - half + 1;
        if (j >= 0 && j < np) m += w[k] * v[j];
      }
      out[2 * i + 1] = m;
    }
    v.swap(out);
  }
  return v;
}

// Neumaier-compensated sum
struct Sum {
  double s = 0.0, c = 0.0;
  void add(double x) {
    const double t = s + x;
    c += std::fabs(s) >= std::fabs(x) ? (s - t) + x : (x - t) + s;
    s = t;
  }
  double value() const { return s + c; }
};

// I(b, d) for d = 0..n (b: Gaussian exponent in grid units)
void gauss_integrals(const std::vector<double>& phi, double b, int n, double* out) {
  const double fine = std::ldexp(1.0, -kFinest);
  if (b <= 1e-4) {
    // wide Gaussian: I = exp(-b d^2) int phi(u) exp(2 b d u - b u^2) du, and the
    // moments 1..15 of phi vanish, so the integral is 1 up to (2 b d)^16 M_16 / 16!
    // (below 1e-25 here for d <= 128)
    for (int d = 0; d <= n; ++d) out[d] = std::exp(-b * (double)d * d);
    return;
  }
  // sampling level: exponent b / 4^L <= 2.5e-4 on the sampling scale
  int L = (int)std::ceil(std::log(std::max(b, 1e-300) / 2.5e-4) / std::log(4.0));
  L = std::max(L, 6);
  if (L > kFinest) {  // narrower than the finest sampling: small-width expansion
    for (int d = 0; d <= n; ++d) {
      out[d] = 0.0;
      if (d >= kSupport) continue;
      const size_t i = (size_t)(d + kSupport) << kFinest;
      const double d2 = (phi[i + 1] - 2.0 * phi[i] + phi[i - 1]) / (fine * fine);
      out[d] = std::sqrt(M_PI / b) * ((d == 0 ? 1.0 : 0.0) + d2 / (4.0 * b));
    }
    return;
  }
  const int stride = 1 << (kFinest - L);
  const double step = std::ldexp(1.0, -L);
  const double reach = std::sqrt(40.0 / b);  // exp(-b x^2) < e^-40 beyond
  const int per_unit = 1 << L;
  for (int d = 0; d <= n; ++d) {
    const double lo = std::max(-(double)kSupport, d - reach);
    const double hi = std::min((double)kSupport, d + reach);
    out[d] = 0.0;
    if (lo > hi) continue;
    const long i0 = (long)std::floor((lo + kSupport) * per_unit);
    const long i1 = std::min<long>((long)std::ceil((hi + kSupport) * per_unit), 2L * kSupport * per_unit);
    Sum s;
    for (long i = i0; i <= i1; ++i) {
      const double u = -kSupport + i * step;
      const double x = d - u;
      s.add(phi[(size_t)i * stride] * std::exp(-b * x * x));
    }
    out[d] = step * s.value();
  }
}

}  // namespace

std::vector<double> isf_octant(int n, double hx, double hy, double hz) {
  const std::vector<double> phi = isf_samples();
  const double h[3] = {hx, hy, hz};
  const double hmin = std::min(hx, std::min(hy, hz)), hmax = std::max(hx, std::max(hy, hz));
  // 1/r as Gaussians over [r_min, r_max] (bohr): every |H (d - u)| of the doubled
  // box is below sqrt(3) (n + 16) hmax; r_min leaves out ~2 pi r_min^2 of the
  // singular integral
  const double r_min = 1e-7 * hmin, r_max = std::sqrt(3.0) * (n + kOrder) * hmax;
  const double delta = 0.15;
  const double s_lo = std::log(1e-16 / r_max), s_hi = std::log(std::sqrt(40.0) / r_min);
  const int nq = (int)std::floor((s_hi - s_lo) / delta) + 1;
  // cos(pi f d / n) for 0 <= f, d <= n, exact multiples of 2 pi folded first
  std::vector<double> cs((size_t)(n + 1) * (n + 1));
  for (int f = 0; f <= n; ++f)
    for (int d = 0; d <= n; ++d) cs[(size_t)f * (n + 1) + d] = std::cos(M_PI * ((f * d) % (2 * n)) / n);
  const int e = n + 1;
  std::vector<double> tab((size_t)e * e * e, 0.0);
  std::vector<double> I(e), G[3];
  for (auto& g : G) g.resize(e);
  for (int q = 0; q < nq; ++q) {
    const double s = s_lo + q * delta;
    const double w = 2.0 / std::sqrt(M_PI) * delta * std::exp(s), a = std::exp(2.0 * s);
    for (int ax = 0; ax < 3; ++ax) {
      if (ax > 0 && h[ax] == h[ax - 1]) {  // same spacing: same transform
        G[ax] = G[ax - 1];
        continue;
      }
      gauss_integrals(phi, a * h[ax] * h[ax], n, I.data());
      // 2n-point DFT of the even sequence I(0), I(1), .., I(n), .., I(1)
      for (int f = 0; f <= n; ++f) {
        const double* c = &cs[(size_t)f * (n + 1)];
        double acc = I[0] + I[n] * c[n];
        for (int d = 1; d < n; ++d) acc += 2.0 * I[d] * c[d];
        G[ax][f] = acc;
      }
    }
    for (int fx = 0; fx <= n; ++fx) {
      const double wx = w * G[0][fx];
      for (int fy = 0; fy <= n; ++fy) {
        const double wxy = wx * G[1][fy];
        double* t = &tab[((size_t)fx * e + fy) * e];
        for (int fz = 0; fz <= n; ++fz) t[fz] += wxy * G[2][fz];
      }
    }
  }
  const double scale = hx * hy * hz / (8.0 * (double)n * n * n);  // hx hy hz / (2n)^3
  for (double& v : tab) v *= scale;
  return tab;
}

}  // namespace exx
