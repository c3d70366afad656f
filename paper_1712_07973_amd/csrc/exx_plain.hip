// exx_plain.hip -- the plain FP64 GPU path (reference implementation on the GPU).
//
// One orbital pair per complex transform (imaginary part zero for real
// orbitals; rho_ij = conj(psi_j) psi_i of Eq. 2 for complex ones), the full
// zero-padded grid (2n on isolated axes, n on periodic ones) stored in HBM, and one launch per stage: pair build,
// three forward axis transforms, kernel multiply, three inverse axis
// transforms, reduction with FP64 atomics.  It follows the pair-sum scheme of
// arXiv:1712.07973 (Eq. 5 with the kernels 1-3 of Section 2.1.1) with no
// packing, pruning or fusion, and serves as the baseline the fused FP32 path
// is measured against.
#include "exx_fft.hpp"
#include "exx_internal.hpp"

namespace exx {

namespace {

constexpr int kLines = 16;  // lines per block in the axis transforms
constexpr int kPitch = kLines + 1;

__device__ __forceinline__ int foldk(int k, int M) { return k <= M - k ? k : M - k; }

// CPLX: psi holds interleaved (re, im) values and the pair is conj(psi_j) psi_i
template <bool CPLX>
__global__ void k_plain_build(const double* __restrict__ psi, const Slot* __restrict__ slots,
                              int slot0, int n, Dims m, cpx<double>* __restrict__ Z) {
  const size_t m3 = (size_t)m.x * m.y * m.z;
  const size_t n3 = (size_t)n * n * n;
  const int p = blockIdx.y;
  const Slot sl = slots[slot0 + p];
  cpx<double>* zp = Z + (size_t)p * m3;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < m3;
       idx += (size_t)gridDim.x * blockDim.x) {
    int x = (int)(idx % m.x), y = (int)((idx / m.x) % m.y), z = (int)(idx / ((size_t)m.x * m.y));
    cpx<double> r{0.0, 0.0};
    if (x < n && y < n && z < n) {
      size_t o = ((size_t)z * n + y) * n + x;
      if constexpr (CPLX) {
        const auto* pc = reinterpret_cast<const cpx<double>*>(psi);
        r = cmulc(pc[(size_t)sl.ia * n3 + o], pc[(size_t)sl.ja * n3 + o]);
      } else {
        r.x = psi[(size_t)sl.ia * n3 + o] * psi[(size_t)sl.ja * n3 + o];
      }
    }
    zp[idx] = r;
  }
}

// Transforms of length L along one axis of the [z][y][x] array (x fastest),
// kLines lines per block; the lines of a block are consecutive in x for the
// y and z axes and consecutive rows for the x axis.
template <int L, int DIR>
__global__ __launch_bounds__(256) void k_plain_axis(cpx<double>* __restrict__ Z, Dims m,
                                                    int axis, const cpx<double>* __restrict__ twg) {
  using S = Split<L>;
  constexpr int L1 = S::L1, L2 = S::L2;
  constexpr int NT = 256;
  __shared__ cpx<double> buf[L * kPitch];
  __shared__ cpx<double> tw[L];
  const int tid = threadIdx.x;
  const size_t m3 = (size_t)m.x * m.y * m.z;
  const int groups = (int)(m3 / L / kLines);
  const int p = blockIdx.x / groups, g = blockIdx.x % groups;
  size_t base;
  size_t es, lstr;
  if (axis == 0) {  // lines along x: rows (z, y), kLines consecutive rows
    base = (size_t)p * m3 + (size_t)g * kLines * m.x;
    es = 1;
    lstr = m.x;
  } else if (axis == 1) {  // lines along y: (z, x), kLines consecutive x
    int z = g / (m.x / kLines), x0 = (g % (m.x / kLines)) * kLines;
    base = (size_t)p * m3 + (size_t)z * m.x * m.y + x0;
    es = m.x;
    lstr = 1;
  } else {  // lines along z: (y, x), kLines consecutive x
    int y = g / (m.x / kLines), x0 = (g % (m.x / kLines)) * kLines;
    base = (size_t)p * m3 + (size_t)y * m.x + x0;
    es = (size_t)m.x * m.y;
    lstr = 1;
  }
  for (int k = tid; k < L; k += NT) tw[k] = twg[k];
  for (int q = tid; q < kLines * L; q += NT) {
    int l, e;
    if (axis == 0) {
      e = q % L;
      l = q / L;
    } else {
      l = q % kLines;
      e = q / kLines;
    }
    buf[e * kPitch + l] = Z[base + e * es + l * lstr];
  }
  __syncthreads();
  constexpr int C1 = kLines * L2;
  for (int it = tid; it < C1; it += NT) {
    int l = it % kLines, t = it / kLines;
    cpx<double> v[L1];
#pragma unroll
    for (int k1 = 0; k1 < L1; ++k1) v[k1] = buf[(t + L2 * k1) * kPitch + l];
    Dft<L1, DIR, double>::run(v);
#pragma unroll
    for (int q1 = 1; q1 < L1; ++q1)
      v[q1] = DIR < 0 ? cmul(v[q1], tw[t * q1]) : cmulc(v[q1], tw[t * q1]);
#pragma unroll
    for (int q1 = 0; q1 < L1; ++q1) buf[(t + L2 * q1) * kPitch + l] = v[q1];
  }
  __syncthreads();
  constexpr int C2 = kLines * L1;
  static_assert(C2 <= NT, "one step-2 item per thread");
  cpx<double> w[L2];
  const bool act = tid < C2;
  const int l2 = tid % kLines, q1 = tid / kLines;
  if (act) {
#pragma unroll
    for (int t = 0; t < L2; ++t) w[t] = buf[(t + L2 * q1) * kPitch + l2];
    Dft<L2, DIR, double>::run(w);
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int q2 = 0; q2 < L2; ++q2) buf[(q1 + L1 * q2) * kPitch + l2] = w[q2];
  }
  __syncthreads();
  for (int q = tid; q < kLines * L; q += NT) {
    int l, e;
    if (axis == 0) {
      e = q % L;
      l = q / L;
    } else {
      l = q % kLines;
      e = q / kLines;
    }
    Z[base + e * es + l * lstr] = buf[e * kPitch + l];
  }
}

__global__ void k_plain_kmul(cpx<double>* __restrict__ Z, Dims m, const double* __restrict__ kt) {
  const size_t m3 = (size_t)m.x * m.y * m.z;
  const int hy = m.y / 2 + 1, hz = m.z / 2 + 1;
  cpx<double>* zp = Z + (size_t)blockIdx.y * m3;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < m3;
       idx += (size_t)gridDim.x * blockDim.x) {
    int kx = (int)(idx % m.x), ky = (int)((idx / m.x) % m.y), kz = (int)(idx / ((size_t)m.x * m.y));
    double k = kt[((size_t)foldk(kx, m.x) * hy + foldk(ky, m.y)) * hz + foldk(kz, m.z)];
    cpx<double> v = zp[idx];
    zp[idx] = {v.x * k, v.y * k};
  }
}

// CPLX: e += Re(conj(rho) V), (K psi)_i += f_j V psi_j, (K psi)_j += f_i conj(V) psi_i
template <bool CPLX>
__global__ __launch_bounds__(256) void k_plain_reduce(const cpx<double>* __restrict__ Z,
                                                      const double* __restrict__ psi,
                                                      const double* __restrict__ occ,
                                                      const Slot* __restrict__ slots, int slot0,
                                                      int n, Dims m, double* __restrict__ kpsi,
                                                      double* __restrict__ e_slot, int want_k,
                                                      int want_e) {
  __shared__ double red[4];
  const size_t m3 = (size_t)m.x * m.y * m.z;
  const size_t n3 = (size_t)n * n * n;
  const int p = blockIdx.y;
  const Slot sl = slots[slot0 + p];
  const cpx<double>* zp = Z + (size_t)p * m3;
  const int vals = CPLX ? 2 : 1;  // doubles per grid value
  const double* pi = psi + (size_t)sl.ia * n3 * vals;
  const double* pj = psi + (size_t)sl.ja * n3 * vals;
  double* ki = kpsi + (size_t)sl.ia * n3 * vals;
  double* kj = kpsi + (size_t)sl.ja * n3 * vals;
  const double fi = occ[sl.ia], fj = occ[sl.ja];
  double e = 0.0;
  for (size_t o = (size_t)blockIdx.x * blockDim.x + threadIdx.x; o < n3;
       o += (size_t)gridDim.x * blockDim.x) {
    int x = (int)(o % n), y = (int)((o / n) % n), z = (int)(o / ((size_t)n * n));
    const cpx<double> V = zp[((size_t)z * m.y + y) * m.x + x];
    if constexpr (CPLX) {
      const cpx<double> a{pi[2 * o], pi[2 * o + 1]}, b{pj[2 * o], pj[2 * o + 1]};
      const cpx<double> rho = cmulc(a, b);
      e += rho.x * V.x + rho.y * V.y;
      if (want_k) {
        const cpx<double> u = cmul(V, b), w = cmulc(a, V);  // V psi_j, conj(V) psi_i
        atomicAdd(&ki[2 * o], fj * u.x);
        atomicAdd(&ki[2 * o + 1], fj * u.y);
        if (sl.ia != sl.ja) {
          atomicAdd(&kj[2 * o], fi * w.x);
          atomicAdd(&kj[2 * o + 1], fi * w.y);
        }
      }
    } else {
      double a = pi[o], b = pj[o];
      e += a * b * V.x;
      if (want_k) {
        atomicAdd(&ki[o], fj * V.x * b);
        if (sl.ia != sl.ja) atomicAdd(&kj[o], fi * V.x * a);
      }
    }
  }
  if (!want_e) return;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(&e_slot[2 * (slot0 + p)], red[0] + red[1] + red[2] + red[3]);
}

template <typename F>
hipError_t dispatch_m(int m, F&& f) {
  switch (m) {
    case 16: return f.template operator()<16>();
    case 32: return f.template operator()<32>();
    case 48: return f.template operator()<48>();
    case 64: return f.template operator()<64>();
    case 80: return f.template operator()<80>();
    case 96: return f.template operator()<96>();
    case 112: return f.template operator()<112>();
    case 128: return f.template operator()<128>();
    case 160: return f.template operator()<160>();
    case 192: return f.template operator()<192>();
    case 224: return f.template operator()<224>();
    case 256: return f.template operator()<256>();
    default: return hipErrorInvalidValue;
  }
}

unsigned grid_for(size_t count) {
  size_t b = (count + 255) / 256;
  return (unsigned)(b > 4096 ? 4096 : (b ? b : 1));
}

}  // namespace

hipError_t plain_build(const double* psi, const Slot* slots, int slot0, int npairs, int n, Dims m,
                       void* Z, bool cplx, hipStream_t s) {
  if (npairs <= 0) return hipSuccess;
  size_t m3 = (size_t)m.x * m.y * m.z;
  auto* Zc = static_cast<cpx<double>*>(Z);
  if (cplx)
    hipLaunchKernelGGL(k_plain_build<true>, dim3(grid_for(m3), npairs), dim3(256), 0, s, psi,
                       slots, slot0, n, m, Zc);
  else
    hipLaunchKernelGGL(k_plain_build<false>, dim3(grid_for(m3), npairs), dim3(256), 0, s, psi,
                       slots, slot0, n, m, Zc);
  return hipGetLastError();
}

hipError_t plain_fft_axis(void* Z, int npairs, int n, Dims m, int axis, int dir, const Tables& tb,
                          hipStream_t s) {
  if (npairs <= 0) return hipSuccess;
  const int len = axis == 0 ? m.x : (axis == 1 ? m.y : m.z);
  const size_t m3 = (size_t)m.x * m.y * m.z;
  // roots of the axis length: n points on periodic axes, 2n on padded ones
  auto* tw = static_cast<const cpx<double>*>(len == 2 * n ? tb.tw_2n : tb.tw_n);
  if (!tw || (len != n && len != 2 * n)) return hipErrorInvalidValue;
  return dispatch_m(len, [&]<int L>() -> hipError_t {
    dim3 grid((unsigned)(npairs * (m3 / L / kLines)));
    auto* Zc = static_cast<cpx<double>*>(Z);
    if (dir < 0)
      hipLaunchKernelGGL((k_plain_axis<L, -1>), grid, dim3(256), 0, s, Zc, m, axis, tw);
    else
      hipLaunchKernelGGL((k_plain_axis<L, 1>), grid, dim3(256), 0, s, Zc, m, axis, tw);
    return hipGetLastError();
  });
}

hipError_t plain_kernel_mul(void* Z, int npairs, Dims m, const Tables& tb, hipStream_t s) {
  if (npairs <= 0) return hipSuccess;
  size_t m3 = (size_t)m.x * m.y * m.z;
  hipLaunchKernelGGL(k_plain_kmul, dim3(grid_for(m3), npairs), dim3(256), 0, s,
                     static_cast<cpx<double>*>(Z), m, static_cast<const double*>(tb.ktab_m));
  return hipGetLastError();
}

hipError_t plain_reduce(const void* Z, const double* psi, const double* occ, const Slot* slots,
                        int slot0, int npairs, int n, Dims m, double h3, double* kpsi,
                        double* e_slot, bool want_k, bool want_e, bool cplx, hipStream_t s) {
  (void)h3;
  if (npairs <= 0) return hipSuccess;
  size_t n3 = (size_t)n * n * n;
  auto* Zc = static_cast<const cpx<double>*>(Z);
  if (cplx)
    hipLaunchKernelGGL(k_plain_reduce<true>, dim3(grid_for(n3), npairs), dim3(256), 0, s, Zc, psi,
                       occ, slots, slot0, n, m, kpsi, e_slot, want_k ? 1 : 0, want_e ? 1 : 0);
  else
    hipLaunchKernelGGL(k_plain_reduce<false>, dim3(grid_for(n3), npairs), dim3(256), 0, s, Zc, psi,
                       occ, slots, slot0, n, m, kpsi, e_slot, want_k ? 1 : 0, want_e ? 1 : 0);
  return hipGetLastError();
}

}  // namespace exx
