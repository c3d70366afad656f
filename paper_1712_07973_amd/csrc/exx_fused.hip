// exx_fused.hip -- fused pair-build / FFT / Green multiply / reduction kernels.
//
// Work unit: a packed slot, two unordered orbital pairs whose real
// co-densities rho_a = psi_ia psi_ja and rho_b = psi_ib psi_jb (Eq. 8 of
// arXiv:1712.07973) travel as one complex field Z = rho_a + i rho_b.  The
// Green's kernel is real and even, so the inverse transform returns
// V_a + i V_b exactly.  Three passes per launch of slots:
//
//   pass A  pair build + forward x-transform of every grid row          -> X
//   pass B  per x-frequency slab: forward y,z transforms, multiply by the
//           kernel (Eq. 4 in Fourier space), inverse z,y transforms   X -> X
//   pass C  inverse x-transform, then pair energies h^3 sum rho V (Eq. 5)
//           and K psi accumulation (Eq. 3) over a tile of pairs, in FP64
//
// Free boundary (zero padding to 2n, Section 2.1.2) without materialising the
// padded grid: the 2n-point transform of data supported on [0, n) splits by
// the parity b of the output index into two n-point transforms of the input
// modulated by w_2n^{b r}.  Per axis the padded problem is therefore 2
// "classes" of n-point transforms; the x classes live in X (2 n^3 complex per
// slot), the y/z classes are looped over inside pass B and summed after
// demodulation.  Periodic grids have one class and no modulation.
//
// X layout per slot, z-blocked: [y][z / 16][cx][kx][z % 16].  Passes A and C
// work on the rows (y, 16 consecutive z) of every x-frequency, which is one
// contiguous chunk of 2 n x 16 complex values; pass B gathers its slab
// (cx, kx) as n^2 / 16 runs of 16 consecutive z.
#include "exx_fft.hpp"
#include "exx_internal.hpp"

namespace exx {

template <int N>
struct SplitAC {  // x-lines of passes A and C: 16 work items per line in step 2
  static constexpr int L2 = 16;
  static constexpr int L1 = N / 16;
  static_assert(L1 * L2 == N, "n must be a multiple of 16");
};

__device__ __forceinline__ int fold(int k, int M) { return k <= M - k ? k : M - k; }

// z-block of the spectrum layout; passes A and C move one z-block of rows
constexpr int XZ = 16;

// XCD-ordered grids (xcd_split, exx_schedule.hpp): the blocks resident on one
// XCD at a time share what depends on the item only (orbital rows in pass A,
// the kernel plane in pass B) in that XCD's L2.  The blocks in flight then also
// spread over every slot of the launch instead of a few, which costs where a
// slot is large: measured same-box, 32 and 64 orbitals, ms per evaluation
// (row-major -> XCD order):
//   pass A  free 64^3: 0.224 -> 0.209    free 128^3: 8.82 -> 9.60 (64 orbitals)
//   pass B  free 64^3: 1.284 -> 1.310    free 128^3: 48.7 -> 48.2, and pass C
//           after it 14.2 -> 13.8 (its spectrum reads follow pass B's writes)
// so pass A takes it up to n = 64 and the wave-local pass B from n = 96 on.
constexpr bool pass_a_xcd_order(int n) { return n <= 64; }
constexpr bool pass_b_xcd_order(int n) { return n >= 96; }

// slots per pass A block.  With the non-temporal spectrum stores, up to n = 64 more
// blocks beat reusing a block's set-up (64^3, 32 orbitals: pass A 0.178 ms with one
// slot, 0.212 with 2, 0.219 with 4); larger grids already launch enough blocks per
// slot and gain from two (16 free grids of n = 48..112: 614 against 625 ms).
constexpr int pass_a_slots(int n) { return n <= 64 ? 1 : 2; }

// offset of (cx, kx, y, z) within a slot, and of (y, z) within slab (cx, kx)
template <int N, int NCLS>
__device__ __forceinline__ size_t x_off(int cx, int kx, int y, int z) {
  return ((size_t)(y * (N / XZ) + z / XZ) * NCLS * N + cx * N + kx) * XZ + (z % XZ);
}
__device__ __forceinline__ size_t slab_base(int slab) { return (size_t)slab * XZ; }
template <int N, int NCLS>
__device__ __forceinline__ int slab_off(int y, int z) {
  return (y * (N / XZ) + z / XZ) * (NCLS * N * XZ) + (z % XZ);
}

// Pass A's stores and pass C's loads of the spectrum stream it through HBM
// once: non-temporal accesses keep it from evicting the orbital rows that
// those passes re-read from L2 (measured at 64^3, 32 orbitals: pass A 0.26 ->
// 0.21 ms, pass C 0.37 -> 0.35 ms; complex orbitals 0.62 -> 0.39 and 0.88 -> 0.81 ms).
template <typename T>
__device__ __forceinline__ void store_stream(cpx<T>* p, cpx<T> v) {
  using V2 = T __attribute__((ext_vector_type(2)));
  __builtin_nontemporal_store(V2{v.x, v.y}, reinterpret_cast<V2*>(p));
}
template <typename T>
__device__ __forceinline__ cpx<T> load_stream(const cpx<T>* p) {
  using V2 = T __attribute__((ext_vector_type(2)));
  const V2 v = __builtin_nontemporal_load(reinterpret_cast<const V2*>(p));
  return {v.x, v.y};
}

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__global__ void k_convert(const double* __restrict__ a, float* __restrict__ b, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) b[i] = (float)a[i];
}

__global__ void k_zero(double* __restrict__ p, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = 0.0;
}

hipError_t launch_convert(const double* psi, float* psi32, size_t count, hipStream_t s) {
  unsigned blocks = (unsigned)std::min<size_t>((count + 255) / 256, 65536);
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_convert, dim3(blocks), dim3(256), 0, s, psi, psi32, count);
  return hipGetLastError();
}

// FP32 copies of every member of a merged class (blockIdx.y = member)
__global__ void k_convert_members(const MemberTab m, float* __restrict__ b) {
  const int k = blockIdx.y;
  const double* __restrict__ a = m.psi[k];
  float* __restrict__ d = b + m.dst_off[k];
  const size_t n = m.count[k];
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) d[i] = (float)a[i];
}

hipError_t launch_convert_members(const MemberTab& m, float* psi32, size_t max_count, hipStream_t s) {
  unsigned blocks = (unsigned)std::min<size_t>((max_count + 255) / 256, 65536);
  if (blocks == 0 || m.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_convert_members, dim3(blocks, m.n), dim3(256), 0, s, m, psi32);
  return hipGetLastError();
}

hipError_t launch_zero(double* p, size_t count, hipStream_t s) {
  unsigned blocks = (unsigned)std::min<size_t>((count + 255) / 256, 65536);
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, s, p, count);
  return hipGetLastError();
}

template <typename T>
__device__ __forceinline__ T sqrt_weight(const double* occ, int i, int j) {
  double w = occ[i] * occ[j] * (i == j ? 1.0 : 2.0);
  return (T)sqrt(w > 0.0 ? w : 0.0);
}

// ---------------------------------------------------------------------------
// pass A: co-densities of two pairs packed as Z, forward x-transform per class
// block: rows (y, z0..z0+ZB) of SPB consecutive slots.  The orbital values of
// the next slot are loaded into registers before the current slot's
// transform, so its loads overlap the current slot's LDS work and stores.
// CPLX: complex orbitals (psi holds (re, im) pairs), one pair per slot, and
// Z = conj(psi_j) psi_i (Eq. 2).  swap_yz: the spectrum's (y, z) indices are
// the grid's (z, y), so that pass B transforms the grid's z axis first (wire
// geometry: the periodic axis then serves both y classes).
// ---------------------------------------------------------------------------
template <typename T, int N, int NCLS, int ZB, int NT, int SPB, bool W, bool CPLX>
__global__ __launch_bounds__(NT) void k_pass_a(const T* __restrict__ psi, cpx<T>* __restrict__ X,
                                               const Slot* __restrict__ slots, int slot0,
                                               int nslots, const double* __restrict__ occ,
                                               const cpx<T>* __restrict__ twg,
                                               const cpx<T>* __restrict__ mdg, int swap_yz) {
  using S = SplitAC<N>;
  constexpr int L1 = S::L1, L2 = S::L2;
  constexpr int P = N + 1;
  constexpr int NL = NCLS * ZB;              // lines per block
  constexpr int PV = (ZB * N + NT - 1) / NT;  // grid points per thread
  static_assert(ZB == XZ, "a block's rows are one z-block of the spectrum layout");
  __shared__ cpx<T> zb[ZB * P];
  __shared__ cpx<T> wk[NL * P];
  __shared__ cpx<T> tw[N];
  __shared__ cpx<T> md[N];

  const int tid = threadIdx.x;
  int rb, sg;  // row block (y, z-block) and slot group
  if constexpr (pass_a_xcd_order(N)) {
    xcd_split(blockIdx.x, N * (N / ZB), (nslots + SPB - 1) / SPB, rb, sg);
  } else {
    rb = blockIdx.x;
    sg = blockIdx.y;
  }
  const int y = rb / (N / ZB);
  const int z0 = (rb % (N / ZB)) * ZB;
  const int ls0 = sg * SPB;
  const int ls1 = ls0 + SPB < nslots ? ls0 + SPB : nslots;
  const size_t M3 = (size_t)N * N * N;

  // orbital values of slot ls at the block's points p = tid + q NT -> (zi, x)
  // (CPLX: va = psi_i, vb = psi_j as (re, im))
  T va[PV][2], vb[PV][2];
  auto fetch = [&](int ls) {
    const Slot sl = slots[slot0 + ls];
    if constexpr (CPLX) {
      const cpx<T>* pi = reinterpret_cast<const cpx<T>*>(psi) + (size_t)sl.ia * M3;
      const cpx<T>* pj = reinterpret_cast<const cpx<T>*>(psi) + (size_t)sl.ja * M3;
#pragma unroll
      for (int q = 0; q < PV; ++q) {
        const int p = tid + q * NT;
        if ((ZB * N) % NT == 0 || p < ZB * N) {
          const int zi = p / N, x = p % N;
          const size_t o = swap_yz ? ((size_t)y * N + z0 + zi) * N + x
                                   : ((size_t)(z0 + zi) * N + y) * N + x;
          const cpx<T> u = pi[o], v = pj[o];
          va[q][0] = u.x;
          va[q][1] = u.y;
          vb[q][0] = v.x;
          vb[q][1] = v.y;
        }
      }
      return;
    }
    const bool ha = sl.ia >= 0, hb = sl.ib >= 0;  // either half may be empty
    const T* pia = psi + (size_t)(ha ? sl.ia : 0) * M3;
    const T* pja = psi + (size_t)(ha ? sl.ja : 0) * M3;
    const T* pib = psi + (size_t)(hb ? sl.ib : 0) * M3;
    const T* pjb = psi + (size_t)(hb ? sl.jb : 0) * M3;
#pragma unroll
    for (int q = 0; q < PV; ++q) {
      const int p = tid + q * NT;
      if ((ZB * N) % NT == 0 || p < ZB * N) {
        const int zi = p / N, x = p % N;
        const size_t o = swap_yz ? ((size_t)y * N + z0 + zi) * N + x
                                 : ((size_t)(z0 + zi) * N + y) * N + x;
        va[q][0] = ha ? pia[o] : T(0);
        va[q][1] = ha ? pja[o] : T(0);
        vb[q][0] = hb ? pib[o] : T(0);
        vb[q][1] = hb ? pjb[o] : T(0);
      }
    }
  };
  if (ls0 < ls1) fetch(ls0);
  // the tables, loaded while the first slot's orbital values are in flight
  // (first read after the loop's first barrier)
  for (int k = tid; k < N; k += NT) {
    tw[k] = twg[k];
    if (NCLS == 2) md[k] = mdg[k];
  }

#pragma unroll 1
  for (int ls = ls0; ls < ls1; ++ls) {
    T wa = T(1), wb = T(1);
    if (W) {
      const Slot sl = slots[slot0 + ls];
      if (sl.ia >= 0) wa = sqrt_weight<T>(occ, sl.ia, sl.ja);
      if (sl.ib >= 0) wb = sqrt_weight<T>(occ, sl.ib, sl.jb);
    }
    // zb was last read by the previous slot's step 1, before its second barrier
#pragma unroll
    for (int q = 0; q < PV; ++q) {
      const int p = tid + q * NT;
      if ((ZB * N) % NT == 0 || p < ZB * N) {
        const int zi = p / N, x = p % N;
        if constexpr (CPLX)
          zb[zi * P + x] = {(va[q][0] * vb[q][0] + va[q][1] * vb[q][1]) * wa,
                            (va[q][1] * vb[q][0] - va[q][0] * vb[q][1]) * wa};
        else
          zb[zi * P + x] = {va[q][0] * va[q][1] * wa, vb[q][0] * vb[q][1] * wb};
      }
    }
    if (ls + 1 < ls1) fetch(ls + 1);
    __syncthreads();

    // step 1: items (line, t), line = cx*ZB + zi fastest; wk was last read by the
    // previous slot's step 2, before the barrier above
    constexpr int C1 = NL * L2;
#pragma unroll
    for (int it0 = 0; it0 < C1; it0 += NT) {
      int it = it0 + tid;
      if (C1 % NT == 0 || it < C1) {
        int line = it % NL, t = it / NL;
        int cx = line / ZB, zi = line % ZB;
        cpx<T> v[L1];
#pragma unroll
        for (int k1 = 0; k1 < L1; ++k1) {
          int x = t + L2 * k1;
          v[k1] = zb[zi * P + x];
          if (NCLS == 2 && cx == 1) v[k1] = cmul(v[k1], md[x]);
        }
        Dft<L1, -1, T>::run(v);
#pragma unroll
        for (int q1 = 1; q1 < L1; ++q1) v[q1] = cmul(v[q1], tw[t * q1]);
#pragma unroll
        for (int q1 = 0; q1 < L1; ++q1) wk[line * P + t + L2 * q1] = v[q1];
      }
    }
    __syncthreads();

    // step 2: items (line, q1); DFT_L2 over t -> kx = q1 + L1 q2, written to X
    constexpr int C2 = NL * L1;
    cpx<T>* Xs = X + (size_t)ls * NCLS * M3;
#pragma unroll
    for (int it0 = 0; it0 < C2; it0 += NT) {
      int it = it0 + tid;
      if (C2 % NT == 0 || it < C2) {
        int line = it % NL, q1 = it / NL;
        int cx = line / ZB, zi = line % ZB;
        cpx<T> v[L2];
#pragma unroll
        for (int t = 0; t < L2; ++t) v[t] = wk[line * P + t + L2 * q1];
        Dft<L2, -1, T>::run(v);
#pragma unroll
        for (int q2 = 0; q2 < L2; ++q2) {
          int kx = q1 + L1 * q2;
          store_stream(&Xs[x_off<N, NCLS>(cx, kx, y, z0 + zi)], v[q2]);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// pass B: per (slot, cx, kx) slab [y][z]: 2-D forward transform per (cy, cz)
// class, kernel multiply (Eq. 4 in Fourier space), 2-D inverse transform,
// demodulation and sum over classes.  A z-modulation is constant along y, so
// it commutes with the y-transform: with SHARE_Y the forward and inverse
// y-transforms are done once per cy and shared by both z classes (the
// y-transformed columns and the partial z sums then live in registers); for
// large slabs whose registers would spill, each class is transformed
// separately.  Energy-only variant: accumulate sum K |Z|^2 (Parseval).
// LDS layouts: A = [y][z] (pitch N), B = [z][y] (pitch N+1), same storage.
// Register arrays indexed by items (line, t), t < L2, holding L1 values:
//   acc : output, items (z, t) holding y = t + L2 k1
//   yv  : y-transformed columns, items (ky, t) holding z = t + L2 k1
//   wacc: sum over cz of the z-convolved columns, items (ky, t)
// ---------------------------------------------------------------------------
template <typename T, int N, int NT>
struct SlabFft {
  using S = Split<N>;
  static constexpr int L1 = S::L1, L2 = S::L2;
  static constexpr int PB = N + 1;
  static constexpr int C1 = N * L2;  // items (line, t)
  static constexpr int C2 = N * L1;  // items (line, q1)
  static constexpr int I1 = (C1 + NT - 1) / NT;
  static constexpr int I2 = (C2 + NT - 1) / NT;
  static __device__ __forceinline__ bool ok1(int it) { return C1 % NT == 0 || it < C1; }
  static __device__ __forceinline__ bool ok2(int it) { return C2 % NT == 0 || it < C2; }

  // y forward step 1 from the global slab (modulated by md^(cy y + cz z)) -> layout A
  template <int NCLS>
  static __device__ __forceinline__ void y_fwd1(const cpx<T>* g, cpx<T>* lds, const cpx<T>* tw,
                                                const cpx<T>* md, int cy, int cz, int tid) {
#pragma unroll
    for (int ii = 0; ii < I1; ++ii) {
      int it = tid + ii * NT;
      if (ok1(it)) {
        int z = it % N, t = it / N;
        cpx<T> v[L1];
        cpx<T> mz = cz ? md[z] : cpx<T>{T(1), T(0)};
#pragma unroll
        for (int k1 = 0; k1 < L1; ++k1) {
          cpx<T> a = g[slab_off<N, NCLS>(t + L2 * k1, z)];
          if (cy) a = cmul(a, md[t + L2 * k1]);
          if (cz) a = cmul(a, mz);
          v[k1] = a;
        }
        y_fwd1_tail(v, lds, tw, z, t);
      }
    }
  }
  // the same for class (1, 0) from slab values already in registers
  static __device__ __forceinline__ void y_fwd1_odd_vals(const cpx<T> (&vals)[I1][L1], cpx<T>* lds,
                                                         const cpx<T>* tw, const cpx<T>* md,
                                                         int tid) {
#pragma unroll
    for (int ii = 0; ii < I1; ++ii) {
      int it = tid + ii * NT;
      if (ok1(it)) {
        int z = it % N, t = it / N;
        cpx<T> v[L1];
#pragma unroll
        for (int k1 = 0; k1 < L1; ++k1) v[k1] = cmul(vals[ii][k1], md[t + L2 * k1]);
        y_fwd1_tail(v, lds, tw, z, t);
      }
    }
  }
  // slab values of items (z, t), y = t + L2 k1, into registers
  template <int NCLS>
  static __device__ __forceinline__ void load_slab(const cpx<T>* g, cpx<T> (&vals)[I1][L1], int tid) {
#pragma unroll
    for (int ii = 0; ii < I1; ++ii) {
      int it = tid + ii * NT;
      if (ok1(it)) {
        int z = it % N, t = it / N;
#pragma unroll
        for (int k1 = 0; k1 < L1; ++k1) vals[ii][k1] = g[slab_off<N, NCLS>(t + L2 * k1, z)];
      }
    }
  }
  static __device__ __forceinline__ void y_fwd1_tail(cpx<T>* v, cpx<T>* lds, const cpx<T>* tw,
                                                     int z, int t) {
    Dft<L1, -1, T>::run(v);
#pragma unroll
    for (int q1 = 1; q1 < L1; ++q1) v[q1] = cmul(v[q1], tw[t * q1]);
#pragma unroll
    for (int q1 = 0; q1 < L1; ++q1) lds[(t + L2 * q1) * N + z] = v[q1];
  }
  // y forward step 2: layout A (src) -> layout B (dst), ky in natural order;
  // in place (src == dst) every item is loaded before any is stored
  template <bool INPLACE>
  static __device__ __forceinline__ void y_fwd2(const cpx<T>* src, cpx<T>* dst, int tid) {
    cpx<T> w[I2][L2];
#pragma unroll
    for (int ii = 0; ii < I2; ++ii) {
      int it = tid + ii * NT;
      if (ok2(it)) {
        int z = it % N, q1 = it / N;
#pragma unroll
        for (int t = 0; t < L2; ++t) w[ii][t] = src[(t + L2 * q1) * N + z];
        Dft<L2, -1, T>::run(w[ii]);
      }
    }
    if (INPLACE) __syncthreads();
#pragma unroll
    for (int ii = 0; ii < I2; ++ii) {
      int it = tid + ii * NT;
      if (ok2(it)) {
        int z = it % N, q1 = it / N;
#pragma unroll
        for (int q2 = 0; q2 < L2; ++q2) dst[z * PB + q1 + L1 * q2] = w[ii][q2];
      }
    }
  }
  // z forward step 1 on one item: values v (z = t + L2 k1) -> layout B in place
  static __device__ __forceinline__ void z_fwd1_item(cpx<T>* v, cpx<T>* lds, const cpx<T>* tw,
                                                     int ky, int t) {
    Dft<L1, -1, T>::run(v);
#pragma unroll
    for (int q1 = 1; q1 < L1; ++q1) v[q1] = cmul(v[q1], tw[t * q1]);
#pragma unroll
    for (int q1 = 0; q1 < L1; ++q1) lds[(t + L2 * q1) * PB + ky] = v[q1];
  }
  // z forward step 2, kernel multiply (or Parseval sum), inverse step 2, in place
  // kt: the kernel table plane of this slab, [fold ky][fold kz] with MY, MZ
  // FFT points along y and z (2N on a zero-padded axis)
  template <bool EONLY, int MY, int MZ>
  static __device__ __forceinline__ void z_mid(cpx<T>* lds, const cpx<T>* tw, const T* kt,
                                               int cy, int cz, double& esum, int tid) {
    constexpr int HZ = MZ / 2 + 1;
    constexpr bool PADY = (MY == 2 * N), PADZ = (MZ == 2 * N);
#pragma unroll
    for (int ii = 0; ii < I2; ++ii) {
      int it = tid + ii * NT;
      if (ok2(it)) {
        int ky = it % N, q1 = it / N;
        cpx<T> v[L2];
#pragma unroll
        for (int t = 0; t < L2; ++t) v[t] = lds[(t + L2 * q1) * PB + ky];
        Dft<L2, -1, T>::run(v);
        const int kyf = PADY ? 2 * ky + cy : ky;
        const T* kr = kt + (size_t)fold(kyf, MY) * HZ;
        // kz = q1 + L1 q2 and its kernel index kzf = c + step q2 (c = 2 q1 + cz
        // padded, q1 periodic): below half the range fold(kzf) = kzf, above it
        // MZ - kzf, with the switch exactly at q2 = L2 / 2, so both halves are a
        // base pointer plus compile-time offsets.
        constexpr int step = PADZ ? 2 * L1 : L1;
        const int c = PADZ ? 2 * q1 + cz : q1;
        const T* k_lo = kr + c;
        const T* k_hi = kr + (MZ - c);
#pragma unroll
        for (int q2 = 0; q2 < L2; ++q2) {
          T kv = (2 * q2 < L2) ? k_lo[step * q2] : k_hi[-step * q2];
          if (EONLY) {
            esum += (double)kv *
                    ((double)v[q2].x * (double)v[q2].x + (double)v[q2].y * (double)v[q2].y);
          } else {
            v[q2].x *= kv;
            v[q2].y *= kv;
          }
        }
        if (!EONLY) {
          Dft<L2, 1, T>::run(v);
#pragma unroll
          for (int t = 1; t < L2; ++t) v[t] = cmulc(v[t], tw[t * q1]);
#pragma unroll
          for (int t = 0; t < L2; ++t) lds[(t + L2 * q1) * PB + ky] = v[t];
        }
      }
    }
  }
  // z inverse step 1 on one item: layout B -> values v (z = t + L2 k1)
  static __device__ __forceinline__ void z_inv1_item(cpx<T>* v, const cpx<T>* lds, int ky, int t) {
#pragma unroll
    for (int q1 = 0; q1 < L1; ++q1) v[q1] = lds[(t + L2 * q1) * PB + ky];
    Dft<L1, 1, T>::run(v);
  }
  // y inverse step 2: layout B (src) -> layout A (dst)
  template <bool INPLACE>
  static __device__ __forceinline__ void y_inv2(const cpx<T>* src, cpx<T>* dst, const cpx<T>* tw,
                                                int tid) {
    cpx<T> w[I2][L2];
#pragma unroll
    for (int ii = 0; ii < I2; ++ii) {
      int it = tid + ii * NT;
      if (ok2(it)) {
        int z = it % N, q1 = it / N;
#pragma unroll
        for (int q2 = 0; q2 < L2; ++q2) w[ii][q2] = src[z * PB + q1 + L1 * q2];
        Dft<L2, 1, T>::run(w[ii]);
#pragma unroll
        for (int t = 1; t < L2; ++t) w[ii][t] = cmulc(w[ii][t], tw[t * q1]);
      }
    }
    if (INPLACE) __syncthreads();
#pragma unroll
    for (int ii = 0; ii < I2; ++ii) {
      int it = tid + ii * NT;
      if (ok2(it)) {
        int z = it % N, q1 = it / N;
#pragma unroll
        for (int t = 0; t < L2; ++t) dst[(t + L2 * q1) * N + z] = w[ii][t];
      }
    }
  }
  // y inverse step 1, demodulate (cy, cz) and accumulate into acc
  static __device__ __forceinline__ void y_inv1(const cpx<T>* lds, const cpx<T>* md, int cy, int cz,
                                                cpx<T> (&acc)[I1][L1], int tid) {
#pragma unroll
    for (int ii = 0; ii < I1; ++ii) {
      int it = tid + ii * NT;
      if (ok1(it)) {
        int z = it % N, t = it / N;
        cpx<T> v[L1];
#pragma unroll
        for (int q1 = 0; q1 < L1; ++q1) v[q1] = lds[(t + L2 * q1) * N + z];
        Dft<L1, 1, T>::run(v);
        cpx<T> mz = cz ? md[z] : cpx<T>{T(1), T(0)};
#pragma unroll
        for (int k1 = 0; k1 < L1; ++k1) {
          cpx<T> a = v[k1];
          if (cy) a = cmulc(a, md[t + L2 * k1]);
          if (cz) a = cmulc(a, mz);
          acc[ii][k1] = cadd(acc[ii][k1], a);
        }
      }
    }
  }
};

// The wide (512-thread) shared-y variant asks for two blocks per CU, i.e. a
// budget of 128 registers (4 waves per SIMD); other variants take the
// compiler's choice.
template <typename T, int N, int NT, bool SHARE_Y>
constexpr int pass_b_min_waves() {
  return (SHARE_Y && NT == 512 && sizeof(T) == 4) ? 4 : 1;
}

template <typename T, int N, int CX, int CY, int CZ, int NT, bool EONLY, bool SHARE_Y>
__global__ __launch_bounds__(NT, (pass_b_min_waves<T, N, NT, SHARE_Y>())) void k_pass_b(cpx<T>* __restrict__ X, const T* __restrict__ ktab,
                                               const cpx<T>* __restrict__ twg,
                                               const cpx<T>* __restrict__ mdg,
                                               double* __restrict__ e_slot, int slot0,
                                               int kparts) {
  using F = SlabFft<T, N, NT>;
  constexpr int L1 = F::L1, L2 = F::L2, PB = F::PB, I1 = F::I1;
  constexpr int MX = CX * N, MY = CY * N, MZ = CZ * N;  // FFT points per axis
  constexpr int HY = MY / 2 + 1, HZ = MZ / 2 + 1;       // kernel table extents
  constexpr bool ANY_PAD = CX == 2 || CY == 2 || CZ == 2;
  __shared__ cpx<T> lds[(SHARE_Y ? 2 : 1) * N * PB];
  __shared__ cpx<T> tw[N];
  __shared__ cpx<T> md[N];

  const int tid = threadIdx.x;
  const int slab = blockIdx.x;  // cx * N + kx
  const int ls = blockIdx.y;
  const int cx = slab / N, kxp = slab % N;
  const int kxf = CX == 2 ? 2 * kxp + cx : kxp;
  const T* kt = ktab + (size_t)fold(kxf, MX) * HY * HZ;
  cpx<T>* g = X + (size_t)ls * CX * N * N * N + slab_base(slab);

  for (int k = tid; k < N; k += NT) {
    tw[k] = twg[k];
    if (ANY_PAD) md[k] = mdg[k];
  }
  cpx<T> acc[I1][L1];
#pragma unroll
  for (int ii = 0; ii < I1; ++ii)
#pragma unroll
    for (int k1 = 0; k1 < L1; ++k1) acc[ii][k1] = {T(0), T(0)};
  double esum = 0.0;
  __syncthreads();

  if constexpr (SHARE_Y) {
    // two LDS buffers U, V: every step reads one and writes the other (or
    // registers), which removes the in-place and write-after-read barriers
    cpx<T>* U = lds;
    cpx<T>* Vb = lds + N * PB;
    static_assert(!SHARE_Y || CZ == 2, "shared y-transforms serve two z classes");
    // the slab again for the odd y class, loaded (an L2 hit) while the even
    // class finishes, into registers its y-columns no longer need
    // (up to n = 80; at n = 96 those registers would spill, and the odd class
    // reads its slab again)
    constexpr bool PRE_ODD = N <= 80;
    cpx<T> odd[PRE_ODD ? I1 : 1][L1];
#pragma unroll
    for (int cy = 0; cy < CY; ++cy) {
      if (cy == 0 || !PRE_ODD)
        F::template y_fwd1<CX>(g, U, tw, md, cy, 0, tid);
      else
        F::y_fwd1_odd_vals(odd, U, tw, md, tid);
      __syncthreads();
      F::template y_fwd2<false>(U, Vb, tid);
      __syncthreads();
      cpx<T> yv[I1][L1];
      cpx<T> wacc[I1][L1];
#pragma unroll
      for (int ii = 0; ii < I1; ++ii) {
        int it = tid + ii * NT;
        if (F::ok1(it)) {
          int ky = it % N, t = it / N;
#pragma unroll
          for (int k1 = 0; k1 < L1; ++k1) {
            yv[ii][k1] = Vb[(t + L2 * k1) * PB + ky];
            wacc[ii][k1] = {T(0), T(0)};
          }
        }
      }
      if constexpr (N <= 80) {
        // both z classes side by side, class 0 in U and class 1 in Vb: each phase
        // holds two independent items per thread (measured at n = 64: pass B
        // 1.16 -> 1.12 ms; n = 80 4.05 -> 3.79 ms; at n = 96 the registers spill)
        __syncthreads();  // every yv read of Vb precedes class 1's writes to it
#pragma unroll
        for (int ii = 0; ii < I1; ++ii) {
          int it = tid + ii * NT;
          if (F::ok1(it)) {
            int ky = it % N, t = it / N;
            cpx<T> v0[L1], v1[L1];
#pragma unroll
            for (int k1 = 0; k1 < L1; ++k1) {
              v0[k1] = yv[ii][k1];
              v1[k1] = cmul(yv[ii][k1], md[t + L2 * k1]);
            }
            F::z_fwd1_item(v0, U, tw, ky, t);
            F::z_fwd1_item(v1, Vb, tw, ky, t);
          }
        }
        __syncthreads();
        F::template z_mid<EONLY, MY, MZ>(U, tw, kt, cy, 0, esum, tid);
        F::template z_mid<EONLY, MY, MZ>(Vb, tw, kt, cy, 1, esum, tid);
        __syncthreads();
        if (!EONLY) {
#pragma unroll
          for (int ii = 0; ii < I1; ++ii) {
            int it = tid + ii * NT;
            if (F::ok1(it)) {
              int ky = it % N, t = it / N;
              cpx<T> v0[L1], v1[L1];
              F::z_inv1_item(v0, U, ky, t);
              F::z_inv1_item(v1, Vb, ky, t);
#pragma unroll
              for (int k1 = 0; k1 < L1; ++k1)
                wacc[ii][k1] = cadd(cadd(wacc[ii][k1], v0[k1]), cmulc(v1[k1], md[t + L2 * k1]));
            }
          }
          __syncthreads();  // the inverse z steps' reads of U precede its rewrite below
        }
      } else {
#pragma unroll
        for (int cz = 0; cz < CZ; ++cz) {
          cpx<T>* B = cz ? Vb : U;  // class cz works in its own buffer
#pragma unroll
          for (int ii = 0; ii < I1; ++ii) {
            int it = tid + ii * NT;
            if (F::ok1(it)) {
              int ky = it % N, t = it / N;
              cpx<T> v[L1];
#pragma unroll
              for (int k1 = 0; k1 < L1; ++k1)
                v[k1] = cz ? cmul(yv[ii][k1], md[t + L2 * k1]) : yv[ii][k1];
              F::z_fwd1_item(v, B, tw, ky, t);
            }
          }
          __syncthreads();
          F::template z_mid<EONLY, MY, MZ>(B, tw, kt, cy, cz, esum, tid);
          __syncthreads();
          if (EONLY) continue;
#pragma unroll
          for (int ii = 0; ii < I1; ++ii) {
            int it = tid + ii * NT;
            if (F::ok1(it)) {
              int ky = it % N, t = it / N;
              cpx<T> v[L1];
              F::z_inv1_item(v, B, ky, t);
#pragma unroll
              for (int k1 = 0; k1 < L1; ++k1)
                wacc[ii][k1] = cadd(wacc[ii][k1], cz ? cmulc(v[k1], md[t + L2 * k1]) : v[k1]);
            }
          }
        }
      }
      if (EONLY) {
        if constexpr (PRE_ODD) {
          if (cy == 0 && CY == 2) F::template load_slab<CX>(g, odd, tid);
        }
        __syncthreads();
        continue;
      }
      // U was last read by the cz = 0 inverse step, before the previous barrier
      // (the interleaved form: before the barrier that closes its inverse steps)
#pragma unroll
      for (int ii = 0; ii < I1; ++ii) {
        int it = tid + ii * NT;
        if (F::ok1(it)) {
          int ky = it % N, t = it / N;
#pragma unroll
          for (int k1 = 0; k1 < L1; ++k1) U[(t + L2 * k1) * PB + ky] = wacc[ii][k1];
        }
      }
      if constexpr (PRE_ODD) {
        if (cy == 0 && CY == 2) F::template load_slab<CX>(g, odd, tid);
      }
      __syncthreads();
      F::template y_inv2<false>(U, Vb, tw, tid);
      __syncthreads();
      F::y_inv1(Vb, md, cy, 0, acc, tid);
      // the next y_fwd1 writes U, whose last reads (y_inv2) precede the barrier above
    }
  } else {
#pragma unroll 1
    for (int cls = 0; cls < CY * CZ; ++cls) {
      const int cy = cls / CZ;
      const int cz = cls % CZ;
      F::template y_fwd1<CX>(g, lds, tw, md, cy, cz, tid);
      __syncthreads();
      F::template y_fwd2<true>(lds, lds, tid);
      __syncthreads();
#pragma unroll
      for (int ii = 0; ii < I1; ++ii) {
        int it = tid + ii * NT;
        if (F::ok1(it)) {
          int ky = it % N, t = it / N;
          cpx<T> v[L1];
#pragma unroll
          for (int k1 = 0; k1 < L1; ++k1) v[k1] = lds[(t + L2 * k1) * PB + ky];
          F::z_fwd1_item(v, lds, tw, ky, t);
        }
      }
      __syncthreads();
      F::template z_mid<EONLY, MY, MZ>(lds, tw, kt, cy, cz, esum, tid);
      __syncthreads();
      if (EONLY) continue;
#pragma unroll
      for (int ii = 0; ii < I1; ++ii) {
        int it = tid + ii * NT;
        if (F::ok1(it)) {
          int ky = it % N, t = it / N;
          cpx<T> v[L1];
          F::z_inv1_item(v, lds, ky, t);
#pragma unroll
          for (int k1 = 0; k1 < L1; ++k1) lds[(t + L2 * k1) * PB + ky] = v[k1];
        }
      }
      __syncthreads();
      F::template y_inv2<true>(lds, lds, tw, tid);
      __syncthreads();
      F::y_inv1(lds, md, cy, cz, acc, tid);
      __syncthreads();
    }
  }

  if (EONLY) {
    // block reduction of the Parseval sum into this (slot, slab)'s partial
    __shared__ double red[NT / 64];
    double v = esum;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    if (tid == 0) {
      double sum = 0.0;
      for (int w = 0; w < NT / 64; ++w) sum += red[w];
      // one partial per (slot, slab); summed in a fixed order by k_slot_reduce
      e_slot[(size_t)(2 * (slot0 + ls)) * kparts + slab] = sum;
    }
    return;
  } else {
    // every block has read its whole slab (first class) before any write here
#pragma unroll
    for (int ii = 0; ii < I1; ++ii) {
      int it = tid + ii * NT;
      if (F::ok1(it)) {
        int z = it % N, t = it / N;
#pragma unroll
        for (int k1 = 0; k1 < L1; ++k1) g[slab_off<N, CX>(t + L2 * k1, z)] = acc[ii][k1];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// pass B, wave-local form.  One slab (slot, cx, kx) per workgroup of 8 N
// threads (N / 8 wavefronts).  Every n-point line transform is two register
// steps, DFT_{N/8} per lane over points t + 8 k1 and DFT_8 across the line's 8
// lanes, with one LDS exchange between them.  The 8 lanes of a line sit in one
// wavefront, and a wavefront owns 8 whole columns of the slab while it
// transforms along y and 8 whole rows while it transforms along z, so inside a
// phase every exchange stays within one wavefront: it synchronises with itself
// only (the LDS operations of a wavefront take effect in issue order).  Only
// the two transpositions per y class, columns -> rows before the z phase and
// rows -> columns after it, need a workgroup barrier.
//
// Per y class cy: forward y (columns), then per z class cz the forward z
// transform of the y-transformed rows (modulated by w_2n^z for cz = 1), the
// kernel multiply (or the Parseval sum), the inverse z transform and the
// demodulated sum over cz (rows), then the inverse y transform, demodulated
// (columns).  With two y classes the class-0 result waits in HBM-backed global
// memory (the slab itself, after its class-1 input has been read) or, for
// small slabs, in registers; the class-1 result is added to it.
//
// LDS: one slab buffer, row pitch PB, element (row, col) at row PB + col +
// col / 8 (one spare word per 8 columns spreads a row's stride-8 accesses over
// the banks), PB = 8 mod 16 (so rows an odd number of rows apart, or two rows
// apart, fall on different bank halves).  Within the y phase the values
// between the two steps sit at row p ^ ((p / 8) & 3) of their column instead
// of row p = t + 8 q1, which keeps both steps' accesses free of bank conflicts.
// ---------------------------------------------------------------------------
// LDS load of one complex value that the compiler keeps as a single 8-byte
// (16-byte for FP64) read: on gfx950 a paired read (ds_read2_b64) of two such
// values measured 7.3 LDS cycles against 2 x 2.1 for two single reads, and
// pairing is what the compiler does with nearby addresses of one base.
template <typename T>
__device__ __forceinline__ cpx<T> lds_ld(const cpx<T>* p) {
  using V2 = T __attribute__((ext_vector_type(2)));
  using LV = __attribute__((address_space(3))) volatile V2;
  const V2 v = *(const LV*)(p);  // generic -> LDS address space
  return {v.x, v.y};
}

// Two consecutive complex values (16-byte aligned) in one 16-byte LDS read.
template <typename T>
__device__ __forceinline__ void lds_ld2(const cpx<T>* p, cpx<T>& a, cpx<T>& b) {
  using V4 = T __attribute__((ext_vector_type(4)));
  using LV = __attribute__((address_space(3))) volatile V4;
  const V4 v = *(const LV*)(p);
  a = {v.x, v.y};
  b = {v.z, v.w};
}

// Twiddle and modulation tables of the wave-local pass in LDS, laid out so
// that the values a lane needs are contiguous (paired 16-byte reads) and the
// eight rows that the lanes of a wavefront read fall on different banks:
//   rowT[r TS + k] = w_N^{r k}    (the twiddles of step 1, lane row r = t)
//   modT[r TS + k] = w_2N^{r + 8k} (the class-1 modulation at point r + 8 k)
//   colA[q TA + t] = w_N^{q t}    (the twiddles of step 2, row q = q1)
constexpr int WAVE_TS = 18, WAVE_TA = 10;
template <typename T>
struct WaveTabs {
  const cpx<T>* rowT;
  const cpx<T>* modT;
  const cpx<T>* colA;
};

// v[k] *= r[k] (C = false) or conj(r[k]) (C = true) for k in [K0, L), with r in
// LDS, 16-byte aligned at even k.  PAIR: two values per 16-byte read, fewer LDS
// instructions for a few more VALU ones: it pays where the wave-local pass waits
// on the LDS (one 1024-thread block per CU from n = 96 on: free 128^3, pass B
// -6 %), not at n = 64, where several blocks share a CU and VALU issue limits
template <bool C, int K0, int L, bool PAIR, typename T>
__device__ __forceinline__ void lds_scale(cpx<T>* v, const cpx<T>* r) {
  static_assert(L % 2 == 0, "even length");
  if constexpr (!PAIR) {
#pragma unroll
    for (int k = K0; k < L; ++k) v[k] = C ? cmulc(v[k], lds_ld(r + k)) : cmul(v[k], lds_ld(r + k));
    return;
  }
  if constexpr (K0 == 1) {
    const cpx<T> a = lds_ld(r + 1);
    v[1] = C ? cmulc(v[1], a) : cmul(v[1], a);
  }
#pragma unroll
  for (int k = (K0 == 1 ? 2 : K0); k < L; k += 2) {
    cpx<T> a, b;
    lds_ld2(r + k, a, b);
    v[k] = C ? cmulc(v[k], a) : cmul(v[k], a);
    v[k + 1] = C ? cmulc(v[k + 1], b) : cmul(v[k + 1], b);
  }
}

template <int N>
constexpr int wave_pitch() {
  int p = 9 * N / 8;
  while (p % 16 != 8) ++p;
  return p;
}

// The class-0 output of the y classes is held in registers (instead of being
// parked in the slab and read back) where the registers allow it: up to n = 64,
// and at n = 96, whose 768-thread block (3 waves per SIMD) may use 168 registers
// a lane (143 with the held values; pass B -5 % at free 96^3).  The 896- and
// 1024-thread blocks of n = 112, 128 have 128, all in use.
template <typename T, int N>
constexpr bool wave_hold_p0() {
  return sizeof(T) == 4 && (N <= 64 || N == 96);
}

// A value the compiler must treat as unknown from here on: keeps it from
// carrying addresses computed in one phase over to the next (their registers
// would stay live, and spill, across the phases in between).
__device__ __forceinline__ unsigned opaque(unsigned v) {
  asm volatile("" : "+v"(v));
  return v;
}

// Vector loads of one complex value through a buffer resource: a lane's byte
// offset in a register, a block-uniform offset in a scalar register, so the
// rows of a column share one address register.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void* base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, 0x7fffffff, 0x00020000);
}
template <typename T>
__device__ __forceinline__ cpx<T> buffer_load_cpx(__amdgpu_buffer_rsrc_t r, unsigned voff,
                                                  unsigned soff) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(cpx<T>, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  } else {
    return __builtin_bit_cast(cpx<T>, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
  }
}

__device__ __forceinline__ void wave_lds_sync() {
  // orders this wavefront's LDS accesses before and after this point (the
  // hardware keeps a wavefront's LDS operations in order; the fences keep the
  // compiler from moving accesses across)
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One y class of the wave-local pass B (CYI = 0 or 1, compile time).  P holds
// the class-0 output of this lane's column points between the classes.
template <typename T, int N, int CX, int CY, int CZ, bool EONLY, int CYI>
__device__ __forceinline__ void wave_y_class(cpx<T>* __restrict__ S, const WaveTabs<T> tb, cpx<T>* g,
                                             __amdgpu_buffer_rsrc_t grs, const T* kt,
                                             cpx<T> (&P)[N / 8], cpx<T> (&V1)[N / 8],
                                             double& esum) {
  constexpr int L1 = N / 8, PB = wave_pitch<N>();
  constexpr int NJ = (L1 + 7) / 8;  // step-2 items per lane
  constexpr int MY = CY * N, MZ = CZ * N;
  constexpr int HZ = MZ / 2 + 1;
  constexpr bool PADY = CY == 2, PADZ = CZ == 2;
  constexpr bool HOLD = wave_hold_p0<T, N>();
  // with two y classes the class-1 input is loaded during class 0's inverse y
  // phase, and (n > 64) the parked class-0 result during class 1's, so that
  // their latency overlaps the inverse transforms
  constexpr bool EARLY = CY == 2 && !EONLY;
  constexpr bool WPAIR = N > 64;  // paired table reads (see lds_scale)
  constexpr unsigned KSTRIDE = 8u * CX * N * N * sizeof(cpx<T>);  // slab rows y -> y + 8

  // lane coordinates, laundered per class (see opaque)
  const unsigned tid = opaque(threadIdx.x);
  const int lane = tid & 63, wv = tid >> 6;
  // column phases: column zc, position ty; row phase: row kr, position tz
  const int zc = 8 * wv + (lane & 7), ty = lane >> 3;
  cpx<T>* Scol = S + (zc + (zc >> 3));
  const int kr = 8 * wv + (lane >> 3), tz = lane & 7;
  cpx<T>* Srow = S + kr * PB;
  // slab element (ty + 8 k1, zc): this lane's byte offset plus k1 KSTRIDE
  // (a slab spans less than CX N^3 values of one slot: 32-bit offsets)
  const unsigned goff = (unsigned)(((size_t)ty * CX * N * N + (size_t)(zc / XZ) * (CX * N * XZ) +
                                    zc % XZ) * sizeof(cpx<T>));
  auto gat = [&](int k1) -> cpx<T>* {
    return reinterpret_cast<cpx<T>*>(reinterpret_cast<char*>(g) + goff + (size_t)k1 * KSTRIDE);
  };

  // ---- forward y, step 1: DFT_L1 over y = ty + 8 k1 of column zc
  {
    cpx<T> v[L1];
#pragma unroll
    for (int k1 = 0; k1 < L1; ++k1)
      v[k1] = (EARLY && CYI == 1) ? V1[k1] : buffer_load_cpx<T>(grs, goff, k1 * KSTRIDE);
    if constexpr (CYI == 1) lds_scale<false, 0, L1, WPAIR>(v, tb.modT + ty * WAVE_TS);
    if constexpr (CYI == 1 && !EONLY && !HOLD) {
      // the class-1 input is in registers: park the class-0 output in the slab
#pragma unroll
      for (int k1 = 0; k1 < L1; ++k1) *gat(k1) = P[k1];
    }
    Dft<L1, -1, T>::run(v);
    lds_scale<false, 1, L1, WPAIR>(v, tb.rowT + ty * WAVE_TS);
#pragma unroll
    for (int q1 = 0; q1 < L1; ++q1) Scol[((ty ^ (q1 & 3)) + 8 * q1) * PB] = v[q1];
  }
  wave_lds_sync();
  // ---- forward y, step 2: DFT_8 over t for q1 = ty + 8 j -> ky = q1 + L1 q2
  {
    cpx<T> w[NJ][8];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int q1 = ty + 8 * j;
      if (q1 < L1) {
#pragma unroll
        for (int t = 0; t < 8; ++t) w[j][t] = lds_ld(&Scol[((t ^ (ty & 3)) + 8 * q1) * PB]);
      }
    }
    wave_lds_sync();  // every lane's reads precede the in-place writes
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int q1 = ty + 8 * j;
      if (q1 < L1) {
        Dft<8, -1, T>::run(w[j]);
#pragma unroll
        for (int q2 = 0; q2 < 8; ++q2) Scol[(q1 + L1 * q2) * PB] = w[j][q2];
      }
    }
  }
  __syncthreads();  // columns -> rows

  // ---- z phase on row kr (ky): values z = tz + 8 k1 at column tz + 9 k1.
  // Both z classes take their forward step 1 from the row at once; class 1's
  // result waits in registers while class 0 finishes in the row.
  {
    const int kyf = PADY ? 2 * kr + CYI : kr;
    const T* krow = kt + (size_t)fold(kyf, MY) * HZ;
    // kernel values of one z class at this lane's (q1 = tz + 8 j, q2): kernel
    // index kzf = c + step q2; below half the range fold(kzf) = kzf, above it
    // MZ - kzf, switching exactly at q2 = 4.  Where the registers allow it
    // (FP32 except n = 112, which then spills) they are loaded ahead of their
    // use, so the latency overlaps the transforms; else where they are used.
    constexpr int step = PADZ ? 2 * L1 : L1;
    constexpr bool KPRE = sizeof(T) == 4 && N != 112;
    auto k_load = [&](int cz, auto& kv) {
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int q1 = tz + 8 * j;
        if (q1 < L1) {
          const int c = PADZ ? 2 * q1 + cz : q1;
          const T* k_lo = krow + c;
          const T* k_hi = krow + (MZ - c);
#pragma unroll
          for (int q2 = 0; q2 < 8; ++q2) kv[j][q2] = (q2 < 4) ? k_lo[step * q2] : k_hi[-step * q2];
        }
      }
    };
    // step 2 of one class, in place in the row: per q1 = tz + 8 j, DFT_8,
    // kernel (kz = q1 + L1 q2) or the Parseval sum, inverse DFT_8
    auto z_mid = [&](int cz, const auto& kv) {
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int q1 = tz + 8 * j;
        if (q1 < L1) {
          cpx<T> w[8];
#pragma unroll
          for (int t = 0; t < 8; ++t) w[t] = lds_ld(&Srow[t + 9 * q1]);
          Dft<8, -1, T>::run(w);
#pragma unroll
          for (int q2 = 0; q2 < 8; ++q2) {
            T k;
            if constexpr (KPRE) {
              k = kv[j][q2];
            } else {
              const int c = PADZ ? 2 * q1 + cz : q1;
              k = (q2 < 4) ? krow[c + step * q2] : krow[MZ - c - step * q2];
            }
            if (EONLY) {
              esum += (double)k * ((double)w[q2].x * (double)w[q2].x + (double)w[q2].y * (double)w[q2].y);
            } else {
              w[q2].x *= k;
              w[q2].y *= k;
            }
          }
          if (!EONLY) {
            Dft<8, 1, T>::run(w);
            lds_scale<true, 1, 8, WPAIR>(w, tb.colA + q1 * WAVE_TA);
#pragma unroll
            for (int t = 0; t < 8; ++t) Srow[t + 9 * q1] = w[t];
          }
        }
      }
    };
    T kv0[KPRE ? NJ : 1][8], kv1[KPRE && CZ == 2 ? NJ : 1][8];
    cpx<T> u1[CZ == 2 ? L1 : 1];
    {
      cpx<T> u0[L1];
#pragma unroll
      for (int k1 = 0; k1 < L1; ++k1) {
        u0[k1] = lds_ld(&Srow[tz + 9 * k1]);
        if constexpr (CZ == 2) u1[k1] = u0[k1];
      }
      if constexpr (CZ == 2) lds_scale<false, 0, L1, WPAIR>(u1, tb.modT + tz * WAVE_TS);
      Dft<L1, -1, T>::run(u0);
      lds_scale<false, 1, L1, WPAIR>(u0, tb.rowT + tz * WAVE_TS);
#pragma unroll
      for (int q1 = 0; q1 < L1; ++q1) Srow[tz + 9 * q1] = u0[q1];
    }
    if constexpr (KPRE) k_load(0, kv0);
    if constexpr (CZ == 2) {
      Dft<L1, -1, T>::run(u1);
      lds_scale<false, 1, L1, WPAIR>(u1, tb.rowT + tz * WAVE_TS);
    }
    wave_lds_sync();
    z_mid(0, kv0);
    if constexpr (CZ == 2 && KPRE) k_load(1, kv1);
    wave_lds_sync();  // step 2 of class 0 precedes the reads and stores below
    cpx<T> acc[L1];
    if constexpr (!EONLY) {
      // inverse step 1 of class 0: IDFT_L1 over q1 -> z = tz + 8 k1
#pragma unroll
      for (int q1 = 0; q1 < L1; ++q1) acc[q1] = lds_ld(&Srow[tz + 9 * q1]);
      Dft<L1, 1, T>::run(acc);
    }
    if constexpr (CZ == 2) {
      // class 1 into the row (this lane's own step-1 addresses)
#pragma unroll
      for (int q1 = 0; q1 < L1; ++q1) Srow[tz + 9 * q1] = u1[q1];
      wave_lds_sync();
      z_mid(1, kv1);
      wave_lds_sync();
      if constexpr (!EONLY) {
        cpx<T> v[L1];
#pragma unroll
        for (int q1 = 0; q1 < L1; ++q1) v[q1] = lds_ld(&Srow[tz + 9 * q1]);
        Dft<L1, 1, T>::run(v);
        lds_scale<true, 0, L1, WPAIR>(v, tb.modT + tz * WAVE_TS);
#pragma unroll
        for (int k1 = 0; k1 < L1; ++k1) acc[k1] = cadd(acc[k1], v[k1]);
      }
    }
    if constexpr (EONLY) {
      __syncthreads();  // rows -> columns: the next class rewrites every column
      return;
    } else {
#pragma unroll
      for (int k1 = 0; k1 < L1; ++k1) Srow[tz + 9 * k1] = acc[k1];
    }
  }
  __syncthreads();  // rows -> columns

  // ---- inverse y (column zc again), step 2: IDFT_8 over q2 (ky = q1 + L1 q2),
  // conjugate twiddle; lane coordinates laundered again for this phase
  const unsigned tid2 = opaque(threadIdx.x);
  const int zc2 = 8 * (int)(tid2 >> 6) + (int)(tid2 & 7), ty2 = (int)((tid2 & 63) >> 3);
  cpx<T>* Scol2 = S + (zc2 + (zc2 >> 3));
  const unsigned off2 = (unsigned)(((size_t)ty2 * CX * N * N + (size_t)(zc2 / XZ) * (CX * N * XZ) +
                                    zc2 % XZ) * sizeof(cpx<T>));
  cpx<T> pk[EARLY && CYI == 1 && !HOLD ? L1 : 1];
  if constexpr (EARLY) {
    // no workgroup barrier remains before these values are used, so nothing
    // forces the loads to complete before the transforms below
#pragma unroll
    for (int k1 = 0; k1 < L1; ++k1) {
      if constexpr (CYI == 0)
        V1[k1] = buffer_load_cpx<T>(grs, off2, k1 * KSTRIDE);  // the class-1 input
      else if constexpr (!HOLD)
        pk[k1] = buffer_load_cpx<T>(grs, off2, k1 * KSTRIDE);  // the parked class-0 result
    }
  }
  {
    cpx<T> w[NJ][8];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int q1 = ty2 + 8 * j;
      if (q1 < L1) {
#pragma unroll
        for (int q2 = 0; q2 < 8; ++q2) w[j][q2] = lds_ld(&Scol2[(q1 + L1 * q2) * PB]);
      }
    }
    wave_lds_sync();
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int q1 = ty2 + 8 * j;
      if (q1 < L1) {
        Dft<8, 1, T>::run(w[j]);
        lds_scale<true, 1, 8, WPAIR>(w[j], tb.colA + q1 * WAVE_TA);
#pragma unroll
        for (int t = 0; t < 8; ++t) Scol2[((t ^ (ty2 & 3)) + 8 * q1) * PB] = w[j][t];
      }
    }
  }
  wave_lds_sync();
  // ---- inverse y, step 1: IDFT_L1 over q1 -> y = ty + 8 k1, demodulate
  {
    cpx<T> o[L1];
#pragma unroll
    for (int q1 = 0; q1 < L1; ++q1) o[q1] = lds_ld(&Scol2[((ty2 ^ (q1 & 3)) + 8 * q1) * PB]);
    Dft<L1, 1, T>::run(o);
    if constexpr (CYI == 1) lds_scale<true, 0, L1, WPAIR>(o, tb.modT + ty2 * WAVE_TS);
    if constexpr (CY == 2 && CYI == 0) {
#pragma unroll
      for (int k1 = 0; k1 < L1; ++k1) P[k1] = o[k1];
    } else {
#pragma unroll
      for (int k1 = 0; k1 < L1; ++k1) {
        cpx<T>* dst = reinterpret_cast<cpx<T>*>(reinterpret_cast<char*>(g) + off2 + (size_t)k1 * KSTRIDE);
        if (CY == 2) o[k1] = cadd(o[k1], HOLD ? P[k1] : pk[(EARLY && !HOLD) ? k1 : 0]);
        // pass C reads the result only after the launch: at n = 128 a
        // non-temporal store keeps it from evicting what the blocks in flight
        // re-read (kernel planes, parked and class-1 slab data; pass B -1 %,
        // no gain at n <= 96)
        if constexpr (N >= 128)
          store_stream(dst, o[k1]);
        else
          *dst = o[k1];
      }
    }
  }
  // the next class's forward y stores go to this wavefront's own columns
  wave_lds_sync();
}

template <typename T, int N, int CX, int CY, int CZ, bool EONLY>
__global__ __launch_bounds__(8 * N) void k_pass_b_wave(cpx<T>* __restrict__ X,
                                                       const T* __restrict__ ktab,
                                                       const cpx<T>* __restrict__ twg,
                                                       const cpx<T>* __restrict__ mdg,
                                                       double* __restrict__ e_slot, int slot0,
                                                       int kparts, int nslots) {
  constexpr int NT = 8 * N, L1 = N / 8, PB = wave_pitch<N>();
  constexpr int MX = CX * N, MY = CY * N, MZ = CZ * N;
  constexpr int HY = MY / 2 + 1, HZ = MZ / 2 + 1;
  constexpr bool ANY_PAD = CX == 2 || CY == 2 || CZ == 2;
  static_assert(N % 8 == 0 && L1 <= 16, "line length 8 L1 with L1 <= 16");
  __shared__ cpx<T> S[N * PB];
  __shared__ __align__(16) cpx<T> rowT[8 * WAVE_TS];
  __shared__ __align__(16) cpx<T> modT[ANY_PAD ? 8 * WAVE_TS : 2];
  __shared__ __align__(16) cpx<T> colA[L1 * WAVE_TA];

  const int tid = threadIdx.x;
  int slab, ls;  // slab = cx * N + kx, slot of the launch
  if constexpr (pass_b_xcd_order(N)) {
    xcd_split(blockIdx.x, CX * N, nslots, slab, ls);
  } else {
    slab = blockIdx.x;
    ls = blockIdx.y;
  }
  const int cx = slab / N, kxp = slab % N;
  const int kxf = CX == 2 ? 2 * kxp + cx : kxp;
  const T* kt = ktab + (size_t)fold(kxf, MX) * HY * HZ;
  cpx<T>* g = X + (size_t)ls * CX * N * N * N + slab_base(slab);
  const __amdgpu_buffer_rsrc_t grs = buffer_rsrc(g);

  // every entry a lane reads (k < L1 of a row, t < 8) from the global tables
  // w_N^k (twg) and w_2N^k (mdg), k < N; 8 L1 = N <= NT threads, one entry of
  // each table per thread
  static_assert(8 * L1 <= NT, "one table entry per thread");
  if (tid < 8 * L1) {
    const int lo = tid & 7, hi = tid >> 3;  // hi < L1
    rowT[lo * WAVE_TS + hi] = twg[lo * hi];
    if (ANY_PAD) modT[lo * WAVE_TS + hi] = mdg[lo + 8 * hi];
    colA[hi * WAVE_TA + lo] = twg[hi * lo];
  }
  __syncthreads();

  const WaveTabs<T> tb{rowT, modT, colA};
  double esum = 0.0;
  cpx<T> P[L1], V1[L1];
  wave_y_class<T, N, CX, CY, CZ, EONLY, 0>(S, tb, g, grs, kt, P, V1, esum);
  if constexpr (CY == 2) wave_y_class<T, N, CX, CY, CZ, EONLY, 1>(S, tb, g, grs, kt, P, V1, esum);

  if constexpr (EONLY) {
    // block reduction of the Parseval sum into this (slot, slab)'s partial
    __shared__ double red[NT / 64];
    double v = esum;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    if (tid == 0) {
      double sum = 0.0;
      for (int w = 0; w < NT / 64; ++w) sum += red[w];
      e_slot[(size_t)(2 * (slot0 + ls)) * kparts + slab] = sum;
    }
  }
}

// ---------------------------------------------------------------------------
// pass B split in three launches for slabs whose two LDS buffers do not fit
// (n >= 112 with a zero-padded z axis).  The 2-D transform of a
// slab factorises into independent 1-D transforms along y (per z column) and
// along z (per ky line), so each launch works on chunks of SC columns or
// lines with small LDS tiles and many blocks per CU; the y-transformed
// classes travel through a scratch Y[slot][slab][cy][ky][z] (L2 / memory-side
// cache resident for the few slots of one launch):
//   B1  per z-chunk: y-transform of every class cy       X -> Y
//   B2  per ky-chunk: per cy, z-transform of every class cz, kernel multiply
//       (or the Parseval sum), inverse z, demodulate, sum over cz   Y -> Y
//   B3  per z-chunk: inverse y of every class, demodulate, sum     Y -> X
// ---------------------------------------------------------------------------
constexpr int SC = 16;  // columns (B1, B3) or lines (B2) per block

template <typename T, int N, int CX, int CY, int NT>
__global__ __launch_bounds__(NT) void k_pass_b1(const cpx<T>* __restrict__ X, cpx<T>* __restrict__ Y,
                                                const cpx<T>* __restrict__ twg,
                                                const cpx<T>* __restrict__ mdg) {
  using S = Split<N>;
  constexpr int L1 = S::L1, L2 = S::L2;
  constexpr int P = SC + 1;
  __shared__ cpx<T> buf[N * P];  // [y][zi]
  __shared__ cpx<T> tw[N];
  __shared__ cpx<T> md[N];
  const int tid = threadIdx.x;
  const int z0 = blockIdx.x * SC, slab = blockIdx.y, ls = blockIdx.z;
  const cpx<T>* g = X + (size_t)ls * CX * N * N * N + slab_base(slab);
  cpx<T>* yo = Y + ((size_t)ls * CX * N + slab) * CY * N * N;
  for (int k = tid; k < N; k += NT) {
    tw[k] = twg[k];
    md[k] = mdg[k];
  }
  __syncthreads();
  constexpr int C1 = SC * L2, C2 = SC * L1;
#pragma unroll 1
  for (int cy = 0; cy < CY; ++cy) {
    // step 1, items (zi, t): y = t + L2 k1
    for (int it = tid; it < C1; it += NT) {
      const int zi = it % SC, t = it / SC;
      cpx<T> v[L1];
#pragma unroll
      for (int k1 = 0; k1 < L1; ++k1) {
        const int y = t + L2 * k1;
        cpx<T> a = g[slab_off<N, CX>(y, z0 + zi)];
        v[k1] = cy ? cmul(a, md[y]) : a;
      }
      Dft<L1, -1, T>::run(v);
#pragma unroll
      for (int q1 = 1; q1 < L1; ++q1) v[q1] = cmul(v[q1], tw[t * q1]);
#pragma unroll
      for (int q1 = 0; q1 < L1; ++q1) buf[(t + L2 * q1) * P + zi] = v[q1];
    }
    __syncthreads();
    // step 2, items (zi, q1): ky = q1 + L1 q2
    cpx<T>* yc = yo + (size_t)cy * N * N;
    for (int it = tid; it < C2; it += NT) {
      const int zi = it % SC, q1 = it / SC;
      cpx<T> w[L2];
#pragma unroll
      for (int t = 0; t < L2; ++t) w[t] = buf[(t + L2 * q1) * P + zi];
      Dft<L2, -1, T>::run(w);
#pragma unroll
      for (int q2 = 0; q2 < L2; ++q2) yc[(size_t)(q1 + L1 * q2) * N + z0 + zi] = w[q2];
    }
    __syncthreads();  // buf is rewritten by the next class
  }
}

template <typename T, int N, int CX, int CY, int CZ, int NT, bool EONLY>
__global__ __launch_bounds__(NT) void k_pass_b2(cpx<T>* __restrict__ Y, const T* __restrict__ ktab,
                                                const cpx<T>* __restrict__ twg,
                                                const cpx<T>* __restrict__ mdg,
                                                double* __restrict__ e_part, int slot0,
                                                int kparts) {
  using S = Split<N>;
  constexpr int L1 = S::L1, L2 = S::L2;
  constexpr int P = SC + 1;
  constexpr int MX = CX * N, MY = CY * N, MZ = CZ * N;
  constexpr int HY = MY / 2 + 1, HZ = MZ / 2 + 1;
  constexpr bool PADY = CY == 2, PADZ = CZ == 2;
  __shared__ cpx<T> buf[N * P];  // [z'][kyi]
  __shared__ cpx<T> tw[N];
  __shared__ cpx<T> md[N];
  __shared__ double red[NT / 64];
  const int tid = threadIdx.x;
  const int k0 = blockIdx.x * SC, slab = blockIdx.y, ls = blockIdx.z;
  const int cx = slab / N, kxp = slab % N;
  const int kxf = CX == 2 ? 2 * kxp + cx : kxp;
  const T* kt = ktab + (size_t)fold(kxf, MX) * HY * HZ;
  cpx<T>* yo = Y + ((size_t)ls * CX * N + slab) * CY * N * N;
  for (int k = tid; k < N; k += NT) {
    tw[k] = twg[k];
    md[k] = mdg[k];
  }
  __syncthreads();
  constexpr int C1 = SC * L2, C2 = SC * L1;
  constexpr int I1 = (C1 + NT - 1) / NT;
  double esum = 0.0;
#pragma unroll 1
  for (int cy = 0; cy < CY; ++cy) {
    cpx<T>* yc = yo + (size_t)cy * N * N;
    // the lines' values, items (kyi, t): z = t + L2 k1, and their z-class sums;
    // t runs fastest across lanes, so global accesses cover runs of L2 z values
    cpx<T> vals[I1][L1], wacc[I1][L1];
#pragma unroll
    for (int ii = 0; ii < I1; ++ii) {
      const int it = tid + ii * NT;
      if (C1 % NT == 0 || it < C1) {
        const int t = it % L2, kyi = it / L2;
#pragma unroll
        for (int k1 = 0; k1 < L1; ++k1) {
          vals[ii][k1] = yc[(size_t)(k0 + kyi) * N + t + L2 * k1];
          wacc[ii][k1] = {T(0), T(0)};
        }
      }
    }
#pragma unroll
    for (int cz = 0; cz < CZ; ++cz) {
      // forward step 1 (per t) -> buf [z'][kyi]
#pragma unroll
      for (int ii = 0; ii < I1; ++ii) {
        const int it = tid + ii * NT;
        if (C1 % NT == 0 || it < C1) {
          const int t = it % L2, kyi = it / L2;
          cpx<T> v[L1];
#pragma unroll
          for (int k1 = 0; k1 < L1; ++k1) v[k1] = cz ? cmul(vals[ii][k1], md[t + L2 * k1]) : vals[ii][k1];
          Dft<L1, -1, T>::run(v);
#pragma unroll
          for (int q1 = 1; q1 < L1; ++q1) v[q1] = cmul(v[q1], tw[t * q1]);
#pragma unroll
          for (int q1 = 0; q1 < L1; ++q1) buf[(t + L2 * q1) * P + kyi] = v[q1];
        }
      }
      __syncthreads();
      // forward step 2 (per q1), kernel multiply, inverse step 2, in place
      for (int it = tid; it < C2; it += NT) {
        const int kyi = it % SC, q1 = it / SC;
        cpx<T> v[L2];
#pragma unroll
        for (int t = 0; t < L2; ++t) v[t] = buf[(t + L2 * q1) * P + kyi];
        Dft<L2, -1, T>::run(v);
        const int ky = k0 + kyi;
        const int kyf = PADY ? 2 * ky + cy : ky;
        const T* kr = kt + (size_t)fold(kyf, MY) * HZ;
        // kz = q1 + L1 q2, kernel index c + step q2 folded at q2 = L2 / 2
        constexpr int step = PADZ ? 2 * L1 : L1;
        const int c = PADZ ? 2 * q1 + cz : q1;
        const T* k_lo = kr + c;
        const T* k_hi = kr + (MZ - c);
#pragma unroll
        for (int q2 = 0; q2 < L2; ++q2) {
          const T kv = (2 * q2 < L2) ? k_lo[step * q2] : k_hi[-step * q2];
          if (EONLY) {
            esum += (double)kv * ((double)v[q2].x * (double)v[q2].x + (double)v[q2].y * (double)v[q2].y);
          } else {
            v[q2].x *= kv;
            v[q2].y *= kv;
          }
        }
        if (!EONLY) {
          Dft<L2, 1, T>::run(v);
#pragma unroll
          for (int t = 1; t < L2; ++t) v[t] = cmulc(v[t], tw[t * q1]);
#pragma unroll
          for (int t = 0; t < L2; ++t) buf[(t + L2 * q1) * P + kyi] = v[t];
        }
      }
      __syncthreads();
      if (!EONLY) {
        // inverse step 1 (per t), demodulate, sum over cz
#pragma unroll
        for (int ii = 0; ii < I1; ++ii) {
          const int it = tid + ii * NT;
          if (C1 % NT == 0 || it < C1) {
            const int t = it % L2, kyi = it / L2;
            cpx<T> v[L1];
#pragma unroll
            for (int q1 = 0; q1 < L1; ++q1) v[q1] = buf[(t + L2 * q1) * P + kyi];
            Dft<L1, 1, T>::run(v);
#pragma unroll
            for (int k1 = 0; k1 < L1; ++k1)
              wacc[ii][k1] = cadd(wacc[ii][k1], cz ? cmulc(v[k1], md[t + L2 * k1]) : v[k1]);
          }
        }
        __syncthreads();  // buf is rewritten by the next class
      }
    }
    if (!EONLY) {
#pragma unroll
      for (int ii = 0; ii < I1; ++ii) {
        const int it = tid + ii * NT;
        if (C1 % NT == 0 || it < C1) {
          const int t = it % L2, kyi = it / L2;
#pragma unroll
          for (int k1 = 0; k1 < L1; ++k1) yc[(size_t)(k0 + kyi) * N + t + L2 * k1] = wacc[ii][k1];
        }
      }
    }
  }
  if (EONLY) {
    // one partial per (slot, slab, ky-chunk), summed in a fixed order later
    double v = esum;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    if (tid == 0) {
      double sum = 0.0;
      for (int k = 0; k < NT / 64; ++k) sum += red[k];
      e_part[(size_t)(2 * (slot0 + ls)) * kparts + (size_t)slab * (N / SC) + blockIdx.x] = sum;
    }
  }
}

template <typename T, int N, int CX, int CY, int NT>
__global__ __launch_bounds__(NT) void k_pass_b3(cpx<T>* __restrict__ X, const cpx<T>* __restrict__ Y,
                                                const cpx<T>* __restrict__ twg,
                                                const cpx<T>* __restrict__ mdg) {
  using S = Split<N>;
  constexpr int L1 = S::L1, L2 = S::L2;
  constexpr int P = SC + 1;
  __shared__ cpx<T> buf[N * P];  // [y'][zi]
  __shared__ cpx<T> tw[N];
  __shared__ cpx<T> md[N];
  const int tid = threadIdx.x;
  const int z0 = blockIdx.x * SC, slab = blockIdx.y, ls = blockIdx.z;
  cpx<T>* g = X + (size_t)ls * CX * N * N * N + slab_base(slab);
  const cpx<T>* yo = Y + ((size_t)ls * CX * N + slab) * CY * N * N;
  for (int k = tid; k < N; k += NT) {
    tw[k] = twg[k];
    md[k] = mdg[k];
  }
  __syncthreads();
  constexpr int C1 = SC * L2, C2 = SC * L1;
  constexpr int I1 = (C1 + NT - 1) / NT;
  cpx<T> acc[I1][L1];
#pragma unroll
  for (int ii = 0; ii < I1; ++ii)
#pragma unroll
    for (int k1 = 0; k1 < L1; ++k1) acc[ii][k1] = {T(0), T(0)};
#pragma unroll 1
  for (int cy = 0; cy < CY; ++cy) {
    const cpx<T>* yc = yo + (size_t)cy * N * N;
    // inverse step 2, items (zi, q1): ky = q1 + L1 q2
    for (int it = tid; it < C2; it += NT) {
      const int zi = it % SC, q1 = it / SC;
      cpx<T> w[L2];
#pragma unroll
      for (int q2 = 0; q2 < L2; ++q2) w[q2] = yc[(size_t)(q1 + L1 * q2) * N + z0 + zi];
      Dft<L2, 1, T>::run(w);
#pragma unroll
      for (int t = 1; t < L2; ++t) w[t] = cmulc(w[t], tw[t * q1]);
#pragma unroll
      for (int t = 0; t < L2; ++t) buf[(t + L2 * q1) * P + zi] = w[t];
    }
    __syncthreads();
    // inverse step 1, items (zi, t): y = t + L2 k1, demodulate, sum over cy
#pragma unroll
    for (int ii = 0; ii < I1; ++ii) {
      const int it = tid + ii * NT;
      if (C1 % NT == 0 || it < C1) {
        const int zi = it % SC, t = it / SC;
        cpx<T> v[L1];
#pragma unroll
        for (int q1 = 0; q1 < L1; ++q1) v[q1] = buf[(t + L2 * q1) * P + zi];
        Dft<L1, 1, T>::run(v);
#pragma unroll
        for (int k1 = 0; k1 < L1; ++k1)
          acc[ii][k1] = cadd(acc[ii][k1], cy ? cmulc(v[k1], md[t + L2 * k1]) : v[k1]);
      }
    }
    __syncthreads();  // buf is rewritten by the next class
  }
  // write back the z-chunk of the slab (B1 has read it in an earlier launch)
#pragma unroll
  for (int ii = 0; ii < I1; ++ii) {
    const int it = tid + ii * NT;
    if (C1 % NT == 0 || it < C1) {
      const int zi = it % SC, t = it / SC;
#pragma unroll
      for (int k1 = 0; k1 < L1; ++k1) g[slab_off<N, CX>(t + L2 * k1, z0 + zi)] = acc[ii][k1];
    }
  }
}

// ---------------------------------------------------------------------------
// pass C: inverse x-transform of every slot of a pair tile for the rows
// (y, z0..z0+ZB), then FP64 pair energies h^3 sum rho V (Eq. 5) and the
// K psi sums (Eq. 3) of the tile's orbitals at the rows' points.
//
// Each thread owns L1 fixed grid points (x = t + 16 k1 of one row).  Slots
// come in tile order (row a, column pair bb) holding the pairs (a, 2bb) and
// (a, 2bb+1), so the K psi sums of the J-side orbitals sit in FP64 registers
// at compile-time indices, and the I-side orbital a has one register set that
// is added into K psi when its row is done.  The tile pairs of one launch
// share no orbital (round-robin schedule), so every update of K psi is a plain
// read-modify-write: no atomics, and results do not depend on scheduling.
// A block issues its first global loads together (the first slot's spectrum
// rows, the J-side orbital values, tables, occupations, slots); the next slot's
// spectrum rows go into the step-2 threads' registers while the current slot
// is reduced, the K psi of row a is read when the row starts, and a slot takes
// one workgroup barrier (two row buffers in LDS).
// Energies: with pair_out, one partial per (slot half, block) for the
// pair-energy matrix; otherwise one weighted partial per block
// (sum over the block's pairs of w f_i f_j e_ij, w = 2 off the diagonal).
// want_k: 0 no K psi; 1 add into K psi; 2 as 1, except that the diagonal tile
// pairs (the first round, which holds every orbital once) store their row
// sums, so K psi needs no clearing beforehand.
// ---------------------------------------------------------------------------
// Threads per owned row segment: from n = 96 on two threads share each (row, t)
// segment of L1 = n / 16 points, the first reducing ceil(L1 / 2) of them and the
// second the rest, so that a pair tile of 8 orbitals fits the registers (its K
// psi sums are (tile + 1) ceil(L1 / HP) FP64 values per thread) and K psi is
// read and written half as often as with a tile of 4.  At n = 80 the one-thread
// form with a tile of 4 is faster (two 256-thread blocks per CU against one
// 512-thread block: 4.6 against 6.2 ms of pass C for 67 orbitals).
template <typename T, int N>
constexpr int pass_c_halves() {
  return (sizeof(T) == 4 && N >= 96) ? 2 : 1;
}

// pair-tile edge of the variant with HP threads per segment: the K psi register
// budget is (tile + 1) L1 / HP FP64 values per thread.  Where two threads per
// segment are possible a schedule tile above the one-thread tile selects them,
// so a tile of 4 at n = 96, 128 runs the one-thread, 256-thread variant.
template <typename T, int N, int HP = pass_c_halves<T, N>()>
constexpr int pass_c_tile() {
  return (N / 16 <= 4 || HP == 2) ? 8 : 4;
}

// FP32 at n <= 32: ask for 3 waves per SIMD (168 registers); larger grids
// need more registers for the per-thread points
template <typename T, int N>
constexpr int pass_c_min_waves() {
  return (sizeof(T) == 4 && N <= 32) ? 3 : 1;
}

// b where the mask is all ones, a where it is zero, bit by bit.  The mask comes
// through opaque(), so the compiler cannot turn the choice between two elements
// of a register array into one load at a run-time index (a stack array).
template <typename T>
__device__ __forceinline__ T pick(unsigned m, T a, T b) {
  if constexpr (sizeof(T) == 4) {
    return __uint_as_float((__float_as_uint(a) & ~m) | (__float_as_uint(b) & m));
  } else {
    const unsigned long long m2 = ((unsigned long long)m << 32) | m;
    return __longlong_as_double((long long)(((unsigned long long)__double_as_longlong(a) & ~m2) |
                                            ((unsigned long long)__double_as_longlong(b) & m2)));
  }
}

template <typename T, int N, int NCLS, int ZB, int NT, int TM, int HP>
__global__ __launch_bounds__(NT, (pass_c_min_waves<T, N>())) void k_pass_c(const cpx<T>* __restrict__ X,
                                               const T* __restrict__ psi,
                                               const double* __restrict__ occ,
                                               const Slot* __restrict__ slots,
                                               const TilePair* __restrict__ tiles, int t0,
                                               int slot_base, double* __restrict__ kpsi,
                                               double* __restrict__ e_part, int want_k,
                                               int want_e, int pair_out,
                                               const cpx<T>* __restrict__ twg,
                                               const cpx<T>* __restrict__ mdg, int kparts,
                                               int swap_yz, const SysTab systab) {
  using S = SplitAC<N>;
  constexpr int L1 = S::L1, L2 = S::L2;
  constexpr int P = N + 1;
  constexpr int NL = NCLS * ZB;
  constexpr int HB = (TM + 1) / 2;            // column pairs per tile row
  constexpr int MAXS = TM * HB;               // slots per tile pair
  constexpr int NW = NT / 64;
  constexpr int C2 = NL * L1;                 // step-2 items (line, q1), one per thread
  constexpr int LP = (L1 + HP - 1) / HP;      // points per thread (the last half may own one less)
  constexpr bool EVEN = L1 % HP == 0;
  static_assert(ZB * L2 * HP == NT, "HP point-owner threads per (row, t)");
  static_assert(ZB == XZ, "a block's rows are one z-block of the spectrum layout");
  static_assert(C2 <= NT, "one step-2 item per thread");
  // Rows after the inverse step 2, two buffers: slot k's step 1 reads buffer
  // k & 1 while the step-2 threads fill the other one for slot k + 1, and the
  // one barrier per slot orders the step 1 of slot k - 1 before that fill.
  __shared__ cpx<T> xo[2][NL * P];
  __shared__ cpx<T> tw[N];
  __shared__ cpx<T> md[N];
  __shared__ Slot st[MAXS];
  __shared__ int smap[TM][HB];
  __shared__ double fI[TM], fJ[TM];
  __shared__ double ered[MAXS][2][NW];
  __shared__ double etot[NW];
  // J-side orbital values at the owned points (slot [b][k1 NT + tid], read back
  // by the same thread only)
  __shared__ T pJs[TM][LP * NT];

  const int tid = threadIdx.x;
  const int y = blockIdx.x / (N / ZB);
  const int z0 = (blockIdx.x % (N / ZB)) * ZB;
  const TilePair tp = tiles[t0 + blockIdx.y];
  // this tile pair's system (merged batch schedules) or the launch's own buffers
  const double* __restrict__ occ_s = systab.n ? systab.occ[tp.sys] : occ;
  double* __restrict__ kpsi_s = systab.n ? systab.kpsi[tp.sys] : kpsi;
  const size_t M3 = (size_t)N * N * N;
  // owner of (row zi_own, t_own), points x = t_own + 16 k1 for k1 in [k0, k0 + LP)
  // clipped to L1 (a half's threads are whole wavefronts, so the clipped point is
  // skipped without divergence; it is read at the last valid point and
  // contributes zeros)
  // (threads of one half are contiguous, so K psi updates stay 128-byte runs)
  const int h_own = tid / (ZB * L2), rt = tid % (ZB * L2);
  const int t_own = rt % L2, zi_own = rt / L2;
  const int k0 = h_own * LP;
  auto kok = [&](int k1) { return EVEN || k0 + k1 < L1; };
  auto kcl = [&](int k1) { return EVEN ? k0 + k1 : min(k0 + k1, L1 - 1); };
  const unsigned hmask = opaque(h_own ? ~0u : 0u);  // second half of a segment
  // offset of the owned row (swap_yz: spectrum (y, z) = grid (z, y))
  const size_t row = swap_yz ? ((size_t)y * N + z0 + zi_own) * N : ((size_t)(z0 + zi_own) * N + y) * N;
  const int ns = tp.s1 - tp.s0;

  // spectrum rows of a slot: the block's rows are one contiguous z-block chunk
  // of the slot, value (cx, kx, zi) at (cx N + kx) ZB + zi.  Step-2 item (line,
  // q1) = (tid mod NL, tid / NL), line = cx ZB + zi, takes kx = q1 + L1 q2: its
  // thread loads them straight into registers, one slot ahead (each load of a
  // wavefront reads whole 128-byte runs of 16 zi at consecutive kx)
  const bool s2 = tid < C2;
  const int line2 = tid % NL, q12 = tid / NL;
  cpx<T> nw[L2];
  auto fetch = [&](int k) {
    const cpx<T>* Xs = X + (size_t)(tp.s0 + k - slot_base) * NCLS * M3 + (size_t)blockIdx.x * NL * N +
                       (size_t)((line2 / ZB) * N + q12) * ZB + line2 % ZB;
    if (s2) {
#pragma unroll
      for (int q2 = 0; q2 < L2; ++q2) nw[q2] = load_stream(Xs + (size_t)L1 * q2 * ZB);
    }
  };
  // The block's first global loads go out together, so that their latencies
  // overlap: the first slot's spectrum rows, the orbital values at the owned
  // points (every J-side orbital of the tile once, parked in LDS below; the
  // I-side orbital once per row), then the tables, occupations and slots.
  if (ns > 0) fetch(0);
  T pjr[TM][LP];
#pragma unroll
  for (int b = 0; b < TM; ++b) {
    const T* po = psi + (size_t)(tp.J0 + b) * M3 + row;
#pragma unroll
    for (int k1 = 0; k1 < LP; ++k1)
      pjr[b][k1] = (b < tp.nJ && kok(k1)) ? po[t_own + L2 * kcl(k1)] : T(0);
  }
  for (int k = tid; k < N; k += NT) {
    tw[k] = twg[k];
    if (NCLS == 2) md[k] = mdg[k];
  }
  for (int k = tid; k < TM * HB; k += NT) smap[k / HB][k % HB] = -1;
  for (int k = tid; k < TM; k += NT) {
    fI[k] = k < tp.nI ? occ_s[tp.I0 + k] : 0.0;
    fJ[k] = k < tp.nJ ? occ_s[tp.J0 + k] : 0.0;
  }
  __syncthreads();
  for (int k = tid; k < ns; k += NT) {
    const Slot sl = slots[tp.s0 + k];
    st[k] = sl;
    const int a = (sl.ia >= 0 ? sl.ia : sl.ib) - tp.I0;
    const int bb = ((sl.ia >= 0 ? sl.ja : sl.jb) - tp.J0) >> 1;
    smap[a][bb] = k;
  }
  double accJ[TM][LP];
#pragma unroll
  for (int b = 0; b < TM; ++b)
#pragma unroll
    for (int k1 = 0; k1 < LP; ++k1) accJ[b][k1] = 0.0;
  double ew = 0.0;

  // the J-side orbital values into LDS (slot [b][k1 NT + tid], read back by the
  // same thread only)
#pragma unroll
  for (int b = 0; b < TM; ++b)
#pragma unroll
    for (int k1 = 0; k1 < LP; ++k1) pJs[b][k1 * NT + tid] = pjr[b][k1];
  __syncthreads();

  int k = 0;  // running slot index (uniform)
#pragma unroll 1
  for (int a = 0; a < tp.nI; ++a) {
    double accI[LP];
    T pI[LP];
    {
      const T* po = psi + (size_t)(tp.I0 + a) * M3 + row;
#pragma unroll
      for (int k1 = 0; k1 < LP; ++k1) {
        accI[k1] = 0.0;
        pI[k1] = kok(k1) ? po[t_own + L2 * kcl(k1)] : T(0);
      }
    }
    // K psi of row a at the owned points, read here so that the read overlaps
    // the row's slots (no other block of the launch touches these points, and
    // this block writes them only at the row's end)
    double kold[LP];
    const bool rmw = want_k && !(want_k == 2 && tp.diag);
    if (rmw) {
      const double* ko = kpsi_s + (size_t)(tp.I0 + a) * M3 + row;
#pragma unroll
      for (int k1 = 0; k1 < LP; ++k1) kold[k1] = kok(k1) ? ko[t_own + L2 * (k0 + k1)] : 0.0;
    }
    const double fa = fI[a];
#pragma unroll
    for (int bb = 0; bb < HB; ++bb) {
      if (smap[a][bb] < 0) continue;
      const Slot sl = st[k];
      cpx<T>* xb = xo[k & 1];
      if (s2) {
        // inverse step 2 of item (line2, q12): IDFT_L2 over q2, conjugate twiddle
        cpx<T> w[L2];
#pragma unroll
        for (int q2 = 0; q2 < L2; ++q2) w[q2] = nw[q2];
        if (k + 1 < ns) fetch(k + 1);  // spectrum rows of the next slot
        Dft<L2, 1, T>::run(w);
#pragma unroll
        for (int t = 1; t < L2; ++t) w[t] = cmulc(w[t], tw[t * q12]);
#pragma unroll
        for (int t = 0; t < L2; ++t) xb[line2 * P + t + L2 * q12] = w[t];
      }
      __syncthreads();
      // inverse step 1 (per t) of both x classes, demodulated: V_a + i V_b at the
      // owned points (with two owners per segment both transform, each keeps half)
      cpx<T> V[LP];
      {
        cpx<T> v[L1];
#pragma unroll
        for (int q1 = 0; q1 < L1; ++q1) v[q1] = xb[zi_own * P + t_own + L2 * q1];
        Dft<L1, 1, T>::run(v);
#pragma unroll
        for (int k1 = 0; k1 < LP; ++k1)
          V[k1] = HP == 1 ? v[k1]
                          : cpx<T>{pick(hmask, v[k1].x, v[min(LP % L1 + k1, L1 - 1)].x),
                                   pick(hmask, v[k1].y, v[min(LP % L1 + k1, L1 - 1)].y)};
        if (NCLS == 2) {
#pragma unroll
          for (int q1 = 0; q1 < L1; ++q1) v[q1] = xb[(ZB + zi_own) * P + t_own + L2 * q1];
          Dft<L1, 1, T>::run(v);
#pragma unroll
          for (int k1 = 0; k1 < LP; ++k1) {
            const cpx<T> w = HP == 1 ? v[k1]
                                     : cpx<T>{pick(hmask, v[k1].x, v[min(LP % L1 + k1, L1 - 1)].x),
                                              pick(hmask, v[k1].y, v[min(LP % L1 + k1, L1 - 1)].y)};
            V[k1] = cadd(V[k1], cmulc(w, md[t_own + L2 * kcl(k1)]));
          }
        }
      }
      // the two halves: J columns 2bb and 2bb + 1 (compile-time register indices)
      double eh[2] = {0.0, 0.0};
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int b = 2 * bb + h;
        if (b >= TM) continue;
        const bool valid = h ? sl.ib >= 0 : sl.ia >= 0;
        if (!valid) continue;
        const bool self = tp.diag && b == a;  // the (a, a) pair updates (K psi)_a once
        const double fb = fJ[b];
        double e = 0.0;
#pragma unroll
        for (int k1 = 0; k1 < LP; ++k1) {
          const T pa = pI[k1], pb = pJs[b][k1 * NT + tid];
          const double Vv = (double)(h ? V[k1].y : V[k1].x);
          e += (double)(pa * pb) * Vv;
          if (want_k) {
            accI[k1] += fb * Vv * (double)pb;
            if (!self) accJ[b][k1] += fa * Vv * (double)pa;
          }
        }
        eh[h] = e;
        if (!pair_out) ew += (self ? 1.0 : 2.0) * fa * fb * e;
      }
      if (want_e && pair_out) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
          eh[0] += __shfl_xor(eh[0], off);
          eh[1] += __shfl_xor(eh[1], off);
        }
        if ((tid & 63) == 0) {
          ered[k][0][tid >> 6] = eh[0];
          ered[k][1][tid >> 6] = eh[1];
        }
      }
      ++k;
    }
    if (want_k) {
      double* ko = kpsi_s + (size_t)(tp.I0 + a) * M3 + row;
      if (tp.diag) {
        // on a diagonal tile orbital a's column sums (from rows a' < a) are
        // complete here: one write carries both
#pragma unroll
        for (int b = 0; b < TM; ++b)
          if (b == a)
#pragma unroll
            for (int k1 = 0; k1 < LP; ++k1) accI[k1] += accJ[b][k1];
      }
      if (!rmw) {  // first write of this orbital row in the evaluation
#pragma unroll
        for (int k1 = 0; k1 < LP; ++k1)
          if (kok(k1)) ko[t_own + L2 * (k0 + k1)] = accI[k1];
      } else {
#pragma unroll
        for (int k1 = 0; k1 < LP; ++k1)
          if (kok(k1)) ko[t_own + L2 * (k0 + k1)] = kold[k1] + accI[k1];
      }
    }
  }
  if (want_k && !tp.diag) {
    // J-side sums of an off-diagonal tile
#pragma unroll
    for (int b = 0; b < TM; ++b) {
      if (b >= tp.nJ) continue;
      double* ko = kpsi_s + (size_t)(tp.J0 + b) * M3 + row;
#pragma unroll
      for (int k1 = 0; k1 < LP; ++k1)
        if (kok(k1)) ko[t_own + L2 * (k0 + k1)] += accJ[b][k1];
    }
  }
  if (!want_e) return;
  if (pair_out) {
    __syncthreads();
    // one partial per (slot half, row block), summed in a fixed order later
    for (int q = tid; q < 2 * ns; q += NT) {
      const int kk = q >> 1, half = q & 1;
      double sum = 0.0;
      if (half ? st[kk].ib >= 0 : st[kk].ia >= 0) {
#pragma unroll
        for (int w2 = 0; w2 < NW; ++w2) sum += ered[kk][half][w2];
      }
      e_part[(size_t)(2 * (tp.s0 + kk) + half) * kparts + blockIdx.x] = sum;
    }
  } else {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) ew += __shfl_xor(ew, off);
    if ((tid & 63) == 0) etot[tid >> 6] = ew;
    __syncthreads();
    if (tid == 0) {
      double sum = 0.0;
#pragma unroll
      for (int w2 = 0; w2 < NW; ++w2) sum += etot[w2];
      e_part[(size_t)tp.eidx * kparts + blockIdx.x] = sum;
    }
  }
}

// ---------------------------------------------------------------------------
// pass C for complex orbitals: one pair per slot.  Slot (a, b) of a tile pair
// holds (I0 + a, J0 + b); its inverse transform is the complex V_ij of
// rho_ij = conj(psi_j) psi_i (Eq. 2).  (K psi)_i gains f_j V_ij psi_j and
// (K psi)_j gains f_i conj(V_ij) psi_i, since V_ji = conj(V_ij) for a real, even
// kernel; e_ij = h^3 sum Re(conj(rho_ij) V_ij) is real and symmetric.  K psi
// is complex FP64; the energy partials keep the two-half layout of the packed
// pass with the b half zero.
// ---------------------------------------------------------------------------
template <typename T, int N>
constexpr int pass_c_tile_cplx() {
  // accumulators (tile + 1) * L1 complex FP64 per thread, and the tile's J-side
  // orbitals in LDS: tile * n * 16 * 2 sizeof(T) bytes beside the two row buffers.
  // FP32 at n = 64: a tile of 8 fits one block per CU (256 registers, 100 KB of
  // LDS) and measured 1.16 ms of pass C per evaluation of 32 orbitals against
  // 0.90 ms with a tile of 4 (two blocks per CU, 80 % more K psi updates)
  if (sizeof(T) == 8) return N <= 32 ? 8 : (N <= 64 ? 4 : 2);
  return N <= 48 ? 8 : 4;
}

// FP32 at n = 16: 3 waves per SIMD; from n = 32 on the complex accumulators
// need the registers of one wave
template <typename T, int N>
constexpr int pass_c_cplx_min_waves() {
  return (sizeof(T) == 4 && N <= 16) ? 3 : 1;
}

template <typename T, int N, int NCLS, int ZB, int NT, int TM>
__global__ __launch_bounds__(NT, (pass_c_cplx_min_waves<T, N>())) void k_pass_c_cplx(
    const cpx<T>* __restrict__ X, const cpx<T>* __restrict__ psi, const double* __restrict__ occ,
    const Slot* __restrict__ slots, const TilePair* __restrict__ tiles, int t0, int slot_base,
    cpx<double>* __restrict__ kpsi, double* __restrict__ e_part, int want_k, int want_e,
    int pair_out, const cpx<T>* __restrict__ twg, const cpx<T>* __restrict__ mdg, int kparts,
    int swap_yz, const SysTab systab) {
  using S = SplitAC<N>;
  constexpr int L1 = S::L1, L2 = S::L2;
  constexpr int P = N + 1;
  constexpr int NL = NCLS * ZB;
  constexpr int MAXS = TM * TM;               // slots per tile pair
  constexpr int NW = NT / 64;
  constexpr int PF = (NL * N + NT - 1) / NT;  // prefetched spectrum values per thread
  static_assert(ZB * L2 == NT, "one point-owner item per thread");
  static_assert(ZB == XZ, "a block's rows are one z-block of the spectrum layout");
  __shared__ cpx<T> xs[NL * P];
  __shared__ cpx<T> xo[NL * P];
  __shared__ cpx<T> tw[N];
  __shared__ cpx<T> md[N];
  __shared__ int smap[TM][TM];
  __shared__ double fI[TM], fJ[TM];
  __shared__ double ered[MAXS][NW];
  __shared__ double etot[NW];
  __shared__ cpx<T> pJs[TM][L1 * NT];

  const int tid = threadIdx.x;
  const int y = blockIdx.x / (N / ZB);
  const int z0 = (blockIdx.x % (N / ZB)) * ZB;
  const TilePair tp = tiles[t0 + blockIdx.y];
  // this tile pair's system (merged batch schedules) or the launch's own buffers
  const double* __restrict__ occ_s = systab.n ? systab.occ[tp.sys] : occ;
  cpx<double>* __restrict__ kpsi_s = systab.n ? reinterpret_cast<cpx<double>*>(systab.kpsi[tp.sys]) : kpsi;
  const size_t M3 = (size_t)N * N * N;
  const int t_own = tid % L2, zi_own = tid / L2;
  // offset of the owned row (swap_yz: spectrum (y, z) = grid (z, y))
  const size_t row = swap_yz ? ((size_t)y * N + z0 + zi_own) * N : ((size_t)(z0 + zi_own) * N + y) * N;
  const int ns = tp.s1 - tp.s0;

  cpx<T> pf[PF];
  auto fetch = [&](int k) {
    const cpx<T>* Xs = X + (size_t)(tp.s0 + k - slot_base) * NCLS * M3 + (size_t)blockIdx.x * NL * N;
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      int p = tid + q * NT;
      if ((NL * N) % NT == 0 || p < NL * N) pf[q] = load_stream(Xs + p);
    }
  };
  // the block's first global loads go out together (as in the real pass C):
  // the first slot's spectrum rows, the tile's J-side orbital values, then the
  // tables, occupations and slots
  if (ns > 0) fetch(0);
  cpx<T> pjr[TM][L1];
#pragma unroll
  for (int b = 0; b < TM; ++b) {
    const cpx<T>* po = psi + (size_t)(tp.J0 + b) * M3 + row;
#pragma unroll
    for (int k1 = 0; k1 < L1; ++k1)
      pjr[b][k1] = b < tp.nJ ? po[t_own + L2 * k1] : cpx<T>{T(0), T(0)};
  }
  for (int k = tid; k < N; k += NT) {
    tw[k] = twg[k];
    if (NCLS == 2) md[k] = mdg[k];
  }
  for (int k = tid; k < TM * TM; k += NT) smap[k / TM][k % TM] = -1;
  for (int k = tid; k < TM; k += NT) {
    fI[k] = k < tp.nI ? occ_s[tp.I0 + k] : 0.0;
    fJ[k] = k < tp.nJ ? occ_s[tp.J0 + k] : 0.0;
  }
  __syncthreads();
  for (int k = tid; k < ns; k += NT) {
    const Slot sl = slots[tp.s0 + k];
    smap[sl.ia - tp.I0][sl.ja - tp.J0] = k;
  }
  double accJ[TM][L1][2];
#pragma unroll
  for (int b = 0; b < TM; ++b)
#pragma unroll
    for (int k1 = 0; k1 < L1; ++k1) accJ[b][k1][0] = accJ[b][k1][1] = 0.0;
  double ew = 0.0;

  // the J-side orbital values into LDS (slot [b][k1 NT + tid], read back by the
  // same thread only)
#pragma unroll
  for (int b = 0; b < TM; ++b)
#pragma unroll
    for (int k1 = 0; k1 < L1; ++k1) pJs[b][k1 * NT + tid] = pjr[b][k1];
  __syncthreads();

  int k = 0;  // running slot index (uniform)
#pragma unroll 1
  for (int a = 0; a < tp.nI; ++a) {
    double accI[L1][2];
    cpx<T> pI[L1];
    {
      const cpx<T>* po = psi + (size_t)(tp.I0 + a) * M3 + row;
#pragma unroll
      for (int k1 = 0; k1 < L1; ++k1) {
        accI[k1][0] = accI[k1][1] = 0.0;
        pI[k1] = po[t_own + L2 * k1];
      }
    }
    // K psi of row a, read here so that the read overlaps the row's slots (no
    // other block of the launch touches these points; this block writes them
    // at the row's end); zero where the row's first write of the evaluation is
    const bool first = want_k == 2 && tp.diag;
    cpx<double> kold[L1];
    if (want_k) {
      const cpx<double>* ko = kpsi_s + (size_t)(tp.I0 + a) * M3 + row;
#pragma unroll
      for (int k1 = 0; k1 < L1; ++k1) kold[k1] = first ? cpx<double>{0.0, 0.0} : ko[t_own + L2 * k1];
    }
    const double fa = fI[a];
#pragma unroll
    for (int b = 0; b < TM; ++b) {
      if (smap[a][b] < 0) continue;
#pragma unroll
      for (int q = 0; q < PF; ++q) {
        int p = tid + q * NT;
        if ((NL * N) % NT == 0 || p < NL * N) {
          int zi = p % ZB, kx = (p / ZB) % N, cx = p / (ZB * N);
          xs[(cx * ZB + zi) * P + kx] = pf[q];
        }
      }
      if (k + 1 < ns) fetch(k + 1);  // spectrum rows of the next slot
      __syncthreads();
      // inverse step 2 (per q1): IDFT_L2 over q2, conjugate twiddle; xs -> xo
      constexpr int C2 = NL * L1;
#pragma unroll
      for (int it = tid; it < C2; it += NT) {
        int line = it % NL, q1 = it / NL;
        cpx<T> w[L2];
#pragma unroll
        for (int q2 = 0; q2 < L2; ++q2) w[q2] = xs[line * P + q1 + L1 * q2];
        Dft<L2, 1, T>::run(w);
#pragma unroll
        for (int t = 1; t < L2; ++t) w[t] = cmulc(w[t], tw[t * q1]);
#pragma unroll
        for (int t = 0; t < L2; ++t) xo[line * P + t + L2 * q1] = w[t];
      }
      __syncthreads();
      // inverse step 1 (per t) of both x classes, demodulated: V_ij
      cpx<T> V[L1];
      {
        cpx<T> v[L1];
#pragma unroll
        for (int q1 = 0; q1 < L1; ++q1) v[q1] = xo[zi_own * P + t_own + L2 * q1];
        Dft<L1, 1, T>::run(v);
#pragma unroll
        for (int k1 = 0; k1 < L1; ++k1) V[k1] = v[k1];
        if (NCLS == 2) {
#pragma unroll
          for (int q1 = 0; q1 < L1; ++q1) v[q1] = xo[(ZB + zi_own) * P + t_own + L2 * q1];
          Dft<L1, 1, T>::run(v);
#pragma unroll
          for (int k1 = 0; k1 < L1; ++k1) V[k1] = cadd(V[k1], cmulc(v[k1], md[t_own + L2 * k1]));
        }
      }
      const bool self = tp.diag && b == a;  // the (a, a) pair updates (K psi)_a once
      const double fb = fJ[b];
      double e = 0.0;
#pragma unroll
      for (int k1 = 0; k1 < L1; ++k1) {
        const cpx<T> pa = pI[k1], pb = pJs[b][k1 * NT + tid];
        const cpx<T> rho = cmulc(pa, pb);
        const double vr = (double)V[k1].x, vi = (double)V[k1].y;
        e += (double)rho.x * vr + (double)rho.y * vi;
        if (want_k) {
          const double ar = pa.x, ai = pa.y, br = pb.x, bi = pb.y;
          accI[k1][0] += fb * (vr * br - vi * bi);  // V psi_j
          accI[k1][1] += fb * (vr * bi + vi * br);
          if (!self) {
            accJ[b][k1][0] += fa * (vr * ar + vi * ai);  // conj(V) psi_i
            accJ[b][k1][1] += fa * (vr * ai - vi * ar);
          }
        }
      }
      if (want_e && pair_out) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off);
        if ((tid & 63) == 0) ered[k][tid >> 6] = e;
      }
      if (!pair_out) ew += (self ? 1.0 : 2.0) * fa * fb * e;
      ++k;
    }
    if (want_k) {
      cpx<double>* ko = kpsi_s + (size_t)(tp.I0 + a) * M3 + row;
      if (tp.diag) {
        // on a diagonal tile orbital a's column sums (from rows a' < a) are
        // complete here: one write carries both
#pragma unroll
        for (int b = 0; b < TM; ++b)
          if (b == a)
#pragma unroll
            for (int k1 = 0; k1 < L1; ++k1) {
              accI[k1][0] += accJ[b][k1][0];
              accI[k1][1] += accJ[b][k1][1];
            }
      }
#pragma unroll
      for (int k1 = 0; k1 < L1; ++k1) {
        cpx<double> v = kold[k1];
        v.x += accI[k1][0];
        v.y += accI[k1][1];
        ko[t_own + L2 * k1] = v;
      }
    }
  }
  if (want_k && !tp.diag) {
    // J-side sums of an off-diagonal tile
#pragma unroll
    for (int b = 0; b < TM; ++b) {
      if (b >= tp.nJ) continue;
      cpx<double>* ko = kpsi_s + (size_t)(tp.J0 + b) * M3 + row;
#pragma unroll
      for (int k1 = 0; k1 < L1; ++k1) {
        cpx<double> v = ko[t_own + L2 * k1];
        v.x += accJ[b][k1][0];
        v.y += accJ[b][k1][1];
        ko[t_own + L2 * k1] = v;
      }
    }
  }
  if (!want_e) return;
  if (pair_out) {
    __syncthreads();
    // one partial per (slot half, row block); the b half of a slot is empty
    for (int q = tid; q < 2 * ns; q += NT) {
      const int kk = q >> 1, half = q & 1;
      double sum = 0.0;
      if (!half) {
#pragma unroll
        for (int w2 = 0; w2 < NW; ++w2) sum += ered[kk][w2];
      }
      e_part[(size_t)(2 * (tp.s0 + kk) + half) * kparts + blockIdx.x] = sum;
    }
  } else {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) ew += __shfl_xor(ew, off);
    if ((tid & 63) == 0) etot[tid >> 6] = ew;
    __syncthreads();
    if (tid == 0) {
      double sum = 0.0;
#pragma unroll
      for (int w2 = 0; w2 < NW; ++w2) sum += etot[w2];
      e_part[(size_t)tp.eidx * kparts + blockIdx.x] = sum;
    }
  }
}

// ---------------------------------------------------------------------------
// pair-energy partials: pass C writes one per (slot half, row block of 16
// z-rows: n^2/16 of them), the energy-only pass B one per (slot, slab: at most
// 2n); k_slot_reduce sums each slot half's partials in a fixed order, so the
// energies do not depend on block scheduling.
// ---------------------------------------------------------------------------
int energy_parts(int n) { return std::max(n * n / 8, 2 * n); }

__global__ __launch_bounds__(256) void k_slot_reduce(const double* __restrict__ parts, int kparts,
                                                     int count, int nhalves,
                                                     double* __restrict__ e_slot) {
  const int lane = threadIdx.x & 63;
  const int h = blockIdx.x * 4 + (threadIdx.x >> 6);  // one wave per slot half
  if (h >= nhalves) return;
  const double* p = parts + (size_t)h * kparts;
  double sum = 0.0;
  for (int k = lane; k < count; k += 64) sum += p[k];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
  if (lane == 0) e_slot[h] = sum;
}

hipError_t launch_slot_reduce(const double* parts, int kparts, int count, int nhalves,
                              double* e_slot, hipStream_t s) {
  if (nhalves <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_slot_reduce, dim3((nhalves + 3) / 4), dim3(256), 0, s, parts, kparts, count,
                     nhalves, e_slot);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// finalize: E_x = -1/2 sum_ij f_i f_j e_ij in a fixed order, pair-energy matrix
// ---------------------------------------------------------------------------
// sum_mode 0: per-pair energies e_slot[2s + h] (weights f_i f_j, 2 off the
// diagonal; pair-energy matrix written if requested); 1: Parseval sums of
// weighted slots e_slot[2s]; 2: nvals weighted partial sums e_slot[0..nvals).
__global__ __launch_bounds__(1024) void k_finalize(const Slot* __restrict__ slots, int nvals,
                                                   const double* __restrict__ occ,
                                                   const double* __restrict__ e_slot, int n_orb,
                                                   double h3, int sum_mode,
                                                   double* __restrict__ ex_out,
                                                   double* __restrict__ pair_e) {
  __shared__ double red[16];
  const int tid = threadIdx.x;
  double sum = 0.0;
  for (int s = tid; s < nvals; s += 1024) {
    if (sum_mode == 2) {
      sum += h3 * e_slot[s];
      continue;
    }
    if (sum_mode == 1) {
      sum += h3 * e_slot[2 * s];
      continue;
    }
    const Slot sl = slots[s];
    for (int half = 0; half < 2; ++half) {
      int i = half ? sl.ib : sl.ia, j = half ? sl.jb : sl.ja;
      if (i < 0) continue;
      double e = h3 * e_slot[2 * s + half];
      sum += occ[i] * occ[j] * (i == j ? 1.0 : 2.0) * e;
      if (pair_e) {
        pair_e[(size_t)i * n_orb + j] = e;
        pair_e[(size_t)j * n_orb + i] = e;
      }
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
  if ((tid & 63) == 0) red[tid >> 6] = sum;
  __syncthreads();
  if (tid == 0 && ex_out) {
    double s = 0.0;
    for (int w = 0; w < 16; ++w) s += red[w];
    *ex_out = -0.5 * s;
  }
}

// E_x of every member of a merged class (blockIdx.x = member): the sum of
// k_finalize's mode 2 over the member's rows, in the same order
__global__ __launch_bounds__(1024) void k_finalize_members(const MemberTab m,
                                                           const double* __restrict__ e_slot, double h3) {
  __shared__ double red[16];
  const int tid = threadIdx.x, k = blockIdx.x;
  const int r0 = m.row0[k], nvals = m.row0[k + 1] - r0;
  double sum = 0.0;
  for (int s = tid; s < nvals; s += 1024) sum += h3 * e_slot[r0 + s];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
  if ((tid & 63) == 0) red[tid >> 6] = sum;
  __syncthreads();
  if (tid == 0 && m.ex_out[k]) {
    double s = 0.0;
    for (int w = 0; w < 16; ++w) s += red[w];
    *m.ex_out[k] = -0.5 * s;
  }
}

hipError_t launch_finalize_members(const MemberTab& m, const double* e_slot, double h3, hipStream_t s) {
  if (m.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_finalize_members, dim3(m.n), dim3(1024), 0, s, m, e_slot, h3);
  return hipGetLastError();
}

hipError_t launch_finalize(const Slot* slots, int nvals, const double* occ, const double* e_slot,
                           int n_orb, double h3, int sum_mode, double* ex_out, double* pair_e,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, s, slots, nvals, occ, e_slot, n_orb, h3,
                     sum_mode, ex_out, pair_e);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gradient of E_x (reverse mode).  E_x = -1/2 sum_ij f_i f_j e_ij with
// e_ij = h^3 <rho_ij, V_ij> is a quartic in psi whose derivative with respect
// to psi_k at a grid point is -2 f_k h^3 (K psi)_k (Eq. 3: K psi = -D_X psi),
// and whose derivative with respect to f_k is -sum_j f_j e_kj.  Both are
// scaled by the upstream derivative gbar (a device scalar, so the backward of
// a captured or asynchronous evaluation needs no host sync).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_grad_psi(double* __restrict__ g, size_t per_orb,
                                                  const double* __restrict__ occ,
                                                  const double* __restrict__ gbar, double h3) {
  const int k = blockIdx.y;
  const double c = -2.0 * h3 * occ[k] * gbar[0];
  double2* row = reinterpret_cast<double2*>(g + (size_t)k * per_orb);
  const size_t n2 = per_orb / 2;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n2; i += (size_t)gridDim.x * 256) {
    double2 v = row[i];
    v.x *= c;
    v.y *= c;
    row[i] = v;
  }
}

__global__ __launch_bounds__(256) void k_grad_occ(const double* __restrict__ pair_e, int n_orb,
                                                  const double* __restrict__ occ,
                                                  const double* __restrict__ gbar,
                                                  double* __restrict__ g_occ) {
  __shared__ double red[4];
  const int k = blockIdx.x, tid = threadIdx.x;
  double s = 0.0;
  for (int j = tid; j < n_orb; j += 256) s += occ[j] * pair_e[(size_t)k * n_orb + j];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  if (tid == 0) g_occ[k] = -gbar[0] * (((red[0] + red[1]) + red[2]) + red[3]);
}

hipError_t launch_gradient(double* grad_psi, size_t per_orb, int n_orb, const double* occ,
                           const double* gbar, double h3, const double* pair_e, double* grad_occ,
                           hipStream_t s) {
  if (per_orb % 2 != 0) return hipErrorInvalidValue;  // rows are whole double2 runs
  const size_t n2 = per_orb / 2;
  const unsigned bx = (unsigned)std::min<size_t>((n2 + 255) / 256, 1024);
  hipLaunchKernelGGL(k_grad_psi, dim3(bx, n_orb), dim3(256), 0, s, grad_psi, per_orb, occ, gbar, h3);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !grad_occ) return e;
  hipLaunchKernelGGL(k_grad_occ, dim3(n_orb), dim3(256), 0, s, pair_e, n_orb, occ, gbar, grad_occ);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// host dispatch over the supported grid sizes
// ---------------------------------------------------------------------------
template <typename F>
static hipError_t dispatch_n(int n, F&& f) {
  switch (n) {
    case 16: return f.template operator()<16>();
    case 32: return f.template operator()<32>();
    case 48: return f.template operator()<48>();
    case 64: return f.template operator()<64>();
    case 80: return f.template operator()<80>();
    case 96: return f.template operator()<96>();
    case 112: return f.template operator()<112>();
    case 128: return f.template operator()<128>();
    default: return hipErrorInvalidValue;
  }
}

bool fused_supported(int precision, int n) {
  if (n % 16 != 0 || n < 16 || n > 128) return false;
  if (precision == EXX_PREC_FP64_FUSED) return n <= 96;
  return true;
}

template <typename T, int N, bool SY>
constexpr int pass_b_threads() {
  // a few items per thread; where LDS allows one block per CU (the shared-y
  // variant from N = 80 on, the single-buffer one from N = 96 on) the block
  // takes the whole CU (16 waves) to keep per-thread arrays small; the shared-y
  // block at N = 96 has 768 threads (one item each, 168 registers)
  if (N <= 32) return 128;
  if (N <= 64) return 256;
  if (sizeof(T) == 8) return 512;
  if (SY && N == 96) return 768;
  return (SY || N > 80) ? 1024 : 512;
}

template <typename T>
hipError_t launch_pass_a(const Launch& L, const T* psi, void* X, const Slot* slots, int slot0,
                         int nslots, const double* occ, bool weighted, const Tables& tb) {
  if (nslots <= 0) return hipSuccess;
  return dispatch_n(L.n, [&]<int N>() -> hipError_t {
    constexpr int ZB = XZ;
    constexpr int NT = 256;
    constexpr int SPB = pass_a_slots(N);
    dim3 grid = pass_a_xcd_order(N) ? dim3(N * (N / ZB) * ((nslots + SPB - 1) / SPB))
                            : dim3(N * (N / ZB), (nslots + SPB - 1) / SPB);
    auto* Xc = static_cast<cpx<T>*>(X);
    auto* tw = static_cast<const cpx<T>*>(tb.tw);
    auto* md = static_cast<const cpx<T>*>(tb.md);
    auto go = [&]<int NCLS, bool W, bool CPLX>() {
      hipLaunchKernelGGL((k_pass_a<T, N, NCLS, ZB, NT, SPB, W, CPLX>), grid, dim3(NT), 0, L.stream,
                         psi, Xc, slots, slot0, nslots, occ, tw, md, L.swap_yz);
    };
    auto by_w = [&]<int NCLS, bool CPLX>() {
      if (weighted)
        go.template operator()<NCLS, true, CPLX>();
      else
        go.template operator()<NCLS, false, CPLX>();
    };
    auto by_cls = [&]<bool CPLX>() {
      if (L.ncls == 2)
        by_w.template operator()<2, CPLX>();
      else
        by_w.template operator()<1, CPLX>();
    };
    if (L.cplx)
      by_cls.template operator()<true>();
    else
      by_cls.template operator()<false>();
    return hipGetLastError();
  });
}

template <typename T, int N, int CY, int CZ>
constexpr bool pass_b_share_y() {
  // sharing the y-transforms needs two z classes, two slab buffers in LDS
  // (2 N (N+1) complex values) and keeps two more slab-sized register arrays
  // live; used where two buffers fit (measured at n = 80: pass B 6.98 -> 4.09 ms
  // free, 2.44 -> 1.16 ms surface; n = 96 surface 4.34 -> 1.79, free 9.09 -> 6.67
  // against the split form)
  if (CZ != 2) return false;
  if (sizeof(T) == 8) return N <= 32;
  return N <= 96;
}

template <typename T, int N, int CX, int CY, int CZ, int NT, bool SY>
hipError_t launch_pass_b_cls(const Launch& L, cpx<T>* Xc, int nslots, bool energy_only,
                             double* e_slot, int slot0, const Tables& tb) {
  auto* kt = static_cast<const T*>(tb.ktab);
  auto* tw = static_cast<const cpx<T>*>(tb.tw);
  auto* md = static_cast<const cpx<T>*>(tb.md);
  dim3 grid(CX * N, nslots);
  if (energy_only)
    hipLaunchKernelGGL((k_pass_b<T, N, CX, CY, CZ, NT, true, SY>), grid, dim3(NT), 0, L.stream,
                       Xc, kt, tw, md, e_slot, slot0, energy_parts(N));
  else
    hipLaunchKernelGGL((k_pass_b<T, N, CX, CY, CZ, NT, false, SY>), grid, dim3(NT), 0, L.stream,
                       Xc, kt, tw, md, e_slot, slot0, energy_parts(N));
  return hipGetLastError();
}

// parity classes (x, y, z) of the boundary conditions: free (2, 2, 2),
// surface (1, 1, 2), periodic (1, 1, 1); the wire's (2, 2, 1) runs as (2, 1, 2)
// with the spectrum's y and z exchanged (passes A and C swap_yz, kernel table
// [fx][fz][fy]), so that its periodic axis is transformed once for both
// y classes (6 instead of 8 line sets per slab)
template <typename T, int N>
constexpr bool wave_form_fits() {  // one slab buffer plus the tables in LDS
  return (size_t)N * wave_pitch<N>() * sizeof(cpx<T>) + 2 * N * sizeof(cpx<T>) <= 160 * 1024;
}

template <typename T, int N, int CX, int CY, int CZ>
hipError_t launch_pass_b_wave(const Launch& L, cpx<T>* Xc, int nslots, bool energy_only,
                              double* e_slot, int slot0, const Tables& tb) {
  if constexpr (!wave_form_fits<T, N>()) {
    return hipErrorInvalidValue;
  } else {
    auto* kt = static_cast<const T*>(tb.ktab);
    auto* tw = static_cast<const cpx<T>*>(tb.tw);
    auto* md = static_cast<const cpx<T>*>(tb.md);
    dim3 grid = pass_b_xcd_order(N) ? dim3(CX * N * nslots) : dim3(CX * N, nslots);
    if (energy_only)
      hipLaunchKernelGGL((k_pass_b_wave<T, N, CX, CY, CZ, true>), grid, dim3(8 * N), 0, L.stream,
                         Xc, kt, tw, md, e_slot, slot0, energy_parts(N), nslots);
    else
      hipLaunchKernelGGL((k_pass_b_wave<T, N, CX, CY, CZ, false>), grid, dim3(8 * N), 0, L.stream,
                         Xc, kt, tw, md, e_slot, slot0, energy_parts(N), nslots);
    return hipGetLastError();
  }
}

bool pass_b_wave_supported(int precision, int n) {
  bool ok = false;
  (void)dispatch_n(n, [&]<int N>() -> hipError_t {
    ok = precision == EXX_PREC_FP64_FUSED ? wave_form_fits<double, N>() : wave_form_fits<float, N>();
    return hipSuccess;
  });
  return ok;
}

template <typename T, int N, int CX, int CY, int CZ>
hipError_t launch_pass_b_for(const Launch& L, cpx<T>* Xc, int nslots, bool energy_only,
                             double* e_slot, int slot0, const Tables& tb, int slab_threads,
                             int form) {
  if (form == EXX_SLAB_WAVE)
    return launch_pass_b_wave<T, N, CX, CY, CZ>(L, Xc, nslots, energy_only, e_slot, slot0, tb);
  constexpr bool SY = pass_b_share_y<T, N, CY, CZ>();
  constexpr int NT = pass_b_threads<T, N, SY>();
  if constexpr (SY && NT == 256 && sizeof(T) == 4 && N == 64) {
    // the 512-thread variant: one item per thread, 4 waves per SIMD
    if (slab_threads == 512)
      return launch_pass_b_cls<T, N, CX, CY, CZ, 512, SY>(L, Xc, nslots, energy_only, e_slot,
                                                           slot0, tb);
  }
  return launch_pass_b_cls<T, N, CX, CY, CZ, NT, SY>(L, Xc, nslots, energy_only, e_slot, slot0,
                                                      tb);
}

template <typename T>
hipError_t launch_pass_b(const Launch& L, void* X, int nslots, bool energy_only, double* e_slot,
                         int slot0, const Tables& tb, int slab_threads, int form) {
  if (nslots <= 0) return hipSuccess;
  return dispatch_n(L.n, [&]<int N>() -> hipError_t {
    if constexpr (sizeof(T) == 8 && N > 96) {
      return hipErrorInvalidValue;
    } else {
      auto* Xc = static_cast<cpx<T>*>(X);
      if (L.ncls == 2 && L.cy == 2 && L.cz == 2)
        return launch_pass_b_for<T, N, 2, 2, 2>(L, Xc, nslots, energy_only, e_slot, slot0, tb,
                                                slab_threads, form);
      if (L.ncls == 1 && L.cy == 1 && L.cz == 2)
        return launch_pass_b_for<T, N, 1, 1, 2>(L, Xc, nslots, energy_only, e_slot, slot0, tb,
                                                slab_threads, form);
      if (L.ncls == 1 && L.cy == 1 && L.cz == 1)
        return launch_pass_b_for<T, N, 1, 1, 1>(L, Xc, nslots, energy_only, e_slot, slot0, tb,
                                                slab_threads, form);
      if (L.ncls == 2 && L.cy == 1 && L.cz == 2)  // wire, y and z exchanged
        return launch_pass_b_for<T, N, 2, 1, 2>(L, Xc, nslots, energy_only, e_slot, slot0, tb,
                                                slab_threads, form);
      return hipErrorInvalidValue;
    }
  });
}

// ---- split pass B (three launches) ------------------------------------------
template <typename T, int N, int CX, int CY, int CZ>
hipError_t launch_split_for(const Launch& L, cpx<T>* X, cpx<T>* Y, int nslots, bool energy_only,
                            double* e_part, int slot0, const Tables& tb) {
  constexpr int NT = 128;
  auto* kt = static_cast<const T*>(tb.ktab);
  auto* tw = static_cast<const cpx<T>*>(tb.tw);
  auto* md = static_cast<const cpx<T>*>(tb.md);
  dim3 grid(N / SC, CX * N, nslots);
  hipLaunchKernelGGL((k_pass_b1<T, N, CX, CY, NT>), grid, dim3(NT), 0, L.stream, X, Y, tw, md);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (energy_only) {
    hipLaunchKernelGGL((k_pass_b2<T, N, CX, CY, CZ, NT, true>), grid, dim3(NT), 0, L.stream, Y, kt,
                       tw, md, e_part, slot0, energy_parts(N));
    return hipGetLastError();
  }
  hipLaunchKernelGGL((k_pass_b2<T, N, CX, CY, CZ, NT, false>), grid, dim3(NT), 0, L.stream, Y, kt,
                     tw, md, e_part, slot0, energy_parts(N));
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_pass_b3<T, N, CX, CY, NT>), grid, dim3(NT), 0, L.stream, X, Y, tw, md);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_pass_b_split(const Launch& L, void* X, void* Y, int nslots, bool energy_only,
                               double* e_part, int slot0, const Tables& tb) {
  if (nslots <= 0) return hipSuccess;
  if (nslots > 65535) return hipErrorInvalidValue;
  return dispatch_n(L.n, [&]<int N>() -> hipError_t {
    auto* Xc = static_cast<cpx<T>*>(X);
    auto* Yc = static_cast<cpx<T>*>(Y);
    if (L.ncls == 2 && L.cy == 2 && L.cz == 2)
      return launch_split_for<T, N, 2, 2, 2>(L, Xc, Yc, nslots, energy_only, e_part, slot0, tb);
    if (L.ncls == 1 && L.cy == 1 && L.cz == 2)
      return launch_split_for<T, N, 1, 1, 2>(L, Xc, Yc, nslots, energy_only, e_part, slot0, tb);
    if (L.ncls == 1 && L.cy == 1 && L.cz == 1)
      return launch_split_for<T, N, 1, 1, 1>(L, Xc, Yc, nslots, energy_only, e_part, slot0, tb);
    if (L.ncls == 2 && L.cy == 1 && L.cz == 2)  // wire, y and z exchanged
      return launch_split_for<T, N, 2, 1, 2>(L, Xc, Yc, nslots, energy_only, e_part, slot0, tb);
    return hipErrorInvalidValue;
  });
}

// Large FP32 slabs with a zero-padded z axis and without the shared-y variant
// take the split pass B (n >= 112: two slab buffers no longer fit in LDS).  Periodic slabs have
// a quarter of the classes and stay faster in one launch (n = 96: pass B 1.35
// vs 2.22 ms split; n = 128: 2.82 vs 5.46 ms at 32 orbitals).
bool pass_b_split(int precision, int n, int ncls, int cy, int cz) {
  if (precision != EXX_PREC_FP32 || n < 96 || cz != 2) return false;
  bool sy = false;
  (void)dispatch_n(n, [&]<int N>() -> hipError_t {
    if (ncls == 2 && cy == 2 && cz == 2) sy = pass_b_share_y<float, N, 2, 2>();
    else if (ncls == 1 && cy == 1 && cz == 2) sy = pass_b_share_y<float, N, 1, 2>();
    return hipSuccess;
  });
  return !sy;
}

// Energy partials per slot half written by the split pass B (one per slab and ky-chunk).
int split_energy_parts_used(int n, int ncls) { return ncls * n * (n / SC); }

int pass_c_max_tile(int precision, int n, bool cplx) {
  int t = 0;
  (void)dispatch_n(n, [&]<int N>() -> hipError_t {
    if (!cplx)
      t = precision == EXX_PREC_FP64_FUSED ? pass_c_tile<double, N>() : pass_c_tile<float, N>();
    else if (precision == EXX_PREC_FP64_FUSED)
      t = pass_c_tile_cplx<double, N>();
    else
      t = pass_c_tile_cplx<float, N>();
    return hipSuccess;
  });
  return t > 0 ? t : pass_c_tile<float, 128>();
}

template <typename T>
hipError_t launch_pass_c(const Launch& L, const void* X, const T* psi, const double* occ,
                         const Slot* slots, const TilePair* tiles, int t0, int ntiles,
                         int slot_base, double* kpsi, double* e_slot, int k_mode, bool want_e,
                         bool pair_out, int tmax, const Tables& tb, const SysTab* sys) {
  if (ntiles <= 0) return hipSuccess;
  const SysTab systab = sys ? *sys : SysTab{};
  return dispatch_n(L.n, [&]<int N>() -> hipError_t {
    if constexpr (sizeof(T) == 8 && N > 96) {
      return hipErrorInvalidValue;
    } else {
      constexpr int ZB = XZ;
      dim3 grid(N * (N / ZB), ntiles);
      auto* Xc = static_cast<const cpx<T>*>(X);
      auto* tw = static_cast<const cpx<T>*>(tb.tw);
      auto* md = static_cast<const cpx<T>*>(tb.md);
      if (L.cplx) {
        constexpr int TMC = pass_c_tile_cplx<T, N>();
        if (tmax > TMC) return hipErrorInvalidValue;
        auto* pc = reinterpret_cast<const cpx<T>*>(psi);
        auto* kc = reinterpret_cast<cpx<double>*>(kpsi);
        if (L.ncls == 2)
          hipLaunchKernelGGL((k_pass_c_cplx<T, N, 2, ZB, ZB * 16, TMC>), grid, dim3(ZB * 16), 0, L.stream, Xc,
                             pc, occ, slots, tiles, t0, slot_base, kc, e_slot, k_mode,
                             want_e ? 1 : 0, pair_out ? 1 : 0, tw, md, energy_parts(N), L.swap_yz,
                             systab);
        else
          hipLaunchKernelGGL((k_pass_c_cplx<T, N, 1, ZB, ZB * 16, TMC>), grid, dim3(ZB * 16), 0, L.stream, Xc,
                             pc, occ, slots, tiles, t0, slot_base, kc, e_slot, k_mode,
                             want_e ? 1 : 0, pair_out ? 1 : 0, tw, md, energy_parts(N), L.swap_yz,
                             systab);
        return hipGetLastError();
      }
      auto run = [&]<int HP>() -> hipError_t {
        constexpr int NT = ZB * 16 * HP;
        constexpr int TM = pass_c_tile<T, N, HP>();
        if (tmax > TM) return hipErrorInvalidValue;
        if (L.ncls == 2)
          hipLaunchKernelGGL((k_pass_c<T, N, 2, ZB, NT, TM, HP>), grid, dim3(NT), 0, L.stream, Xc,
                             psi, occ, slots, tiles, t0, slot_base, kpsi, e_slot, k_mode,
                             want_e ? 1 : 0, pair_out ? 1 : 0, tw, md, energy_parts(N), L.swap_yz,
                             systab);
        else
          hipLaunchKernelGGL((k_pass_c<T, N, 1, ZB, NT, TM, HP>), grid, dim3(NT), 0, L.stream, Xc,
                             psi, occ, slots, tiles, t0, slot_base, kpsi, e_slot, k_mode,
                             want_e ? 1 : 0, pair_out ? 1 : 0, tw, md, energy_parts(N), L.swap_yz,
                             systab);
        return hipGetLastError();
      };
      if constexpr (pass_c_halves<T, N>() == 2) {
        if (tmax > pass_c_tile<T, N, 1>()) return run.template operator()<2>();
      }
      return run.template operator()<1>();
    }
  });
}

template hipError_t launch_pass_a<float>(const Launch&, const float*, void*, const Slot*, int, int,
                                         const double*, bool, const Tables&);
template hipError_t launch_pass_a<double>(const Launch&, const double*, void*, const Slot*, int,
                                          int, const double*, bool, const Tables&);
template hipError_t launch_pass_b<float>(const Launch&, void*, int, bool, double*, int,
                                         const Tables&, int, int);
template hipError_t launch_pass_b<double>(const Launch&, void*, int, bool, double*, int,
                                          const Tables&, int, int);
template hipError_t launch_pass_b_split<float>(const Launch&, void*, void*, int, bool, double*, int,
                                               const Tables&);
template hipError_t launch_pass_c<float>(const Launch&, const void*, const float*, const double*,
                                         const Slot*, const TilePair*, int, int, int, double*,
                                         double*, int, bool, bool, int, const Tables&,
                                         const SysTab*);
template hipError_t launch_pass_c<double>(const Launch&, const void*, const double*,
                                          const double*, const Slot*, const TilePair*, int, int,
                                          int, double*, double*, int, bool, bool, int,
                                          const Tables&, const SysTab*);

}  // namespace exx
