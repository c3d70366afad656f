// exx_api.cpp -- C ABI: validation, plans (twiddle and kernel tables), pair
// schedules, workspace layout and the launch sequence of one evaluation.
//
// Pair-sum scheme of arXiv:1712.07973 (Section 2, Eq. 5): all N(N+1)/2
// unordered pairs i <= j are solved once; an off-diagonal pair enters E_x
// twice (f_i f_j e_ij + f_j f_i e_ji) and updates both (K psi)_i and
// (K psi)_j, which is the single-device analogue of returning each pair
// potential to both orbital owners (Section 2.1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "exx_fft.hpp"
#include "exx_internal.hpp"

using namespace exx;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  g_last_error = std::string(where) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
  return EXX_ERR_HIP;
}

}  // namespace

int exx::record_error(int code, const std::string& msg) { return fail(code, msg); }
int exx::record_hip_error(hipError_t e, const char* where) { return hip_fail(e, where); }

namespace {

#define EXX_HIP(call)                            \
  do {                                           \
    hipError_t e_ = (call);                      \
    if (e_ != hipSuccess) return hip_fail(e_, #call); \
  } while (0)

constexpr double kPi = 3.14159265358979323846;

bool supported_n(int n) { return n >= 16 && n <= 128 && n % 16 == 0; }

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Green's kernel in Fourier space (real, even), FP64 on the host, at the
// wave vector with in-plane (x, y) part Gp2 = Gx^2 + Gy^2 and normal part Gz.
double kernel_value(const exx_grid& g, double R, double Gp2, double Gz) {
  const double G2 = Gp2 + Gz * Gz;
  if (g.kernel == EXX_KERNEL_SCREENED) {
    double w2 = g.omega * g.omega;
    if (G2 == 0.0) return kPi / w2;
    return 4.0 * kPi * (-std::expm1(-G2 / (4.0 * w2))) / G2;
  }
  if (g.bc == EXX_BC_PERIODIC) {
    if (G2 == 0.0) return 0.0;
    return 4.0 * kPi / G2;
  }
  if (g.bc == EXX_BC_SURFACE) {  // Coulomb cut at |z| = R, periodic in-plane
    if (Gp2 > 0.0) {
      const double Gp = std::sqrt(Gp2);
      return 4.0 * kPi / G2 *
             (1.0 + std::exp(-Gp * R) * (Gz / Gp * std::sin(Gz * R) - std::cos(Gz * R)));
    }
    if (Gz != 0.0) return 4.0 * kPi / G2 * (1.0 - std::cos(Gz * R) - Gz * R * std::sin(Gz * R));
    return -2.0 * kPi * R * R;
  }
  if (g.bc == EXX_BC_WIRE) {  // Coulomb cut at in-plane distance R, periodic along z
    const double Gp = std::sqrt(Gp2), az = std::fabs(Gz);
    if (az > 0.0)
      return 4.0 * kPi / G2 *
             (1.0 + R * (Gp * std::cyl_bessel_j(1.0, Gp * R) * std::cyl_bessel_k(0.0, az * R) -
                         az * std::cyl_bessel_j(0.0, Gp * R) * std::cyl_bessel_k(1.0, az * R)));
    if (Gp > 0.0) {
      const double x = Gp * R;
      return 4.0 * kPi / G2 *
             (1.0 - std::cyl_bessel_j(0.0, x) - x * std::cyl_bessel_j(1.0, x) * std::log(R));
    }
    return kPi * R * R * (1.0 - 2.0 * std::log(R));
  }
  if (G2 == 0.0) return 2.0 * kPi * R * R;
  double G = std::sqrt(G2);
  double s = std::sin(0.5 * G * R);
  return 8.0 * kPi * s * s / G2;
}

// Octant table K(fx, fy, fz) / (mx my mz) for folded indices 0..m/2 per axis
// (fz fastest).
std::vector<double> kernel_octant(const exx_grid& g, double R, Dims m) {
  if (g.kernel == EXX_KERNEL_ISF) return isf_octant(g.nx, g.hx, g.hy, g.hz);
  const int hx = m.x / 2 + 1, hy = m.y / 2 + 1, hz = m.z / 2 + 1;
  std::vector<double> t((size_t)hx * hy * hz);
  const double inv = 1.0 / ((double)m.x * m.y * m.z);
  auto wave = [](int f, int mm, double h) { return 2.0 * kPi * f / (mm * h); };
  for (int fx = 0; fx < hx; ++fx)
    for (int fy = 0; fy < hy; ++fy)
      for (int fz = 0; fz < hz; ++fz) {
        const double gx = wave(fx, m.x, g.hx), gy = wave(fy, m.y, g.hy);
        t[((size_t)fx * hy + fy) * hz + fz] =
            kernel_value(g, R, gx * gx + gy * gy, wave(fz, m.z, g.hz)) * inv;
      }
  return t;
}

// exp(-2 pi i k / L) for k < count, FP64 (libm) then stored as T.
template <typename T>
std::vector<cpx<T>> roots(int L, int count) {
  std::vector<cpx<T>> v(count);
  for (int k = 0; k < count; ++k) {
    double a = -2.0 * kPi * (double)k / (double)L;
    v[k] = {(T)std::cos(a), (T)std::sin(a)};
  }
  return v;
}

template <typename V>
int upload(void** dst, const V& v) {
  size_t bytes = v.size() * sizeof(typename V::value_type);
  EXX_HIP(hipMalloc(dst, bytes));
  EXX_HIP(hipMemcpy(*dst, v.data(), bytes, hipMemcpyHostToDevice));
  return EXX_OK;
}

bool is_fp32(const exx_plan* p) { return p->precision == EXX_PREC_FP32; }
bool is_plain(const exx_plan* p) { return p->precision == EXX_PREC_FP64_PLAIN; }

size_t slot_bytes(const exx_plan* p) {
  // fused: ncls * n^3 complex of the compute type; plain: the padded grid, complex FP64 per pair
  if (is_plain(p)) return (size_t)p->m.x * p->m.y * p->m.z * 16;
  size_t c = is_fp32(p) ? 8 : 16;
  return (size_t)p->ncls * p->n * p->n * p->n * c;
}

int max_tile(const exx_plan* p) { return pass_c_max_tile(p->precision, p->n, p->cplx); }

// Default form of the y/z pass (FP32, 32 orbitals, ms of pass B per evaluation,
// shared / wave): free n = 32 0.13 / 0.19, 64 1.32 / 1.30, 96 6.8 / 6.1,
// 128 23.6 / 14.5; periodic n = 80 0.60 / 0.86, 128 2.78 / 2.58.  The wave-local
// form wins from n = 48 on except on the periodic 80^3 grid.  FP64 plans keep
// the workgroup-shared form by default (their wave-local form, n <= 80, is
// selectable and tested but not the timed configuration).
int default_slab_form(const exx_plan* p) {
  if (!is_fp32(p) || !pass_b_wave_supported(p->precision, p->n)) return EXX_SLAB_SHARED;
  if (p->n <= 32) return EXX_SLAB_SHARED;
  if (p->ncls == 1 && p->cy == 1 && p->cz == 1 && p->n == 80) return EXX_SLAB_SHARED;
  return EXX_SLAB_WAVE;
}

void default_tuning(exx_plan* p) {
  p->tuning.tile = max_tile(p);
  const size_t budget = (size_t)4 << 30;  // bytes of spectrum workspace per launch chunk
  size_t per = slot_bytes(p);
  p->tuning.batch_slots = (int)std::max<size_t>(1, std::min<size_t>(budget / per, 1 << 20));
  p->tuning.slab_threads = (p->n == 64 && is_fp32(p)) ? 512 : 256;
  p->tuning.streams = 1;
  p->tuning.slab_form = default_slab_form(p);
}

int schedule_tile(const exx_plan* p) {
  return is_plain(p) ? 0 : std::max(1, std::min(p->tuning.tile, max_tile(p)));
}

void build_schedule(const exx_plan* p, int N, Schedule& s) {
  const int packing = is_plain(p) ? kPlain : (p->cplx ? kTiled : kPacked);
  build_schedule_host(N, schedule_tile(p), p->tuning.batch_slots, packing, s);
}

int cap_slots(const exx_plan* p, const Schedule& s) {
  int cap = 0;
  for (auto& c : s.chunks) cap = std::max(cap, c.s1 - c.s0);
  return cap;
}

struct WsLayout {
  size_t psi32 = 0, e_slot = 0, e_part = 0, X = 0, Y = 0, total = 0;
  int split_slots = 0;  // slots per launch of the split pass B (0: not split)
};

bool uses_split(const exx_plan* p) {
  return p->tuning.slab_form != EXX_SLAB_WAVE && pass_b_split(p->precision, p->n, p->ncls, p->cy, p->cz);
}

// bytes per slot of the split pass B scratch: ncls cy n^3 complex FP32
size_t split_slot_bytes(const exx_plan* p) { return (size_t)p->ncls * p->cy * p->n * p->n * p->n * 8; }

WsLayout layout(const exx_plan* p, const Schedule& s) {
  WsLayout w;
  size_t off = 0;
  w.psi32 = off;
  if (is_fp32(p))
    off += align_up((size_t)s.n_orb * p->n * p->n * p->n * sizeof(float) * (p->cplx ? 2 : 1), 256);
  w.e_slot = off;
  off += align_up(2 * s.slots.size() * sizeof(double), 256);
  w.e_part = off;
  if (!is_plain(p)) off += align_up(2 * s.slots.size() * (size_t)energy_parts(p->n) * sizeof(double), 256);
  w.X = off;
  off += align_up((size_t)cap_slots(p, s) * slot_bytes(p), 256);
  w.Y = off;
  if (!is_plain(p) && uses_split(p)) {
    // a few slots per launch: the scratch stays near the memory-side cache size
    const size_t budget = (size_t)512 << 20;
    w.split_slots = (int)std::max<size_t>(1, std::min<size_t>(cap_slots(p, s), budget / split_slot_bytes(p)));
    off += align_up((size_t)w.split_slots * split_slot_bytes(p), 256);
  }
  w.total = off;
  return w;
}

int get_schedule(exx_plan* p, int N, Schedule** out, bool allow_build) {
  auto it = p->schedules.find(N);
  if (it != p->schedules.end() &&
      it->second.tile == schedule_tile(p) &&
      it->second.batch_slots == p->tuning.batch_slots) {
    *out = &it->second;
    return EXX_OK;
  }
  if (!allow_build) return fail(EXX_ERR_NOT_PREPARED, "schedule for this n_orb is not prepared (call exx_plan_prepare before graph capture)");
  if (it != p->schedules.end()) {
    (void)hipFree(it->second.d_slots);
    (void)hipFree(it->second.d_tiles);
    p->schedules.erase(it);
  }
  Schedule s;
  build_schedule(p, N, s);
  int dev = 0;
  EXX_HIP(hipGetDevice(&dev));
  EXX_HIP(hipSetDevice(p->device));
  EXX_HIP(hipMalloc((void**)&s.d_slots, std::max<size_t>(1, s.slots.size()) * sizeof(Slot)));
  EXX_HIP(hipMemcpy(s.d_slots, s.slots.data(), s.slots.size() * sizeof(Slot), hipMemcpyHostToDevice));
  if (!s.tiles.empty()) {
    EXX_HIP(hipMalloc((void**)&s.d_tiles, s.tiles.size() * sizeof(TilePair)));
    EXX_HIP(hipMemcpy(s.d_tiles, s.tiles.data(), s.tiles.size() * sizeof(TilePair), hipMemcpyHostToDevice));
  }
  // fork/join events of the overlapped rounds: one fork, then per round one
  // event after pass A, one after pass B and one after pass C
  const size_t need = 1 + 3 * s.segments.size();
  while (p->sync_ev.size() < need) {
    hipEvent_t e;
    EXX_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    p->sync_ev.push_back(e);
  }
  EXX_HIP(hipSetDevice(dev));
  auto res = p->schedules.emplace(N, std::move(s));
  *out = &res.first->second;
  return EXX_OK;
}

bool aligned(const void* ptr, size_t a) { return ((uintptr_t)ptr % a) == 0; }

// Brackets one launch with a pair of events when profiling is on.
struct Prof {
  exx_plan* p;
  hipStream_t st;
  size_t idx = (size_t)-1;
  Prof(exx_plan* p_, int kind, hipStream_t st_) : p(p_), st(st_) {
    if (!p->profile || !p->recording) return;
    if (p->ev_used == p->ev_start.size()) {
      hipEvent_t a, b;
      if (hipEventCreate(&a) != hipSuccess) return;
      if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return;
      }
      p->ev_start.push_back(a);
      p->ev_stop.push_back(b);
      p->ev_kind.push_back(kind);
    }
    idx = p->ev_used++;
    p->ev_kind[idx] = kind;
    (void)hipEventRecord(p->ev_start[idx], st);
  }
  ~Prof() {
    if (idx != (size_t)-1) (void)hipEventRecord(p->ev_stop[idx], st);
  }
};
#define EXX_PROF(kind) Prof prof_##__LINE__(p, kind, st)
#define EXX_PROF_ON(kind, stream) Prof prof_##__LINE__(p, kind, stream)

// Slots of one round (segment) of a chunk: its tile pairs' slots are contiguous.
void segment_slots(const Schedule& s, int g, int* a, int* b) {
  *a = s.tiles[s.segments[g].t0].s0;
  *b = s.tiles[s.segments[g].t1 - 1].s1;
}

template <typename T>
int run_fused(exx_plan* p, const Schedule& s, const WsLayout& w, const double* psi,
              const double* occ, int N, int mode, unsigned flags, double* ex_out, double* kpsi,
              double* pair_e, char* ws, hipStream_t st) {
  const bool want_k = (mode & EXX_MODE_KPSI) != 0;
  const bool want_e = (mode & EXX_MODE_ENERGY) != 0 || pair_e != nullptr;
  const bool parseval = (mode == EXX_MODE_ENERGY) && pair_e == nullptr;
  // values per orbital: n^3 doubles, or n^3 (re, im) pairs for complex orbitals
  const size_t n3 = (size_t)p->n * p->n * p->n * (p->cplx ? 2 : 1);
  const T* psiT;
  if constexpr (sizeof(T) == 4) {
    float* p32 = reinterpret_cast<float*>(ws + w.psi32);
    {
      EXX_PROF(EXX_PASS_CONVERT);
      EXX_HIP(launch_convert(psi, p32, (size_t)N * n3, st));
    }
    psiT = p32;
  } else {
    psiT = psi;
  }
  double* e_slot = reinterpret_cast<double*>(ws + w.e_slot);
  double* e_part = reinterpret_cast<double*>(ws + w.e_part);
  const int kparts = energy_parts(p->n);
  char* X = ws + w.X;
  const size_t sb = slot_bytes(p);
  // K psi needs no clearing: pass C's diagonal tile pairs (the first round,
  // every orbital once) store their row sums unless the caller accumulates
  const int k_mode = !want_k ? 0 : ((flags & EXX_FLAG_ACCUMULATE) ? 1 : 2);
  Launch L{p->n, p->ncls, p->cy, p->cz, p->h3, st, p->cplx ? 1 : 0, p->swap_yz ? 1 : 0};
  // pass B over ns slots from slot s0 (spectra at Xs) on the stream of Lb: one
  // launch, or the split form in groups of w.split_slots
  auto pass_b = [&](const Launch& Lb, char* Xs, int s0, int ns) -> int {
    if (w.split_slots == 0) {
      EXX_PROF_ON(EXX_PASS_B, Lb.stream);
      EXX_HIP(launch_pass_b<T>(Lb, Xs, ns, parseval, e_part, s0, p->tables, p->tuning.slab_threads,
                               p->tuning.slab_form));
      return EXX_OK;
    }
    if constexpr (sizeof(T) == 4) {
      for (int a = 0; a < ns; a += w.split_slots) {
        const int k = std::min(w.split_slots, ns - a);
        EXX_PROF_ON(EXX_PASS_B, Lb.stream);
        EXX_HIP(launch_pass_b_split<T>(Lb, Xs + (size_t)a * sb, ws + w.Y, k, parseval, e_part, s0 + a,
                                       p->tables));
      }
      return EXX_OK;
    }
    return fail(EXX_ERR_INTERNAL, "split pass B is FP32 only");
  };
  const bool overlap = p->tuning.streams == 3 && p->side[0] && p->side[1] &&
                       p->sync_ev.size() >= 1 + 3 * s.segments.size();
  if (!overlap) {
    for (const auto& c : s.chunks) {
      const int ns = c.s1 - c.s0;
      {
        EXX_PROF(EXX_PASS_A);
        EXX_HIP(launch_pass_a<T>(L, psiT, X, s.d_slots, c.s0, ns, occ, parseval, p->tables));
      }
      if (int r = pass_b(L, X, c.s0, ns)) return r;
      if (!parseval) {
        for (int g = c.seg0; g < c.seg1; ++g) {
          const auto& sg = s.segments[g];
          EXX_PROF(EXX_PASS_C);
          EXX_HIP(launch_pass_c<T>(L, X, psiT, occ, s.d_slots, s.d_tiles, sg.t0, sg.t1 - sg.t0, c.s0,
                                   kpsi, e_part, k_mode, want_e, pair_e != nullptr, s.tile,
                                   p->tables));
        }
      }
    }
  } else {
    // Rounds in a pipeline over three streams: pass A of round g on sa, pass B
    // on the caller's stream once A(g) is done, pass C on sc once B(g) is done.
    // Rounds of a chunk own disjoint slots of X, so A(g+1) and C(g-1) may run
    // beside B(g); the next chunk's pass A reuses X only after the previous
    // chunk's last reader of X is done (its last pass C, or its last pass B in
    // the energy-only mode, which has no pass C).  Pass C launches stay in
    // round order on sc, so the K psi updates keep the order of the serial path.
    hipStream_t sa = p->side[0], sc = p->side[1];
    Launch La = L, Lc = L;
    La.stream = sa;
    Lc.stream = sc;
    size_t ev = 0;
    hipEvent_t fork = p->sync_ev[ev++];
    EXX_HIP(hipEventRecord(fork, st));
    EXX_HIP(hipStreamWaitEvent(sa, fork, 0));
    if (!parseval) EXX_HIP(hipStreamWaitEvent(sc, fork, 0));
    hipEvent_t last_c = nullptr, last_use = nullptr;
    for (const auto& c : s.chunks) {
      if (last_use) EXX_HIP(hipStreamWaitEvent(sa, last_use, 0));
      for (int g = c.seg0; g < c.seg1; ++g) {
        int a0, a1;
        segment_slots(s, g, &a0, &a1);
        char* Xg = X + (size_t)(a0 - c.s0) * sb;
        {
          EXX_PROF_ON(EXX_PASS_A, sa);
          EXX_HIP(launch_pass_a<T>(La, psiT, Xg, s.d_slots, a0, a1 - a0, occ, parseval, p->tables));
        }
        hipEvent_t ea = p->sync_ev[ev++];
        EXX_HIP(hipEventRecord(ea, sa));
        EXX_HIP(hipStreamWaitEvent(st, ea, 0));
        if (int r = pass_b(L, Xg, a0, a1 - a0)) return r;
        hipEvent_t eb = p->sync_ev[ev++];
        EXX_HIP(hipEventRecord(eb, st));
        if (parseval) {
          last_use = eb;
          continue;
        }
        EXX_HIP(hipStreamWaitEvent(sc, eb, 0));
        {
          const auto& sg = s.segments[g];
          EXX_PROF_ON(EXX_PASS_C, sc);
          EXX_HIP(launch_pass_c<T>(Lc, X, psiT, occ, s.d_slots, s.d_tiles, sg.t0, sg.t1 - sg.t0,
                                   c.s0, kpsi, e_part, k_mode, want_e, pair_e != nullptr, s.tile,
                                   p->tables));
        }
        last_c = p->sync_ev[ev++];
        EXX_HIP(hipEventRecord(last_c, sc));
        last_use = last_c;
      }
    }
    // sa's last pass A is already joined by the pass B that waited for it
    if (last_c) EXX_HIP(hipStreamWaitEvent(st, last_c, 0));
  }
  if (want_e) {
    EXX_PROF(EXX_PASS_FINALIZE);
    double* eo = (mode & EXX_MODE_ENERGY) ? ex_out : nullptr;
    if (parseval) {  // one partial per (slot, slab)
      const int count = w.split_slots ? split_energy_parts_used(p->n, p->ncls) : p->ncls * p->n;
      EXX_HIP(launch_slot_reduce(e_part, kparts, count, 2 * (int)s.slots.size(), e_slot, st));
      EXX_HIP(launch_finalize(s.d_slots, (int)s.slots.size(), occ, e_slot, N, p->h3, 1, eo, nullptr, st));
    } else if (pair_e) {  // one partial per (slot half, row block)
      EXX_HIP(launch_slot_reduce(e_part, kparts, p->n * p->n / 16, 2 * (int)s.slots.size(), e_slot, st));
      EXX_HIP(launch_finalize(s.d_slots, (int)s.slots.size(), occ, e_slot, N, p->h3, 0, eo, pair_e, st));
    } else {  // one weighted partial per (tile pair, row block)
      EXX_HIP(launch_slot_reduce(e_part, kparts, p->n * p->n / 16, (int)s.tiles.size(), e_slot, st));
      EXX_HIP(launch_finalize(s.d_slots, (int)s.tiles.size(), occ, e_slot, N, p->h3, 2, eo, nullptr, st));
    }
  }
  return EXX_OK;
}

int run_plain(exx_plan* p, const Schedule& s, const WsLayout& w, const double* psi,
              const double* occ, int N, int mode, unsigned flags, double* ex_out, double* kpsi,
              double* pair_e, char* ws, hipStream_t st) {
  const bool want_k = (mode & EXX_MODE_KPSI) != 0;
  const bool want_e = (mode & EXX_MODE_ENERGY) != 0 || pair_e != nullptr;
  const size_t n3 = (size_t)p->n * p->n * p->n * (p->cplx ? 2 : 1);  // doubles per orbital
  double* e_slot = reinterpret_cast<double*>(ws + w.e_slot);
  void* Z = ws + w.X;
  {
    EXX_PROF(EXX_PASS_ZERO);
    if (want_e) EXX_HIP(launch_zero(e_slot, 2 * s.slots.size(), st));
    if (want_k && !(flags & EXX_FLAG_ACCUMULATE)) EXX_HIP(launch_zero(kpsi, (size_t)N * n3, st));
  }
  for (const auto& c : s.chunks) {
    const int np = c.s1 - c.s0;
    {
      EXX_PROF(EXX_PASS_PLAIN_OTHER);
      EXX_HIP(plain_build(psi, s.d_slots, c.s0, np, p->n, p->m, Z, p->cplx, st));
    }
    for (int a = 0; a < 3; ++a) {
      EXX_PROF(EXX_PASS_PLAIN_FFT);
      EXX_HIP(plain_fft_axis(Z, np, p->n, p->m, a, -1, p->tables, st));
    }
    {
      EXX_PROF(EXX_PASS_PLAIN_OTHER);
      EXX_HIP(plain_kernel_mul(Z, np, p->m, p->tables, st));
    }
    for (int a = 0; a < 3; ++a) {
      EXX_PROF(EXX_PASS_PLAIN_FFT);
      EXX_HIP(plain_fft_axis(Z, np, p->n, p->m, a, +1, p->tables, st));
    }
    {
      EXX_PROF(EXX_PASS_PLAIN_OTHER);
      EXX_HIP(plain_reduce(Z, psi, occ, s.d_slots, c.s0, np, p->n, p->m, p->h3, kpsi, e_slot, want_k,
                           want_e, p->cplx, st));
    }
  }
  if (want_e) {
    EXX_PROF(EXX_PASS_FINALIZE);
    EXX_HIP(launch_finalize(s.d_slots, (int)s.slots.size(), occ, e_slot, N, p->h3, 0,
                            (mode & EXX_MODE_ENERGY) ? ex_out : nullptr, pair_e, st));
  }
  return EXX_OK;
}

int validate_grid(const exx_grid* g, int precision) {
  if (!g) return fail(EXX_ERR_INVALID_ARG, "grid is NULL");
  if (g->nx <= 0 || g->ny <= 0 || g->nz <= 0) return fail(EXX_ERR_INVALID_ARG, "grid sizes must be positive");
  if (!(g->hx > 0) || !(g->hy > 0) || !(g->hz > 0) || !std::isfinite(g->hx) || !std::isfinite(g->hy) ||
      !std::isfinite(g->hz))
    return fail(EXX_ERR_INVALID_ARG, "grid spacings must be positive and finite");
  if (g->bc != EXX_BC_PERIODIC && g->bc != EXX_BC_FREE && g->bc != EXX_BC_SURFACE &&
      g->bc != EXX_BC_WIRE)
    return fail(EXX_ERR_INVALID_ARG, "unknown boundary condition");
  if (g->kernel != EXX_KERNEL_COULOMB && g->kernel != EXX_KERNEL_SCREENED && g->kernel != EXX_KERNEL_ISF)
    return fail(EXX_ERR_INVALID_ARG, "unknown kernel");
  if (g->kernel == EXX_KERNEL_SCREENED && (!(g->omega > 0) || g->bc != EXX_BC_PERIODIC))
    return fail(EXX_ERR_INVALID_ARG, "screened kernel needs omega > 0 and a periodic grid");
  if (g->kernel == EXX_KERNEL_ISF && g->bc != EXX_BC_FREE)
    return fail(EXX_ERR_INVALID_ARG, "the ISF kernel is built for the free boundary");
  if (precision != EXX_PREC_FP32 && precision != EXX_PREC_FP64_PLAIN && precision != EXX_PREC_FP64_FUSED)
    return fail(EXX_ERR_INVALID_ARG, "unknown precision");
  if (g->nx != g->ny || g->nx != g->nz) return fail(EXX_ERR_UNSUPPORTED_SIZE, "grid must be cubic (nx == ny == nz)");
  if (!supported_n(g->nx))
    return fail(EXX_ERR_UNSUPPORTED_SIZE, "n must be one of 16, 32, 48, 64, 80, 96, 112, 128");
  if (precision == EXX_PREC_FP64_FUSED && g->nx > 96)
    return fail(EXX_ERR_UNSUPPORTED_SIZE, "FP64_FUSED supports n <= 96 (LDS capacity)");
  return EXX_OK;
}

}  // namespace

int exx::build_merged_class(const std::vector<exx_plan*>& plans, const std::vector<int>& n_orb,
                            MergedClass& mc) {
  if (mc.members.empty() || (int)mc.members.size() > kMaxMergedSystems)
    return fail(EXX_ERR_INVALID_ARG, "a merged class holds 1 to 32 systems");
  exx_plan* p = plans[mc.members[0]];
  if (!is_fp32(p)) return fail(EXX_ERR_INVALID_ARG, "merged launches need the FP32 path");
  std::vector<const Schedule*> parts;
  for (int s : mc.members) {
    Schedule* sc = nullptr;
    if (int rc = get_schedule(plans[s], n_orb[s], &sc, true)) return rc;
    parts.push_back(sc);
  }
  merge_schedules(parts, p->tuning.batch_slots, mc.sched, mc.orb_base, mc.tile_base);
  Schedule& s = mc.sched;
  EXX_HIP(hipSetDevice(p->device));
  EXX_HIP(hipMalloc((void**)&s.d_slots, std::max<size_t>(1, s.slots.size()) * sizeof(Slot)));
  EXX_HIP(hipMemcpy(s.d_slots, s.slots.data(), s.slots.size() * sizeof(Slot), hipMemcpyHostToDevice));
  EXX_HIP(hipMalloc((void**)&s.d_tiles, std::max<size_t>(1, s.tiles.size()) * sizeof(TilePair)));
  EXX_HIP(hipMemcpy(s.d_tiles, s.tiles.data(), s.tiles.size() * sizeof(TilePair), hipMemcpyHostToDevice));
  // class workspace: FP32 orbitals of every member end to end, per-tile energy
  // partials and sums, the spectrum of the largest chunk, the split pass B scratch
  const size_t orbs = (size_t)s.n_orb * p->n * p->n * p->n * (p->cplx ? 2 : 1);
  size_t off = 0;
  mc.psi32 = off;
  off += align_up(orbs * sizeof(float), 256);
  mc.e_part = off;
  off += align_up(s.tiles.size() * (size_t)energy_parts(p->n) * sizeof(double), 256);
  mc.e_slot = off;
  off += align_up(s.tiles.size() * sizeof(double), 256);
  mc.X = off;
  off += align_up((size_t)cap_slots(p, s) * slot_bytes(p), 256);
  mc.Y = off;
  mc.split_slots = 0;
  if (uses_split(p)) {
    const size_t budget = (size_t)512 << 20;
    mc.split_slots = (int)std::max<size_t>(1, std::min<size_t>(cap_slots(p, s), budget / split_slot_bytes(p)));
    off += align_up((size_t)mc.split_slots * split_slot_bytes(p), 256);
  }
  mc.ws_bytes = off;
  return EXX_OK;
}

void exx::free_merged_class(MergedClass& mc) {
  if (mc.sched.d_slots) (void)hipFree(mc.sched.d_slots);
  if (mc.sched.d_tiles) (void)hipFree(mc.sched.d_tiles);
  mc.sched.d_slots = nullptr;
  mc.sched.d_tiles = nullptr;
}

int exx::run_merged_class(const std::vector<exx_plan*>& plans, const MergedClass& mc,
                          const exx_system* sys, int mode, unsigned flags, char* ws, hipStream_t st) {
  exx_plan* p = plans[mc.members[0]];
  const Schedule& s = mc.sched;
  const bool want_e = (mode & EXX_MODE_ENERGY) != 0;
  const size_t n3 = (size_t)p->n * p->n * p->n * (p->cplx ? 2 : 1);
  char* base = ws + mc.ws_off;
  float* psi32 = reinterpret_cast<float*>(base + mc.psi32);
  double* e_part = reinterpret_cast<double*>(base + mc.e_part);
  double* e_slot = reinterpret_cast<double*>(base + mc.e_slot);
  char* X = base + mc.X;
  const size_t sb = slot_bytes(p);
  const int kparts = energy_parts(p->n);
  const int k_mode = (flags & EXX_FLAG_ACCUMULATE) ? 1 : 2;
  Launch L{p->n, p->ncls, p->cy, p->cz, p->h3, st, p->cplx ? 1 : 0, p->swap_yz ? 1 : 0};
  // every member's orbitals into the class's FP32 copy (one launch), and its
  // outputs addressed with merged orbital indices (pointers offset back by its
  // first merged orbital)
  SysTab tab;
  MemberTab mt;
  tab.n = mt.n = (int)mc.members.size();
  size_t max_count = 0;
  for (size_t k = 0; k < mc.members.size(); ++k) {
    const exx_system& y = sys[mc.members[k]];
    const int N = (k + 1 < mc.members.size() ? mc.orb_base[k + 1] : s.n_orb) - mc.orb_base[k];
    mt.psi[k] = y.psi;
    mt.count[k] = (size_t)N * n3;
    mt.dst_off[k] = (size_t)mc.orb_base[k] * n3;
    mt.row0[k] = mc.tile_base[k];
    mt.ex_out[k] = y.ex_out;
    max_count = std::max(max_count, mt.count[k]);
    tab.kpsi[k] = reinterpret_cast<double*>(reinterpret_cast<uintptr_t>(y.kpsi) -
                                            (uintptr_t)mc.orb_base[k] * n3 * sizeof(double));
    tab.occ[k] = reinterpret_cast<const double*>(reinterpret_cast<uintptr_t>(y.occ) -
                                                 (uintptr_t)mc.orb_base[k] * sizeof(double));
  }
  mt.row0[mt.n] = (int)s.tiles.size();
  EXX_HIP(launch_convert_members(mt, psi32, max_count, st));
  for (const auto& c : s.chunks) {
    const int ns = c.s1 - c.s0;
    EXX_HIP(launch_pass_a<float>(L, psi32, X, s.d_slots, c.s0, ns, nullptr, false, p->tables));
    if (mc.split_slots == 0) {
      EXX_HIP(launch_pass_b<float>(L, X, ns, false, e_part, c.s0, p->tables, p->tuning.slab_threads,
                                   p->tuning.slab_form));
    } else {
      for (int a = 0; a < ns; a += mc.split_slots) {
        const int k = std::min(mc.split_slots, ns - a);
        EXX_HIP(launch_pass_b_split<float>(L, X + (size_t)a * sb, base + mc.Y, k, false, e_part,
                                           c.s0 + a, p->tables));
      }
    }
    for (int g = c.seg0; g < c.seg1; ++g) {
      const auto& sg = s.segments[g];
      EXX_HIP(launch_pass_c<float>(L, X, psi32, nullptr, s.d_slots, s.d_tiles, sg.t0, sg.t1 - sg.t0,
                                   c.s0, nullptr, e_part, k_mode, want_e, false, s.tile, p->tables,
                                   &tab));
    }
  }
  if (want_e) {
    // every tile pair's weighted partials, then per member the sum of its rows,
    // each in the fixed order of the unmerged evaluation
    EXX_HIP(launch_slot_reduce(e_part, kparts, p->n * p->n / 16, (int)s.tiles.size(), e_slot, st));
    EXX_HIP(launch_finalize_members(mt, e_slot, p->h3, st));
  }
  return EXX_OK;
}

int exx::compute_impl(exx_plan* p, const double* psi, const double* occ, int n_orb, int mode,
                      unsigned flags, double* ex_out, double* kpsi, double* pair_e, void* ws,
                      size_t ws_bytes, void* stream, bool may_allocate) {
  if (!p) return fail(EXX_ERR_INVALID_ARG, "plan is NULL");
  if (!psi || !occ) return fail(EXX_ERR_INVALID_ARG, "psi and occ are required");
  if (n_orb <= 0) return fail(EXX_ERR_INVALID_ARG, "n_orb must be positive");
  if (n_orb > p->n_orb_max) return fail(EXX_ERR_CAPACITY, "n_orb exceeds the plan's n_orb_max");
  if (mode != EXX_MODE_ENERGY && mode != EXX_MODE_KPSI && mode != EXX_MODE_ENERGY_KPSI)
    return fail(EXX_ERR_INVALID_ARG, "unknown mode");
  if ((flags & ~EXX_FLAG_ACCUMULATE) != 0) return fail(EXX_ERR_INVALID_ARG, "unknown flags");
  if ((mode & EXX_MODE_ENERGY) && !ex_out) return fail(EXX_ERR_INVALID_ARG, "ex_out is required for ENERGY modes");
  if ((mode & EXX_MODE_KPSI) && !kpsi) return fail(EXX_ERR_INVALID_ARG, "kpsi is required for KPSI modes");
  if (!aligned(psi, 16) || (kpsi && !aligned(kpsi, 16)) || !aligned(occ, 8) ||
      (pair_e && !aligned(pair_e, 8)) || (ex_out && !aligned(ex_out, 8)))
    return fail(EXX_ERR_ALIGNMENT, "psi/kpsi must be 16-byte aligned, scalars 8-byte aligned");
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  EXX_HIP(hipStreamIsCapturing(st, &cap));
  Schedule* s = nullptr;
  // without allocation the schedule must already exist (exx_plan_prepare)
  int rc = get_schedule(p, n_orb, &s, may_allocate && cap == hipStreamCaptureStatusNone);
  if (rc) return rc;
  WsLayout w = layout(p, *s);
  if (!ws || ws_bytes < w.total)
    return fail(EXX_ERR_WORKSPACE, "workspace smaller than exx_workspace_bytes(): need " + std::to_string(w.total));
  if (!aligned(ws, 256)) return fail(EXX_ERR_ALIGNMENT, "workspace must be 256-byte aligned");
  char* wsc = static_cast<char*>(ws);
  // profiling events are created on first use: not in the allocation-free call
  p->recording = (cap == hipStreamCaptureStatusNone) && may_allocate;
  if (is_plain(p)) return run_plain(p, *s, w, psi, occ, n_orb, mode, flags, ex_out, kpsi, pair_e, wsc, st);
  if (is_fp32(p)) return run_fused<float>(p, *s, w, psi, occ, n_orb, mode, flags, ex_out, kpsi, pair_e, wsc, st);
  return run_fused<double>(p, *s, w, psi, occ, n_orb, mode, flags, ex_out, kpsi, pair_e, wsc, st);
}

extern "C" {

const char* exx_version(void) { return "exx 0.1 gfx950"; }

const char* exx_last_error(void) { return g_last_error.c_str(); }

const char* exx_error_string(int code) {
  switch (code) {
    case EXX_OK: return "ok";
    case EXX_ERR_INVALID_ARG: return "invalid argument";
    case EXX_ERR_UNSUPPORTED_SIZE: return "unsupported size";
    case EXX_ERR_CAPACITY: return "capacity exceeded";
    case EXX_ERR_WORKSPACE: return "workspace missing or too small";
    case EXX_ERR_ALIGNMENT: return "misaligned pointer";
    case EXX_ERR_HIP: return "HIP runtime error";
    case EXX_ERR_NOT_PREPARED: return "schedule not prepared";
    case EXX_ERR_INTERNAL: return "internal error";
    default: return "unknown error code";
  }
}

int exx_plan_create(exx_plan** out, const exx_grid* grid, int precision, int n_orb_max,
                    unsigned flags) {
  if (!out) return fail(EXX_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if ((flags & ~EXX_PLAN_COMPLEX) != 0) return fail(EXX_ERR_INVALID_ARG, "unknown plan flags");
  int rc = validate_grid(grid, precision);
  if (rc) return rc;
  if (n_orb_max <= 0) return fail(EXX_ERR_INVALID_ARG, "n_orb_max must be positive");
  exx_plan* p = new (std::nothrow) exx_plan();
  if (!p) return fail(EXX_ERR_INTERNAL, "out of host memory");
  p->grid = *grid;
  p->n = grid->nx;
  // parity classes per axis: 2 on zero-padded (isolated) axes
  const bool iso_xy = grid->bc == EXX_BC_FREE || grid->bc == EXX_BC_WIRE;
  const bool iso_z = grid->bc == EXX_BC_FREE || grid->bc == EXX_BC_SURFACE;
  p->ncls = iso_xy ? 2 : 1;
  p->cy = iso_xy ? 2 : 1;
  p->cz = iso_z ? 2 : 1;
  p->m = Dims{p->ncls * p->n, p->cy * p->n, p->cz * p->n};
  p->h3 = grid->hx * grid->hy * grid->hz;
  if (grid->R > 0)
    p->R = grid->R;
  else if (grid->bc == EXX_BC_SURFACE)
    p->R = p->n * grid->hz;
  else if (grid->bc == EXX_BC_WIRE)
    p->R = p->n * std::min(grid->hx, grid->hy);
  else
    p->R = p->n * std::min(grid->hx, std::min(grid->hy, grid->hz));
  p->precision = precision;
  p->cplx = (flags & EXX_PLAN_COMPLEX) != 0;
  if (grid->bc == EXX_BC_WIRE && precision != EXX_PREC_FP64_PLAIN) {
    // the fused passes see the wire with y and z exchanged: classes (2, 1, 2),
    // so pass B transforms the periodic axis once for both padded-y classes
    p->swap_yz = true;
    std::swap(p->cy, p->cz);
  }
  p->n_orb_max = n_orb_max;
  default_tuning(p);
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "hipGetDevice");
  }
  if (!is_plain(p)) {
    for (auto& q : p->side) {
      e = hipStreamCreateWithFlags(&q, hipStreamNonBlocking);
      if (e != hipSuccess) {
        exx_plan_destroy(p);
        return hip_fail(e, "hipStreamCreateWithFlags");
      }
    }
  }
  auto kt = kernel_octant(*grid, p->R, p->m);
  if (p->swap_yz) {  // [fx][fy][fz] -> [fx][fz][fy], the fused passes' axis order
    const int ex = p->m.x / 2 + 1, ey = p->m.y / 2 + 1, ez = p->m.z / 2 + 1;
    std::vector<double> t(kt.size());
    for (int fx = 0; fx < ex; ++fx)
      for (int fy = 0; fy < ey; ++fy)
        for (int fz = 0; fz < ez; ++fz)
          t[((size_t)fx * ez + fz) * ey + fy] = kt[((size_t)fx * ey + fy) * ez + fz];
    kt.swap(t);
  }
  int r = EXX_OK;
  if (is_plain(p)) {
    r = upload(&p->tables.tw_n, roots<double>(p->n, p->n));
    if (!r && grid->bc != EXX_BC_PERIODIC) r = upload(&p->tables.tw_2n, roots<double>(2 * p->n, 2 * p->n));
    if (!r) r = upload(&p->tables.ktab_m, kt);
  } else if (is_fp32(p)) {
    std::vector<float> kf(kt.begin(), kt.end());
    r = upload(&p->tables.ktab, kf);
    if (!r) r = upload(&p->tables.tw, roots<float>(p->n, p->n));
    if (!r) r = upload(&p->tables.md, roots<float>(2 * p->n, p->n));
  } else {
    r = upload(&p->tables.ktab, kt);
    if (!r) r = upload(&p->tables.tw, roots<double>(p->n, p->n));
    if (!r) r = upload(&p->tables.md, roots<double>(2 * p->n, p->n));
  }
  if (r) {
    exx_plan_destroy(p);
    return r;
  }
  *out = p;
  return EXX_OK;
}

void exx_plan_destroy(exx_plan* p) {
  if (!p) return;
  for (size_t i = 0; i < p->ev_start.size(); ++i) {
    (void)hipEventDestroy(p->ev_start[i]);
    (void)hipEventDestroy(p->ev_stop[i]);
  }
  for (hipEvent_t e : p->sync_ev) (void)hipEventDestroy(e);
  for (hipStream_t q : p->side)
    if (q) (void)hipStreamDestroy(q);
  void* ptrs[] = {p->tables.tw, p->tables.md, p->tables.ktab, p->tables.tw_n, p->tables.tw_2n,
                  p->tables.ktab_m};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  for (auto& kv : p->schedules) {
    if (kv.second.d_slots) (void)hipFree(kv.second.d_slots);
    if (kv.second.d_tiles) (void)hipFree(kv.second.d_tiles);
  }
  delete p;
}

int exx_plan_prepare(exx_plan* p, int n_orb) {
  if (!p) return fail(EXX_ERR_INVALID_ARG, "plan is NULL");
  if (n_orb <= 0) return fail(EXX_ERR_INVALID_ARG, "n_orb must be positive");
  if (n_orb > p->n_orb_max) return fail(EXX_ERR_CAPACITY, "n_orb exceeds the plan's n_orb_max");
  Schedule* s = nullptr;
  return get_schedule(p, n_orb, &s, true);
}

int exx_plan_schedule_info(exx_plan* p, int n_orb, long long* n_pairs, long long* n_slots) {
  if (!p) return fail(EXX_ERR_INVALID_ARG, "plan is NULL");
  if (n_orb <= 0) return fail(EXX_ERR_INVALID_ARG, "n_orb must be positive");
  Schedule s;
  build_schedule(p, n_orb, s);
  if (n_pairs) *n_pairs = s.n_pairs;
  if (n_slots) *n_slots = (long long)s.slots.size();
  return EXX_OK;
}

int exx_workspace_bytes(const exx_plan* p, int n_orb, size_t* bytes) {
  if (!p || !bytes) return fail(EXX_ERR_INVALID_ARG, "plan or bytes is NULL");
  if (n_orb <= 0) return fail(EXX_ERR_INVALID_ARG, "n_orb must be positive");
  if (n_orb > p->n_orb_max) return fail(EXX_ERR_CAPACITY, "n_orb exceeds the plan's n_orb_max");
  Schedule s;
  build_schedule(p, n_orb, s);
  *bytes = layout(p, s).total;
  return EXX_OK;
}

int exx_plan_get_tuning(const exx_plan* p, exx_tuning* out) {
  if (!p || !out) return fail(EXX_ERR_INVALID_ARG, "plan or out is NULL");
  *out = p->tuning;
  return EXX_OK;
}

int exx_plan_set_tuning(exx_plan* p, const exx_tuning* t) {
  if (!p || !t) return fail(EXX_ERR_INVALID_ARG, "plan or tuning is NULL");
  if (t->tile < 0 || t->tile > 16 || t->batch_slots < 0)
    return fail(EXX_ERR_INVALID_ARG, "tile must be in 1..16 (clamped to the pass limit) and batch_slots >= 0");
  if (t->slab_threads != 0 && t->slab_threads != 256 && t->slab_threads != 512)
    return fail(EXX_ERR_INVALID_ARG, "slab_threads must be 256 or 512");
  if (t->streams != 0 && t->streams != 1 && t->streams != 3)
    return fail(EXX_ERR_INVALID_ARG, "streams must be 1 or 3");
  if (t->slab_form != 0 && t->slab_form != EXX_SLAB_SHARED && t->slab_form != EXX_SLAB_WAVE)
    return fail(EXX_ERR_INVALID_ARG, "slab_form must be EXX_SLAB_SHARED (1) or EXX_SLAB_WAVE (2)");
  if (t->slab_form == EXX_SLAB_WAVE && (is_plain(p) || !pass_b_wave_supported(p->precision, p->n)))
    return fail(EXX_ERR_INVALID_ARG, "the wave-local y/z pass does not fit this grid and precision");
  if (t->tile) p->tuning.tile = t->tile;
  if (t->batch_slots) p->tuning.batch_slots = t->batch_slots;
  if (t->slab_threads) p->tuning.slab_threads = t->slab_threads;
  if (t->streams) p->tuning.streams = t->streams;
  if (t->slab_form) p->tuning.slab_form = t->slab_form;
  return EXX_OK;
}

int exx_compute(exx_plan* p, const double* psi, const double* occ, int n_orb, int mode,
                unsigned flags, double* ex_out, double* kpsi, double* pair_e, void* ws,
                size_t ws_bytes, void* stream) {
  return exx::compute_impl(p, psi, occ, n_orb, mode, flags, ex_out, kpsi, pair_e, ws, ws_bytes,
                           stream, true);
}

int exx_gradient(exx_plan* p, const double* psi, const double* occ, int n_orb,
                 const double* gbar, double* grad_psi, double* grad_occ, double* pair_e, void* ws,
                 size_t ws_bytes, void* stream) {
  if (!p) return fail(EXX_ERR_INVALID_ARG, "plan is NULL");
  if (!gbar || !grad_psi) return fail(EXX_ERR_INVALID_ARG, "gbar and grad_psi are required");
  if (grad_occ && !pair_e) return fail(EXX_ERR_INVALID_ARG, "grad_occ needs the pair_e buffer");
  if (!aligned(gbar, 8) || (grad_occ && !aligned(grad_occ, 8)))
    return fail(EXX_ERR_ALIGNMENT, "gbar and grad_occ must be 8-byte aligned");
  // K psi (and the pair energies when the occupation gradient is wanted) into
  // the output buffers, then the scaling in place on the same stream
  const int rc = exx::compute_impl(p, psi, occ, n_orb, EXX_MODE_KPSI, 0, nullptr, grad_psi,
                                   grad_occ ? pair_e : nullptr, ws, ws_bytes, stream, true);
  if (rc) return rc;
  const size_t per_orb = (size_t)p->n * p->n * p->n * (p->cplx ? 2 : 1);
  EXX_HIP(launch_gradient(grad_psi, per_orb, n_orb, occ, gbar, p->h3, pair_e, grad_occ,
                          static_cast<hipStream_t>(stream)));
  return EXX_OK;
}

int exx_plan_enable_profiling(exx_plan* p, int enable) {
  if (!p) return fail(EXX_ERR_INVALID_ARG, "plan is NULL");
  p->profile = enable != 0;
  return EXX_OK;
}

int exx_plan_read_profile(exx_plan* p, exx_pass_times* out) {
  if (!p || !out) return fail(EXX_ERR_INVALID_ARG, "plan or out is NULL");
  for (size_t i = 0; i < p->ev_used; ++i) {
    EXX_HIP(hipEventSynchronize(p->ev_stop[i]));
    float ms = 0.f;
    EXX_HIP(hipEventElapsedTime(&ms, p->ev_start[i], p->ev_stop[i]));
    p->prof_ms[p->ev_kind[i]] += ms;
    p->prof_launches[p->ev_kind[i]] += 1;
  }
  p->ev_used = 0;
  for (int k = 0; k < EXX_PASS_KINDS; ++k) {
    out->ms[k] = p->prof_ms[k];
    out->launches[k] = p->prof_launches[k];
    p->prof_ms[k] = 0;
    p->prof_launches[k] = 0;
  }
  return EXX_OK;
}

}  // extern "C"
