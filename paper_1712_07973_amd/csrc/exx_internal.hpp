// exx_internal.hpp -- host-side plan structures and kernel launch interfaces.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/exx.h"
#include "exx_isf.hpp"
#include "exx_schedule.hpp"

namespace exx {

// Device tables of one plan (precision-specific arrays are null when unused).
struct Tables {
  void* tw = nullptr;      // w_n^k, k < n (fused paths), cpx<T>
  void* md = nullptr;      // w_{2n}^r, r < n (padded-axis modulation), cpx<T>
  void* ktab = nullptr;    // kernel octant / (fft points), T, [mx/2+1][my/2+1][mz/2+1]
  void* tw_n = nullptr;    // w_n^k, k < n (plain path, unpadded axes), cpx<double>
  void* tw_2n = nullptr;   // w_2n^k, k < 2n (plain path, padded axes), cpx<double>
  void* ktab_m = nullptr;  // kernel octant / (fft points) for the plain path, double
};

// FFT points per axis (n or 2n)
struct Dims {
  int x, y, z;
};

// Parity classes per axis: 2 on a zero-padded axis (the 2n-point transform
// splits into two n-point ones), 1 on a periodic axis.
struct Launch {
  int n;           // grid points per axis
  int ncls;        // x classes (spectrum slots hold ncls n^3 values)
  int cy, cz;      // y and z classes
  double h3;       // volume element
  hipStream_t stream;
  int cplx = 0;    // complex orbitals: one pair per slot, psi and K psi interleaved (re, im)
  int swap_yz = 0; // spectrum (y, z) = grid (z, y): cy, cz above are then the grid's z and y classes
};

// Per-system outputs of a pass C launch over a merged batch schedule: K psi and
// occupations of system k, each pointer offset back by the system's first
// merged orbital so that merged orbital indices address it directly.  n = 0:
// the launch's own kpsi and occ serve every tile pair.
constexpr int kMaxMergedSystems = 32;
struct SysTab {
  int n = 0;
  double* kpsi[kMaxMergedSystems] = {};
  const double* occ[kMaxMergedSystems] = {};
};

// The members of a merged class for the launches that run once per class:
// member k's FP64 orbitals psi[k] (count[k] values) go to the class's FP32 copy
// at dst_off[k]; its energy rows are [row0[k], row0[k + 1]) and its E_x goes to
// ex_out[k].
struct MemberTab {
  int n = 0;
  const double* psi[kMaxMergedSystems] = {};
  size_t count[kMaxMergedSystems] = {};
  size_t dst_off[kMaxMergedSystems] = {};
  int row0[kMaxMergedSystems + 1] = {};
  double* ex_out[kMaxMergedSystems] = {};
};
hipError_t launch_convert_members(const MemberTab& m, float* psi32, size_t max_count, hipStream_t s);
// E_x of every member from its rows of e_slot (as launch_finalize's sum mode 2)
hipError_t launch_finalize_members(const MemberTab& m, const double* e_slot, double h3, hipStream_t s);

}  // namespace exx

struct exx_plan {
  exx_grid grid;
  int n = 0, ncls = 1, cy = 1, cz = 1;  // grid, parity classes per spectrum axis
  bool swap_yz = false;                 // fused wire plans: spectrum y, z = grid z, y
  exx::Dims m{0, 0, 0};                 // FFT points per axis
  double h3 = 0, R = 0;
  int precision = 0;
  bool cplx = false;  // complex orbitals (EXX_PLAN_COMPLEX)
  int n_orb_max = 0;
  int device = 0;
  exx_tuning tuning{};
  exx::Tables tables;
  std::map<int, exx::Schedule> schedules;  // keyed by n_orb (schedule depends on tuning.tile)
  // profiling: event pairs recorded around launches, consumed by exx_plan_read_profile
  bool profile = false;
  bool recording = false;  // false while the stream is being captured
  std::vector<hipEvent_t> ev_start, ev_stop;
  std::vector<int> ev_kind;
  size_t ev_used = 0;
  double prof_ms[EXX_PASS_KINDS] = {};
  long long prof_launches[EXX_PASS_KINDS] = {};
  // overlapped rounds (tuning.streams == 3): side streams of passes A and C and
  // the fork/join events of one evaluation (created before any graph capture)
  hipStream_t side[2] = {nullptr, nullptr};
  std::vector<hipEvent_t> sync_ev;
};

namespace exx {

// ---- fused kernels (FP32 and FP64 instantiations), exx_fused.hip ----------
// All return hipSuccess or the launch error.
hipError_t launch_convert(const double* psi, float* psi32, size_t count, hipStream_t s);
hipError_t launch_zero(double* p, size_t count, hipStream_t s);

template <typename T>
hipError_t launch_pass_a(const Launch& L, const T* psi, void* X, const Slot* slots, int slot0,
                         int nslots, const double* occ, bool weighted, const Tables& tb);
template <typename T>
hipError_t launch_pass_b(const Launch& L, void* X, int nslots, bool energy_only, double* e_slot,
                         int slot0, const Tables& tb, int slab_threads, int form);
// whether the wave-local y/z pass (EXX_SLAB_WAVE) fits a grid of n points
bool pass_b_wave_supported(int precision, int n);
template <typename T>
hipError_t launch_pass_c(const Launch& L, const void* X, const T* psi, const double* occ,
                         const Slot* slots, const TilePair* tiles, int t0, int ntiles,
                         int slot_base, double* kpsi, double* e_slot, int k_mode, bool want_e,
                         bool pair_out, int tmax, const Tables& tb,
                         const SysTab* sys = nullptr);  // k_mode: 0 none, 1 add, 2 diagonal tiles store
// pass B in three launches through a scratch of ncls cy n^3 values per slot
// (large slabs, FP32); used when pass_b_split() says so
template <typename T>
hipError_t launch_pass_b_split(const Launch& L, void* X, void* Y, int nslots, bool energy_only,
                               double* e_part, int slot0, const Tables& tb);
bool pass_b_split(int precision, int n, int ncls, int cy, int cz);
int split_energy_parts_used(int n, int ncls);
int energy_parts(int n);  // pair-energy partials per slot half (fused passes)
hipError_t launch_slot_reduce(const double* parts, int kparts, int count, int nhalves,
                              double* e_slot, hipStream_t s);
hipError_t launch_finalize(const Slot* slots, int nvals, const double* occ, const double* e_slot,
                           int n_orb, double h3, int sum_mode, double* ex_out, double* pair_e,
                           hipStream_t s);

bool fused_supported(int precision, int n);
// grad_psi[k] *= -2 h3 f_k gbar over per_orb doubles per orbital (even);
// grad_occ (optional) = -gbar pair_e f
hipError_t launch_gradient(double* grad_psi, size_t per_orb, int n_orb, const double* occ,
                           const double* gbar, double h3, const double* pair_e, double* grad_occ,
                           hipStream_t s);

// Body of exx_compute.  may_allocate = false: no device allocation and no event
// creation (the schedule for n_orb must already be prepared, profiling events
// are not recorded); the workspace is whatever the caller passes.
int compute_impl(exx_plan* p, const double* psi, const double* occ, int n_orb, int mode,
                 unsigned flags, double* ex_out, double* kpsi, double* pair_e, void* ws,
                 size_t ws_bytes, void* stream, bool may_allocate);

// Systems of one grid class of a batch evaluated with shared launches: one
// merged schedule (merge_schedules) over the members' own schedules, so that
// a pass A and a pass B launch cover a chunk of every member's slots and a
// pass C launch a round of every member's tile pairs.  FP32 real or complex
// plans of one grid; at most kMaxMergedSystems members.
struct MergedClass {
  std::vector<int> members;  // system indices of the batch
  Schedule sched;            // merged; device copies in sched.d_slots / d_tiles
  std::vector<int> orb_base, tile_base;
  // workspace region of the class (offsets from the batch workspace) and its parts
  size_t ws_off = 0, ws_bytes = 0;
  size_t psi32 = 0, e_part = 0, e_slot = 0, X = 0, Y = 0;
  int split_slots = 0;
};
// Builds the merged schedule of `members` (their plans prepared for their
// orbital counts), uploads it and sizes the class workspace.
int build_merged_class(const std::vector<exx_plan*>& plans, const std::vector<int>& n_orb,
                       MergedClass& mc);
void free_merged_class(MergedClass& mc);
// One evaluation of the class in KPSI or ENERGY_KPSI mode without pair
// energies (sys: the batch's systems; ws: the batch workspace).
int run_merged_class(const std::vector<exx_plan*>& plans, const MergedClass& mc,
                     const exx_system* sys, int mode, unsigned flags, char* ws, hipStream_t st);

// Record msg (or the HIP error) as this thread's exx_last_error() and return
// the code (EXX_ERR_HIP for the second).
int record_error(int code, const std::string& msg);
int record_hip_error(hipError_t e, const char* where);
// largest pair-tile edge pass C supports at grid n (complex orbitals: its
// complex variant, whose per-tile registers and LDS are twice as large)
int pass_c_max_tile(int precision, int n, bool cplx);

// ---- plain FP64 path, exx_plain.hip ---------------------------------------
// cplx: psi (and kpsi) hold interleaved (re, im) FP64 values
hipError_t plain_build(const double* psi, const Slot* slots, int slot0, int npairs_in_launch,
                       int n, Dims m, void* Z, bool cplx, hipStream_t s);
hipError_t plain_fft_axis(void* Z, int npairs, int n, Dims m, int axis, int dir, const Tables& tb,
                          hipStream_t s);
hipError_t plain_kernel_mul(void* Z, int npairs, Dims m, const Tables& tb, hipStream_t s);
hipError_t plain_reduce(const void* Z, const double* psi, const double* occ, const Slot* slots,
                        int slot0, int npairs_in_launch, int n, Dims m, double h3, double* kpsi,
                        double* e_slot, bool want_k, bool want_e, bool cplx, hipStream_t s);

}  // namespace exx
