// exx_batch.cpp -- batches of independent systems and the autotuner.
//
// A batch owns one plan per system and spreads the systems over a few side
// streams forked from the caller's stream (event fork/join), so independent
// systems overlap on the device; with use_graph the whole evaluation (all
// systems, all passes, the fork and the join) is captured once into a HIP
// graph with parallel branches and replayed, so a batch costs one graph
// launch.  The autotuner times a small grid of tunings
// with hipEvents and keeps the fastest; results persist in a text cache.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "exx_internal.hpp"

struct exx_batch {
  std::vector<exx_plan*> plans;  // one per system (plans may repeat grids)
  std::vector<int> n_orb;
  std::vector<size_t> ws_off;
  size_t ws_total = 0;
  int use_graph = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<exx_system> captured;  // pointers the graph was captured with
  int captured_mode = 0;
  unsigned captured_flags = 0;
  void* captured_ws = nullptr;
  hipStream_t captured_stream = nullptr;
  std::vector<hipStream_t> side;  // default-priority, non-blocking
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
  bool merge = false;                    // EXX_BATCH_MERGE
  std::vector<exx::MergedClass> classes;  // with merge: every system in one class
};

namespace {
constexpr int kSideStreams = 4;
}

namespace {

using exx::record_error;
using exx::record_hip_error;

#define EXX_BATCH_HIP(call)                                    \
  do {                                                         \
    hipError_t e_ = (call);                                    \
    if (e_ != hipSuccess) return record_hip_error(e_, #call);  \
  } while (0)

bool same_systems(const std::vector<exx_system>& a, const exx_system* b, size_t n) {
  if (a.size() != n) return false;
  for (size_t i = 0; i < n; ++i)
    if (std::memcmp(&a[i], &b[i], sizeof(exx_system)) != 0) return false;
  return true;
}

// Two grids that give the same kernels and kernel table.
bool same_grid(const exx_grid& a, const exx_grid& c) {
  return a.nx == c.nx && a.ny == c.ny && a.nz == c.nz && a.hx == c.hx && a.hy == c.hy &&
         a.hz == c.hz && a.bc == c.bc && a.kernel == c.kernel && a.R == c.R && a.omega == c.omega;
}

}  // namespace

extern "C" {

int exx_batch_create(exx_batch** out, const exx_grid* grids, const int* n_orb, int n_systems,
                     int precision, unsigned flags) {
  if (!out || !grids || !n_orb || n_systems <= 0)
    return record_error(EXX_ERR_INVALID_ARG, "out, grids and n_orb are required and n_systems > 0");
  if ((flags & ~(EXX_BATCH_GRAPH | EXX_BATCH_COMPLEX | EXX_BATCH_MERGE)) != 0)
    return record_error(EXX_ERR_INVALID_ARG, "unknown batch flags");
  if ((flags & EXX_BATCH_MERGE) && precision != EXX_PREC_FP32)
    return record_error(EXX_ERR_INVALID_ARG, "EXX_BATCH_MERGE needs the FP32 path");
  *out = nullptr;
  exx_batch* b = new (std::nothrow) exx_batch();
  if (!b) return record_error(EXX_ERR_INTERNAL, "out of host memory");
  b->use_graph = (flags & EXX_BATCH_GRAPH) != 0;
  const unsigned plan_flags = (flags & EXX_BATCH_COMPLEX) ? EXX_PLAN_COMPLEX : 0u;
  size_t off = 0;
  for (int s = 0; s < n_systems; ++s) {
    exx_plan* p = nullptr;
    int rc = exx_plan_create(&p, &grids[s], precision, n_orb[s], plan_flags);
    if (rc == EXX_OK) rc = exx_plan_prepare(p, n_orb[s]);
    size_t bytes = 0;
    if (rc == EXX_OK) rc = exx_workspace_bytes(p, n_orb[s], &bytes);
    if (rc != EXX_OK) {
      if (p) exx_plan_destroy(p);
      exx_batch_destroy(b);
      return rc;
    }
    b->plans.push_back(p);
    b->n_orb.push_back(n_orb[s]);
    b->ws_off.push_back(off);
    off += (bytes + 255) / 256 * 256;
  }
  b->ws_total = off;
  if (flags & EXX_BATCH_MERGE) {
    // classes of systems on one grid (at most kMaxMergedSystems each); the
    // workspace becomes one region per class
    b->merge = true;
    std::vector<int> cls(n_systems, -1);
    for (int s = 0; s < n_systems; ++s) {
      if (cls[s] >= 0) continue;
      exx::MergedClass mc;
      for (int c = s; c < n_systems && (int)mc.members.size() < exx::kMaxMergedSystems; ++c)
        if (cls[c] < 0 && same_grid(grids[s], grids[c])) {
          cls[c] = (int)b->classes.size();
          mc.members.push_back(c);
        }
      b->classes.push_back(mc);
    }
    off = 0;
    for (auto& mc : b->classes) {
      int rc = exx::build_merged_class(b->plans, b->n_orb, mc);
      if (rc != EXX_OK) {
        exx_batch_destroy(b);
        return rc;
      }
      mc.ws_off = off;
      off += (mc.ws_bytes + 255) / 256 * 256;
    }
    b->ws_total = off;
  }
  const int ns = std::min<int>(kSideStreams, n_systems);
  if (hipError_t e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming); e != hipSuccess) {
    exx_batch_destroy(b);
    return record_hip_error(e, "hipEventCreateWithFlags");
  }
  for (int k = 0; k < ns; ++k) {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) {
      if (st) (void)hipStreamDestroy(st);
      exx_batch_destroy(b);
      return record_hip_error(e, "side stream / join event creation");
    }
    b->side.push_back(st);
    b->join.push_back(ev);
  }
  *out = b;
  return EXX_OK;
}

void exx_batch_destroy(exx_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (auto& mc : b->classes) exx::free_merged_class(mc);
  for (auto* p : b->plans) exx_plan_destroy(p);
  for (auto st : b->side) (void)hipStreamDestroy(st);
  for (auto ev : b->join) (void)hipEventDestroy(ev);
  if (b->fork) (void)hipEventDestroy(b->fork);
  delete b;
}

int exx_batch_workspace_bytes(const exx_batch* b, size_t* bytes) {
  if (!b || !bytes) return record_error(EXX_ERR_INVALID_ARG, "batch or bytes is NULL");
  *bytes = b->ws_total;
  return EXX_OK;
}

// Issues every system: fork the side streams from st, system s on side stream
// s mod K (largest systems first), join back into st.
static int batch_issue(exx_batch* b, const exx_system* sys, int mode, unsigned flags, char* ws,
                       hipStream_t st) {
  EXX_BATCH_HIP(hipEventRecord(b->fork, st));
  for (auto side : b->side) EXX_BATCH_HIP(hipStreamWaitEvent(side, b->fork, 0));
  if (b->merge) {
    // one merged class per side stream in turn
    int rc = EXX_OK;
    for (size_t k = 0; k < b->classes.size() && rc == EXX_OK; ++k)
      rc = exx::run_merged_class(b->plans, b->classes[k], sys, mode, flags, ws,
                                 b->side[k % b->side.size()]);
    for (size_t k = 0; k < b->side.size(); ++k) {
      EXX_BATCH_HIP(hipEventRecord(b->join[k], b->side[k]));
      EXX_BATCH_HIP(hipStreamWaitEvent(st, b->join[k], 0));
    }
    return rc;
  }
  std::vector<size_t> order(b->plans.size());
  for (size_t s = 0; s < order.size(); ++s) order[s] = s;
  auto work = [&](size_t s) {
    double n3 = (double)b->plans[s]->n * b->plans[s]->n * b->plans[s]->n * b->plans[s]->ncls;
    return n3 * b->n_orb[s] * (b->n_orb[s] + 1);
  };
  std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t c) { return work(a) > work(c); });
  int rc = EXX_OK;
  for (size_t k = 0; k < order.size() && rc == EXX_OK; ++k) {
    const size_t s = order[k];
    size_t bytes = 0;
    exx_workspace_bytes(b->plans[s], b->n_orb[s], &bytes);
    rc = exx_compute(b->plans[s], sys[s].psi, sys[s].occ, b->n_orb[s], mode, flags, sys[s].ex_out,
                     sys[s].kpsi, sys[s].pair_e, ws + b->ws_off[s], bytes,
                     b->side[k % b->side.size()]);
  }
  for (size_t k = 0; k < b->side.size(); ++k) {
    EXX_BATCH_HIP(hipEventRecord(b->join[k], b->side[k]));
    EXX_BATCH_HIP(hipStreamWaitEvent(st, b->join[k], 0));
  }
  return rc;
}

int exx_batch_compute(exx_batch* b, const exx_system* sys, int mode, unsigned flags, void* ws,
                      size_t ws_bytes, void* stream) {
  if (!b || !sys) return record_error(EXX_ERR_INVALID_ARG, "batch or systems is NULL");
  if (!ws || ws_bytes < b->ws_total)
    return record_error(EXX_ERR_WORKSPACE, "workspace smaller than exx_batch_workspace_bytes(): need " +
                                               std::to_string(b->ws_total));
  if (((uintptr_t)ws % 256) != 0) return record_error(EXX_ERR_ALIGNMENT, "workspace must be 256-byte aligned");
  if (b->merge) {
    if (mode != EXX_MODE_KPSI && mode != EXX_MODE_ENERGY_KPSI)
      return record_error(EXX_ERR_INVALID_ARG, "a merged batch evaluates the KPSI and ENERGY_KPSI modes");
    if ((flags & ~EXX_FLAG_ACCUMULATE) != 0) return record_error(EXX_ERR_INVALID_ARG, "unknown flags");
    for (size_t s = 0; s < b->plans.size(); ++s) {
      if (sys[s].pair_e) return record_error(EXX_ERR_INVALID_ARG, "a merged batch gives no pair energies");
      if (!sys[s].psi || !sys[s].occ || !sys[s].kpsi || ((mode & EXX_MODE_ENERGY) && !sys[s].ex_out))
        return record_error(EXX_ERR_INVALID_ARG, "psi, occ, kpsi (and ex_out for energies) are required");
    }
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* wsc = static_cast<char*>(ws);
  if (!b->use_graph) return batch_issue(b, sys, mode, flags, wsc, st);
  const size_t n = b->plans.size();
  bool reuse = b->exec && same_systems(b->captured, sys, n) && b->captured_mode == mode &&
               b->captured_flags == flags && b->captured_ws == ws && b->captured_stream == st;
  if (!reuse) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    hipStream_t cs = st;
    bool own = false;
    if (cs == nullptr) {  // the legacy default stream cannot be captured
      EXX_BATCH_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
      own = true;
    }
    if (hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal); e != hipSuccess) {
      if (own) (void)hipStreamDestroy(cs);
      return record_hip_error(e, "hipStreamBeginCapture");
    }
    int rc = batch_issue(b, sys, mode, flags, wsc, cs);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(cs, &g);
    if (own) (void)hipStreamDestroy(cs);
    if (rc != EXX_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return record_hip_error(e, "hipStreamEndCapture");
    b->graph = g;
    EXX_BATCH_HIP(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
    b->captured.assign(sys, sys + n);
    b->captured_mode = mode;
    b->captured_flags = flags;
    b->captured_ws = ws;
    b->captured_stream = st;
  }
  EXX_BATCH_HIP(hipGraphLaunch(b->exec, st));
  return EXX_OK;
}

int exx_batch_autotune(exx_batch* b, const exx_system* sys, void* ws, size_t ws_bytes,
                       void* stream, int budget_ms, const char* cache_path) {
  if (!b || !sys) return record_error(EXX_ERR_INVALID_ARG, "batch or systems is NULL");
  if (b->merge) return record_error(EXX_ERR_INVALID_ARG, "a merged batch is not autotuned");
  if (!ws || ws_bytes < b->ws_total)
    return record_error(EXX_ERR_WORKSPACE, "workspace smaller than exx_batch_workspace_bytes(): need " +
                                               std::to_string(b->ws_total));
  const size_t n = b->plans.size();
  // classes: systems on the same grid (same kernels and kernel table); each is
  // tuned on its member with the most orbitals
  auto same_class = [&](size_t a, size_t c) {
    return same_grid(b->plans[a]->grid, b->plans[c]->grid) &&
           b->plans[a]->precision == b->plans[c]->precision;
  };
  std::vector<int> cls(n, -1);
  std::vector<size_t> rep;
  for (size_t s = 0; s < n; ++s) {
    if (cls[s] >= 0) continue;
    cls[s] = (int)rep.size();
    size_t best = s;
    for (size_t c = s + 1; c < n; ++c)
      if (cls[c] < 0 && same_class(s, c)) {
        cls[c] = cls[s];
        if (b->n_orb[c] > b->n_orb[best]) best = c;
      }
    rep.push_back(best);
  }
  const int per_class = std::max(1, (budget_ms > 0 ? budget_ms : 20000) / (int)rep.size());
  char* wsc = static_cast<char*>(ws);
  for (size_t k = 0; k < rep.size(); ++k) {
    const size_t s = rep[k];
    if (!sys[s].kpsi)
      return record_error(EXX_ERR_INVALID_ARG, "exx_batch_autotune needs each class's K psi buffer as scratch");
    const size_t slice = (s + 1 < n ? b->ws_off[s + 1] : b->ws_total) - b->ws_off[s];
    int rc = exx_autotune(b->plans[s], sys[s].psi, sys[s].occ, b->n_orb[s], sys[s].kpsi,
                          wsc + b->ws_off[s], slice, stream, per_class, cache_path);
    if (rc != EXX_OK) return rc;
    exx_tuning t{};
    exx_plan_get_tuning(b->plans[s], &t);
    for (size_t c = 0; c < n; ++c) {
      if (cls[c] != (int)k || c == s) continue;
      // the class's tuning where it fits this member's share of the workspace
      exx_tuning old{};
      exx_plan_get_tuning(b->plans[c], &old);
      rc = exx_plan_set_tuning(b->plans[c], &t);
      size_t need = 0;
      const size_t share = (c + 1 < n ? b->ws_off[c + 1] : b->ws_total) - b->ws_off[c];
      if (rc == EXX_OK) rc = exx_workspace_bytes(b->plans[c], b->n_orb[c], &need);
      if (rc != EXX_OK || need > share) (void)exx_plan_set_tuning(b->plans[c], &old);
      rc = exx_plan_prepare(b->plans[c], b->n_orb[c]);
      if (rc != EXX_OK) return rc;
    }
  }
  // the captured graph holds the old launches: capture again on the next call
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  return EXX_OK;
}

int exx_batch_get_tuning(const exx_batch* b, int system, exx_tuning* out) {
  if (!b || !out || system < 0 || system >= (int)b->plans.size())
    return record_error(EXX_ERR_INVALID_ARG, "batch, system index or out is invalid");
  return exx_plan_get_tuning(b->plans[system], out);
}

int exx_autotune(exx_plan* p, const double* psi, const double* occ, int n_orb, double* kpsi,
                 void* ws, size_t ws_bytes, void* stream, int budget_ms, const char* cache_path) {
  if (!p || !psi || !occ || !kpsi) return record_error(EXX_ERR_INVALID_ARG, "plan, psi, occ and kpsi are required");
  const auto t_start = std::chrono::steady_clock::now();
  const double budget = budget_ms > 0 ? (double)budget_ms : 20000.0;
  auto spent = [&]() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start)
               .count() > budget;
  };
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipDeviceProp_t prop;
  EXX_BATCH_HIP(hipGetDeviceProperties(&prop, p->device));
  std::ostringstream key;
  key << prop.gcnArchName << " n=" << p->n << " bc=" << p->grid.bc << " kernel=" << p->grid.kernel
      << " prec=" << p->precision << " complex=" << (p->cplx ? 1 : 0) << " N=" << n_orb;
  // cache lookup
  if (cache_path) {
    std::ifstream f(cache_path);
    std::string line;
    while (std::getline(f, line)) {
      auto bar = line.find('|');
      if (bar == std::string::npos || line.substr(0, bar) != key.str()) continue;
      exx_tuning t{};
      if (std::sscanf(line.c_str() + bar + 1, "%d %d %d %d %d", &t.tile, &t.batch_slots,
                      &t.slab_threads, &t.streams, &t.slab_form) == 5)
        return exx_plan_set_tuning(p, &t);
    }
  }
  exx_tuning base = p->tuning, best = base;
  float best_ms = 1e30f;
  // pair-tile edges up to pass C's limit for this plan (complex plans stop lower)
  std::vector<int> tiles;
  for (int t : {4, 8})
    if (t <= exx::pass_c_max_tile(p->precision, p->n, p->cplx)) tiles.push_back(t);
  if (tiles.empty()) tiles.push_back(exx::pass_c_max_tile(p->precision, p->n, p->cplx));
  std::vector<int> batches = {64, 256, 1 << 20};
  const bool fused = p->precision != EXX_PREC_FP64_PLAIN;
  // the 512-thread slab variant exists for the FP32 path at n = 64 only
  std::vector<int> slab_threads = (p->n == 64 && p->precision == EXX_PREC_FP32)
                                      ? std::vector<int>{256, 512}
                                      : std::vector<int>{p->tuning.slab_threads};
  std::vector<int> streams = fused ? std::vector<int>{1, 3} : std::vector<int>{1};
  // y/z pass forms: the workgroup-shared one always, the wave-local one where it fits
  std::vector<int> forms = {EXX_SLAB_SHARED};
  if (fused && exx::pass_b_wave_supported(p->precision, p->n)) forms.push_back(EXX_SLAB_WAVE);
  std::vector<exx_tuning> cands;
  for (int t : tiles)
    for (int bs : batches)
      for (int form : forms)
        for (int sth : slab_threads) {
          if (form == EXX_SLAB_WAVE && sth != slab_threads.front()) continue;  // no thread choice
          for (int nst : streams) {
            exx_tuning cand = base;
            cand.tile = t;
            cand.batch_slots = bs;
            cand.slab_threads = sth;
            cand.streams = nst;
            cand.slab_form = form;
            cands.push_back(cand);
          }
        }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  double* ex_dev = nullptr;
  hipError_t he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  if (he == hipSuccess) he = hipMalloc((void**)&ex_dev, sizeof(double));
  if (he != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return record_hip_error(he, "autotune events / scratch scalar");
  }
  int rc = EXX_OK;
  for (const exx_tuning& cand : cands) {
    if (best_ms < 1e30f && spent()) break;  // budget spent: keep the best so far
    if (exx_plan_set_tuning(p, &cand) != EXX_OK) continue;
    size_t need = 0;
    if (exx_workspace_bytes(p, n_orb, &need) != EXX_OK || need > ws_bytes) continue;
    if (exx_plan_prepare(p, n_orb) != EXX_OK) continue;
    rc = exx_compute(p, psi, occ, n_orb, EXX_MODE_ENERGY_KPSI, 0, ex_dev, kpsi, nullptr, ws, ws_bytes, st);
    if (rc != EXX_OK) break;
    (void)hipEventRecord(e0, st);
    const int reps = 3;
    for (int r = 0; r < reps && rc == EXX_OK; ++r)
      rc = exx_compute(p, psi, occ, n_orb, EXX_MODE_ENERGY_KPSI, 0, ex_dev, kpsi, nullptr, ws, ws_bytes, st);
    (void)hipEventRecord(e1, st);
    (void)hipEventSynchronize(e1);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (rc != EXX_OK) break;
    if (ms < best_ms) {
      best_ms = ms;
      best = cand;
    }
  }
  (void)hipFree(ex_dev);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  exx_plan_set_tuning(p, &best);
  if (rc != EXX_OK) return rc;
  if (cache_path) {
    std::ofstream f(cache_path, std::ios::app);
    f << key.str() << "|" << best.tile << " " << best.batch_slots << " " << best.slab_threads
      << " " << best.streams << " " << best.slab_form << "\n";
  }
  return exx_plan_prepare(p, n_orb);
}

}  // extern "C"
