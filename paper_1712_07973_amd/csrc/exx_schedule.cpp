// exx_schedule.cpp -- pair schedule of one evaluation (host only).
//
// Pair-sum scheme of arXiv:1712.07973 (Section 2, Eq. 5): every unordered
// pair i <= j is solved once.
#include "exx_schedule.hpp"

#include <algorithm>

namespace exx {

// Orbital tiles of edge T; tile pairs (I <= J) in rounds of a round-robin
// tournament (the diagonal pairs (I, I) form one extra round), so the tile
// pairs of one round share no orbital.  This is the single-device image of the
// round-robin pair distribution of Section 2.1: there every process pairs its
// orbitals with those received at step s; here each round is a set of
// independent blocks that can update K psi without atomics.
std::vector<std::vector<std::pair<int, int>>> tile_rounds(int nt) {
  std::vector<std::vector<std::pair<int, int>>> rounds;
  std::vector<std::pair<int, int>> diag;
  for (int I = 0; I < nt; ++I) diag.push_back({I, I});
  rounds.push_back(diag);
  const int M = nt + (nt % 2);  // even number of teams; team M-1 is a bye when nt is odd
  for (int r = 0; r + 1 < M; ++r) {
    std::vector<std::pair<int, int>> rd;
    auto add = [&](int a, int b) {
      if (a >= nt || b >= nt || a == b) return;
      rd.push_back({std::min(a, b), std::max(a, b)});
    };
    add(r, M - 1);
    for (int k = 1; k < M / 2; ++k) add((r + k) % (M - 1), (r - k + (M - 1)) % (M - 1));
    if (!rd.empty()) rounds.push_back(rd);
  }
  return rounds;
}

// Chunks of whole tile pairs whose slots fit `cap`, each split into segments
// (runs of one round) for the pass C launches.
static void chunk_tiles(Schedule& s, int cap) {
  int t0 = 0;
  while (t0 < (int)s.tiles.size()) {
    int t1 = t0;
    while (t1 < (int)s.tiles.size() && s.tiles[t1].s1 - s.tiles[t0].s0 <= cap) ++t1;
    if (t1 == t0) t1 = t0 + 1;
    Schedule::Chunk c{t0, t1, s.tiles[t0].s0, s.tiles[t1 - 1].s1, (int)s.segments.size(), 0};
    int a = t0;
    while (a < t1) {
      int b = a;
      while (b < t1 && s.tile_round[b] == s.tile_round[a]) ++b;
      s.segments.push_back({a, b});
      a = b;
    }
    c.seg1 = (int)s.segments.size();
    s.chunks.push_back(c);
    t0 = t1;
  }
}

void build_schedule_host(int N, int T, int batch_slots, int packing, Schedule& s) {
  s = Schedule();
  s.n_orb = N;
  s.n_pairs = (long long)N * (N + 1) / 2;
  s.batch_slots = batch_slots;
  if (packing == kPlain) {
    s.tile = 0;
    for (int i = 0; i < N; ++i)
      for (int j = i; j < N; ++j) s.slots.push_back({i, j, -1, -1});
    int cap = std::max(1, batch_slots);
    for (int s0 = 0; s0 < (int)s.slots.size(); s0 += cap)
      s.chunks.push_back({0, 0, s0, std::min<int>((int)s.slots.size(), s0 + cap), 0, 0});
    return;
  }
  T = std::max(1, T);
  s.tile = T;
  const int nt = (N + T - 1) / T;
  auto rounds = tile_rounds(nt);
  s.n_rounds = (int)rounds.size();
  std::vector<int> round_of;
  for (size_t r = 0; r < rounds.size(); ++r)
    for (auto [I, J] : rounds[r]) {
      TilePair tp{};
      tp.I0 = I * T;
      tp.nI = std::min(T, N - tp.I0);
      tp.J0 = J * T;
      tp.nJ = std::min(T, N - tp.J0);
      tp.diag = (I == J);
      // kPacked: slot (a, bb) holds the pairs (I0 + a, J0 + 2bb) and
      // (I0 + a, J0 + 2bb + 1); a half outside the tile (ragged edge) or below the
      // diagonal is empty (orbital index -1).  Fully empty slots are not emitted.
      // kTiled: slot (a, b) holds the pair (I0 + a, J0 + b), b >= a on the diagonal.
      tp.s0 = (int)s.slots.size();
      if (packing == kTiled) {
        for (int a = 0; a < tp.nI; ++a)
          for (int b = tp.diag ? a : 0; b < tp.nJ; ++b) s.slots.push_back({tp.I0 + a, tp.J0 + b, -1, -1});
      }
      for (int a = 0; packing == kPacked && a < tp.nI; ++a)
        for (int bb = 0; 2 * bb < tp.nJ; ++bb) {
          Slot sl{-1, -1, -1, -1};
          for (int h = 0; h < 2; ++h) {
            const int b = 2 * bb + h;
            const bool ok = b < tp.nJ && (!tp.diag || b >= a);
            if (!ok) continue;
            (h ? sl.ib : sl.ia) = tp.I0 + a;
            (h ? sl.jb : sl.ja) = tp.J0 + b;
          }
          if (sl.ia >= 0 || sl.ib >= 0) s.slots.push_back(sl);
        }
      tp.s1 = (int)s.slots.size();
      tp.sys = 0;
      tp.eidx = (int)s.tiles.size();
      s.tiles.push_back(tp);
      round_of.push_back((int)r);
    }
  s.tile_round = round_of;
  // chunks of whole tile pairs whose slots fit the launch capacity; pass C
  // segments split chunks at round boundaries
  const int cap = std::max(batch_slots, packing == kTiled ? T * T : T * ((T + 1) / 2));
  chunk_tiles(s, cap);
}

void merge_schedules(const std::vector<const Schedule*>& parts, int cap, Schedule& out,
                     std::vector<int>& orb_base, std::vector<int>& tile_base) {
  out = Schedule();
  orb_base.assign(parts.size(), 0);
  tile_base.assign(parts.size(), 0);
  int rounds = 0, orbs = 0, tiles = 0;
  for (size_t k = 0; k < parts.size(); ++k) {
    orb_base[k] = orbs;
    tile_base[k] = tiles;
    orbs += parts[k]->n_orb;
    tiles += (int)parts[k]->tiles.size();
    rounds = std::max(rounds, parts[k]->n_rounds);
    out.n_pairs += parts[k]->n_pairs;
  }
  out.n_orb = orbs;
  out.n_rounds = rounds;
  out.tile = parts.empty() ? 0 : parts[0]->tile;
  out.batch_slots = cap;
  auto shift = [](int i, int b) { return i < 0 ? i : i + b; };
  int max_tile_slots = 1;
  for (int r = 0; r < rounds; ++r)
    for (size_t k = 0; k < parts.size(); ++k) {
      const Schedule& p = *parts[k];
      const int b = orb_base[k];
      for (size_t t = 0; t < p.tiles.size(); ++t) {
        if (p.tile_round[t] != r) continue;
        TilePair tp = p.tiles[t];
        const int s0 = (int)out.slots.size();
        for (int s = tp.s0; s < tp.s1; ++s) {
          const Slot& sl = p.slots[s];
          out.slots.push_back({shift(sl.ia, b), shift(sl.ja, b), shift(sl.ib, b), shift(sl.jb, b)});
        }
        tp.s0 = s0;
        tp.s1 = (int)out.slots.size();
        tp.I0 += b;
        tp.J0 += b;
        tp.sys = (int)k;
        tp.eidx = tile_base[k] + (int)t;
        max_tile_slots = std::max(max_tile_slots, tp.s1 - tp.s0);
        out.tiles.push_back(tp);
        out.tile_round.push_back(r);
      }
    }
  chunk_tiles(out, std::max(cap, max_tile_slots));
}

}  // namespace exx
