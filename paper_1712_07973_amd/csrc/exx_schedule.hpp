// exx_schedule.hpp -- pair schedule of one evaluation (host only, no HIP).
#pragma once

#include <utility>
#include <vector>

namespace exx {

// One packed slot = two unordered pairs (ia, ja) and (ib, jb) sharing one
// complex transform (real part: pair a, imaginary part: pair b); a negative
// orbital index marks an empty half.  Within a pair tile the slot of row a and
// column pair bb holds (I0 + a, J0 + 2bb) and (I0 + a, J0 + 2bb + 1).  With
// complex orbitals a slot holds one pair (ia, ja) (the b half is empty) and the
// slot of row a and column b holds (I0 + a, J0 + b).
struct Slot {
  int ia, ja, ib, jb;
};

// One pair tile: orbitals [I0, I0+nI) x [J0, J0+nJ) (upper triangle when
// diag), its slots [s0, s1).  sys: the system of a merged batch schedule (0
// otherwise); eidx: the row of its energy partials (the tile index within its
// system plus the system's first row).
struct TilePair {
  int s0, s1, I0, nI, J0, nJ, diag, sys, eidx, pad;
};

struct Schedule {
  int n_orb = 0;
  int tile = 0;
  int batch_slots = 0;
  long long n_pairs = 0;
  std::vector<Slot> slots;
  std::vector<TilePair> tiles;
  // launch chunks: tiles [t0, t1) with slots [s0, s1); pass C is launched once
  // per segment [seg0, seg1) of `segments`, each a run of orbital-disjoint tiles
  struct Chunk {
    int t0, t1, s0, s1, seg0, seg1;
  };
  struct Segment {
    int t0, t1;
  };
  std::vector<Chunk> chunks;
  std::vector<Segment> segments;
  std::vector<int> tile_round;  // round of each tile pair
  int n_rounds = 0;
  Slot* d_slots = nullptr;
  TilePair* d_tiles = nullptr;
};

// Slot packing of a schedule.
enum Packing {
  kPlain = 0,   // one pair per slot in (i <= j) order, chunks of batch_slots (the plain path)
  kPacked = 1,  // tiles of edge `tile`, tile pairs in round-robin rounds, two real pairs
                // per slot, chunks of whole tile pairs within batch_slots
  kTiled = 2    // as kPacked with one pair per slot (complex orbitals)
};

// Builds the schedule for n_orb orbitals.
void build_schedule_host(int n_orb, int tile, int batch_slots, int packing, Schedule& s);

// One schedule over several systems of one grid (a batch's grid class): the
// tile pairs of round r of every system, system by system, then round r + 1,
// so that one pass C launch covers a round of every system.  Orbital indices
// become indices into the systems' orbitals laid end to end (system k's
// orbital i is orb_base[k] + i); each tile pair keeps its system in `sys` and
// its energy row tile_base[sys] + (its index in that system's schedule) in
// `eidx`.  Chunks hold whole tile pairs within `cap` slots (at least one tile
// pair), split into segments at round boundaries as in build_schedule_host.
// The per-system schedules must share one packing.
void merge_schedules(const std::vector<const Schedule*>& parts, int cap, Schedule& out,
                     std::vector<int>& orb_base, std::vector<int>& tile_base);

// Rounds of a round-robin tournament over nt tiles; the first round holds the
// diagonal pairs (I, I).  No two pairs of one round share a tile.
std::vector<std::vector<std::pair<int, int>>> tile_rounds(int nt);

// Launch order of a one-dimensional grid over R items (row blocks or slabs)
// times G slot groups: block b -> (item r, slot group g).  Workgroups are dealt
// to the device's XCDs in turn (b mod kXcds); each XCD takes a contiguous share
// of R / kXcds items and walks the slot groups of one item before the next.  A
// bijection of [0, R G) onto the pairs; for R not a multiple of kXcds, slot
// groups fastest over the whole grid.  (Used by the kernels; constexpr so that
// host code can check it.)
constexpr int kXcds = 8;
constexpr void xcd_split(int b, int R, int G, int& r, int& g) {
  if (R % kXcds == 0) {
    const int x = b % kXcds, i = b / kXcds;
    g = i % G;
    r = x * (R / kXcds) + i / G;
  } else {
    g = b % G;
    r = b / G;
  }
}

}  // namespace exx
