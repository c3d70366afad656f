// Prints the pair schedule for (n_orb, tile, batch_slots, packing) as text, for
// the host-side schedule tests:  S ia ja ib jb / T s0 s1 I0 nI J0 nJ diag /
// C t0 t1 s0 s1 seg0 seg1 / G t0 t1.  With "merge" first, the merged schedule
// of several systems (B orb_base tile_base n_tiles per system; T lines add sys,
// eidx and the round); with "xcd R G", the XCD-ordered launch map.
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../paper_1712_07973_amd/csrc/exx_schedule.hpp"

static int merged(int argc, char** argv) {
  // merge <cap> <packing> <tile> <n_orb of system 0> <n_orb of system 1> ...
  const int cap = std::atoi(argv[2]), packing = std::atoi(argv[3]), T = std::atoi(argv[4]);
  std::vector<exx::Schedule> parts(argc - 5);
  std::vector<const exx::Schedule*> ptrs;
  for (int k = 5; k < argc; ++k) {
    exx::build_schedule_host(std::atoi(argv[k]), T, cap, packing, parts[k - 5]);
    ptrs.push_back(&parts[k - 5]);
  }
  exx::Schedule s;
  std::vector<int> ob, tb;
  exx::merge_schedules(ptrs, cap, s, ob, tb);
  std::printf("P %lld %d %d\n", s.n_pairs, s.tile, s.n_rounds);
  for (size_t k = 0; k < ob.size(); ++k) std::printf("B %d %d %d\n", ob[k], tb[k], (int)parts[k].tiles.size());
  for (auto& x : s.slots) std::printf("S %d %d %d %d\n", x.ia, x.ja, x.ib, x.jb);
  for (size_t i = 0; i < s.tiles.size(); ++i) {
    const auto& t = s.tiles[i];
    std::printf("T %d %d %d %d %d %d %d %d %d %d\n", t.s0, t.s1, t.I0, t.nI, t.J0, t.nJ, t.diag, t.sys, t.eidx,
                s.tile_round[i]);
  }
  for (auto& c : s.chunks) std::printf("C %d %d %d %d %d %d\n", c.t0, c.t1, c.s0, c.s1, c.seg0, c.seg1);
  for (auto& g : s.segments) std::printf("G %d %d\n", g.t0, g.t1);
  return 0;
}

int main(int argc, char** argv) {
  if (argc >= 6 && std::string(argv[1]) == "merge") return merged(argc, argv);
  if (argc == 4 && std::string(argv[1]) == "xcd") {
    // xcd <R> <G>: the launch order, one line X b r g per block
    const int R = std::atoi(argv[2]), G = std::atoi(argv[3]);
    for (int b = 0; b < R * G; ++b) {
      int r = -1, g = -1;
      exx::xcd_split(b, R, G, r, g);
      std::printf("X %d %d %d\n", b, r, g);
    }
    return 0;
  }
  if (argc < 5) return 2;
  int N = std::atoi(argv[1]), T = std::atoi(argv[2]), cap = std::atoi(argv[3]);
  int packing = std::atoi(argv[4]);  // exx::Packing
  exx::Schedule s;
  exx::build_schedule_host(N, T, cap, packing, s);
  std::printf("P %lld %d %d\n", s.n_pairs, s.tile, s.n_rounds);
  for (auto& x : s.slots) std::printf("S %d %d %d %d\n", x.ia, x.ja, x.ib, x.jb);
  for (auto& t : s.tiles) std::printf("T %d %d %d %d %d %d %d\n", t.s0, t.s1, t.I0, t.nI, t.J0, t.nJ, t.diag);
  for (auto& c : s.chunks) std::printf("C %d %d %d %d %d %d\n", c.t0, c.t1, c.s0, c.s1, c.seg0, c.seg1);
  for (auto& g : s.segments) std::printf("G %d %d\n", g.t0, g.t1);
  return 0;
}
