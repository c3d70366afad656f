// Prints the pair schedule for (n_orb, tile, batch_slots, packing) as text, for
// the host-side schedule tests:  S ia ja ib jb / T s0 s1 I0 nI J0 nJ diag /
// C t0 t1 s0 s1 seg0 seg1 / G t0 t1
#include <cstdio>
#include <cstdlib>

#include "../paper_1712_07973_amd/csrc/exx_schedule.hpp"

int main(int argc, char** argv) {
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
