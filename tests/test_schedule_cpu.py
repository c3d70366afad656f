"""The pair schedule (host code of libexx) built with g++ and checked on the CPU.

* every unordered pair i <= j appears exactly once (N(N+1)/2 solves, Section 2);
* packed slots hold two pairs of the same tile pair (at most one half-empty
  slot per tile pair);
* the tile pairs of one pass-C launch (a segment) share no orbital, which is
  what lets pass C update K psi with plain read-modify-writes;
* chunks cover the slots contiguously and respect the slot capacity;
* with complex orbitals (one pair per slot) slot (a, b) of a tile pair holds
  (I0 + a, J0 + b), with the same round and chunk structure.
"""
import itertools
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "paper_1712_07973_amd", "csrc", "exx_schedule.cpp")


@pytest.fixture(scope="module")
def probe(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("sched") / "probe")
    r = subprocess.run(["g++", "-std=c++17", "-O1", "-o", exe,
                        os.path.join(HERE, "schedule_probe.cpp"), SRC],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


PLAIN, PACKED, TILED = 0, 1, 2  # slot packings of exx_schedule.hpp


def run(probe, N, T, cap, packed=True, packing=None):
    if packing is None:
        packing = PACKED if packed else PLAIN
    out = subprocess.run([probe, str(N), str(T), str(cap), str(packing)],
                         capture_output=True, text=True, check=True).stdout.split("\n")
    rec = {"S": [], "T": [], "C": [], "G": []}
    head = None
    for line in out:
        if not line:
            continue
        k, *v = line.split()
        if k == "P":
            head = tuple(int(x) for x in v)
        else:
            rec[k].append(tuple(int(x) for x in v))
    return head, rec


@pytest.mark.parametrize("N,T,cap", [(1, 8, 64), (5, 4, 3), (8, 8, 1 << 20), (32, 8, 1 << 20),
                                     (33, 8, 40), (37, 4, 17), (64, 8, 100), (96, 4, 1 << 20)])
def test_packed_schedule_invariants(probe, N, T, cap):
    head, r = run(probe, N, T, cap)
    assert head[0] == N * (N + 1) // 2
    pairs = []
    for ia, ja, ib, jb in r["S"]:
        if ia >= 0:
            pairs.append((ia, ja))
        if ib >= 0:
            pairs.append((ib, jb))
    assert sorted(pairs) == [(i, j) for i in range(N) for j in range(i, N)]
    # slots of a tile pair belong to it and follow the (row a, column pair bb)
    # layout: halves (I0+a, J0+2bb) and (I0+a, J0+2bb+1), rows in order
    for s0, s1, I0, nI, J0, nJ, diag in r["T"]:
        prev = (-1, -1)
        for ia, ja, ib, jb in r["S"][s0:s1]:
            assert ia >= 0 or ib >= 0
            a = (ia if ia >= 0 else ib) - I0
            bb = ((ja if ia >= 0 else jb) - J0) // 2
            assert (a, bb) > prev
            prev = (a, bb)
            for h, (i, j) in enumerate(((ia, ja), (ib, jb))):
                b = 2 * bb + h
                valid = b < nJ and (not diag or b >= a)
                assert (i >= 0) == valid
                if valid:
                    assert (i, j) == (I0 + a, J0 + b)
    # when T is even and tiles are full, off-diagonal slots are never half empty
    if N % T == 0 and T % 2 == 0:
        for s0, s1, I0, nI, J0, nJ, diag in r["T"]:
            if not diag:
                assert all(x[0] >= 0 and x[2] >= 0 for x in r["S"][s0:s1])
    # segments are orbital-disjoint
    for t0, t1 in r["G"]:
        seen = set()
        for s0, s1, I0, nI, J0, nJ, diag in r["T"][t0:t1]:
            orbs = set(range(I0, I0 + nI)) | set(range(J0, J0 + nJ))
            assert not (orbs & seen)
            seen |= orbs
    # chunks cover slots and tiles contiguously, within capacity when possible
    s_prev, t_prev = 0, 0
    for t0, t1, s0, s1, g0, g1 in r["C"]:
        assert t0 == t_prev and s0 == s_prev
        assert s1 - s0 <= max(cap, T * ((T + 1) // 2))
        assert r["G"][g0][0] == t0 and r["G"][g1 - 1][1] == t1
        t_prev, s_prev = t1, s1
    assert s_prev == len(r["S"]) and t_prev == len(r["T"])


def test_round_robin_round_count(probe):
    # nt tiles: one diagonal round plus nt-1 (even nt) or nt (odd nt) rounds
    for N, T in [(32, 8), (40, 8), (8, 8)]:
        nt = -(-N // T)
        head, _ = run(probe, N, T, 1 << 20)
        expect = 1 + (nt - 1 if nt % 2 == 0 else nt) if nt > 1 else 1
        assert head[2] == expect


def test_plain_schedule_is_one_pair_per_slot(probe):
    head, r = run(probe, 6, 0, 4, packed=False)
    assert [s[:2] for s in r["S"]] == [(i, j) for i in range(6) for j in range(i, 6)]
    assert all(s[2] == -1 for s in r["S"])
    assert [c[2:4] for c in r["C"]] == [(0, 4), (4, 8), (8, 12), (12, 16), (16, 20), (20, 21)]


@pytest.mark.parametrize("N,T,cap", [(1, 4, 64), (5, 4, 3), (8, 4, 1 << 20), (33, 4, 40),
                                     (37, 8, 17), (64, 8, 100)])
def test_single_pair_tiled_schedule_invariants(probe, N, T, cap):
    head, r = run(probe, N, T, cap, packing=TILED)
    assert head[0] == N * (N + 1) // 2
    assert all(s[2] == -1 and s[3] == -1 for s in r["S"])
    assert sorted(s[:2] for s in r["S"]) == [(i, j) for i in range(N) for j in range(i, N)]
    for s0, s1, I0, nI, J0, nJ, diag in r["T"]:
        expect = [(I0 + a, J0 + b) for a in range(nI) for b in range(nJ) if not diag or b >= a]
        assert [s[:2] for s in r["S"][s0:s1]] == expect
    for t0, t1 in r["G"]:
        seen = set()
        for s0, s1, I0, nI, J0, nJ, diag in r["T"][t0:t1]:
            orbs = set(range(I0, I0 + nI)) | set(range(J0, J0 + nJ))
            assert not (orbs & seen)
            seen |= orbs
    s_prev, t_prev = 0, 0
    for t0, t1, s0, s1, g0, g1 in r["C"]:
        assert t0 == t_prev and s0 == s_prev
        assert s1 - s0 <= max(cap, T * T)
        t_prev, s_prev = t1, s1
    assert s_prev == len(r["S"]) and t_prev == len(r["T"])


def test_odd_chunks_with_an_off_diagonal_tile_pair(probe):
    # five orbitals in tiles of 3 (sizes 3 and 2), at most 5 slots per launch
    # (raised to one full tile pair, 6): chunks of 5 and 5 slots, the second
    # holding the small diagonal tile pair and the ragged off-diagonal one; the
    # GPU test of odd pass A chunks above n = 64 relies on exactly this
    head, r = run(probe, 5, 3, 5)
    sizes = [s1 - s0 for (t0, t1, s0, s1, g0, g1) in r["C"]]
    assert sizes == [5, 5]
    t0, t1 = r["C"][1][:2]
    assert any(r["T"][t][6] == 0 for t in range(t0, t1))  # an off-diagonal tile pair
    off = [t for t in range(t0, t1) if r["T"][t][6] == 0][0]
    assert r["T"][off][1] - r["T"][off][0] == 3  # three rows of one column pair


def run_merged(probe, cap, packing, T, sizes):
    out = subprocess.run([probe, "merge", str(cap), str(packing), str(T), *map(str, sizes)],
                         capture_output=True, text=True, check=True).stdout.split("\n")
    rec = {"B": [], "S": [], "T": [], "C": [], "G": []}
    for line in out:
        if not line:
            continue
        k, *v = line.split()
        if k != "P":
            rec[k].append(tuple(int(x) for x in v))
    return rec


@pytest.mark.parametrize("packing", [PACKED, TILED])
@pytest.mark.parametrize("cap,T,sizes", [(40, 4, [5, 9, 3]), (1 << 20, 8, [22, 39, 67, 70]),
                                         (64, 8, [1, 2, 17, 8]), (3, 4, [7, 7])])
def test_merged_schedule_of_several_systems(probe, cap, T, sizes, packing):
    r = run_merged(probe, cap, packing, T, sizes)
    base = [b[0] for b in r["B"]]
    tbase = [b[1] for b in r["B"]]
    ntiles = [b[2] for b in r["B"]]
    assert base == [sum(sizes[:k]) for k in range(len(sizes))]
    # every pair of every system exactly once, in global indices of its own system
    seen = []
    for t in r["T"]:
        s0, s1, I0, nI, J0, nJ, diag, sys, eidx, rnd = t
        lo, hi = base[sys], base[sys] + sizes[sys]
        assert lo <= I0 < hi and lo <= J0 < hi and I0 + nI <= hi and J0 + nJ <= hi
        for sl in r["S"][s0:s1]:
            for i, j in (sl[:2], sl[2:]):
                if i < 0:
                    continue
                assert I0 <= i < I0 + nI and J0 <= j < J0 + nJ
                seen.append((sys, i - lo, j - lo))
    want = [(k, i, j) for k, N in enumerate(sizes) for i in range(N) for j in range(i, N)]
    assert sorted(seen) == sorted(want)
    # energy rows: system k owns tbase[k] .. tbase[k] + ntiles[k] - 1, one per tile pair
    for k in range(len(sizes)):
        rows = sorted(t[8] for t in r["T"] if t[7] == k)
        assert rows == list(range(tbase[k], tbase[k] + ntiles[k]))
    # rounds are in order, so every system's diagonal tile pairs (round 0) come
    # before its other tile pairs; a segment is one round and orbital-disjoint
    rounds = [t[9] for t in r["T"]]
    assert rounds == sorted(rounds)
    assert all(t[6] == (t[9] == 0) for t in r["T"])
    for g0, g1 in r["G"]:
        tiles = r["T"][g0:g1]
        assert len({t[9] for t in tiles}) == 1
        used = set()
        for t in tiles:
            orbs = set(range(t[2], t[2] + t[3])) | set(range(t[4], t[4] + t[5]))
            assert not (orbs & used)
            used |= orbs
    # chunks cover the tile pairs and slots contiguously within the capacity
    # (or one tile pair larger than it)
    t_next, s_next = 0, 0
    for t0, t1, s0, s1, g0, g1 in r["C"]:
        assert t0 == t_next and s0 == s_next and t1 > t0
        assert s1 - s0 <= cap or t1 == t0 + 1
        assert r["G"][g0][0] == t0 and r["G"][g1 - 1][1] == t1
        t_next, s_next = t1, s1
    assert t_next == len(r["T"]) and s_next == len(r["S"])


@pytest.mark.parametrize("R,G", [(1024, 64), (256, 128), (144, 5), (64, 1), (784, 3), (36, 7)])
def test_xcd_ordered_launch_map(probe, R, G):
    """The XCD-ordered grid of passes A and B covers every (item, slot group)
    once; for R a multiple of 8, the blocks one XCD receives (b = x mod 8) stay
    within its contiguous eighth of the items and take an item's slot groups in
    turn before the next item."""
    out = subprocess.run([probe, "xcd", str(R), str(G)], capture_output=True, text=True,
                         check=True).stdout.split()
    rows = [tuple(int(v) for v in out[k + 1:k + 4]) for k in range(0, len(out), 4)]
    assert len(rows) == R * G
    assert sorted((r, g) for _, r, g in rows) == [(r, g) for r in range(R) for g in range(G)]
    if R % 8:
        return
    for x in range(8):
        seq = [(r, g) for b, r, g in rows if b % 8 == x]
        assert all(x * (R // 8) <= r < (x + 1) * (R // 8) for r, _ in seq)
        assert seq == sorted(seq)  # item-major, slot groups fastest
