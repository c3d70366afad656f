#!/usr/bin/env python3
"""Benchmark of the exact-exchange hot path on one MI355X.

One step = one full evaluation of E_x and K psi (pair build, forward
transforms, kernel multiply, inverse transforms, FP64 pair energies and
K psi) for every orbital pair of one synthetic system, with inputs already
resident in HBM.  Default workload: isolated system, 128^3 grid zero-padded
to 256^3, h = 0.4 bohr, 256 Loewdin-orthonormalised Gaussian orbitals (the
last 16 fractionally occupied), truncated Coulomb kernel with R = L, i.e.
32 896 pair Poisson solves per step.

Prints one JSON line: pair-solves/s of the FP32 path (value), the plain FP64
GPU path beside it (on a labelled orbital subset when the full system would
take long, with the FP32 path's accuracy against it on that subset), per-pass
device times from hipEvents recorded on the compute stream, the roofline of
the dominant kernel (its algorithmic bytes per launch over its measured
launch time, against the HBM peak), and the FP64 CPU oracle's rate on a
bounded sample at one core and at all cores.  The timed steps are eager
calls; --graph times replays of one evaluation captured in a HIP graph
instead (the eager rate is then reported beside it).
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, datasheet
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X vector FP32, datasheet
METRIC = "orbital-pair Poisson solves/s (E_x+Kψ) FP32-batched vs FP64, HBM GB/s"


CLASSES = {"free": (2, 2, 2), "surface": (1, 1, 2), "wire": (2, 2, 1),
           "periodic": (1, 1, 1)}  # parity classes per axis x, y, z
# the classes as the FP32 passes see them: the wire runs with y and z exchanged
PASS_CLASSES = dict(CLASSES, wire=(2, 1, 2))


def algorithmic_bytes(n: int, ncls: int, n_orb: int, n_slots: int, cplx: bool = False) -> dict:
    """Minimum HBM bytes of each pass of one evaluation (FP32 path).

    Per slot (two real pairs, or one complex pair) the spectrum X holds
    ncls * n^3 complex FP32 values: pass A writes it, pass B reads and
    rewrites it, pass C reads it.  The orbitals (FP32 copy) are read once by
    A and once by C; K psi (FP64) is written once; complex orbitals double
    both.  Pass B's kernel table is shared by all slots (cache resident) and
    not counted.
    """
    v = 2 if cplx else 1  # reals per orbital value
    x = ncls * n ** 3 * 8
    orb32 = n_orb * n ** 3 * 4 * v
    kps = n_orb * n ** 3 * 8 * v
    return {
        "convert": n_orb * n ** 3 * (8 + 4) * v,
        "pass_a": n_slots * x + orb32,
        "pass_b": n_slots * 2 * x,
        "pass_c": n_slots * x + orb32 + kps,
    }


def model_a_bytes(n: int, grid_classes: tuple, pairs: int, cplx: bool = False) -> dict:
    """Algorithmic HBM bytes of the spectrum in the two-round-trip pipeline.

    Pass A writes the spectrum half-way through the forward transform (x and
    y done), pass B reads it, transforms z, multiplies by the kernel,
    transforms back along z and writes it, pass C reads it.  Two real pairs
    share one complex FP32 array, so a real pair costs 4 bytes per complex
    point (a complex pair 8); the spectrum holds cx cy n^3 points (cx, cy the
    x and y parity classes of the grid, the z axis pruned to the data's n
    planes).  The orbital and K psi traffic, amortised over a pair tile, is
    left out.  These are the bytes the roofline of each pass is quoted on.
    """
    cx, cy, _ = grid_classes
    w = (8 if cplx else 4) * cx * cy * n ** 3 * pairs
    return {"pass_a": w, "pass_b": 2 * w, "pass_c": w}


def fft_flops(n: int, classes: tuple, n_slots: int) -> dict:
    """Nominal 5 L log2 L flops per complex n-point line transform, per pass.

    classes = (cx, cy, cz) parity classes per axis as pass B sees them.  Pass
    A/C: cx x-classes of n^2 lines.  Pass B, per slab (cx n slabs per slot) of
    n^2 points: with two z classes the y-transforms are shared by both (in
    one launch or through the split form's scratch): cy y-line sets forward and
    inverse plus cy cz z-line sets forward and inverse, 2n cy (1 + cz) lines;
    with one z class 4 n cy lines.
    """
    cx, cy, cz = classes
    f = 5.0 * n * math.log2(n)
    a = n_slots * cx * n * n * f
    per_slab = 2 * n * cy * (1 + cz) if cz == 2 else 4 * n * cy * cz
    b = n_slots * cx * n * per_slab * f
    c = n_slots * cx * n * n * f
    return {"pass_a": a, "pass_b": b, "pass_c": c}


PASS_SECTIONS = {"pass_a": ("// pass A:", "// pass B:"), "pass_b": ("// pass B:", "// pass C:"),
                 "pass_c": ("// pass C:", "// pair-energy partials:")}


def kernel_source_sha1(kernel: str) -> str:
    """SHA-1 of the kernel's section of exx_fused.hip, the helpers ahead of
    pass A (spectrum layout, shared device functions) and the DFT header."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1712_07973_amd", "csrc")
    with open(os.path.join(csrc, "exx_fused.hip")) as f:
        text = f.read()
    a, b = PASS_SECTIONS[kernel]
    section = text[:text.index(PASS_SECTIONS["pass_a"][0])] + text[text.index(a):text.index(b)]
    with open(os.path.join(csrc, "exx_fft.hpp")) as f:
        section += f.read()
    return hashlib.sha1(section.encode()).hexdigest()


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed counter summary.

    profiles/<kernel>_<workload>_traffic.json holds FETCH_SIZE and WRITE_SIZE
    per dispatch (rocprofv3 --pmc) scaled by what the same counters read for
    a device copy of known size; it is used only while the kernel source is
    unchanged since the counters were taken (else None).
    """
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_sha1") != kernel_source_sha1(kernel):
        return None
    return t.get("hbm_bytes_per_launch")


def _time_loop(run, steps):
    """ms per step over `steps` calls of run() (hipEvents on the current stream),
    the median step and the host wall time."""
    import torch
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    if torch.distributed.is_available() and torch.distributed.is_initialized():
        torch.distributed.barrier()
    torch.cuda.synchronize()
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(steps - 1)]
    t_host = time.perf_counter()
    e0.record(stream)
    for k in range(steps):
        run()
        if k < steps - 1:
            marks[k].record(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_host
    edges = [e0] + marks + [e1]
    per_step = sorted(edges[k].elapsed_time(edges[k + 1]) for k in range(steps))
    median = (per_step[(steps - 1) // 2] + per_step[steps // 2]) / 2
    return e0.elapsed_time(e1) / steps, median, wall


def timed(plan, psi, occ, kpsi, ex, steps, warmup, use_graph=False):
    """Times `steps` evaluations after `warmup` untimed ones, with no per-launch
    events inside the timed region.  use_graph: the evaluation is captured once
    into a HIP graph (torch.cuda.graph on the plan's stream) and the timed steps
    are replays of it, as an iteration loop over fixed buffers would run it; the
    eager rate is timed too.  Then `steps` more eager evaluations with the plan's
    per-pass hipEvents give the pass breakdown."""
    import torch

    def eager():
        plan.compute(psi, occ, "energy_kpsi", kpsi=kpsi, ex_out=ex)

    for _ in range(warmup):
        eager()
    torch.cuda.synchronize()
    eager_ms, eager_median, eager_wall = _time_loop(eager, steps)
    ms, median, wall = eager_ms, eager_median, eager_wall
    if use_graph:
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            eager()
        for _ in range(warmup):
            graph.replay()
        torch.cuda.synchronize()
        ms, median, wall = _time_loop(graph.replay, steps)
    # pass breakdown: eager evaluations with an event pair around every launch
    plan.enable_profiling(True)
    plan.read_profile()
    for _ in range(steps):
        eager()
    torch.cuda.synchronize()
    prof = plan.read_profile()
    plan.enable_profiling(False)
    prof["_median_ms"] = median
    prof["_eager_ms"] = eager_ms
    return ms, wall, prof


def workload_text(sysm, pairs: int) -> str:
    """What the single-system workload is, with its sizes."""
    n, h, N = sysm.n, sysm.h, sysm.n_orb
    L = n * h
    rtxt = f"R=L={L:g} bohr" if abs(sysm.R - L) < 1e-12 * L else \
        f"R=sqrt(3)L={sysm.R:g} bohr (box diagonal; aliases on the padded grid)"
    geom = {"free": f"free-BC {n}^3 grid padded to {2 * n}^3, h={h} bohr, {rtxt}",
            "surface": f"surface (periodic x, y; isolated z) {n}^3 grid padded to {n}x{n}x{2 * n}, "
                       f"h={h} bohr, R=L={L:g} bohr",
            "wire": f"wire (isolated x, y; periodic z) {n}^3 grid padded to {2 * n}x{2 * n}x{n}, "
                    f"h={h} bohr, R=L={L:g} bohr",
            "periodic": f"periodic {n}^3 grid, h={h} bohr"}[sysm.bc]
    occ = "occupations 2" if float(sysm.occ.min()) == float(sysm.occ.max()) == 2.0 \
        else "occupations 2 with fractional tail"
    kind = (f"complex (phases |k| <= {sysm.recipe.kmax:g} bohr^-1) " if sysm.psi.dtype.kind == "c"
            else "")
    return (f"{geom}, {N} Loewdin-orthonormalised {kind}Gaussian orbitals, {occ}, "
            f"{pairs} pair solves, E_x + K psi")


def copy_bandwidth(dev, reps: int = 5) -> float:
    """Device-to-device copy rate of 1 GiB (bytes read + bytes written per second)."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * src.numel() * 4 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def autograd_times(grid, psi, occ, reps: int = 5) -> dict:
    """Median forward (E_x only) and backward (recomputed K psi) times of exchange_energy."""
    import torch

    import paper_1712_07973_amd as exx
    x = psi.clone().requires_grad_(True)
    for _ in range(2):
        exx.exchange_energy(x, occ, grid).backward()
        x.grad = None
    torch.cuda.synchronize()
    fwd, bwd = [], []
    for _ in range(reps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record()
        y = exx.exchange_energy(x, occ, grid)
        ev[1].record()
        y.backward()
        ev[2].record()
        torch.cuda.synchronize()
        fwd.append(ev[0].elapsed_time(ev[1]))
        bwd.append(ev[1].elapsed_time(ev[2]))
        x.grad = None
    fwd.sort()
    bwd.sort()
    return {"forward_ms": round(fwd[reps // 2], 4), "backward_ms": round(bwd[reps // 2], 4),
            "forward": "E_x only (Parseval, no pass C)",
            "backward": "K psi recomputed, gradient -2 f h^3 K psi"}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sysm, n_sample: int) -> dict:
    """The FP64 oracle as it stands, timed on the first n_sample orbitals (every
    pair among them, E_x and K psi) with scipy.fft on all host cores (at most
    16) and on one core."""
    import oracle
    from oracle import exx_oracle
    psi = sysm.psi[:n_sample].copy()
    occ = sysm.occ[:n_sample].copy()
    pairs = n_sample * (n_sample + 1) // 2
    cores = min(16, os.cpu_count() or 1)
    rate = {}
    for workers in (cores, 1):
        exx_oracle._WORKERS = workers
        t0 = time.perf_counter()
        oracle.exx(psi, occ, sysm.h, sysm.bc, R=sysm.R, symmetric=True)
        rate[workers] = (pairs / (time.perf_counter() - t0), time.perf_counter() - t0)
    return {"value": rate[cores][0], "unit": "pair-solves/s", "cores": cores, "kind": "oracle",
            "sample": f"all {pairs} pairs of the first {n_sample} of {sysm.n_orb} orbitals "
                      f"(E_x and K psi), scipy.fft FP64: {rate[cores][1]:.1f} s with "
                      f"workers={cores}, {rate[1][1]:.1f} s with workers=1",
            "one_core": {"value": rate[1][0], "cores": 1}, "cpu_model": cpu_model()}


def bench_batch(a, dev) -> int:
    """Batches of uneven isolated systems in one captured HIP graph (FP32 path):
    16 systems of n in {48..112} (batch16_free) or 48 small ones of n in
    {32, 48} (batch48_small); with the plans' default tunings, or tuned per grid
    class by exx_batch_autotune first when --batch-tune-ms is given; with
    --merge, systems on one grid share their launches (EXX_BATCH_MERGE), and the
    line also reports the unmerged batch measured the same way."""
    import torch

    import paper_1712_07973_amd as exx
    from exx_inputs import batch_recipes, make_system, pair_count, small_batch_recipes
    small = a.workload == "batch48_small"
    systems = [make_system(r) for r in (small_batch_recipes() if small else batch_recipes())]
    grids = [exx.Grid(n=s.n, h=s.h, bc=s.bc, R=s.R) for s in systems]
    psis = [torch.from_numpy(s.psi).to(dev) for s in systems]
    occs = [torch.from_numpy(s.occ).to(dev) for s in systems]
    pairs = sum(pair_count(s.n_orb) for s in systems)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)

    def run(merge):
        b = exx.Batch(grids, [s.n_orb for s in systems], "fp32", use_graph=True, merge=merge)
        t0 = time.perf_counter()
        tun = (b.autotune(psis, occs, budget_ms=a.batch_tune_ms) if a.batch_tune_ms > 0 and not merge
               else b.tunings())
        tune_s = time.perf_counter() - t0
        outs = None
        for _ in range(max(1, a.warmup)):
            outs = b.compute(psis, occs, outputs=outs)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(a.steps):
            b.compute(psis, occs, outputs=outs)
        e1.record(stream)
        torch.cuda.synchronize()
        E = [float(o[0].item()) for o in outs]
        del b, outs
        torch.cuda.empty_cache()
        return e0.elapsed_time(e1) / a.steps, tun, tune_s, E

    ms, tunings, tune_s, E_x = run(a.merge)
    other = run(False) if a.merge else None
    model = sum(sum(model_a_bytes(s.n, CLASSES[s.bc], pair_count(s.n_orb)).values()) for s in systems)
    gbs = model / (ms * 1e-3) / 1e9
    out = {"metric": METRIC, "value": round(pairs / (ms * 1e-3), 1), "unit": "pair-solves/s",
           "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": (("48 isolated systems, n in {32, 48} padded to 2n, N in [4,16]"
                                    if small else
                                    "16 isolated systems, n in {48..112} padded to 2n, N in [16,96]")
                                   + ", one captured HIP graph per evaluation"
                                   + (", systems on one grid sharing launches" if a.merge else "")),
                      "preset": a.workload, "merge": bool(a.merge),
                      "pairs": pairs, "systems": [[s.n, s.n_orb] for s in systems],
                      "tunings": tunings, "autotune_s": round(tune_s, 1)},
           "roofline": {"bound": "hbm", "kernel": "whole evaluation (every pass of every system)",
                        "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                        "bytes_per_launch": int(model),
                        "bytes_model": "two spectrum round trips, 4 B per real pair per complex "
                                       "point, cx cy n^3 points (z pruned)"},
           "E_x": E_x}
    if other is not None:
        out["unmerged"] = {"value": round(pairs / (other[0] * 1e-3), 1), "ms_per_step": round(other[0], 3),
                           "E_x_equal": other[3] == E_x}
    if not a.no_baselines:
        # FP64 leg: the plain path on the systems of n <= 64 (a labelled subset),
        # one plan per system called in turn, with the FP32 path on the same
        # systems the same way for the accuracy and a like-for-like rate
        sub = [k for k, s in enumerate(systems) if s.n <= 64]
        sp = sum(pair_count(systems[k].n_orb) for k in sub)
        rates = {}
        for prec in ("fp32", "fp64_plain"):
            plans = [exx.Plan(grids[k], prec, n_orb_max=systems[k].n_orb) for k in sub]
            outs_p = [p.compute(psis[k], occs[k], "energy_kpsi") for p, k in zip(plans, sub)]
            torch.cuda.synchronize()
            e0.record(stream)
            reps = 3 if prec == "fp32" else 1
            for _ in range(reps):
                for p, k in zip(plans, sub):
                    p.compute(psis[k], occs[k], "energy_kpsi")
            e1.record(stream)
            torch.cuda.synchronize()
            rates[prec] = (sp / (e0.elapsed_time(e1) / reps * 1e-3), [float(o[0].item()) for o in outs_p])
            del plans, outs_p
            torch.cuda.empty_cache()
        out["fp64_plain"] = {"value": round(rates["fp64_plain"][0], 1),
                             "subset": {"systems": [[systems[k].n, systems[k].n_orb] for k in sub],
                                        "pairs": sp, "fp32_value": round(rates["fp32"][0], 1),
                                        "calls": "one plan per system, called in turn"}}
        out["accuracy_vs_fp64_plain"] = {"dE_x_per_orbital_Ha_max": max(
            abs(e32 - e64) / systems[k].n_orb
            for k, e32, e64 in zip(sub, rates["fp32"][1], rates["fp64_plain"][1]))}
        out["speedup_vs_fp64_plain"] = round(rates["fp32"][0] / rates["fp64_plain"][0], 2)
    if not a.no_cpu_baseline:
        big = max(range(len(systems)), key=lambda k: systems[k].n)
        out["cpu_baseline"] = cpu_baseline(systems[big], a.cpu_sample or 3)
        out["cpu_baseline"]["sample"] += f" (system {big}: n = {systems[big].n})"
    print(json.dumps(out), flush=True)
    return 0


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="free128_n256")
    ap.add_argument("--baseline-steps", type=int, default=3)
    ap.add_argument("--no-baselines", action="store_true", help="skip the FP64 GPU paths")
    ap.add_argument("--fp64-orbitals", type=int, default=0,
                    help="orbitals of the FP64 legs (0: all when they take under ~2 s, else "
                         "the first 32)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="orbitals of the oracle sample (0: 12 up to n = 64, 5 up to n = 96, "
                         "else 3)")
    ap.add_argument("--slab-threads", type=int, default=0,
                    help="threads per slab workgroup of the y/z pass (0: plan default)")
    ap.add_argument("--tile", type=int, default=0, help="pair-tile edge (0: plan default)")
    ap.add_argument("--batch-slots", type=int, default=0,
                    help="slots per launch chunk (0: plan default)")
    ap.add_argument("--slab-form", default="0", choices=["0", "shared", "wave"],
                    help="form of the y/z pass (0: plan default)")
    ap.add_argument("--streams", type=int, default=0,
                    help="1: serial passes, 3: overlapped rounds (0: plan default)")
    ap.add_argument("--graph", action="store_true",
                    help="time replays of one evaluation captured in a HIP graph (measured within "
                         "0.5 %% of eager calls at the default workload)")
    ap.add_argument("--batch-tune-ms", type=int, default=0,
                    help="autotuning budget of the batch workload (0: plan defaults)")
    ap.add_argument("--radius", default="box", choices=["box", "diagonal"],
                    help="free-BC truncation radius: box (R = L = n h, the default) or diagonal "
                         "(R = sqrt(3) L; the 2n-padded grid then aliases periodic images)")
    ap.add_argument("--merge", action="store_true",
                    help="batch workloads: systems on one grid share their launches")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 1 GiB device-to-device 3 times (calibrates memory counters)")
    a = ap.parse_args(argv)

    if a.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {a.gpus} is not supported "
              "(the exchange path here is single-device).", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1712_07973_amd as exx
    from exx_inputs import pair_count, system

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if a.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_per_launch": src.numel() * 4, "launches": 3}))
        return 0
    if a.workload in ("batch16_free", "batch48_small"):
        return bench_batch(a, dev)
    sysm = system(a.workload)
    N, n = sysm.n_orb, sysm.n
    if a.radius == "diagonal":
        if sysm.bc != "free":
            print("--radius diagonal applies to free-BC workloads only", file=sys.stderr)
            return 2
        sysm = dataclasses.replace(sysm, R=math.sqrt(3.0) * n * sysm.h)
    pairs = pair_count(N)
    classes = CLASSES[sysm.bc]
    ncls = classes[0]
    grid = exx.Grid(n=n, h=sysm.h, bc=sysm.bc, R=sysm.R if sysm.bc != "periodic" else None)
    psi = torch.from_numpy(sysm.psi).to(dev)
    occ = torch.from_numpy(sysm.occ).to(dev)
    kpsi = torch.empty_like(psi)
    ex = torch.empty((), dtype=torch.float64, device=dev)
    cplx = psi.is_complex()

    plan = exx.Plan(grid, "fp32", n_orb_max=N, complex_orbitals=cplx)
    plan.set_tuning(tile=a.tile, slab_threads=a.slab_threads, batch_slots=a.batch_slots,
                    streams=a.streams, slab_form=0 if a.slab_form == "0" else a.slab_form)
    plan.workspace(N)
    _, n_slots = plan.schedule_info(N)
    ms, wall, prof = timed(plan, psi, occ, kpsi, ex, a.steps, a.warmup, use_graph=a.graph)
    value = pairs / (ms * 1e-3)
    E32 = float(ex.item())
    K32 = kpsi.clone()

    median_ms = prof.pop("_median_ms")
    eager_ms = prof.pop("_eager_ms")
    # dominant kernel and its roofline
    passes = {k: v for k, v in prof.items() if v[1] > 0}
    dom = max(("pass_a", "pass_b", "pass_c"), key=lambda k: passes.get(k, (0, 0))[0])
    dom_ms, dom_launches = passes[dom]
    per_launch_ms = dom_ms / dom_launches
    launches_per_step = dom_launches / a.steps
    model = model_a_bytes(n, classes, pairs, cplx)
    own = algorithmic_bytes(n, ncls, N, n_slots, cplx)
    flops = fft_flops(n, PASS_CLASSES[sysm.bc], n_slots)
    bytes_per_launch = model[dom] / launches_per_step
    achieved_gbs = bytes_per_launch / (per_launch_ms * 1e-3) / 1e9
    own_per_launch = own[dom] / launches_per_step
    own_gbs = own_per_launch / (per_launch_ms * 1e-3) / 1e9
    achieved_tflops = flops[dom] / launches_per_step / (per_launch_ms * 1e-3) / 1e12
    traffic = measured_traffic(dom, a.workload)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved_gbs, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved_gbs / HBM_PEAK_GBS, 4),
                "traffic": traffic, "launch_ms": round(per_launch_ms, 4),
                "bytes_per_launch": int(bytes_per_launch),
                "bytes_model": "two spectrum round trips, 4 B per real pair per complex point, "
                               "cx cy n^3 points (z pruned)",
                "own_minimum": {"bytes_per_launch": int(own_per_launch),
                                "achieved": round(own_gbs, 1),
                                "frac": round(own_gbs / HBM_PEAK_GBS, 4),
                                "note": "the y,z spectrum never leaves the chip: pass B moves the "
                                        "x-transformed slabs once each way"},
                "fp32_flops": {"achieved": round(achieved_tflops, 2),
                               "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                               "frac": round(achieved_tflops / FP32_VECTOR_PEAK_TFLOPS, 4),
                               "flops": "nominal 5 L log2 L per complex line transform"}}
    if achieved_gbs > HBM_PEAK_GBS:
        # a pass that beats the two-round-trip pipeline's own memory bound
        roofline["frac_note"] = ("above 1: the dominant pass finishes faster than the Model-A "
                                 "pipeline could move its bytes at peak; this design's pass moves "
                                 "own_minimum bytes (the padded spectrum never leaves the chip)")
    whole_model = sum(model.values())

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "pair-solves/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(ms, 4),
        "ms_per_step_median": round(median_ms, 4),
        "timing": "replays of one evaluation captured in a HIP graph (same kernels and launches)"
                  if a.graph else "eager evaluations",
        "eager_ms_per_step": round(eager_ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload_text(sysm, pairs),
                   "preset": a.workload, "n": n,
                   "fft_grid": [c * n for c in classes], "n_orb": N,
                   "orbitals": "complex" if cplx else "real", "pairs": pairs,
                   "slots": n_slots, "pairs_per_slot": 1 if cplx else 2,
                   "tuning": plan.tuning},
        "roofline": roofline,
        "whole_step_model_GBs": round(whole_model / (ms * 1e-3) / 1e9, 1),
        "passes_ms_per_step": {k: round(v[0] / a.steps, 4) for k, v in passes.items()},
        "host_wall_ms_per_step": round(wall * 1e3 / a.steps, 4),
        "E_x": E32,
    }
    if N <= 8:
        out["us_per_call"] = round(ms * 1e3, 1)
    if a.radius == "diagonal":
        gbox = exx.Grid(n=n, h=sysm.h, bc=sysm.bc, R=n * sysm.h)
        pbox = exx.Plan(gbox, "fp32", n_orb_max=N, complex_orbitals=cplx)
        ebox, _, _ = pbox.compute(psi, occ, "energy")
        out["radius_reading"] = {
            "R_bohr": sysm.R, "E_x": E32, "E_x_with_R_eq_L": float(ebox.item()),
            "relative_difference": abs(E32 - float(ebox.item())) / abs(float(ebox.item())),
            "note": "R = box diagonal read literally; on a 2n-padded grid the truncated kernel "
                    "then reaches periodic images, so R = L is the default"}
        del pbox

    if not a.no_baselines:
        # FP64 legs: every orbital when the plain path is quick, else a labelled
        # subset (its rate per pair hardly depends on the orbital count: one pair
        # per transform), with the FP32 path run on the same subset for the
        # accuracy and a like-for-like rate
        plain_pair_ms = 0.9 * (n / 128) ** 3 * (8 if sysm.bc == "free" else 2)
        N64 = a.fp64_orbitals or (N if pair_count(N) * plain_pair_ms < 2000 else 32)
        N64 = min(N64, N)
        sub = {"orbitals": N64, "pairs": pair_count(N64),
               "which": "all" if N64 == N else f"the first {N64} of {N}"}
        psi_s, occ_s = psi[:N64].contiguous(), occ[:N64].contiguous()
        k32s = torch.empty_like(psi_s)
        e32s = torch.empty((), dtype=torch.float64, device=dev)
        if N64 == N:
            k32s.copy_(K32)
            e32s.fill_(E32)
            sub["fp32_value"] = round(value, 1)
        else:
            p32s = exx.Plan(grid, "fp32", n_orb_max=N64, complex_orbitals=cplx)
            ms32s, _, _ = timed(p32s, psi_s, occ_s, k32s, e32s, a.baseline_steps, 1)
            sub["fp32_value"] = round(pair_count(N64) / (ms32s * 1e-3), 1)
            del p32s
        precs = ["fp64_plain"] + (["fp64_fused"] if n <= 96 else [])
        for prec in precs:
            p64 = exx.Plan(grid, prec, n_orb_max=N64, complex_orbitals=cplx)
            p64.workspace(N64)
            k64 = torch.empty_like(psi_s)
            e64 = torch.empty((), dtype=torch.float64, device=dev)
            ms64, _, _ = timed(p64, psi_s, occ_s, k64, e64, a.baseline_steps, 1, use_graph=a.graph)
            out[prec] = {"value": round(pair_count(N64) / (ms64 * 1e-3), 1),
                         "ms_per_step": round(ms64, 3), "subset": sub}
            if prec == "fp64_plain":
                E64 = float(e64.item())
                E32s = float(e32s.item())
                d = (k32s - k64).reshape(N64, -1)
                ref = k64.reshape(N64, -1)
                num = torch.linalg.vector_norm(d, dim=1)
                den = torch.linalg.vector_norm(ref, dim=1)
                out["accuracy_vs_fp64_plain"] = {
                    "dE_x_per_orbital_Ha": abs(E32s - E64) / N64,
                    "kpsi_max_rel_l2": float((num / den).max().item()),
                    "kpsi_max_abs_rel": float((d.abs().amax(1) / ref.abs().amax(1)).max().item()),
                    "orbitals": N64}
                out["speedup_vs_fp64_plain"] = round(sub["fp32_value"] / out[prec]["value"], 2)
            del p64, k64
            torch.cuda.empty_cache()
        copy_gbs = copy_bandwidth(dev)
        out["copy_bandwidth_GBs"] = round(copy_gbs, 1)
        roofline["frac_of_copy_bandwidth"] = round(achieved_gbs / copy_gbs, 4)
        out["autograd"] = autograd_times(grid, psi, occ)

    if not a.no_cpu_baseline:
        ns = a.cpu_sample or (12 if n <= 64 else (5 if n <= 96 else 3))
        out["cpu_baseline"] = cpu_baseline(sysm, min(ns, N))
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
