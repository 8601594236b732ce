#!/usr/bin/env python3
"""Benchmark of the lattice hot path on one MI355X.

Workload (default): steady porous-media flow, 1024x512 D2Q9 lattice, non-overlapping
random circles of radius 8-20 at porosity U(0.6, 0.8), Zou-He velocity inlet
u = 0.05 and pressure outlet rho = 1, tau = 0.6 (synthetic, seed 0).  One bench
step = 1000 fused BGK steps (graph-replayed) plus one FP64 residual / mass
reduction and its host read-back, i.e. one convergence-check interval of the
steady solve.

Prints ONE JSON line: GLUPS over all lattice nodes, the roofline of the dominant
kernel (the fused step) from HIP events on its own stream, the FP64 CPU oracle
timed on this host as a baseline (bounded sample, same workload), and the field
error of the GPU run against that FP64 oracle run.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E
INNER = 1000               # lattice steps per bench step


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the HBM-resident (2.4 GB) roofline lattice")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    return ap.parse_args()


def algorithmic_bytes(fluid: int, total: int) -> int:
    """Per fused step: a fluid node loads 9 and stores 9 float32 populations and
    reads its link byte (73 B); a solid node reads its link byte and mask byte."""
    return 73 * fluid + 2 * (total - fluid)


def time_lattice(G, inner, steps, warmup, report_each=True):
    """Returns (ms per bench step, mean fused-step launch duration in ms)."""
    import torch
    for _ in range(warmup):
        G.step(inner, report=True)
    torch.cuda.synchronize()
    G.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    k0 = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    k1 = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    reps = []
    t0 = time.perf_counter()
    e0.record(G.stream)
    for k in range(steps):
        k0[k].record(G.stream)
        G.step(inner - 1)             # pure fused steps (graph replays + tail)
        k1[k].record(G.stream)
        reps.append(G.step(1, report=report_each))  # last step + FP64 reduction
    e1.record(G.stream)
    G.synchronize()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    total_ms = e0.elapsed_time(e1)
    kern_ms = sum(a.elapsed_time(b) for a, b in zip(k0, k1)) / (steps * (inner - 1))
    return total_ms / steps, kern_ms, wall / steps, reps[-1]


def porous_large(seed):
    """8192x4096 porous lattice: the 1024x512 obstacle layout tiled 8x8 (2.4 GB of
    population stores, far above the 256 MB last-level cache)."""
    from paper_2604_27158_amd import workloads as W
    base = W.porous_circles(seed)
    shapes = []
    for ty in range(8):
        for tx in range(8):
            for (cx, cy, A, B, C, F, R) in base.shapes:
                shapes.append((cx + 1024 * tx, cy + 512 * ty, A, B, C, F, R))
    return W.Lattice(nx=8192, ny=4096, tau=base.tau, bc_x=base.bc_x, bc_y=base.bc_y,
                     u_in=base.u_in, rho_out=base.rho_out, shapes=shapes, wrap_x=False,
                     wrap_y=True, seed=seed, name=f"porous8192x4096-tiled-s{seed}")


def cpu_baseline(lat, seconds):
    """FP64 oracle (C, OpenMP over rows) on this host: MLUPS on a bounded number of
    steps of the same workload; returns (dict, oracle Sim after those steps)."""
    import numpy as np
    from oracle import lbm as olbm
    mask = olbm.raster(lat.nx, lat.ny, lat.shapes_array(), lat.wrap_x, lat.wrap_y)
    sim = olbm.Sim(lat, mask).init()
    t = time.perf_counter()
    sim.run(10)
    dt = (time.perf_counter() - t) / 10
    n = int(max(20, min(2000, seconds / max(dt, 1e-9))))
    n -= n % 10
    t = time.perf_counter()
    sim.run(n - 10)
    el = time.perf_counter() - t
    lups = (n - 10) * lat.nx * lat.ny
    return ({"value": lups / el / 1e9, "unit": "GLUPS", "cores": olbm.threads(),
             "kind": "oracle", "sample": f"{lat.name}: {n - 10} FP64 steps "
             f"({el:.1f} s) after 10 untimed, all nodes counted"}, sim, mask, n)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported by this build "
              "(the lattice and FNO paths run on a single MI355X)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2604_27158_amd import lbmfno
    from paper_2604_27158_amd import workloads as W

    lbmfno.load()
    lat = W.porous_circles(args.seed)
    G = lbmfno.Lattice.from_workload(lat)
    fluid, _ = G.info()
    N = lat.nx * lat.ny
    ms_step, kern_ms, wall_ms, rep = time_lattice(G, INNER, args.steps, args.warmup)
    glups = INNER * N / (ms_step * 1e6)
    bytes_launch = algorithmic_bytes(fluid, N)
    achieved = bytes_launch / (kern_ms * 1e-3) / 1e9
    out = {
        "metric": "D2Q9 GLUPS & %HBM peak; hybrid vs plain LBM time-to-steady at fixed error",
        "value": glups,
        "unit": "GLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": lat.name, "nx": lat.nx, "ny": lat.ny, "tau": lat.tau,
                   "bc": "zou-he inlet u=0.05 / outlet rho=1, periodic y",
                   "porosity": fluid / N, "lattice_steps_per_bench_step": INNER,
                   "arith": "fp32 storage, fp64 collision registers"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_bgk_step<zouhe>", "bytes_per_launch": bytes_launch,
                     "launch_ms": kern_ms,
                     "note": "37.7 MB working set: resident in the 256 MB last-level cache"},
        "fluid_glups": INNER * fluid / (ms_step * 1e6),
        "residual": rep["residual"],
        "mass": rep["mass"],
    }
    # achievable copy bandwidth (2 x 1 GiB float32 copy) as the practical ceiling
    n = 1 << 28
    with torch.cuda.stream(G.stream):
        a = torch.empty(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
    for _ in range(3):
        lbmfno.stream_copy(a, b, G.stream)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record(G.stream)
    for _ in range(10):
        lbmfno.stream_copy(a, b, G.stream)
    c1.record(G.stream)
    G.synchronize()
    copy_gbs = 10 * 2 * 4 * n / (c0.elapsed_time(c1) * 1e-3) / 1e9
    out["copy_GBs"] = copy_gbs
    del a, b
    if not args.no_large:
        big = porous_large(args.seed)
        GB = lbmfno.Lattice.from_workload(big)
        fl_b, _ = GB.info()
        msb, kb, _, _ = time_lattice(GB, 100, 5, 1)
        bb = algorithmic_bytes(fl_b, big.nx * big.ny)
        ach = bb / (kb * 1e-3) / 1e9
        out["roofline_hbm_resident"] = {
            "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "frac_of_copy": ach / copy_gbs, "traffic": None,
            "workload": big.name, "glups": 100 * big.nx * big.ny / (msb * 1e6),
            "bytes_per_launch": bb, "launch_ms": kb}
        GB.close()
        del GB
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        cb, sim, mask, nsteps = cpu_baseline(lat, args.cpu_seconds)
        out["cpu_baseline"] = cb
        # error of the GPU against FP64 over the same number of steps
        G2 = lbmfno.Lattice.from_workload(lat)
        G2.step(nsteps)
        g = G2.macros().cpu().numpy().astype(np.float64)
        r = sim.macros()
        fl = mask == 0
        out["error_vs_fp64"] = {
            k: float(np.linalg.norm((a_ - b_)[fl]) / np.linalg.norm(b_[fl]))
            for k, a_, b_ in zip(("rho", "ux", "uy"), g, r)}
        out["error_vs_fp64"]["steps"] = nsteps
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
