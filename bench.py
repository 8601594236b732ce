#!/usr/bin/env python3
"""Benchmark of the lattice hot path on one MI355X.

Workload (default): steady porous-media flow, 1024x512 D2Q9 lattice, non-overlapping
random circles of radius 8-20 at porosity U(0.6, 0.8), Zou-He velocity inlet
u = 0.02 and pressure outlet rho = 1, tau = 0.6 (synthetic, seed 0).  One bench
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
INNER = 1001               # lattice steps per bench step: 1000 in whole fused launches + a report step


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
    ap.add_argument("--no-extras", action="store_true",
                    help="only the main workload (for profiler runs)")
    ap.add_argument("--steady-max", type=int, default=400_000,
                    help="step budget of the time-to-steady run")
    ap.add_argument("--steady-seeds", type=int, default=20,
                    help="porous geometries in the FNO-initialised time-to-steady study")
    return ap.parse_args()


def profiled_traffic(name: str):
    """HBM bytes per launch of the step kernel on workload `name`, from the
    counter summary committed under profiles/, or None when the kernel source has
    changed since the counters were taken (the summary records its hash)."""
    import glob
    import hashlib
    src = os.path.join(ROOT, "paper_2604_27158_amd", "csrc", "lbm.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    for md in glob.glob(os.path.join(ROOT, "profiles", "*.md")):
        for line in open(md):
            f = line.split()
            if len(f) == 5 and f[0] == "traffic_bytes_per_launch" and f[1] == name and f[3] == "source":
                return float(f[2]) if f[4] == sha else None
    return None


def algorithmic_bytes(fluid: int, total: int) -> int:
    """Per launch of a step kernel: a fluid node loads 9 and stores 9 float32
    populations and reads its link byte (73 B); a solid node reads its link byte and
    mask byte.  A one-step kernel moves this once per step; a fused S-step kernel
    once per S steps (the intermediate states stay in LDS)."""
    return 73 * fluid + 2 * (total - fluid)


def steps_per_launch(kname: str) -> int:
    """Lattice steps per launch of the kernel named by lbm_step_kernel
    ("pair-64x8/lean": 2, "deep3-64x16/lean": 3, "node/lean": 1)."""
    shape = kname.split("/")[0]
    if shape.startswith("pair"):
        return 2
    if shape.startswith("deep"):
        return int(shape[4:].split("-")[0])
    return 1


def roofline(G, fluid, N, kern_ms, traffic_name):
    """Roofline of the step kernel from the mean per-step time (HIP events on the
    lattice's stream): per-launch algorithmic bytes over the launch duration, and
    the one-step equivalent (the bandwidth a one-step-per-launch kernel would need
    for the same lattice updates per second)."""
    kname = G.step_kernel()
    per_launch = steps_per_launch(kname)
    launch_ms = kern_ms * per_launch
    b = algorithmic_bytes(fluid, N)
    ach = b / (launch_ms * 1e-3) / 1e9
    eq = b / (kern_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": profiled_traffic(traffic_name),
            "kernel": ("k_bgk_multi " if per_launch > 1 else "k_bgk_step ") + kname,
            "steps_per_launch": per_launch, "bytes_per_launch": b, "launch_ms": launch_ms,
            "one_step_equivalent": {"achieved": eq, "frac": eq / HBM_PEAK_GBS}}


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


def fno_flops(spec, H, W):
    """Algorithmic flops of one FNO sample (real multiply-adds x 2; complex products
    as four real ones; DFTs as dense truncated transforms)."""
    C, m1, m2 = spec.width, spec.m1, spec.m2
    Hp, Wp = H + spec.padding, W + spec.padding
    K1 = 2 * m1
    cl = spec.cin + (2 if spec.coords else 0)
    lift = 2 * H * W * (cl * C // 2 + C // 2 * C)
    per_layer = (2 * (2 * m2) * Wp * C * Hp          # row forward DFT
                 + 2 * (2 * K1) * (2 * Hp) * C * m2  # column forward DFT (real form)
                 + 8 * C * C * K1 * m2               # complex mode mixing
                 + 2 * (2 * Hp) * (2 * K1) * C * m2  # column inverse DFT
                 + 2 * Wp * (2 * m2) * C * Hp        # row inverse DFT
                 + 2 * Wp * C * C * Hp)              # 1x1 convolution
    din, dec = C, 0
    for _ in range(spec.dec_layers):
        dec += 2 * H * W * din * spec.dec_size
        din = spec.dec_size
    dec += 2 * H * W * din * spec.cout
    return lift + spec.layers * per_layer + dec


def bench_fno(out):
    """FNO forward latency / throughput at B = 1 and B = 100 (flagship 4 -> 3 model
    on the 256x128 lattice grid, random weights)."""
    import torch
    from paper_2604_27158_amd import fno as gfno
    from paper_2604_27158_amd import workloads as W
    from paper_2604_27158_amd.hybrid import time_call
    import numpy as np
    spec = W.FnoSpec()
    H, Wd = 128, 256
    layout = gfno.param_layout(spec)
    params = 0.05 * W.fno_random_params(0, layout, spec.width)
    params[sum(int(np.prod(sh)) for _, sh in layout[:-1])] = 1.0   # output density bias
    model = gfno.Fno(spec, params, H, Wd)
    flops = fno_flops(spec, H, Wd)
    res = {"model": "FNO 4->3 width 32, 4 layers, 12x12 modes, decoder 1x32",
           "params": gfno.param_count(spec), "grid": [H, Wd], "gflop_per_sample": flops / 1e9}
    s = torch.cuda.Stream()
    for B in (1, 100):
        with torch.cuda.stream(s):
            x = torch.randn((B, 4, H, Wd), device="cuda")
            y = torch.empty((B, 3, H, Wd), device="cuda")
        for _ in range(3):
            model.forward(x, out=y, stream=s)
        reps = 20 if B == 1 else 5
        ms = time_call(lambda: model.forward(x, out=y, stream=s), s, reps)
        res[f"B{B}"] = {"ms": ms, "samples_per_s": B / (ms * 1e-3),
                        "tflops": flops * B / (ms * 1e-3) / 1e12}
    out["fno"] = res
    return model


def bench_hybrid(out, ellipse_seeds=4, shear_seeds=10):
    """The trained hybrids on this GPU, wall time against the plain lattice on the
    same GPU (eps_T) next to the step reduction (eps_N) and the field errors:
    (a) flows past ellipses at 256x128 with the flagship FNO: 20 cycles of 5 FNO
        calls of dt = 100, re-initialisation and 200 lattice steps;
    (b) the double shear layer at 128x128 with the small surrogate pair (a density
        and a velocity model), 1:k hybrids with Delta T = 223 lattice steps over 30
        outputs; error reductions against the pure surrogate rollout."""
    import os
    from paper_2604_27158_amd import unsteady as U, shear as S
    if os.path.exists(U.DEFAULT_WEIGHTS):
        r = U.hybrid_study(U.TrainedFno(), list(U.TEST_SEEDS)[:ellipse_seeds])
        r.pop("per_seed", None)
        r["workload"] = "ellipses256x128 (1-5 ellipses, Re 100-200), trained flagship FNO"
        out["hybrid"] = r
    else:
        out["hybrid"] = {"skipped": "trained ellipse surrogate weights not present"}
    if os.path.exists(S.weights_path("small")):
        r = S.study("small", list(S.TEST_SEEDS)[:shear_seeds])
        r.pop("curves", None)
        r["workload"] = "double-shear128x128, small surrogate pair (dT = 223 steps)"
        r["paper_eps_T_pct_context"] = {"1:1": 11.8, "1:2": 7.7, "1:3": 5.7,
                                        "hardware": "RTX A4000, 2.6M-parameter pair"}
        out["shear_hybrid"] = r
    else:
        out["shear_hybrid"] = {"skipped": "trained shear surrogate weights not present"}


def bench_adjoint(out, reps=3):
    """The differentiable coupling at the configured size: a flagship-shaped FNO
    (4 -> 3, width 32, 4 layers, 12 x 12 modes; seeded small random weights) hands
    (rho - 1, u, v) to a 512x256 walled channel with 40 obstacles, 200 lattice steps
    checkpointed every 50, MSE against the plain lattice's own state; gradient
    through the lattice adjoint and the FNO backward kernels, then AdamW.  Reports
    milliseconds per training step (all of it on the GPU)."""
    import numpy as np
    import torch
    from paper_2604_27158_amd import lbmfno, fno as gfno
    from paper_2604_27158_amd import workloads as W
    from paper_2604_27158_amd.adjoint import fno_through_lattice
    lat = W.channel_walls_circles(4, nx=512, ny=256, n_circles=40, rmin=6, rmax=14, tau=0.8, g=0.0)
    G = lbmfno.Lattice.from_workload(lat)
    spec = W.FnoSpec()
    params = 0.05 * W.fno_random_params(3, gfno.param_layout(spec), spec.width)
    tr = gfno.Trainer(gfno.Fno(spec, params, lat.ny, lat.nx), params, lr=1e-3)
    r0, u0, v0 = W.random_macro_fields(7, lat.nx, lat.ny, amp_u=0.02)
    mask = G.mask.to(torch.float32)
    G.reinit(*(torch.from_numpy(a).float() for a in (r0, u0, v0)))
    G.step(200)
    tgt = G.macros().clone()
    x = torch.stack([torch.from_numpy(a).float().cuda() for a in (r0 - 1.0, u0, v0)] + [mask])[None].contiguous()
    fluid = G.mask == 0

    def one():
        loss, _ = fno_through_lattice(tr, x, G, 200, tgt, fluid, ckpt_every=50)
        tr.adamw()
        return loss
    one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = [one() for _ in range(reps)]
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / reps * 1e3
    out["adjoint_fno_training"] = {"workload": f"{lat.name}, 200 steps, checkpoints every 50",
                                   "fno": "4->3 width 32, 4 layers, 12x12 modes", "ms_per_training_step": ms,
                                   "per_training_step": "200 lattice steps, 200 recomputed from checkpoints, 200 adjoint steps, FNO forward + backward + AdamW",
                                   "losses": losses}


def bench_batch(out, steps=20000, trt_lambda=0.0, key="batch"):
    """100 trajectories of flows past 1-5 ellipses, sizes from {256x128, 384x192,
    512x256}, one launch per step (graph-replayed), autotuned kernel; with
    trt_lambda > 0 the same flows with the TRT collision."""
    import dataclasses
    import torch
    from paper_2604_27158_amd import lbmfno
    from paper_2604_27158_amd import workloads as W
    lats = [dataclasses.replace(W.ellipse_flow(s), trt_lambda=trt_lambda) for s in range(100)]
    B = lbmfno.Batch(lats)
    for i, lat in enumerate(lats):
        B.trajectory(i).reinit(*(torch.from_numpy(a) for a in W.plug_flow(lat)))
    B.step(64)
    B.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(B.stream)
    B.step(steps)
    e1.record(B.stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1)
    fluid = 0
    for i in range(len(lats)):
        fluid += B.trajectory(i).info()[0]
    bytes_step = algorithmic_bytes(fluid, B.nodes)   # per one-step launch
    nonfinite = 0
    for i in range(len(lats)):
        t = B.trajectory(i)
        m = t.macros()
        nonfinite += int(t.check_fields(m[0], m[1], m[2])["nonfinite"] > 0)
    per_launch = steps_per_launch(B.choice.split()[1].split("+")[0])   # "tuned deep4+nt ..."
    ach = bytes_step * steps / per_launch / (ms * 1e-3) / 1e9
    eq = bytes_step * steps / (ms * 1e-3) / 1e9
    out[key] = {"collision": f"TRT lambda {trt_lambda:g}" if trt_lambda > 0 else "BGK",
                "trajectories": len(lats), "nodes": B.nodes, "steps": steps,
                    "glups": B.nodes * steps / (ms * 1e6), "seconds": ms / 1e3,
                    "kernel": B.choice, "steps_per_launch": per_launch, "achieved_GBs": ach,
                    "frac": ach / HBM_PEAK_GBS, "one_step_equivalent_GBs": eq,
                    "one_step_equivalent_frac": eq / HBM_PEAK_GBS,
                    "diverged_trajectories": nonfinite}
    B.close()


def bench_steady(out, lat, max_steps):
    """Plain time-to-steady on the main workload: from rest until the density
    residual (every 1000 steps) is below 1e-8."""
    from paper_2604_27158_amd import lbmfno
    from paper_2604_27158_amd.hybrid import steady_solve
    G = lbmfno.Lattice.from_workload(lat)
    steps, sec, rep, hist = steady_solve(G, tol=1e-8, check_every=1000, max_steps=max_steps)
    out["time_to_steady_plain"] = {"tol": 1e-8, "steps": steps, "seconds": sec,
                                   "residual": rep["residual"], "converged": rep["residual"] < 1e-8,
                                   "residual_every_10k": [h[1] for h in hist[9::10]]}


# speed-ups (%) of FNO initialisation over plain LBM printed in the paper's
# steady-convergence table (RTX A4000; geometric means over 20 trajectories)
PAPER_STEADY_SPEEDUP = {"u@0.0001": 32.7, "v@0.0001": 11.7, "rho@0.0001": 70.0, "dp@0.0001": 42.5,
                        "u@1e-05": 8.57, "rho@1e-05": 50.0, "dp@1e-05": 28.4, "rho@1e-06": 38.1,
                        "rho@2e-07": 31.4}


def bench_time_to_steady(out, seeds):
    """Hybrid (FNO-initialised) vs plain time-to-steady on 512 x 256 porous
    geometries held out from training: outputs (223 lattice steps each) to each
    tolerance against each run's own steady reference, and the wall time on this
    GPU including the two FNO calls and the re-initialisation."""
    from paper_2604_27158_amd import steady_init as S
    if not os.path.exists(S.DEFAULT_WEIGHTS):
        out["time_to_steady_fno"] = {"skipped": "trained surrogate weights not present"}
        return
    log = lambda m: print(m, file=sys.stderr, flush=True)
    res = S.time_to_steady_study(S.SteadyInit(), list(S.TEST_SEEDS)[:seeds], outputs=500, log=log)
    rows = {}
    for r in res["table"]:
        key = f"{r['quantity']}@{r['tol']:g}"
        rows[key] = {"lbm_outputs": r["lbm"], "fno_outputs": r["fno"], "steady_init_outputs": r["steady"],
                     "reached_lbm_fno": [r["lbm_reached"], r["fno_reached"]],
                     "paired_seeds": r["paired_seeds"],
                     "speedup_pct": r["speedup_pct"], "time_speedup_pct": r.get("time_speedup_pct"),
                     "seconds_lbm": r.get("seconds_lbm"), "seconds_fno": r.get("seconds_fno"),
                     "paper_speedup_pct": PAPER_STEADY_SPEEDUP.get(key)}
    lat = S.geometry(S.TEST_SEEDS[0])
    out["time_to_steady_fno"] = {
        "workload": f"porous {lat.nx}x{lat.ny}, r 8-20, phi U(0.75,0.9), u_in {lat.u_in}, tau {lat.tau:.4f}",
        "seeds": len(res["seeds"]), "output_every_steps": res["output_every"], "outputs": res["outputs"],
        "reference": res["reference"], "seconds_per_lattice_step": res["seconds_per_step"],
        "seconds_fno_init": res["seconds_fno_init"],
        "median_final_state_fno_vs_lbm": res["median_final_state_fno_vs_lbm"], "rows": rows}


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
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
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
    roof = roofline(G, fluid, N, kern_ms, "porous1024x512")
    roof["note"] = "37.7 MB working set: resident in the 256 MB last-level cache"
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
                   "bc": f"zou-he inlet u={lat.u_in} / outlet rho=1, periodic y",
                   "porosity": fluid / N, "lattice_steps_per_bench_step": INNER,
                   "arith": "fp32 storage; fp32 collision with the velocity and linear "
                            "equilibrium term in fp64"},
        "roofline": roof,
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
        inner_b = 101                 # 100 fused steps per bench step: whole launches of 2 or 4
        msb, kb, _, _ = time_lattice(GB, inner_b, 5, 1)
        rb = roofline(GB, fl_b, big.nx * big.ny, kb, "porous8192x4096")
        rb.update({"frac_of_copy": rb["achieved"] / copy_gbs,
                   "one_step_equivalent_frac_of_copy": rb["one_step_equivalent"]["achieved"] / copy_gbs,
                   "workload": big.name, "glups": inner_b * big.nx * big.ny / (msb * 1e6)})
        out["roofline_hbm_resident"] = rb
        GB.close()
        del GB
        torch.cuda.empty_cache()
    if not args.no_extras:
        bench_fno(out)
        bench_hybrid(out)
        bench_batch(out)
        bench_batch(out, trt_lambda=0.25, key="batch_trt")
        bench_adjoint(out)
        bench_steady(out, lat, args.steady_max)
        bench_time_to_steady(out, args.steady_seeds)
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
