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
    """Algorithmic HBM bytes of one lattice step: a fluid node loads 9 and stores 9
    float32 populations and reads its link byte (73 B); a solid node only has its
    link byte read (1 B)."""
    return 73 * fluid + 1 * (total - fluid)


def steps_per_launch(kname: str) -> int:
    """Lattice steps per launch of the kernel named by lbm_step_kernel
    ("pair-64x8/lean": 2, "deep3-64x16/lean": 3, "node/lean": 1)."""
    shape = kname.split("/")[0]
    if shape.startswith("pair"):
        return 2
    if shape.startswith("deep"):
        return int(shape[4:].split("-")[0])
    return 1


ROOFLINE_FORMULA = ("frac = S x (73 B x fluid nodes + 1 B x solid nodes) / mean launch time / 8 TB/s, "
                    "S = lattice steps per launch; frac_physical = the same bytes once per launch "
                    "(one read of f(n) and one write of f(n+S); the S - 1 states between stay in LDS); "
                    "traffic_ratio = counted HBM bytes per launch / that one-pass minimum")


def roofline(G, fluid, N, kern_ms, traffic_name):
    """Roofline of the step kernel.  achieved = the algorithmic bytes of the S lattice
    steps one launch performs, over the mean launch duration (HIP events on the
    lattice's stream); frac_physical counts the state's bytes once per launch."""
    kname = G.step_kernel()
    S = steps_per_launch(kname)
    launch_ms = kern_ms * S
    b = algorithmic_bytes(fluid, N)
    ach = S * b / (launch_ms * 1e-3) / 1e9
    phys = b / (launch_ms * 1e-3) / 1e9
    traffic = profiled_traffic(traffic_name)
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": ("k_bgk_multi " if S > 1 else "k_bgk_step ") + kname,
            "steps_per_launch": S, "bytes_per_step": b, "bytes_per_launch": S * b,
            "launch_ms": launch_ms, "frac_physical": phys / HBM_PEAK_GBS,
            "traffic_ratio": traffic / b if traffic else None, "formula": ROOFLINE_FORMULA}


# (result key, closure) pairs: each closure compares one result of this run with the
# FP64 oracle; they run only in the CPU-baseline leg (skipped with --no-cpu-baseline)
FP64_CHECKS = []


def rel_fluid(a, b, fl):
    import numpy as np
    a, b = np.asarray(a, np.float64)[..., fl], np.asarray(b, np.float64)[..., fl]
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def lattice_vs_fp64(lat, gpu_fields, nsteps, init=None):
    """rel-L2 over fluid nodes of the GPU fields (rho - 1, ux, uy) after nsteps against
    the FP64 oracle run from the same start (rest, or f_eq of `init`)."""
    import numpy as np
    from oracle import lbm as olbm
    mask = olbm.raster(lat.nx, lat.ny, lat.shapes_array(), lat.wrap_x, lat.wrap_y)
    if init is not None:   # the float32 fields the GPU lattice was given
        init = tuple(np.asarray(a, np.float64).astype(np.float32).astype(np.float64) for a in init)
    O = olbm.Sim(lat, mask).init(*(init or ())).run(nsteps)
    r = O.macros()
    fl = mask == 0
    g = gpu_fields
    return {"steps": nsteps, "rho-1": rel_fluid(g[0], r[0] - 1.0, fl), "ux": rel_fluid(g[1], r[1], fl),
            "uy": rel_fluid(g[2], r[2], fl)}


def gpu_run_fields(lat, nsteps, init=None):
    """(rho - 1, ux, uy) float64 host fields of a fresh GPU lattice after nsteps."""
    import numpy as np
    import torch
    from paper_2604_27158_amd import lbmfno
    G = lbmfno.Lattice.from_workload(lat)
    if init is not None:
        G.reinit(*(torch.from_numpy(np.asarray(a, np.float64)).float() for a in init))
    G.step(nsteps)
    out = G.macros(rho_minus_one=True).cpu().numpy().astype(np.float64)
    G.close()
    return out


def plain_check(lat, nsteps, init, tag):
    """A closure for FP64_CHECKS: a fresh GPU lattice run now (from rest, or f_eq of
    `init`), compared with the FP64 oracle when the closure is called."""
    g = gpu_run_fields(lat, nsteps, init)
    return lambda: {tag: dict(lattice_vs_fp64(lat, g, nsteps, init), workload=lat.name)}


def fno_algorithmic_bytes(spec, H, W):
    """Minimum HBM bytes of one FNO sample: the float32 input and output read and
    written once, and per Fourier layer one read and one write of the bf16 latent
    [H'][W'][width] plus one write and one read of its row-transform and
    column-inverse coefficients (bf16)."""
    C, m2 = spec.width, spec.m2
    Hp, Wp = H + spec.padding, W + spec.padding
    io = 4 * H * W * (spec.cin + spec.cout)
    latent = 2 * 2 * Hp * Wp * C
    coef = 2 * (2 * m2 * C * Hp * 2 + 2 * m2 * Hp * C * 2)
    return io + spec.layers * (latent + coef)


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
    params = W.fno_random_params(0, layout, spec.width)
    model = gfno.Fno(spec, params, H, Wd)
    # the sample checked against FP64: smooth (rho, ux, uy) fields and an obstacle mask
    r0, u0, v0 = W.random_macro_fields(5, Wd, H, amp_rho=0.02, amp_u=0.05)
    x_chk = np.stack([r0, u0, v0, (W.random_array(12, (H, Wd)) > 1.2).astype(np.float64)])[None]
    flops = fno_flops(spec, H, Wd)
    res = {"model": "FNO 4->3 width 32, 4 layers, 12x12 modes, decoder 1x32",
           "params": gfno.param_count(spec), "grid": [H, Wd], "gflop_per_sample": flops / 1e9}
    nbytes = fno_algorithmic_bytes(spec, H, Wd)
    res["bytes_per_sample"] = nbytes
    s = torch.cuda.Stream()
    samples = {}
    for B in (1, 100):
        k = 0 if B == 1 else 37
        with torch.cuda.stream(s):
            x = torch.randn((B, 4, H, Wd), device="cuda", generator=torch.Generator("cuda").manual_seed(B))
            x[k] = torch.from_numpy(x_chk[0]).float().cuda()
            y = torch.empty((B, 3, H, Wd), device="cuda")
        for _ in range(3):
            model.forward(x, out=y, stream=s)
        reps = 20 if B == 1 else 5
        ms = time_call(lambda: model.forward(x, out=y, stream=s), s, reps)
        res[f"B{B}"] = {"ms": ms, "samples_per_s": B / (ms * 1e-3),
                        "tflops": flops * B / (ms * 1e-3) / 1e12}
        if B == 1:
            # the hybrids' form: the launches replayed from a captured HIP graph
            for _ in range(3):
                model.forward(x, out=y, stream=s, graph=True)
            res["B1"]["ms_graph"] = time_call(lambda: model.forward(x, out=y, stream=s, graph=True), s, reps)
        s.synchronize()
        samples[B] = (x[k:k + 1].cpu().numpy().astype(np.float64), y[k:k + 1].cpu().numpy().astype(np.float64))
    # roofline at batch 100: achieved FLOP/s against min(dense bf16 MFMA peak,
    # arithmetic intensity x HBM peak)
    ms100 = res["B100"]["ms"]
    ai = flops / nbytes
    mfma_peak, hbm_ceiling = 2500.0, ai * HBM_PEAK_GBS / 1000.0
    ceiling = min(mfma_peak, hbm_ceiling)
    ach = flops * 100 / (ms100 * 1e-3) / 1e12
    res["roofline"] = {"bound": "hbm" if hbm_ceiling < mfma_peak else "mfma", "achieved": ach,
                       "peak": ceiling, "unit": "TFLOP/s", "frac": ach / ceiling,
                       "arithmetic_intensity_flop_per_byte": ai,
                       "achieved_GBs": nbytes * 100 / (ms100 * 1e-3) / 1e9,
                       "formula": "achieved = algorithmic flops of 100 samples / forward time; peak = "
                                  "min(2.5 PFLOP/s dense bf16 MFMA, flops/bytes x 8 TB/s), bytes = "
                                  "float32 input + output, and per Fourier layer one read + one write of "
                                  "the bf16 latent and of its row / column coefficients"}
    out["fno"] = res

    def check():
        from oracle import fno as ofno
        ospec = ofno.Spec()   # the same 4 -> 3, width 32, 4 layers, 12 x 12 modes, decoder 1 x 32
        rep = {}
        for B, (xs, ys) in samples.items():
            r64 = ofno.forward(ospec, params, xs, "fp64")
            rbf = ofno.forward(ospec, params, xs, "bf16")
            rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
            rep[f"B{B}"] = {"sample": 0 if B == 1 else 37, "rel_l2_vs_fp64": rel(ys, r64),
                            "rel_l2_vs_bf16_policy_oracle": rel(ys, rbf)}
        return rep
    FP64_CHECKS.append(("fno", check))
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
    from paper_2604_27158_amd import workloads as W
    if os.path.exists(U.DEFAULT_WEIGHTS):
        fno = U.TrainedFno()
        r = U.hybrid_study(fno, list(U.TEST_SEEDS)[:ellipse_seeds])
        per_seed = r.pop("per_seed", None)
        r["workload"] = "ellipses256x128 (1-5 ellipses, Re 100-200), trained flagship FNO"
        # wall time against the velocity error at the 14 000-step horizon over a
        # sweep of cadences (mean over >= 6 stable seeds), and time to error
        r["cadence_sweep"] = U.cadence_study(fno, list(U.TEST_SEEDS)[:10])
        out["hybrid"] = r
        # the plain lattice (the hybrid's reference) over spin-up + horizon, vs FP64
        lat = U.geometry(per_seed[0]["seed"])
        n = U.SPINUP + r["horizon_steps"]
        FP64_CHECKS.append(("hybrid", plain_check(lat, n, W.plug_flow(lat), "plain_lattice_reference")))
    else:
        out["hybrid"] = {"skipped": "trained ellipse surrogate weights not present"}
    if os.path.exists(S.weights_path("small")):
        r = S.study("small", list(S.TEST_SEEDS)[:shear_seeds])
        r.pop("curves", None)
        r["cadence_sweep"] = S.cadence_sweep("small", list(S.TEST_SEEDS)[:6])
        r["workload"] = "double-shear128x128, small surrogate pair (dT = 223 steps)"
        r["paper_eps_T_pct_context"] = {"1:1": 11.8, "1:2": 7.7, "1:3": 5.7,
                                        "hardware": "RTX A4000, 2.6M-parameter pair"}
        out["shear_hybrid"] = r
        slat, r0, u0, v0 = W.double_shear_layer(S.TEST_SEEDS[0], S.N)
        FP64_CHECKS.append(("shear_hybrid", plain_check(slat, S.OUTPUTS * S.DT, (r0, u0, v0),
                                                        "plain_lattice_reference")))
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

    def one():
        loss, _ = fno_through_lattice(tr, x, G, 200, tgt, ckpt_every=50)
        tr.adamw()
        return loss
    one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = [one() for _ in range(reps)]
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / reps * 1e3
    # gradient of the loss w.r.t. the fields the FNO hands over (the lattice adjoint
    # through 200 steps, checkpoints every 50), GPU against the FP64 oracle
    from paper_2604_27158_amd.adjoint import CheckpointedRollout
    y = tr.forward(x)
    torch.cuda.synchronize()
    fields = [(y[0, 0] + 1.0).clone(), y[0, 1].clone(), y[0, 2].clone()]
    roll = CheckpointedRollout(G, 200, 50)
    m = roll.forward(*fields)
    gl, dm = tr.mse(m, tgt.contiguous())
    gg = [t.cpu().numpy().astype(np.float64) for t in roll.backward(dm[0], dm[1], dm[2])]
    f0 = [t.cpu().numpy().astype(np.float64) for t in fields]
    tg = tgt.cpu().numpy().astype(np.float64)

    def check():
        from oracle import lbm as olbm
        mask = olbm.raster(lat.nx, lat.ny, lat.shapes_array(), lat.wrap_x, lat.wrap_y)
        scale = float((mask == 0).sum()) / mask.size   # the oracle's loss is a fluid-node mean
        ref = olbm.rollout_grad(lat, mask, *f0, 200, tg)
        lref = scale * olbm.rollout_loss(lat, mask, *f0, 200, tg)
        fl = mask == 0
        return {"field_gradient_rel_l2": {k: rel_fluid(a, scale * b, fl)
                                          for k, a, b in zip(("rho", "ux", "uy"), gg, ref)},
                "loss": gl, "loss_fp64": lref, "steps": 200}
    FP64_CHECKS.append(("adjoint_fno_training", check))
    out["adjoint_fno_training"] = {"workload": f"{lat.name}, 200 steps, checkpoints every 50",
                                   "fno": "4->3 width 32, 4 layers, 12x12 modes", "ms_per_training_step": ms,
                                   "per_training_step": "200 lattice steps, 200 recomputed from checkpoints, 200 adjoint steps, FNO forward + backward + AdamW",
                                   "losses": losses}


def bench_batch(out, steps=20000, trt_lambda=0.0, key="batch"):
    """100 trajectories of flows past 1-5 ellipses (Re 100-200 on the channel
    half-height), sizes from {256x128, 384x192, 512x256}, one launch per 3-4 fused
    steps (graph-replayed), autotuned kernel; with trt_lambda > 0 the same flows
    with the TRT collision."""
    import dataclasses
    import torch
    from paper_2604_27158_amd import lbmfno
    from paper_2604_27158_amd import workloads as W
    lats = [dataclasses.replace(W.batch_flow(s), trt_lambda=trt_lambda) for s in range(100)]
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
    ach = bytes_step * steps / (ms * 1e-3) / 1e9
    phys = bytes_step * steps / per_launch / (ms * 1e-3) / 1e9
    out[key] = {"collision": f"TRT lambda {trt_lambda:g}" if trt_lambda > 0 else "BGK",
                "trajectories": len(lats), "nodes": B.nodes, "steps": steps,
                "glups": B.nodes * steps / (ms * 1e6), "seconds": ms / 1e3,
                "kernel": B.choice, "steps_per_launch": per_launch, "achieved_GBs": ach,
                "frac": ach / HBM_PEAK_GBS, "frac_physical": phys / HBM_PEAK_GBS,
                "formula": ROOFLINE_FORMULA + " (summed over trajectories; whole-run wall time "
                           "of the graph-replayed launches)",
                "diverged_trajectories": nonfinite}
    B.close()
    if trt_lambda == 0.0:
        picks = (0, 50)
        S2 = lbmfno.Batch([lats[i] for i in picks])
        for k, i in enumerate(picks):
            S2.trajectory(k).reinit(*(torch.from_numpy(a) for a in W.plug_flow(lats[i])))
        S2.step(1000)
        g = [S2.trajectory(k).macros(rho_minus_one=True).cpu().numpy().astype("float64")
             for k in range(len(picks))]
        S2.close()
        sampled = [(lats[i], g[k]) for k, i in enumerate(picks)]
        FP64_CHECKS.append((key, lambda: {"sampled_trajectories": [
            dict(lattice_vs_fp64(lt, gk, 1000, W.plug_flow(lt)), workload=lt.name) for lt, gk in sampled]}))


def bench_steady(out, lat, max_steps):
    """Plain time-to-steady on the main workload: from rest until the density
    residual (every 1000 steps) is below 1e-8."""
    from paper_2604_27158_amd import lbmfno
    from paper_2604_27158_amd.hybrid import steady_solve
    G = lbmfno.Lattice.from_workload(lat)
    steps, sec, rep, hist = steady_solve(G, tol=1e-8, check_every=1000, max_steps=max_steps)
    m = G.macros(rho_minus_one=True)
    dp = G.compare(m, m)["dp"]    # c_s^2 (mean rho on the inlet column - on the outlet column)
    out["time_to_steady_plain"] = {"tol": 1e-8, "steps": steps, "seconds": sec,
                                   "residual": rep["residual"], "converged": rep["residual"] < 1e-8,
                                   "pressure_drop": dp, "glups": steps * lat.nx * lat.ny / sec / 1e9,
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
    FP64_CHECKS.append(("time_to_steady_fno", plain_check(lat, 2000, None, "plain_lattice_2000_steps")))
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
        rb.update({"frac_physical_of_copy": rb["frac_physical"] * HBM_PEAK_GBS / copy_gbs,
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
        # error of the GPU against FP64 over the same number of steps: the density
        # deviation (pressure) at full resolution, the velocity and the pressure drop
        G2 = lbmfno.Lattice.from_workload(lat)
        G2.step(nsteps)
        gm = G2.macros(rho_minus_one=True)
        g = gm.cpu().numpy().astype(np.float64)
        r = sim.macros()
        fl = mask == 0
        err = {"steps": nsteps, "rho-1": rel_fluid(g[0], r[0] - 1.0, fl),
               "rho": rel_fluid(1.0 + g[0], r[0], fl), "ux": rel_fluid(g[1], r[1], fl),
               "uy": rel_fluid(g[2], r[2], fl)}
        c0, c1 = fl[:, 0], fl[:, -1]
        dp64 = float(((r[0][:, 0][c0]).mean() - (r[0][:, -1][c1]).mean()) / 3.0)
        dp32 = G2.compare(gm, gm)["dp"]
        err["pressure_drop"] = {"gpu": dp32, "fp64": dp64, "rel": abs(dp32 - dp64) / abs(dp64)}
        out["error_vs_fp64"] = err
        # every other result against the FP64 oracle
        for key, fn in FP64_CHECKS:
            if isinstance(out.get(key), dict):
                out[key]["error_vs_fp64"] = fn()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
