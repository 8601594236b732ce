"""Fixed kernel sequences for hardware-counter runs (rocprofv3 --pmc).

Launches the step kernel of a workload directly (no graph replay, so every
dispatch is visible to the counter collector; each call advances the lattice by
the steps of one launch of the fused kernel the workload runs by default) and the
library's copy kernel on a buffer of known size, which calibrates the byte
counters:

    python -m paper_2604_27158_amd.profile_run --workload porous1024 --steps 50

The fno workloads run the flagship FNO forward (4 -> 3 channels, width 32, four
layers of 12 x 12 modes, 128 x 256 grid, seeded random weights) at batch 1 and
batch 100, eagerly, `--steps` times each:

    python -m paper_2604_27158_amd.profile_run --workload fno --steps 20
"""
import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

COPY_FLOATS = 1 << 26   # 256 MiB per buffer: 512 MiB moved per copy launch


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="porous1024", choices=["porous1024", "large", "fno"])
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--copies", type=int, default=5)
    args = ap.parse_args()
    import torch
    from paper_2604_27158_amd import lbmfno
    from paper_2604_27158_amd import workloads as W
    if args.workload == "fno":
        run_fno(args.steps)
        return
    import bench
    lat = W.porous_circles(0) if args.workload == "porous1024" else bench.porous_large(0)
    G = lbmfno.Lattice.from_workload(lat)
    spl = bench.steps_per_launch(G.step_kernel())
    for _ in range(args.steps // spl):
        G.step(spl)
    G.synchronize()
    fluid, _ = G.info()
    a = torch.ones(COPY_FLOATS, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(args.copies):
        lbmfno.stream_copy(a, b)
    torch.cuda.synchronize()
    print(f"profile_run: {lat.name} {args.steps} steps ({G.step_kernel()}), fluid {fluid} of {lat.nx * lat.ny}; "
          f"{args.copies} copies of {COPY_FLOATS * 4} bytes", flush=True)


def run_fno(reps):
    import numpy as np
    import torch
    from paper_2604_27158_amd import fno as gfno
    from paper_2604_27158_amd import workloads as W
    spec = W.FnoSpec()
    model = gfno.Fno(spec, W.fno_random_params(0, gfno.param_layout(spec), spec.width), 128, 256)
    for B in (1, 100):
        x = torch.from_numpy(W.random_array(1, (B, spec.cin, 128, 256)).astype(np.float32)).cuda()
        y = torch.empty((B, spec.cout, 128, 256), dtype=torch.float32, device="cuda")
        for _ in range(reps):
            model.forward(x, out=y)
        torch.cuda.synchronize()
        print(f"profile_run: flagship FNO forward, batch {B}, {reps} calls", flush=True)


if __name__ == "__main__":
    main()
