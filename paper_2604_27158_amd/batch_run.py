"""Fixed run of the batched launch for kernel traces (rocprofv3 --kernel-trace):
100 ellipse-flow trajectories of the batch workload (sizes from {256x128, 384x192,
512x256}), plug-flow
start, `--steps` lattice steps issued as the benchmark issues them (graph-replayed
chunks of whole fused launches).

    python -m paper_2604_27158_amd.batch_run --steps 2000
"""
import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=2000)
    args = ap.parse_args()
    import torch
    from paper_2604_27158_amd import lbmfno
    from paper_2604_27158_amd import workloads as W
    lats = [W.batch_flow(s) for s in range(100)]
    B = lbmfno.Batch(lats)
    for i, lat in enumerate(lats):
        B.trajectory(i).reinit(*(torch.from_numpy(a) for a in W.plug_flow(lat)))
    B.step(64)
    B.synchronize()
    B.step(args.steps)
    B.synchronize()
    print(f"batch_run: {len(lats)} trajectories, {B.nodes} nodes, {args.steps} steps, kernel {B.choice}",
          flush=True)


if __name__ == "__main__":
    main()
