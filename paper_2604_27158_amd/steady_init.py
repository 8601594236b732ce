"""FNO initialisation of steady porous-media runs (the paper's Sec. 3.1 and its
porous-media tables): two FNO surrogates map the binary obstacle mask to the steady
density and velocity fields, the lattice is re-initialised from their prediction
(f = f_eq(rho, u)) and plain lattice steps run from there; the convergence of rho,
u, v and the pressure drop towards the steady reference is compared with the naive
start (rho = 1, u = 0).

Everything on the device runs in liblbmfno kernels: the lattice (data generation,
reference, convergence runs), the FNO forward/backward/AdamW (training) and the
field comparison.  This module only sequences the calls, keeps the tensors and
folds the output normalisation into the decoder's last layer.

Models (the paper's porous hyperparameter tables): density 1 -> 1 channel, width 16,
3 Fourier layers, 6 modes, padding 9, decoder 3 x 32; velocity 1 -> 2 channels,
width 16, 6 layers, 12 modes, padding 9, decoder 3 x 64.  AdamW, learning rate
1e-2 multiplied by 0.85 every 10 epochs.  Dataset: porous geometries at 512 x 256
(the paper's dataset resolution), each run to its steady state by the lattice.

    python -m paper_2604_27158_amd.steady_init train --out weights.npz
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2604_27158_amd import workloads as W  # noqa: E402

NX, NY = 512, 256
OUTPUT_EVERY = 223        # one output interval (the paper's Delta T = 223 lattice steps)
RHO_SPEC = W.FnoSpec(cin=1, width=16, layers=3, m1=6, m2=6, dec_layers=3, dec_size=32, cout=1,
                     padding=9)
U_SPEC = W.FnoSpec(cin=1, width=16, layers=6, m1=12, m2=12, dec_layers=3, dec_size=64, cout=2,
                   padding=9)
TRAIN_SEEDS = range(100000, 101700)      # 1700 training geometries
VAL_SEEDS = range(200000, 200200)        # 200 validation geometries
TEST_SEEDS = range(300000, 300020)       # 20 evaluation geometries
DEFAULT_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights",
                               "porous_steady_512x256.npz")


GAP = 2   # minimum free cells between obstacle discs
# Reynolds number of the paper's porous setup on the domain height,
# U L / nu = 0.5 * 1.0 / 0.01 = 50, at inlet speed 0.01: nu = 0.01 * 256 / 50
U_IN = 0.01
TAU = 0.5 + 3.0 * U_IN * NY / 50.0


def geometry(seed: int) -> W.Lattice:
    """Porous medium at 512 x 256: the porous generator with the obstacle radii of
    the 1024 x 512 case (8-20 cells), inlet/outlet keep-out halved, and the porosity
    range of the paper's porous-media setup, phi ~ U(0.75, 0.9); inlet speed and
    viscosity give its Reynolds number on the domain height, 50.  The paper gives no
    obstacle sizes; obstacles of 16-40 cells are resolved by the surrogates' 6 and
    12 retained modes (about 20 cells at this grid), smaller ones are not."""
    return W.porous_circles(seed, nx=NX, ny=NY, rmin=8, rmax=20, phi_lo=0.75, phi_hi=0.9,
                            gap=GAP, keepout=20, u_in=U_IN, tau=TAU)


def make_dataset(seeds, steps: int, log=None, per_launch: int = 100):
    """Device tensors X [n][1][ny][nx] (mask) and Y [n][3][ny][nx] (rho - 1, ux, uy):
    each geometry run `steps` lattice steps from rest, `per_launch` geometries at a
    time through the batched launcher (one launch per step for all of them)."""
    import torch
    from paper_2604_27158_amd import lbmfno
    seeds = list(seeds)
    X = torch.empty((len(seeds), 1, NY, NX), dtype=torch.float32, device="cuda")
    Y = torch.empty((len(seeds), 3, NY, NX), dtype=torch.float32, device="cuda")
    t0 = time.perf_counter()
    for k0 in range(0, len(seeds), per_launch):
        lats = [geometry(s) for s in seeds[k0:k0 + per_launch]]
        batch = lbmfno.Batch(lats)
        batch.step(steps - OUTPUT_EVERY)
        prev = [batch.trajectory(i).macros(rho_minus_one=True) for i in range(min(len(lats), 8))]
        batch.step(OUTPUT_EVERY)
        if log and k0 == 0:
            ch = [batch.trajectory(i).compare(batch.trajectory(i).macros(rho_minus_one=True), p)["rel_l1_ux"]
                  for i, p in enumerate(prev)]
            log(f"dataset: relative L1 change of ux over the last {OUTPUT_EVERY} of {steps} steps, "
                f"median of {len(ch)}: {float(np.median(ch)):.2e}")
        for i in range(len(lats)):
            view = batch.trajectory(i)
            f = view.macros(rho_minus_one=True)
            X[k0 + i, 0].copy_(view.mask.to(torch.float32))
            Y[k0 + i].copy_(f)
        torch.cuda.synchronize()
        batch.close()
        if log:
            log(f"dataset: {k0 + len(lats)}/{len(seeds)} geometries, {steps} steps each "
                f"({time.perf_counter() - t0:.1f} s)")
    return X, Y


def pow2_scale(t) -> float:
    """Power of two nearest the RMS of t (so that folding it into weights is exact)."""
    rms = float(t.double().pow(2).mean().sqrt())
    return 2.0 ** round(math.log2(max(rms, 1e-30)))


def fold_output_scale(spec, params: np.ndarray, scale: float) -> np.ndarray:
    """Packed parameters of the network scale * f(x): the decoder's last weights and
    biases multiplied by `scale` (exact for a power of two)."""
    from paper_2604_27158_amd import fno as gfno
    p = np.array(params, dtype=np.float64, copy=True)
    off = 0
    for name, shp in gfno.param_layout(spec):
        n = int(np.prod(shp))
        if name in ("dec_out.w", "dec_out.b"):
            p[off:off + n] *= scale
        off += n
    return p


def train_model(spec, X, Y, Xv, Yv, epochs: int, batch: int = 8, lr: float = 1e-2,
                decay: float = 0.85, decay_every: int = 10, weight_decay: float = 1e-2,
                seed: int = 0, log=None):
    """AdamW training of one model on device tensors (targets already normalised).
    Returns (the parameters of the epoch with the lowest validation loss,
    [(epoch, train loss, validation loss)])."""
    import torch
    from paper_2604_27158_amd import fno as gfno
    params = W.fno_random_params(seed, gfno.param_layout(spec), spec.width)
    model = gfno.Fno(spec, params, NY, NX)
    tr = gfno.Trainer(model, params, lr=lr, weight_decay=weight_decay)
    n = X.shape[0]
    g = torch.Generator().manual_seed(seed)
    hist = []
    best = (float("inf"), None)
    t0 = time.perf_counter()
    for ep in range(epochs):
        tr.lr = lr * decay ** (ep // decay_every)
        perm = torch.randperm(n, generator=g)
        tot, cnt = 0.0, 0
        for b0 in range(0, n - batch + 1, batch):
            idx = perm[b0:b0 + batch].cuda()
            xb = X.index_select(0, idx).contiguous()
            yb = Y.index_select(0, idx).contiguous()
            tot += tr.step(xb, yb)
            cnt += 1
        vl = evaluate(tr, Xv, Yv, batch)
        hist.append((ep, tot / max(cnt, 1), vl))
        if vl < best[0]:
            best = (vl, tr.params())
        if log:
            log(f"{spec.cout}-output model: epoch {ep + 1}/{epochs} train {tot / max(cnt, 1):.4e} "
                f"val {vl:.4e} lr {tr.lr:.2e} ({time.perf_counter() - t0:.0f} s)")
    return best[1], hist


def evaluate(tr, X, Y, batch: int = 8) -> float:
    """Mean squared error of a trainer's model over a device dataset."""
    tot, n = 0.0, 0
    for b0 in range(0, X.shape[0], batch):
        xb = X[b0:b0 + batch].contiguous()
        yb = Y[b0:b0 + batch].contiguous()
        out = tr.fno.forward(xb)
        loss, _ = tr.mse(out, yb)
        tot += loss * xb.shape[0]
        n += xb.shape[0]
    return tot / max(n, 1)


class SteadyInit:
    """The two trained surrogates bound to the 512 x 256 grid; predict() gives
    (rho, ux, uy) float32 device fields for a lattice's mask."""

    def __init__(self, path: str = DEFAULT_WEIGHTS):
        from paper_2604_27158_amd import fno as gfno
        with np.load(path, allow_pickle=False) as z:
            p_rho, p_u = z["rho_params"], z["u_params"]
        self.rho = gfno.Fno(RHO_SPEC, p_rho, NY, NX)
        self.u = gfno.Fno(U_SPEC, p_u, NY, NX)

    def predict(self, lattice):
        """Fields for lattice.reinit: rho = 1 + drho, ux, uy (device, lattice stream)."""
        import torch
        with torch.cuda.stream(lattice.stream):
            x = lattice.mask.to(torch.float32).reshape(1, 1, NY, NX)
            drho = self.rho.forward(x, stream=lattice.stream)
            u = self.u.forward(x, stream=lattice.stream)
            rho = drho[0, 0] + 1.0
        return rho, u[0, 0], u[0, 1]


def outputs_to_tolerance(errs, key: str, eps: float):
    """First output index (1-based) at which errs[k][key] <= eps and stays so for the
    rest of the recorded run; None if never."""
    last_bad = -1
    for k, e in enumerate(errs):
        if not e[key] <= eps:
            last_bad = k
    return last_bad + 2 if last_bad + 1 < len(errs) else None


QUANTITIES = (("u", "rel_l1_ux"), ("v", "rel_l1_uy"), ("rho", "rel_l1_rho"), ("dp", "rel_dp"))
TOLERANCES = (1e-4, 1e-5, 1e-6, 2e-7)


def geo_mean(xs):
    xs = [x for x in xs if x is not None]
    return float(np.exp(np.mean(np.log(xs)))) if xs else None


def run_outputs(lats, inits, outputs: int, log=None, tag=""):
    """Run trajectories side by side in one batch for `outputs` output intervals;
    inits[i] is None (rest: rho = 1, u = 0) or a callable(view) giving (rho, ux,
    uy) to re-initialise from.  Returns (batch, fields [n][outputs][3][ny][nx] as
    (rho - 1, ux, uy) on the device)."""
    import torch
    from paper_2604_27158_amd import lbmfno
    batch = lbmfno.Batch(lats)
    n = len(lats)
    for i, init in enumerate(inits):
        if init is not None:
            view = batch.trajectory(i)
            view.reinit(*init(view))
    store = torch.empty((n, outputs, 3, NY, NX), dtype=torch.float32, device="cuda")
    t0 = time.perf_counter()
    for o in range(outputs):
        batch.step(OUTPUT_EVERY)
        for i in range(n):
            store[i, o].copy_(batch.trajectory(i).macros(rho_minus_one=True))
        if log and (o + 1) % 50 == 0:
            torch.cuda.synchronize()
            log(f"{tag}: {o + 1}/{outputs} outputs of {n} trajectories ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    return batch, store


def own_reference(store_i):
    """The paper's steady reference of one trajectory: the mean of its last 10 outputs."""
    return store_i[-10:].double().mean(dim=0).to(store_i.dtype).contiguous()


def time_to_steady_study(init: "SteadyInit", seeds, outputs: int = 500, log=None):
    """Outputs (of 223 lattice steps) each start needs to bring u, v, rho and the
    pressure drop within each tolerance of its own steady reference (the mean of
    its last 10 outputs): rest (plain lattice), the FNO prediction, and the plain
    run's converged fields ("steady" start); per seed and as geometric means over
    seeds; the distance between the starts' final states; and the wall time per
    lattice step and of the FNO start (two models + equilibrium re-initialisation)."""
    import torch
    from paper_2604_27158_amd import lbmfno
    seeds = list(seeds)
    lats = [geometry(s) for s in seeds]
    ns = len(seeds)
    # rest and FNO starts side by side
    batch, store = run_outputs(lats + lats, [None] * ns + [init.predict] * ns, outputs, log, "lbm+fno")
    refs = {"lbm": [own_reference(store[i]) for i in range(ns)],
            "fno": [own_reference(store[ns + i]) for i in range(ns)]}
    errs = {"lbm": [], "fno": []}
    for i in range(ns):
        for name, j in (("lbm", i), ("fno", ns + i)):
            view = batch.trajectory(j)
            errs[name].append([view.compare(store[j, o], refs[name][i]) for o in range(outputs)])
    final_gap = [batch.trajectory(i).compare(refs["fno"][i], refs["lbm"][i]) for i in range(ns)]
    last_change = {name: [batch.trajectory(j).compare(store[j, -1], store[j, -2])
                          for j in (range(ns) if name == "lbm" else range(ns, 2 * ns))]
                   for name in ("lbm", "fno")}
    batch.close()
    del store
    torch.cuda.empty_cache()
    # "steady" start from the plain run's converged fields
    steady_fields = [(refs["lbm"][i][0] + 1.0, refs["lbm"][i][1], refs["lbm"][i][2]) for i in range(ns)]
    batch, store = run_outputs(lats, [(lambda v, f=f: f) for f in steady_fields], outputs, log, "steady")
    refs["steady"] = [own_reference(store[i]) for i in range(ns)]
    errs["steady"] = [[batch.trajectory(i).compare(store[i, o], refs["steady"][i]) for o in range(outputs)]
                      for i in range(ns)]
    batch.close()
    del store
    torch.cuda.empty_cache()
    per_seed = []
    for i, sd in enumerate(seeds):
        rec = {"seed": sd, "name": lats[i].name,
               "final_state_fno_vs_lbm": {q: final_gap[i][key] for q, key in QUANTITIES},
               "last_output_change": {n: {q: last_change[n][i][key] for q, key in QUANTITIES}
                                      for n in last_change}}
        for name in ("lbm", "fno", "steady"):
            rec[name] = {q: {str(e): outputs_to_tolerance(errs[name][i], key, e) for e in TOLERANCES}
                         for q, key in QUANTITIES}
            rec["first_output_" + name] = {q: errs[name][i][0][key] for q, key in QUANTITIES}
        per_seed.append(rec)
        if log:
            log(f"seed {sd}: outputs to 1e-4 (lbm/fno/steady) " +
                ", ".join(f"{q} {rec['lbm'][q]['0.0001']}/{rec['fno'][q]['0.0001']}/{rec['steady'][q]['0.0001']}"
                          for q, _ in QUANTITIES))
    table = []
    for e in TOLERANCES:
        for q, _ in QUANTITIES:
            row = {"tol": e, "quantity": q}
            for name in ("lbm", "fno", "steady"):
                vals = [r[name][q][str(e)] for r in per_seed]
                row[name] = geo_mean(vals)
                row[name + "_reached"] = sum(v is not None for v in vals)
            # speed-up over the seeds where both the rest and the FNO start reach e
            pairs = [(r["lbm"][q][str(e)], r["fno"][q][str(e)]) for r in per_seed
                     if r["lbm"][q][str(e)] is not None and r["fno"][q][str(e)] is not None]
            row["paired_seeds"] = len(pairs)
            if pairs:
                gl, gf = geo_mean([p[0] for p in pairs]), geo_mean([p[1] for p in pairs])
                row["lbm_paired"], row["fno_paired"] = gl, gf
                row["speedup_pct"] = 100.0 * (gl - gf) / gl
            else:
                row["speedup_pct"] = None
            table.append(row)
    # wall-clock costs on this GPU: one lattice on its own, and the FNO start
    G = lbmfno.Lattice.from_workload(lats[0])
    G.step(1000)
    G.synchronize()
    t0 = time.perf_counter()
    G.step(20000)
    G.synchronize()
    t_step = (time.perf_counter() - t0) / 20000
    for _ in range(3):
        G.reinit(*init.predict(G))
    G.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        G.reinit(*init.predict(G))
    G.synchronize()
    t_init = (time.perf_counter() - t0) / 10
    for row in table:
        if row["speedup_pct"] is not None:
            t_l = row["lbm_paired"] * OUTPUT_EVERY * t_step
            t_f = row["fno_paired"] * OUTPUT_EVERY * t_step + t_init
            row["seconds_lbm"], row["seconds_fno"] = t_l, t_f
            row["time_speedup_pct"] = 100.0 * (t_l - t_f) / t_l
    gaps = {q: float(np.median([r["final_state_fno_vs_lbm"][q] for r in per_seed])) for q, _ in QUANTITIES}
    return {"seeds": seeds, "output_every": OUTPUT_EVERY, "outputs": outputs,
            "reference": "mean of each trajectory's last 10 outputs",
            "seconds_per_step": t_step, "seconds_fno_init": t_init,
            "median_final_state_fno_vs_lbm": gaps, "table": table, "per_seed": per_seed}


def log_print(msg):
    print(msg, flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--out", default=DEFAULT_WEIGHTS)
    t.add_argument("--train", type=int, default=len(TRAIN_SEEDS))
    t.add_argument("--val", type=int, default=len(VAL_SEEDS))
    t.add_argument("--steps", type=int, default=20000, help="lattice steps per sample")
    t.add_argument("--epochs", type=int, default=40)
    t.add_argument("--batch", type=int, default=8)
    e = sub.add_parser("eval")
    e.add_argument("--weights", default=DEFAULT_WEIGHTS)
    e.add_argument("--seeds", type=int, default=len(TEST_SEEDS))
    e.add_argument("--json", default=None)
    e.add_argument("--outputs", type=int, default=500)
    args = ap.parse_args()
    if args.cmd == "eval":
        import json
        from paper_2604_27158_amd import lbmfno
        lbmfno.load()
        res = time_to_steady_study(SteadyInit(args.weights), list(TEST_SEEDS)[:args.seeds],
                                   outputs=args.outputs, log=log_print)
        for row in res["table"]:
            log_print(json.dumps({k: v for k, v in row.items()}))
        if args.json:
            with open(args.json, "w") as f:
                json.dump(res, f, indent=1)
        return
    import torch
    from paper_2604_27158_amd import lbmfno
    lbmfno.load()
    t0 = time.perf_counter()
    X, Y = make_dataset(list(TRAIN_SEEDS)[:args.train], args.steps, log_print)
    Xv, Yv = make_dataset(list(VAL_SEEDS)[:args.val], args.steps, log_print)
    log_print(f"datasets ready in {time.perf_counter() - t0:.1f} s")
    s_rho = pow2_scale(Y[:, 0])
    s_u = pow2_scale(Y[:, 1:])
    Yr, Yvr = (Y[:, :1] / s_rho).contiguous(), (Yv[:, :1] / s_rho).contiguous()
    Yu, Yvu = (Y[:, 1:] / s_u).contiguous(), (Yv[:, 1:] / s_u).contiguous()
    del Y, Yv
    p_rho, h_rho = train_model(RHO_SPEC, X, Yr, Xv, Yvr, args.epochs, args.batch, seed=1, log=log_print)
    p_u, h_u = train_model(U_SPEC, X, Yu, Xv, Yvu, args.epochs, args.batch, seed=2, log=log_print)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    np.savez(args.out,
             rho_params=fold_output_scale(RHO_SPEC, p_rho, s_rho).astype(np.float32),
             u_params=fold_output_scale(U_SPEC, p_u, s_u).astype(np.float32),
             rho_scale=np.float64(s_rho), u_scale=np.float64(s_u),
             rho_history=np.array(h_rho, dtype=np.float64), u_history=np.array(h_u, dtype=np.float64),
             samples=np.int64(args.train), steps=np.int64(args.steps), epochs=np.int64(args.epochs))
    log_print(f"wrote {args.out} ({time.perf_counter() - t0:.0f} s total)")


if __name__ == "__main__":
    main()
