"""Double shear layer with hybrid FNO-LBM super-time-stepping (the paper's Sec. 3.2
and Appendix B): periodic 128 x 128, initial condition of Eqs. 9-10 with randomised
layer centres and Reynolds numbers 8-50, outputs every Delta T = 223 lattice steps
over 30 Delta T.

Surrogates: a density model (rho -> rho) and a velocity model ((u, v) -> (u, v)),
each predicting one Delta T ahead; the paper's two groups:
  small (2.6M): density width 14, 3 layers, 8 modes; velocity width 14, 3 layers,
                32 modes; decoder 1 x 32, padding 9;
  large (11.2M): both with 7 layers and 32 modes.
Trained on 3000 pairs (100 lattice trajectories x 30 steps of Delta T), validated
on ~1000 pairs, AdamW, lr 1e-2 x 0.85 every 8 epochs; normalisation folded into the
weights (powers of two), so the runtime path feeds raw fields to the FNO kernels.

Rollouts over the 30 Delta T horizon from the analytic initial condition: plain
lattice (the reference), pure FNO (30 chained calls), and 1:k hybrids (one Delta T by
the FNO, then k Delta T by the lattice after an equilibrium re-initialisation,
k = 1, 2, 3).  Errors per output against the reference: mean squared error over
(rho, u, v) and the relative L2 error of the vorticity (central differences);
global errors are their means over the 30 outputs.  Wall times on this GPU give
eps_T; eps_N is the share of lattice steps the FNO replaces.

    python -m paper_2604_27158_amd.shear train --group small
    python -m paper_2604_27158_amd.shear eval --group small
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

N = 128
DT = W.SHEAR_DT_OUT
OUTPUTS = W.SHEAR_OUTPUTS
GROUPS = {
    "small": (W.FnoSpec(cin=1, width=14, layers=3, m1=8, m2=8, dec_layers=1, dec_size=32, cout=1, padding=9),
              W.FnoSpec(cin=2, width=14, layers=3, m1=32, m2=32, dec_layers=1, dec_size=32, cout=2, padding=9)),
    "large": (W.FnoSpec(cin=1, width=14, layers=7, m1=32, m2=32, dec_layers=1, dec_size=32, cout=1, padding=9),
              W.FnoSpec(cin=2, width=14, layers=7, m1=32, m2=32, dec_layers=1, dec_size=32, cout=2, padding=9)),
}
TRAIN_SEEDS = range(40000, 40100)     # 100 trajectories -> 3000 pairs
VAL_SEEDS = range(41000, 41034)       # 34 trajectories -> 1020 pairs
TEST_SEEDS = range(42000, 42100)      # 100 inference trajectories
HYBRIDS = (1, 2, 3)


def weights_path(group: str) -> str:
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", f"shear_{group}_128.npz")


def simulate(seeds, log=None):
    """Lattice fields (rho - 1, ux, uy) at t = 0, 1, ..., 30 Delta T for each seed, run
    side by side by the batched launcher: device tensor [n][31][3][N][N]."""
    import torch
    from paper_2604_27158_amd import lbmfno
    seeds = list(seeds)
    F = torch.empty((len(seeds), OUTPUTS + 1, 3, N, N), dtype=torch.float32, device="cuda")
    t0 = time.perf_counter()
    for k0 in range(0, len(seeds), 100):
        cases = [W.double_shear_layer(s, N) for s in seeds[k0:k0 + 100]]
        batch = lbmfno.Batch([c[0] for c in cases])
        for i, (_, r, u, v) in enumerate(cases):
            batch.trajectory(i).reinit(*(torch.from_numpy(a) for a in (r, u, v)))
        for t in range(OUTPUTS + 1):
            if t:
                batch.step(DT)
            for i in range(len(cases)):
                F[k0 + i, t].copy_(batch.trajectory(i).macros(rho_minus_one=True))
        torch.cuda.synchronize()
        batch.close()
        if log:
            log(f"shear trajectories: {k0 + len(cases)}/{len(seeds)} ({time.perf_counter() - t0:.1f} s)")
    return F


def pow2(x: float) -> float:
    return 2.0 ** round(math.log2(max(x, 1e-30)))


def pairs(F):
    """Normalised training pairs of both models and the scales: density
    ((rho - 1)/s_r at t -> at t + 1) and velocity (u / s_u at t -> at t + 1)."""
    s_r = pow2(float(F[:, :, 0].double().pow(2).mean().sqrt()))
    s_u = pow2(float(F[:, :, 1:].double().pow(2).mean().sqrt()))
    x, y = F[:, :-1].flatten(0, 1), F[:, 1:].flatten(0, 1)
    return ((x[:, :1] / s_r).contiguous(), (y[:, :1] / s_r).contiguous(),
            (x[:, 1:] / s_u).contiguous(), (y[:, 1:] / s_u).contiguous(), s_r, s_u)


def train_model(spec, X, Y, Xv, Yv, epochs: int, batch: int = 16, lr: float = 1e-2, seed: int = 7,
                log=None, tag=""):
    """AdamW (lr x 0.85 every 8 epochs); returns (best-validation parameters, history)."""
    import torch
    from paper_2604_27158_amd import fno as gfno
    from paper_2604_27158_amd import steady_init as SI
    params = W.fno_random_params(seed, gfno.param_layout(spec), spec.width)
    tr = gfno.Trainer(gfno.Fno(spec, params, N, N), params, lr=lr, weight_decay=1e-2)
    n = X.shape[0]
    g = torch.Generator().manual_seed(seed)
    hist, best = [], (float("inf"), None)
    t0 = time.perf_counter()
    for ep in range(epochs):
        tr.lr = lr * 0.85 ** (ep // 8)
        perm = torch.randperm(n, generator=g)
        tot, cnt = 0.0, 0
        for b0 in range(0, n - batch + 1, batch):
            idx = perm[b0:b0 + batch].cuda()
            tot += tr.step(X.index_select(0, idx).contiguous(), Y.index_select(0, idx).contiguous())
            cnt += 1
        vl = SI.evaluate(tr, Xv, Yv, batch)
        hist.append((ep, tot / max(cnt, 1), vl))
        if vl < best[0]:
            best = (vl, tr.params())
        if log:
            log(f"{tag} epoch {ep + 1}/{epochs} train {tot / max(cnt, 1):.4e} val {vl:.4e} "
                f"({time.perf_counter() - t0:.0f} s)")
    return best[1], hist


class Surrogate:
    """Both trained models of a group on the 128 x 128 grid.  step(fields) maps raw
    (rho, ux, uy) [3][N][N] (device) one Delta T ahead."""

    def __init__(self, group: str, path: str | None = None, graph: bool = False):
        import torch
        from paper_2604_27158_amd import fno as gfno
        spec_r, spec_u = GROUPS[group]
        with np.load(path or weights_path(group), allow_pickle=False) as z:
            self.rho = gfno.Fno(spec_r, z["rho_params"], N, N)
            self.u = gfno.Fno(spec_u, z["u_params"], N, N)
        self.group = group
        self.graph = graph
        # fixed input and output buffers (graph=True: the two forwards replay captured
        # graphs, which on MI355X is no faster than launching them)
        self.x = torch.empty((3, N, N), dtype=torch.float32, device="cuda")
        self.y = torch.empty((3, N, N), dtype=torch.float32, device="cuda")

    def step(self, fields=None):
        """One Delta T ahead from raw (rho, ux, uy) [3][N][N] on the device; with
        fields=None the input is what the caller already wrote into self.x (for
        instance Lattice.macros(out=sur.x)).  Returns self.y, which the next step
        overwrites."""
        if fields is not None and fields.data_ptr() != self.x.data_ptr():
            self.x.copy_(fields)
        x, y = self.x, self.y
        self.rho.forward(x[0:1].view(1, 1, N, N), out=y[0:1].view(1, 1, N, N), graph=self.graph)
        self.u.forward(x[1:3].view(1, 2, N, N), out=y[1:3].view(1, 2, N, N), graph=self.graph)
        return y


def vorticity(f):
    """dv/dx - du/dy by periodic central differences (lattice units), f [3][N][N]."""
    u, v = f[1], f[2]
    return 0.5 * (np.roll(v, -1, 1) - np.roll(v, 1, 1)) - 0.5 * (np.roll(u, -1, 0) - np.roll(u, 1, 0))


def errors(pred, ref):
    """(MSE over (rho, u, v), relative L2 vorticity error) of raw fields [3][N][N];
    infinite for a prediction that is no longer finite."""
    if not np.isfinite(pred).all():
        return float("inf"), float("inf")
    mse = float(np.mean((pred - ref) ** 2))
    wr = vorticity(ref)
    return mse, float(np.linalg.norm(vorticity(pred) - wr) / np.linalg.norm(wr))


def is_fno_interval(t: int, k: int) -> bool:
    """Interval t (0-based) of a 1:k hybrid is predicted by the FNO."""
    return t % (k + 1) == 0


def host_fields(G):
    """(rho, ux, uy) of a lattice as float64 host fields, rho = 1 + (rho - 1) from the
    library's full-resolution density deviation."""
    m = G.macros(rho_minus_one=True).cpu().numpy().astype(np.float64)
    m[0] += 1.0
    return m


def rollouts(sur: Surrogate, seed: int, neq: bool = False, mass: bool = False, ks=HYBRIDS):
    """Outputs 1..30 of the plain lattice, the pure FNO and the 1:k hybrids (k in ks)
    from one initial condition, as raw (rho, ux, uy) numpy fields."""
    import torch
    from paper_2604_27158_amd import lbmfno
    lat, r0, u0, v0 = W.double_shear_layer(seed, N)
    ic = torch.from_numpy(np.stack([r0, u0, v0]).astype(np.float32)).cuda()
    G = lbmfno.Lattice.from_workload(lat)
    G.reinit(ic[0], ic[1], ic[2])
    ref = []
    for _ in range(OUTPUTS):
        G.step(DT)
        ref.append(host_fields(G))
    x = ic.clone()
    pure = []
    for _ in range(OUTPUTS):
        x = sur.step(x)
        pure.append(x.cpu().numpy().astype(np.float64))
    hyb = {}
    for k in ks:
        H = lbmfno.Lattice.from_workload(lat)
        out = []
        with torch.cuda.stream(H.stream):
            H.reinit(ic[0], ic[1], ic[2])
            for t in range(OUTPUTS):
                if is_fno_interval(t, k):
                    H.macros(out=sur.x)
                    y = sur.step()
                    H.reinit(y[0], y[1], y[2], neq=neq, mass=mass)
                    out.append(y.cpu().numpy().astype(np.float64))
                else:
                    H.step(DT)
                    out.append(host_fields(H))
        hyb[k] = out
    return ref, pure, hyb


def timed_runs(sur: Surrogate, seed: int, reps: int = 3, neq: bool = False, mass: bool = False,
               ks=HYBRIDS):
    """Wall time of the 30 Delta T horizon on this GPU: plain lattice and each 1:k
    hybrid (FNO calls, re-initialisations and lattice steps; no measurements)."""
    import torch
    from paper_2604_27158_amd import lbmfno
    lat, r0, u0, v0 = W.double_shear_layer(seed, N)
    ic = torch.from_numpy(np.stack([r0, u0, v0]).astype(np.float32)).cuda()
    G = lbmfno.Lattice.from_workload(lat)

    def plain():
        with torch.cuda.stream(G.stream):
            G.reinit(ic[0], ic[1], ic[2])
            G.step(OUTPUTS * DT)

    def hybrid(k):
        # the surrogate runs on the lattice's stream: the hybrid's alternation
        # needs no cross-stream waits
        with torch.cuda.stream(G.stream):
            G.reinit(ic[0], ic[1], ic[2])
            t = 0
            while t < OUTPUTS:
                if is_fno_interval(t, k):
                    G.macros(out=sur.x)
                    y = sur.step()
                    G.reinit(y[0], y[1], y[2], neq=neq, mass=mass)
                    t += 1
                else:
                    n = 1
                    while t + n < OUTPUTS and not is_fno_interval(t + n, k):
                        n += 1
                    G.step(n * DT)
                    t += n

    def clock(fn):
        fn()
        G.synchronize()
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            G.synchronize()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        return best

    res = {"plain": clock(plain)}
    for k in ks:
        res[k] = clock(lambda k=k: hybrid(k))
    return res


SWEEP = (1, 2, 3, 4, 6, 9, 14, 29)   # 1:k cadences of the sweep (1:29: one FNO interval)


def cadence_sweep(group: str, seeds, ks=SWEEP, thresholds=(0.02, 0.05, 0.1), log=None,
                  path: str | None = None):
    """Wall time against error for 1:k hybrids over the 30-output horizon: for every
    cadence the global vorticity error and MSE (means over the outputs and the
    seeds) and eps_T (mean over the seeds of each seed's best-of-three wall times);
    then, for each stated vorticity error, the fastest cadence whose error stays
    within it and its eps_T against the plain lattice (time to error)."""
    sur = Surrogate(group, path)
    errs = {k: [] for k in ks}
    eps_t = {k: [] for k in ks}
    plain_s = []
    for n, s in enumerate(seeds):
        ref, _, hyb = rollouts(sur, s, ks=ks)
        times = timed_runs(sur, s, ks=ks)
        plain_s.append(times["plain"])
        for k in ks:
            e = np.array([errors(p, r) for p, r in zip(hyb[k], ref)])
            errs[k].append(e.mean(axis=0))
            eps_t[k].append((times["plain"] - times[k]) / times["plain"])
        if log:
            log(f"cadence sweep: seed {s} ({n + 1}/{len(seeds)})")
    rows = []
    for k in ks:
        m = np.mean(errs[k], axis=0)
        rows.append({"cadence": f"1:{k}", "k": k,
                     "eps_N_pct": 100.0 * sum(is_fno_interval(t, k) for t in range(OUTPUTS)) / OUTPUTS,
                     "eps_T_pct": 100.0 * float(np.mean(eps_t[k])),
                     "eps_T_pct_std": 100.0 * float(np.std(eps_t[k])),
                     "global_vorticity": float(m[1]), "global_mse": float(m[0])})
    tte = {}
    for eps in thresholds:
        ok = [r for r in rows if r["global_vorticity"] <= eps]
        best = max(ok, key=lambda r: r["eps_T_pct"]) if ok else None
        tte[f"vorticity<={eps:g}"] = ({"cadence": best["cadence"], "eps_T_pct": best["eps_T_pct"],
                                        "global_vorticity": best["global_vorticity"]} if best else None)
    return {"group": group, "seeds": len(seeds), "seconds_plain_mean": float(np.mean(plain_s)),
            "sweep": rows, "time_to_error": tte}


def study(group: str, seeds, log=None, path: str | None = None, neq: bool = False, mass: bool = False):
    """neq: hand the surrogate's fields to the lattice with the first-order
    non-equilibrium part (Lattice.reinit(..., neq=True)) instead of f_eq alone;
    mass: shift the handed-over density so that the lattice keeps its mass
    (Lattice.reinit(..., mass=True))."""
    sur = Surrogate(group, path)
    per = {"pure": [], **{k: [] for k in HYBRIDS}}
    curves = {"pure": np.zeros((OUTPUTS, 2)), **{k: np.zeros((OUTPUTS, 2)) for k in HYBRIDS}}
    t0 = time.perf_counter()
    for n, s in enumerate(seeds):
        ref, pure, hyb = rollouts(sur, s, neq, mass)
        for name, run in (("pure", pure), *((k, hyb[k]) for k in HYBRIDS)):
            e = np.array([errors(p, r) for p, r in zip(run, ref)])
            per[name].append(e.mean(axis=0))
            curves[name] += e
        if log and (n + 1) % 10 == 0:
            log(f"shear study: {n + 1}/{len(seeds)} trajectories ({time.perf_counter() - t0:.1f} s)")
    ns = len(seeds)
    glob = {name: np.mean(per[name], axis=0) for name in per}   # (MSE, vorticity) means
    times = timed_runs(sur, list(seeds)[0], neq=neq, mass=mass)
    out = {"group": group, "reinit": "f_eq + first-order f_neq" if neq else "f_eq, mass-conserving" if mass else "f_eq", "trajectories": ns, "outputs": OUTPUTS, "dt": DT,
           "global_mse": {str(k): float(glob[k][0]) for k in glob},
           "global_vorticity": {str(k): float(glob[k][1]) for k in glob},
           "error_reduction_pct": {}, "eps_T_pct": {}, "eps_N_pct": {},
           "seconds": {"plain": times["plain"], **{f"1:{k}": times[k] for k in HYBRIDS}},
           "curves": {str(k): (curves[k] / ns).tolist() for k in curves}}
    def reduction(a, b):
        if not np.isfinite(a):
            return 100.0 if np.isfinite(b) else None
        return 100.0 * (a - b) / a
    out["pure_fno_diverged"] = int(sum(not np.isfinite(e).all() for e in per["pure"]))
    for k in HYBRIDS:
        out["error_reduction_pct"][f"1:{k}"] = {"mse": reduction(glob["pure"][0], glob[k][0]),
                                                "vorticity": reduction(glob["pure"][1], glob[k][1])}
        n_fno = sum(is_fno_interval(t, k) for t in range(OUTPUTS))
        out["eps_N_pct"][f"1:{k}"] = 100.0 * n_fno / OUTPUTS
        out["eps_T_pct"][f"1:{k}"] = 100.0 * (times["plain"] - times[k]) / times["plain"]
    return out


def log_print(msg):
    print(msg, flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--group", default="small", choices=sorted(GROUPS))
    t.add_argument("--out", default=None)
    t.add_argument("--epochs", type=int, default=60)
    t.add_argument("--batch", type=int, default=16)
    e = sub.add_parser("eval")
    e.add_argument("--group", default="small", choices=sorted(GROUPS))
    e.add_argument("--weights", default=None)
    e.add_argument("--seeds", type=int, default=len(TEST_SEEDS))
    e.add_argument("--json", default=None)
    e.add_argument("--neq", action="store_true", help="re-initialise with the non-equilibrium part")
    e.add_argument("--mass", action="store_true", help="mass-conserving re-initialisation")
    c = sub.add_parser("sweep")
    c.add_argument("--group", default="small", choices=sorted(GROUPS))
    c.add_argument("--weights", default=None)
    c.add_argument("--seeds", type=int, default=6)
    args = ap.parse_args()
    from paper_2604_27158_amd import lbmfno
    lbmfno.load()
    if args.cmd == "sweep":
        import json
        log_print(json.dumps(cadence_sweep(args.group, list(TEST_SEEDS)[:args.seeds], log=log_print,
                                           path=args.weights)))
        return
    if args.cmd == "eval":
        import json
        res = study(args.group, list(TEST_SEEDS)[:args.seeds], log_print, args.weights, neq=args.neq,
                    mass=args.mass)
        log_print(json.dumps({k: v for k, v in res.items() if k != "curves"}))
        if args.json:
            with open(args.json, "w") as f:
                json.dump(res, f, indent=1)
        return
    from paper_2604_27158_amd import fno as gfno
    t0 = time.perf_counter()
    F = simulate(TRAIN_SEEDS, log_print)
    Fv = simulate(VAL_SEEDS, log_print)
    import torch
    bad = int((~torch.isfinite(F).flatten(1).all(dim=1)).sum()) + int((~torch.isfinite(Fv).flatten(1).all(dim=1)).sum())
    if bad:
        raise RuntimeError(f"{bad} shear trajectories lost stability")
    Xr, Yr, Xu, Yu, s_r, s_u = pairs(F)
    xv, yv = Fv[:, :-1].flatten(0, 1), Fv[:, 1:].flatten(0, 1)
    Xrv, Yrv = (xv[:, :1] / s_r).contiguous(), (yv[:, :1] / s_r).contiguous()
    Xuv, Yuv = (xv[:, 1:] / s_u).contiguous(), (yv[:, 1:] / s_u).contiguous()
    del F, Fv
    log_print(f"pairs: train {Xr.shape[0]}, val {Xrv.shape[0]}; scales rho-1 {s_r}, u {s_u} "
              f"({time.perf_counter() - t0:.1f} s)")
    spec_r, spec_u = GROUPS[args.group]
    pr, hr = train_model(spec_r, Xr, Yr, Xrv, Yrv, args.epochs, args.batch, log=log_print, tag="rho")
    pu, hu = train_model(spec_u, Xu, Yu, Xuv, Yuv, args.epochs, args.batch, log=log_print, tag="u")
    out = args.out or weights_path(args.group)
    os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
    np.savez(out,
             rho_params=gfno.fold_affine(spec_r, pr, [s_r], [1.0], [s_r], [1.0]).astype(np.float32),
             u_params=gfno.fold_affine(spec_u, pu, [s_u, s_u], [0.0, 0.0], [s_u, s_u], [0.0, 0.0]).astype(np.float32),
             rho_scale=np.float64(s_r), u_scale=np.float64(s_u),
             rho_history=np.array(hr, dtype=np.float64), u_history=np.array(hu, dtype=np.float64),
             epochs=np.int64(args.epochs))
    log_print(f"wrote {out} ({time.perf_counter() - t0:.0f} s total)")


if __name__ == "__main__":
    main()
