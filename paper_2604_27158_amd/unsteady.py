"""Unsteady hybrid super-time-stepping with a trained FNO (the paper's Sec. 2.3 and
3.2 method, on the configured flow-past-ellipses workload): the flagship FNO
(4 -> 3 channels, width 32, 4 Fourier layers, 12 x 12 modes, GELU, decoder 1 x 32)
maps (rho, ux, uy, mask) at time t to (rho, ux, uy) at t + dt_fno lattice steps; the
hybrid alternates K chained FNO calls with an equilibrium re-initialisation and
n_lbm lattice steps.  Against the plain lattice over the same horizon it reports
the wall time on this GPU and the field error at a stated model time (time to
error), plus the error of a pure FNO rollout.

Data: trajectories of flow past 1-5 random ellipses at 256 x 128 (Re ~ U(100, 200)),
spun up from the plug flow, sampled every dt_fno steps by the batched lattice;
training pairs are consecutive samples.  Training: AdamW (lr 1e-2 x 0.85 every 10
epochs), MSE on normalised fields; the normalisation (power-of-two scales of
rho - 1 and u) is folded into the lift's first layer and the decoder's last layer,
so the runtime path feeds raw fields to the library's FNO kernels.

    python -m paper_2604_27158_amd.unsteady train --out weights.npz
    python -m paper_2604_27158_amd.unsteady eval
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

NX, NY = 256, 128
DT_FNO = 100          # lattice steps per FNO call
K_FNO = 5             # FNO calls per hybrid cycle
N_LBM = 200           # lattice steps per hybrid cycle
CYCLES = 20
SPINUP = 4000         # lattice steps from the plug flow before the first sample
SPEC = W.FnoSpec()    # 4 -> 3, width 32, 4 layers, 12 x 12 modes, GELU, decoder 1 x 32
TRAIN_SEEDS = range(10000, 10200)
VAL_SEEDS = range(20000, 20020)
TEST_SEEDS = range(30000, 30020)
SAMPLES = 40          # samples per training trajectory (39 pairs)
DEFAULT_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights",
                               "ellipse_hybrid_256x128.npz")


def geometry(seed: int) -> W.Lattice:
    return W.ellipse_flow(seed, size=(NX, NY))


def sample_trajectories(seeds, samples: int, log=None, per_launch: int = 100):
    """Fields (rho - 1, ux, uy) every DT_FNO steps after the spin-up, for each seed:
    device tensor [n][samples][3][ny][nx], masks [n][ny][nx] (float), and a flag per
    trajectory that it stayed finite."""
    import torch
    from paper_2604_27158_amd import lbmfno
    seeds = list(seeds)
    n = len(seeds)
    F = torch.empty((n, samples, 3, NY, NX), dtype=torch.float32, device="cuda")
    M = torch.empty((n, NY, NX), dtype=torch.float32, device="cuda")
    ok = torch.ones(n, dtype=torch.bool)
    t0 = time.perf_counter()
    for k0 in range(0, n, per_launch):
        lats = [geometry(s) for s in seeds[k0:k0 + per_launch]]
        batch = lbmfno.Batch(lats)
        for i, lat in enumerate(lats):
            batch.trajectory(i).reinit(*(torch.from_numpy(a) for a in W.plug_flow(lat)))
        batch.step(SPINUP)
        for s in range(samples):
            if s:
                batch.step(DT_FNO)
            for i in range(len(lats)):
                F[k0 + i, s].copy_(batch.trajectory(i).macros(rho_minus_one=True))
        for i in range(len(lats)):
            view = batch.trajectory(i)
            M[k0 + i].copy_(view.mask.to(torch.float32))
        torch.cuda.synchronize()
        batch.close()
        if log:
            log(f"trajectories: {k0 + len(lats)}/{n} ({time.perf_counter() - t0:.1f} s)")
    fin = torch.isfinite(F).flatten(1).all(dim=1).cpu()
    ok &= fin
    # trajectories whose SRT run loses stability (jets past the lattice sound speed)
    ok &= (F[:, :, 1:].abs().flatten(1).amax(dim=1) < 0.35).cpu()
    return F, M, ok


def pow2(x: float) -> float:
    return 2.0 ** round(math.log2(max(x, 1e-30)))


def build_pairs(F, M, ok):
    """Network inputs [P][4][ny][nx] = (rho, ux, uy, mask) and targets [P][3][ny][nx]
    = (rho, ux, uy) one DT_FNO later, from consecutive samples of the stable
    trajectories (absolute rho)."""
    import torch
    idx = torch.nonzero(ok).flatten().tolist()
    xs, ys = [], []
    for i in idx:
        f = F[i]
        x = torch.cat([f[:-1], M[i].expand(f.shape[0] - 1, 1, NY, NX)], dim=1)
        x[:, 0] += 1.0
        y = f[1:].clone()
        y[:, 0] += 1.0
        xs.append(x)
        ys.append(y)
    return torch.cat(xs).contiguous(), torch.cat(ys).contiguous()


def normalisation(X):
    """Power-of-two scales of rho - 1 and of the velocity over the inputs."""
    s_r = pow2(float((X[:, 0] - 1.0).double().pow(2).mean().sqrt()))
    s_u = pow2(float(X[:, 1:3].double().pow(2).mean().sqrt()))
    return s_r, s_u


def normalise(T, s_r, s_u, channels=3):
    """In-place: rho -> (rho - 1) / s_r, u -> u / s_u (first `channels` channels)."""
    T[:, 0] = (T[:, 0] - 1.0) / s_r
    T[:, 1:3] = T[:, 1:3] / s_u
    return T


def fold(params: np.ndarray, s_r: float, s_u: float) -> np.ndarray:
    """Packed parameters of the network on raw fields: the input map
    z' = ((rho - 1)/s_r, ux/s_u, uy/s_u, mask, coords) folded into the lift's first
    layer, and the output map (rho, ux, uy) = (1 + s_r o0, s_u o1, s_u o2) folded into
    the decoder's last layer."""
    from paper_2604_27158_amd import fno as gfno
    return gfno.fold_affine(SPEC, params, [s_r, s_u, s_u, 1.0], [1.0, 0.0, 0.0, 0.0],
                            [s_r, s_u, s_u], [1.0, 0.0, 0.0])


def train(X, Y, Xv, Yv, epochs: int, batch: int = 16, lr: float = 1e-2, seed: int = 3, log=None):
    """AdamW on normalised pairs; returns (best-validation parameters, history)."""
    import torch
    from paper_2604_27158_amd import fno as gfno
    from paper_2604_27158_amd import steady_init as SI
    params = W.fno_random_params(seed, gfno.param_layout(SPEC), SPEC.width)
    model = gfno.Fno(SPEC, params, NY, NX)
    tr = gfno.Trainer(model, params, lr=lr, weight_decay=1e-2)
    n = X.shape[0]
    g = torch.Generator().manual_seed(seed)
    hist, best = [], (float("inf"), None)
    t0 = time.perf_counter()
    for ep in range(epochs):
        tr.lr = lr * 0.85 ** (ep // 10)
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
            log(f"epoch {ep + 1}/{epochs} train {tot / max(cnt, 1):.4e} val {vl:.4e} lr {tr.lr:.2e} "
                f"({time.perf_counter() - t0:.0f} s)")
    return best[1], hist


class TrainedFno:
    """The trained flagship FNO bound to the 256 x 128 grid (raw fields in and out)."""

    def __init__(self, path: str = DEFAULT_WEIGHTS):
        from paper_2604_27158_amd import fno as gfno
        with np.load(path, allow_pickle=False) as z:
            self.params = z["params"]
        self.model = gfno.Fno(SPEC, self.params, NY, NX)


def rel_l2(a, b, fl):
    import torch
    d = ((a - b)[:, fl].double().pow(2).sum(dim=1).sqrt() / b[:, fl].double().pow(2).sum(dim=1).sqrt())
    return [float(v) for v in d]


def hybrid_study(fno: "TrainedFno", seeds, log=None):
    """For each held-out trajectory (after the spin-up): the plain lattice over the
    CYCLES-cycle horizon (reference), the hybrid (K_FNO calls, reinit, N_LBM steps per
    cycle), and a pure FNO rollout, compared at each cycle's end; and wall times."""
    import torch
    from paper_2604_27158_amd import lbmfno
    from paper_2604_27158_amd.hybrid import HybridRunner, Guard, step_reduction
    horizon = CYCLES * (K_FNO * DT_FNO + N_LBM)
    per_seed = []
    for s in seeds:
        lat = geometry(s)
        plain = lbmfno.Lattice.from_workload(lat)
        plain.reinit(*(torch.from_numpy(a) for a in W.plug_flow(lat)))
        plain.step(SPINUP)
        start = plain.save_state()
        fl = plain.mask == 0
        ref = []
        for c in range(CYCLES):
            plain.step(K_FNO * DT_FNO + N_LBM)
            ref.append(plain.macros().clone())
        if not all(bool(torch.isfinite(r).all()) for r in ref) or max(float(r[1:].abs().max()) for r in ref) > 0.35:
            if log:
                log(f"seed {s}: plain run unstable, skipped")
            continue
        # hybrid from the same state
        hyb = lbmfno.Lattice.from_workload(lat)
        hyb.load_state(start)
        runner = HybridRunner(hyb, fno.model, dt_fno=DT_FNO, k_fno=K_FNO, n_lbm=N_LBM,
                              guard=Guard(max_speed=0.35, mass_rel_tol=0.05))
        errs = []
        for c in range(CYCLES):
            runner.cycle()
            errs.append(rel_l2(hyb.macros(), ref[c], fl))
        # pure FNO rollout over the same horizon (every lattice interval replaced by FNO calls)
        pure = []
        m0 = lbmfno.Lattice.from_workload(lat)
        m0.load_state(start)
        x = torch.empty((1, 4, NY, NX), dtype=torch.float32, device="cuda")
        x[0, :3] = m0.macros()
        x[0, 3] = (m0.mask != 0).float()
        calls_per_cycle = (K_FNO * DT_FNO + N_LBM) // DT_FNO
        for c in range(CYCLES):
            for _ in range(calls_per_cycle):
                y = fno.model(x)
                x[0, :3] = y[0]
            pure.append(rel_l2(x[0, :3], ref[c], fl))
        rec = {"seed": s, "name": lat.name, "tau": lat.tau,
               "hybrid_rel_l2": errs, "pure_fno_rel_l2": pure,
               "fallbacks": len(runner.log.fallbacks)}
        per_seed.append(rec)
        if log:
            log(f"seed {s}: final rel-L2 hybrid (rho, ux, uy) " + " ".join(f"{v:.2e}" for v in errs[-1]) +
                " | pure FNO " + " ".join(f"{v:.2e}" for v in pure[-1]) + f" | fallbacks {rec['fallbacks']}")
    # wall time on this GPU for the horizon, plain vs hybrid, on the first stable seed;
    # the hybrid's guard is resolved speculatively (one cycle behind, same results)
    lat = geometry(per_seed[0]["seed"])
    G = lbmfno.Lattice.from_workload(lat)
    G.reinit(*(torch.from_numpy(a) for a in W.plug_flow(lat)))
    G.step(SPINUP)
    start = G.save_state()
    t_plain = t_hyb = float("inf")
    H = lbmfno.Lattice.from_workload(lat)
    H.load_state(start)
    HybridRunner(H, fno.model, dt_fno=DT_FNO, k_fno=K_FNO, n_lbm=N_LBM, speculative=True).run(1)  # warm-up
    for _ in range(3):   # best of three, each from the same state
        G.load_state(start)
        G.synchronize()
        t0 = time.perf_counter()
        with torch.cuda.stream(G.stream):
            G.step(horizon)
        G.synchronize()
        t_plain = min(t_plain, time.perf_counter() - t0)
        H.load_state(start)
        runner = HybridRunner(H, fno.model, dt_fno=DT_FNO, k_fno=K_FNO, n_lbm=N_LBM,
                              guard=Guard(max_speed=0.35, mass_rel_tol=0.05), speculative=True)
        H.synchronize()
        t0 = time.perf_counter()
        runner.run(CYCLES)
        H.synchronize()
        t_hyb = min(t_hyb, time.perf_counter() - t0)
    eps_n = step_reduction(K_FNO, DT_FNO, N_LBM)
    gm = lambda key, c: float(np.exp(np.mean([np.log(max(np.mean(r[key][c]), 1e-30)) for r in per_seed])))
    return {"seeds_evaluated": len(per_seed), "horizon_steps": horizon, "cycles": CYCLES,
            "k_fno": K_FNO, "dt_fno": DT_FNO, "n_lbm": N_LBM, "eps_N": eps_n,
            "seconds_plain": t_plain, "seconds_hybrid": t_hyb,
            "eps_T": (t_plain - t_hyb) / t_plain,
            "geomean_rel_l2_hybrid_final": gm("hybrid_rel_l2", -1),
            "geomean_rel_l2_pure_fno_final": gm("pure_fno_rel_l2", -1),
            "geomean_rel_l2_hybrid_mean_over_cycles": float(np.exp(np.mean(
                [np.log(max(np.mean(np.mean(r["hybrid_rel_l2"], axis=0)), 1e-30)) for r in per_seed]))),
            "per_seed": per_seed}


# (K FNO calls of DT_FNO steps, n lattice steps) per cycle; every cycle length divides
# the 14 000-step horizon.  (5, 200) is the configured cadence.
CADENCES = ((1, 100), (1, 300), (1, 400), (1, 600), (2, 500), (5, 200), (1, 900), (5, 500), (1, 1900),
            (1, 3400))
HORIZON = CYCLES * (K_FNO * DT_FNO + N_LBM)


def velocity_error(a, b, fl):
    """rel-L2 over fluid nodes of the velocity as a vector field, fields [3][ny][nx]."""
    d = (a[1:] - b[1:])[:, fl].double().pow(2).sum().sqrt()
    return float(d / b[1:][:, fl].double().pow(2).sum().sqrt())


def cadence_study(fno: "TrainedFno", seeds, cadences=CADENCES, thresholds=(0.05, 0.1, 0.2),
                  reps: int = 3, log=None):
    """Wall time against error for hybrid cadences over the same 14 000-step horizon
    after the spin-up: for each cadence the velocity error at the horizon against the
    plain lattice (mean over seeds) and eps_T (mean over seeds of best-of-`reps` wall
    times, speculative guard); then, per stated velocity error, the fastest cadence
    within it (time to error).  Seeds whose plain run loses stability are skipped."""
    import torch
    from paper_2604_27158_amd import lbmfno
    from paper_2604_27158_amd.hybrid import HybridRunner, Guard, step_reduction
    err = {c: [] for c in cadences}
    eps_t = {c: [] for c in cadences}
    used = []
    for s in seeds:
        lat = geometry(s)
        G = lbmfno.Lattice.from_workload(lat)
        G.reinit(*(torch.from_numpy(a) for a in W.plug_flow(lat)))
        G.step(SPINUP)
        start = G.save_state()
        G.step(HORIZON)
        ref = G.macros().clone()
        if not bool(torch.isfinite(ref).all()) or float(ref[1:].abs().max()) > 0.35:
            if log:
                log(f"seed {s}: plain run unstable, skipped")
            continue
        used.append(s)
        fl = G.mask == 0
        H = lbmfno.Lattice.from_workload(lat)

        def run_plain():
            G.load_state(start)
            G.synchronize()
            t0 = time.perf_counter()
            with torch.cuda.stream(G.stream):
                G.step(HORIZON)
            G.synchronize()
            return time.perf_counter() - t0

        def run_hybrid(K, n):
            H.load_state(start)
            r = HybridRunner(H, fno.model, dt_fno=DT_FNO, k_fno=K, n_lbm=n,
                             guard=Guard(max_speed=0.35, mass_rel_tol=0.05), speculative=True)
            H.synchronize()
            t0 = time.perf_counter()
            r.run(HORIZON // (K * DT_FNO + n))
            H.synchronize()
            return time.perf_counter() - t0

        run_plain()
        t_plain = min(run_plain() for _ in range(reps))
        for (K, n) in cadences:
            run_hybrid(K, n)
            err[(K, n)].append(velocity_error(H.macros(), ref, fl))
            t = min(run_hybrid(K, n) for _ in range(reps))
            eps_t[(K, n)].append((t_plain - t) / t_plain)
        if log:
            log(f"seed {s}: " + " ".join(f"{K}x{DT_FNO}+{n}: err {err[(K, n)][-1]:.3f} eps_T "
                                          f"{100 * eps_t[(K, n)][-1]:.1f}%" for (K, n) in cadences))
    rows = []
    for (K, n) in cadences:
        rows.append({"cadence": f"{K} x {DT_FNO} FNO + {n} LBM", "k_fno": K, "n_lbm": n,
                     "eps_N_pct": 100.0 * step_reduction(K, DT_FNO, n),
                     "eps_T_pct": 100.0 * float(np.mean(eps_t[(K, n)])),
                     "eps_T_pct_std": 100.0 * float(np.std(eps_t[(K, n)])),
                     "velocity_rel_l2_at_horizon": float(np.mean(err[(K, n)]))})
    tte = {}
    for eps in thresholds:
        ok = [r for r in rows if r["velocity_rel_l2_at_horizon"] <= eps]
        best = max(ok, key=lambda r: r["eps_T_pct"]) if ok else None
        tte[f"velocity<={eps:g}"] = ({k: best[k] for k in ("cadence", "eps_T_pct", "velocity_rel_l2_at_horizon")}
                                      if best else None)
    return {"seeds": len(used), "horizon_steps": HORIZON, "sweep": rows, "time_to_error": tte}


def log_print(msg):
    print(msg, flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--out", default=DEFAULT_WEIGHTS)
    t.add_argument("--train", type=int, default=len(TRAIN_SEEDS))
    t.add_argument("--epochs", type=int, default=40)
    t.add_argument("--batch", type=int, default=16)
    e = sub.add_parser("eval")
    e.add_argument("--weights", default=DEFAULT_WEIGHTS)
    e.add_argument("--seeds", type=int, default=len(TEST_SEEDS))
    e.add_argument("--json", default=None)
    c = sub.add_parser("sweep")
    c.add_argument("--weights", default=DEFAULT_WEIGHTS)
    c.add_argument("--seeds", type=int, default=8)
    args = ap.parse_args()
    import torch
    from paper_2604_27158_amd import lbmfno
    lbmfno.load()
    if args.cmd == "sweep":
        import json
        log_print(json.dumps(cadence_study(TrainedFno(args.weights), list(TEST_SEEDS)[:args.seeds],
                                           log=log_print)))
        return
    if args.cmd == "eval":
        import json
        res = hybrid_study(TrainedFno(args.weights), list(TEST_SEEDS)[:args.seeds], log=log_print)
        log_print(json.dumps({k: v for k, v in res.items() if k != "per_seed"}))
        if args.json:
            with open(args.json, "w") as f:
                json.dump(res, f, indent=1)
        return
    t0 = time.perf_counter()
    F, M, ok = sample_trajectories(list(TRAIN_SEEDS)[:args.train], SAMPLES, log_print)
    Fv, Mv, okv = sample_trajectories(list(VAL_SEEDS), 10, log_print)
    log_print(f"stable trajectories: train {int(ok.sum())}/{len(ok)}, val {int(okv.sum())}/{len(okv)} "
              f"({time.perf_counter() - t0:.1f} s)")
    X, Y = build_pairs(F, M, ok)
    Xv, Yv = build_pairs(Fv, Mv, okv)
    del F, Fv
    s_r, s_u = normalisation(X)
    for T in (X, Xv):
        normalise(T, s_r, s_u)
    for T in (Y, Yv):
        normalise(T, s_r, s_u)
    log_print(f"pairs: train {X.shape[0]}, val {Xv.shape[0]}; scales rho-1 {s_r}, u {s_u}")
    p, hist = train(X, Y, Xv, Yv, args.epochs, args.batch, log=log_print)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    np.savez(args.out, params=fold(p, s_r, s_u).astype(np.float32), rho_scale=np.float64(s_r),
             u_scale=np.float64(s_u), history=np.array(hist, dtype=np.float64),
             pairs=np.int64(X.shape[0]), epochs=np.int64(args.epochs))
    log_print(f"wrote {args.out} ({time.perf_counter() - t0:.0f} s total)")


if __name__ == "__main__":
    main()
