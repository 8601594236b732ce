"""Shared test helpers: error norms and workload construction (no method arithmetic)."""
import numpy as np


def rel_l2(a, b, fluid=None):
    """||a - b||_2 / ||b||_2 over the selected nodes."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if fluid is not None:
        a, b = a[..., fluid], b[..., fluid]
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a - b))


def field_errors(gpu_macros, ref_macros, mask):
    """rel-L2 per field (rho, ux, uy) over fluid nodes, plus that of the density
    deviation rho - 1 (the pressure field, c_s^2 (rho - 1))."""
    fl = mask == 0
    g = [np.asarray(x, dtype=np.float64) for x in gpu_macros]
    r = [np.asarray(x, dtype=np.float64) for x in ref_macros]
    out = {k: rel_l2(gg, rr, fl) for k, gg, rr in zip(("rho", "ux", "uy"), g, r)}
    out["rho-1"] = rel_l2(g[0] - 1.0, r[0] - 1.0, fl)
    return out


def gpu_fields(G):
    """(rho, ux, uy) of a device lattice as float64 arrays, with rho = 1 + (rho - 1)
    from the full-resolution density deviation the library writes (rho itself in
    float32 would round the deviation to 2^-24 absolute, far coarser than the state
    holds it)."""
    m = G.macros(rho_minus_one=True).detach().cpu().numpy().astype(np.float64)
    return 1.0 + m[0], m[1], m[2]


def rho_dev_storage_bound(ref, steps, fluid):
    """Upper bound of the relative L2 error of rho - 1 that float32 population storage
    alone can cause after `steps` steps: every step stores each population once,
    rounding it by up to 2^-25 of its deviation from w, and the deviations are of the
    order of the speed, so the density deviation takes a random walk of at most
    ~2^-24 |u|_max per step; relative to the rms of the reference's rho - 1 (with a
    factor 1.5).  It matters where the flow is fast and its pressure field weak."""
    r = [np.asarray(a, dtype=np.float64)[fluid] for a in ref]
    umax = float(np.sqrt(r[1] ** 2 + r[2] ** 2).max())
    return 1.5 * np.sqrt(steps) * 2.0 ** -24 * umax / float(np.sqrt(np.mean((r[0] - 1.0) ** 2)))
