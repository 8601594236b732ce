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
    """rel-L2 per field (rho, ux, uy) over fluid nodes, plus rho - 1 (informational)."""
    fl = mask == 0
    g = [np.asarray(x, dtype=np.float64) for x in gpu_macros]
    r = [np.asarray(x, dtype=np.float64) for x in ref_macros]
    out = {k: rel_l2(gg, rr, fl) for k, gg, rr in zip(("rho", "ux", "uy"), g, r)}
    out["rho-1"] = rel_l2(g[0] - 1.0, r[0] - 1.0, fl)
    return out
