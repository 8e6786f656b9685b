"""Shared helpers of the GPU parity tests (comparison metrics)."""
import numpy as np


def min_image(d, box):
    box = np.asarray(box, dtype=np.float64)
    return d - box * np.round(d / box)


def rel_err(g, o, ref):
    """max |g - o| / max(|o|, ref) elementwise (the per-component parity
    metric)."""
    g = np.asarray(g, dtype=np.float64)
    o = np.asarray(o, dtype=np.float64)
    return float(np.max(np.abs(g - o) / np.maximum(np.abs(o), ref))) if o.size else 0.0


def compare_states(g, o, box, tol, what=("s", "x", "v", "Te")):
    """Per-component relative errors of a GPU state against the oracle with
    reference scales 1 (spins), 1 A (positions, compared by minimum image),
    the rms velocity, 1 K (electron temperatures)."""
    errs = {}
    if "s" in what:
        errs["s"] = rel_err(g["s"], o["s"], 1.0)
    if "x" in what:
        dx = min_image(g["x"] - o["x"], box)
        errs["x"] = float(np.max(np.abs(dx)))
    if "v" in what:
        vr = max(float(np.sqrt((o["v"] ** 2).mean())), 1e-30)
        errs["v"] = rel_err(g["v"], o["v"], vr)
    if "Te" in what:
        errs["Te"] = rel_err(g["Te"], o["Te"], 1.0)
    bad = {k: v for k, v in errs.items() if not v <= tol}
    return errs, bad
