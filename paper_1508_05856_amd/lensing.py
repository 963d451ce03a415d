"""Volume and lensing instrumentation of Newton-Schulz solves.

The culled volume of a product c = a (x)_tau b is its retained triple count
|R| times b^3, reported by the paper as a percentage of the dense n^3
(the volumes of Secs. 5.4 and 6.2).  Lensing (Sec. 7.2) is the collapse of
that volume onto the plane diagonals of the ijk cube as the iteration
contracts to the identity: in y_k = h_{k-1} (x) y_{k-1} the operand h tends to
I, so the retained triples concentrate on i = k; in z_k = z_{k-1} (x) h_{k-1}
on k = j.  This module exports the retained triples of every product of a
solve, one iteration per step, and measures both.
"""
from __future__ import annotations

import numpy as np

CHANNELS = ("x", "y", "z")


def volume_percent(count: int | np.ndarray, n: int, leaf: int):
    """|R| b^3 as a percentage of the dense n^3 (the logical order n)."""
    return np.asarray(count, dtype=np.float64) * leaf ** 3 * 100.0 / float(n) ** 3


def plane_fractions(triples: np.ndarray, width: int = 0) -> dict:
    """Fractions of the retained triples within `width` leaf blocks of the
    plane diagonals i = k (a's diagonal), k = j (b's) and i = j (c's)."""
    t = np.asarray(triples).reshape(-1, 3).astype(np.int64)
    if t.shape[0] == 0:
        return {"ik": 0.0, "kj": 0.0, "ij": 0.0}
    i, j, k = t[:, 0], t[:, 1], t[:, 2]
    return {"ik": float(np.mean(np.abs(i - k) <= width)),
            "kj": float(np.mean(np.abs(k - j) <= width)),
            "ij": float(np.mean(np.abs(i - j) <= width))}


def trace_solve(ctx, s, tau: float, tol: float, maxit: int, leaf: int = 32, width: int = 0, keep: bool = False,
                **opts) -> list[dict]:
    """Runs one solve an iteration per step and records, after every step,
    the volume and plane-diagonal fractions of its x, y and z products (and
    the triples themselves with keep=True).  Returns one record per step."""
    sv = ctx.solve_begin(s, tau, tol, maxit, leaf=leaf, **opts)
    n = s.shape[0]
    recs = []
    try:
        while True:
            running = ctx.solve_step([sv], 1)
            info = sv.poll()
            # after a step that ended in an update, the x product is that of
            # iteration k - 1; after the stop, that of iteration k
            rec = {"k": info["iterations"], "stopped": running == 0, "resid": info["resid"],
                   "trace_err": info["trace_err"]}
            for w, name in enumerate(CHANNELS):
                t = sv.triples(w).cpu().numpy()
                rec[name] = {"count": int(t.shape[0]), "vol_percent": float(volume_percent(t.shape[0], n, leaf)),
                             **plane_fractions(t, width)}
                if keep:
                    rec[name]["triples"] = t
            recs.append(rec)
            if running == 0:
                break
    finally:
        sv.finish(want_outputs=False)
    return recs
