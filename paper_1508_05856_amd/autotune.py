"""Autotuner for batched and served solves: the leaf block order per
(matrix kind, size bucket, leaf precision, tau).

The leaf block order b sets the cull granularity (smaller b culls more
finely, so fewer flops), the MFMA tile shape and the waves per output tile
(b = 64: four waves of 32 x 32; b = 32 and 16: one wave; BF16x3 at b = 64: a
workgroup of four waves per 2 x 2 quad of tiles), and also which triples are
culled, so it moves the floor the solve stagnates at.  For each kind, size
bucket and tau this times complete Newton-Schulz solves of a representative
instance with every candidate leaf, records each candidate's status, update
count and exact ||I - Y Z||_F, and keeps the fastest of the candidates that
end with status >= 0 and a residual within ACCURACY_FACTOR of the best one,
so a faster leaf is never chosen at a worse accuracy.  The table is cached as
JSON keyed by (arch, precision, tau, kind, n bucket).

    python -m paper_1508_05856_amd.autotune [--prec f32] [--tau 1e-6 1e-4]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuning.json")
ARCH = "gfx950"
BUCKETS = (256, 512, 1024, 2048, 4096)
ACCURACY_FACTOR = 2.0


def candidate_leaves(prec: str):
    return (32, 64) if prec.startswith("bf16") else (16, 32, 64)


def _representative(kind: str, n: int):
    from . import inputs
    if kind == "kms":
        return inputs.kms(n, 0.7)
    m = inputs.smallest_cube(n)
    return inputs.gramian_from_positions(inputs.gauss_positions(m, 1.0, 0.1, 0, n))


def _key(prec: str, tau: float) -> str:
    return f"{ARCH}/{prec}/tau{tau:g}"


def _exact_residual(ctx, Y, Z) -> float:
    """||I - Y Z||_F with a dense FP64 product through the library (tau = 0)."""
    import torch
    C, _, _ = ctx.spamm_multiply(Y, Z, 0.0, 32)
    C.diagonal().sub_(1.0)
    return float(torch.linalg.norm(C))


def choose(cands: dict) -> int | None:
    """The fastest candidate among those with status >= 0 whose exact
    residual is within ACCURACY_FACTOR of the best such residual."""
    ok = {lf: c for lf, c in cands.items() if c["status"] >= 0 and math.isfinite(c["resid"])}
    if not ok:
        return None
    best = min(c["resid"] for c in ok.values())
    fair = {lf: c for lf, c in ok.items() if c["resid"] <= ACCURACY_FACTOR * best}
    return int(min(fair, key=lambda lf: fair[lf]["ms"]))


def tune(ctx, prec: str = "f32", tau: float = 1e-6, tol: float = 1e-6, maxit: int = 40, tau_s_rel: float = 0.01,
         kinds=("kms", "gauss"), buckets=BUCKETS, leaves=None, reps: int = 2, max_n: int = 4096) -> dict:
    """Times every candidate leaf on each (kind, bucket) and returns the table."""
    import torch
    leaves = leaves or candidate_leaves(prec)
    table = {}
    for kind in kinds:
        for n in buckets:
            if n > max_n:
                continue
            s = torch.from_numpy(_representative(kind, n)).cuda()
            cands = {}
            for leaf in leaves:
                best = math.inf
                for _ in range(reps + 1):  # the first run also builds tables and graphs
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    Y, Z, info = ctx.ns_sqrt(s, tau, tol, maxit, leaf=leaf, prec=prec, tau_s=tau_s_rel * tau,
                                             stagnation_stop=True, raise_on_error=False)
                    torch.cuda.synchronize()
                    best = min(best, time.perf_counter() - t0)
                resid = _exact_residual(ctx, Y, Z) if info["status"] >= 0 else math.inf
                cands[leaf] = dict(ms=best * 1e3, status=int(info["status"]), iterations=int(info["iterations"]),
                                   resid=resid)
                del Y, Z
            pick = choose(cands)
            table[f"{kind}/{n}"] = dict(leaf=pick if pick is not None else max(leaves),
                                        valid=pick is not None,
                                        candidates={str(lf): c for lf, c in cands.items()})
            del s
    return table


def load(prec: str = "f32", tau: float = 1e-6, path: str = CACHE) -> dict | None:
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f).get(_key(prec, tau))


def save(table: dict, prec: str, tau: float, path: str = CACHE) -> None:
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    data[_key(prec, tau)] = table
    with open(path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)


def choose_leaf(table: dict | None, kind: str, n: int, default: int = 64) -> int:
    """Leaf of the nearest tuned bucket (log scale) for this kind."""
    if not table:
        return default
    cands = [(abs(math.log(n / int(k.split("/")[1]))), v["leaf"]) for k, v in table.items()
             if k.split("/")[0] == kind]
    return min(cands)[1] if cands else default


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--prec", default="f32")
    p.add_argument("--tau", type=float, nargs="+", default=[1e-6, 1e-4])
    p.add_argument("--tol", type=float, default=1e-6)
    p.add_argument("--max-n", type=int, default=4096)
    p.add_argument("--out", default=CACHE, help="JSON cache to update")
    a = p.parse_args()
    from . import spamm
    ctx = spamm.Context(0)
    for tau in a.tau:
        table = tune(ctx, a.prec, tau, a.tol, max_n=a.max_n)
        save(table, a.prec, tau, a.out)
        print(json.dumps({_key(a.prec, tau): table}, indent=1), flush=True)


if __name__ == "__main__":
    main()
