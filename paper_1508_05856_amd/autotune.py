"""Leaf-size autotuner for batched and served solves.

The leaf block order b sets both the cull granularity (smaller b culls more
finely, so fewer flops) and the MFMA tile (larger b keeps the matrix cores
busier).  For each matrix kind and size bucket this times complete Newton-
Schulz solves of a representative instance with every candidate leaf and keeps
the fastest; the table is cached as JSON keyed by (arch, precision, tau, kind,
n bucket).

    python -m paper_1508_05856_amd.autotune [--prec f32] [--tau 1e-6]
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
BUCKETS = (256, 512, 1024, 2048, 4096, 8192)
LEAVES = (32, 64)


def _representative(kind: str, n: int):
    from . import inputs
    if kind == "kms":
        return inputs.kms(n, 0.7)
    m = inputs.smallest_cube(n)
    return inputs.gramian_from_positions(inputs.gauss_positions(m, 1.0, 0.1, 0, n))


def _key(prec: str, tau: float) -> str:
    return f"{ARCH}/{prec}/tau{tau:g}"


def tune(ctx, prec: str = "f32", tau: float = 1e-6, tol: float = 1e-6, maxit: int = 40,
         kinds=("kms", "gauss"), buckets=BUCKETS, leaves=LEAVES, reps: int = 2, max_n: int = 4096) -> dict:
    """Times every candidate leaf on each (kind, bucket) and returns the table."""
    import torch
    table = {}
    for kind in kinds:
        for n in buckets:
            if n > max_n:
                continue
            s = torch.from_numpy(_representative(kind, n)).cuda()
            times = {}
            for leaf in leaves:
                best = math.inf
                for _ in range(reps + 1):  # the first run also builds tables and graphs
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    ctx.ns_sqrt(s, tau, tol, maxit, leaf=leaf, prec=prec, stagnation_stop=True,
                                raise_on_error=False)
                    torch.cuda.synchronize()
                    best = min(best, time.perf_counter() - t0)
                times[str(leaf)] = best * 1e3
            table[f"{kind}/{n}"] = dict(leaf=int(min(times, key=times.get)), ms=times)
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
    p.add_argument("--tau", type=float, default=1e-6)
    p.add_argument("--tol", type=float, default=1e-6)
    p.add_argument("--max-n", type=int, default=4096)
    p.add_argument("--out", default=CACHE, help="JSON cache to update")
    a = p.parse_args()
    from . import spamm
    ctx = spamm.Context(0)
    table = tune(ctx, a.prec, a.tau, a.tol, max_n=a.max_n)
    save(table, a.prec, a.tau, a.out)
    print(json.dumps(table, indent=1))


if __name__ == "__main__":
    main()
