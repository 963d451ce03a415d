"""Writes the stored expected values under tests/golden/ by running the FP64 CPU
oracle (and nothing else) on the seeded full-size workloads.

    OMP_NUM_THREADS=8 python tests/golden/make_golden.py

Each file records the oracle's per-iteration history of one Newton-Schulz solve
(r_k = ||I - x_k||_F, t_k = (n - tr x_k)/n, |R| of each product), its status
and iteration count, so the GPU tests can compare a whole full-size solve
without re-running the oracle for minutes.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1508_05856_amd import inputs  # noqa: E402

CASES = [
    # name, tau, tau_s, tol, maxit, stagnation_stop
    ("gauss_m16_h1.0_b64_tau1e-08_stag", 1e-8, -1.0, 1e-10, 40, True),
    ("gauss_m16_h1.0_b64_tau1e-06_literal", 1e-6, -1.0, 1e-10, 40, False),
    ("gauss_m16_h1.0_b64_tau1e-04_literal", 1e-4, -1.0, 1e-10, 40, False),
]


def main(names=None):
    s = inputs.gauss_gramian(16, 1.0, 0.1, 0)
    for name, tau, tau_s, tol, maxit, stag in CASES:
        if names and name not in names:
            continue
        t0 = time.time()
        res = oracle.ns_sqrt(s, 64, tau, tol, maxit, tau_s=tau_s, stagnation_stop=stag)
        out = dict(
            source="FP64 CPU oracle (oracle/spamm_oracle.c), written by tests/golden/make_golden.py",
            input="Gaussian Gramian, 16^3 Morton-ordered lattice sites, h=1.0, jitter 0.1, seed 0 (n=4096)",
            leaf=64, tau=tau, tau_s=tau_s, tol=tol, maxit=maxit, stagnation_stop=stag,
            status=res["status"], iterations=res["iterations"], scale=res["scale"],
            r=[float(v) for v in res["r"]], t=[float(v) for v in res["t"]],
            nR=[[int(x) for x in row] for row in res["nR"]],
        )
        with open(os.path.join(HERE, name + ".json"), "w") as f:
            json.dump(out, f, indent=1)
        print(name, res["status"], res["iterations"], f"{time.time() - t0:.1f}s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or None)
