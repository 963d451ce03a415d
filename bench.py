"""Benchmark: Newton-Schulz square-root solves per second on one MI355X.

One step = one complete ns_sqrt solve (ingest, norm pyramids, culls, leaf
products with the fused update, convergence tests, egress) of the 3-D Gaussian
overlap Gramian on 16^3 = 4096 Morton-ordered jittered lattice sites (h = 1.0,
jitter 0.1, seed 0), leaf 64, FP64 leaves, with the input already resident in
HBM.  Prints one JSON line.

The leaf-product kernel is timed live with HIP events that the library records
on its own stream around every leaf-product launch; its algorithmic rate is
2 b^3 |R| per launch over the measured launch time.  The CPU baseline times the
FP64 oracle on a bounded sample of the same solve (its first few updates) and
scales by retained-triple volume.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16x3": 2500.0}
LEAF_SRC = os.path.join(ROOT, "paper_1508_05856_amd", "csrc", "leaf_gemm.hip")
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "leaf_gemm_f64_gauss_n4096_b64_tau1e-8_traffic.md")


def committed_traffic(workload: str, prec: str):
    """HBM bytes per leaf-product launch (FETCH_SIZE + WRITE_SIZE, each
    scaled by the same counter on a plain copy of known size) from the
    committed counter profile of this workload, or None when there is none
    or the leaf-product source has changed since it was taken."""
    import hashlib
    import re
    if not os.path.exists(TRAFFIC_PROFILE):
        return None
    m = re.search(r"```json\n(.*?)\n```", open(TRAFFIC_PROFILE).read(), re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    sha = hashlib.sha256(open(LEAF_SRC, "rb").read()).hexdigest()
    if rec.get("leaf_gemm_sha256") != sha or rec.get("workload") != workload or rec.get("prec") != prec:
        return None
    return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--tau", type=float, default=None)
    p.add_argument("--tau-s", type=float, default=-1.0)
    p.add_argument("--prec", default="f64", choices=["f64", "f32", "bf16x3"])
    p.add_argument("--tol", type=float, default=None)
    p.add_argument("--maxit", type=int, default=40)
    p.add_argument("--literal-stop", action="store_true", help="disable the stagnation stop")
    p.add_argument("--stagnation", action="store_true", help="c1: use the stagnation stop (default: literal)")
    p.add_argument("--damped", action="store_true", help="the damped map (alpha(t), eps(t) of the trace error)")
    p.add_argument("--cpu-sample-iters", type=int, default=8)
    p.add_argument("--m", type=int, default=32, help="c3: lattice side, n = m^3 (16: the n = 4096 analogue, "
                   "which the oracle solves whole for the CPU baseline)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--dump-launches", default=None, help="write per-launch (flops, ms) of the timed steps")
    p.add_argument("--compare-f64", action="store_true", help="also solve in FP64 and report the relative gap")
    p.add_argument("--copy-bytes", type=int, default=1 << 31, help="copy: bytes read (and written) per launch")
    p.add_argument("--workload", default="gauss4096",
                   choices=["gauss4096", "c1", "c3", "batched", "serving", "copy", "product", "norms"],
                   help="gauss4096: the n=4096 Gaussian Gramian (default); batched: 64 uneven solves "
                        "together; serving: a Poisson request stream through the continuous-batching server")
    p.add_argument("--rate", type=float, default=200.0, help="serving: arrivals per second")
    p.add_argument("--duration", type=float, default=60.0, help="serving: seconds of arrivals")
    p.add_argument("--nmax", type=int, default=16384, help="serving: largest n (log-uniform from 512)")
    p.add_argument("--iters-per-step", type=int, default=4, help="batched: iterations per synchronisation")
    p.add_argument("--lanes", default="2048,8192", help="serving: comma-separated largest n of each engine lane "
                   "but the last (each lane has its own stream); empty = one lane")
    a = p.parse_args()
    a.tau_cli, a.tol_cli = a.tau, a.tol
    if a.tau is None:
        a.tau = 1e-8
    if a.tol is None:
        a.tol = 1e-10
    return a


def run_batched(args):
    """64 SPD instances of uneven n solved together through the step API
    (shared launches, one synchronisation per step, captured iterations), and
    the same 64 solved one at a time with ns_sqrt.  Results are bitwise the
    same either way, so the accuracy is equal by construction."""
    import torch

    from paper_1508_05856_amd import autotune, inputs, spamm

    specs = inputs.batch_specs(64, seed=0)
    prec, tol, maxit = "f32", 1e-6, 40
    # the workload leaves the y-channel threshold unstated: the paper's default
    # tau_s = 0.01 tau (with tau_s = tau, 8 of the 64 Gramians bifurcate)
    tsr = 0.01
    table = autotune.load(prec, 1e-6)
    leaves = [autotune.choose_leaf(table, sp["kind"], sp["n"]) for sp in specs]
    mats = [torch.from_numpy(inputs.build_spec(sp)).cuda() for sp in specs]
    outs = [(torch.empty_like(m), torch.empty_like(m)) for m in mats]
    ctx = spamm.Context(0)

    def batched():
        solves = [ctx.solve_begin(m, sp["tau"], tol, maxit, leaf=lf, prec=prec, tau_s=tsr * sp["tau"],
                                  stagnation_stop=True)
                  for m, sp, lf in zip(mats, specs, leaves)]
        while ctx.solve_step(solves, args.iters_per_step) > 0:
            pass
        return [sv.finish(Y, Z)[2] for sv, (Y, Z) in zip(solves, outs)]

    def single():
        return [ctx.ns_sqrt(m, sp["tau"], tol, maxit, leaf=lf, prec=prec, tau_s=tsr * sp["tau"],
                            stagnation_stop=True, Y=Y, Z=Z, raise_on_error=False)[2]
                for m, sp, lf, (Y, Z) in zip(mats, specs, leaves, outs)]

    for _ in range(args.warmup):
        batched()
        single()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        infos = batched()
    torch.cuda.synchronize()
    t_batched = (time.perf_counter() - t0) / args.steps
    t0 = time.perf_counter()
    single_infos = single()
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t0
    # accuracy of the batched results: exact ||I - Y Z||_F per instance
    resid = []
    for (Y, Z), sp, lf in zip(outs, specs, leaves):
        C, _, _ = ctx.spamm_multiply(Y, Z, 0.0, lf)
        C.diagonal().sub_(1.0)
        resid.append(float(torch.linalg.norm(C)))
    # leaf-product rate: one profiled pass with plain launches
    ctx.profile(True)
    prof_infos = batched()
    gemm_ms = ctx.profile_read(spamm.KIND_GEMM)
    ctx.profile(False)
    flops = sum(i["flops_total"] for i in prof_infos)
    achieved = flops / (gemm_ms.sum() * 1e-3) / 1e12
    peak = PEAK_TFLOPS[prec]
    ctx.close()
    nsolve = len(specs)
    # Gaussian Gramians at tau = 1e-4 diverge in FP64 as in FP32 (the culling
    # error exceeds their smallest eigenvalues): they run to their stop like
    # every instance, but only solves that end with status >= 0 count
    nvalid = sum(1 for i in infos if i["status"] >= 0)
    diverged = [dict(kind=sp["kind"], n=sp["n"], tau=sp["tau"]) for sp, i in zip(specs, infos) if i["status"] < 0]
    line = {
        "metric": "NS sqrt solves/sec, 64 uneven SPD instances solved together (batched)",
        "value": nvalid / t_batched, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t_batched * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": prec, "data": "synthetic",
        "config": {
            "workload": "batched_64_kms_gauss_n256-4096", "instances": nsolve,
            "n_range": [min(sp["n"] for sp in specs), max(sp["n"] for sp in specs)],
            "taus": sorted({sp["tau"] for sp in specs}), "tau_s": "0.01 tau", "tol": tol, "maxit": maxit,
            "stop": "stagnation",
            "precision": prec, "leaves": {str(b): leaves.count(b) for b in sorted(set(leaves))},
            "iters_per_step": args.iters_per_step, "graphs": True,
            "valid_solves": nvalid, "diverged": diverged,
            "one_at_a_time_solves_per_s": nvalid / t_single, "speedup_vs_one_at_a_time": t_single / t_batched,
            "statuses": {str(k): [i["status"] for i in infos].count(k) for k in sorted({i["status"] for i in infos})},
            "iterations_max": max(i["iterations"] for i in infos),
            "resid_exact_max_valid": max(r for r, i in zip(resid, infos) if i["status"] >= 0),
            "resid_exact_median_valid": float(np.median([r for r, i in zip(resid, infos) if i["status"] >= 0])),
            "same_iterations_as_one_at_a_time": all(a["iterations"] == b["iterations"]
                                                    for a, b in zip(infos, single_infos)),
        },
        "roofline": {"bound": "mfma", "kernel": "k_leaf_gemm", "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak, "traffic": None,
                     "launches": int(len(gemm_ms)), "avg_launch_ms": float(np.mean(gemm_ms)),
                     "timing": "separate profiled pass with plain launches"},
    }
    print(json.dumps(line), flush=True)


def run_serving(args):
    """Poisson arrivals of sqrt / inverse-sqrt requests (n log-uniform in
    [512, nmax], KMS and Gaussian, tau in {1e-4, 1e-6, 1e-8}, tol 1e-8, FP64)
    submitted in real time to the continuous-batching server; latency is
    arrival to result on the device."""
    import threading

    import torch

    from paper_1508_05856_amd import inputs, serve

    reqs = inputs.serving_requests(args.rate, args.duration, seed=0, nmin=512, nmax=args.nmax)
    dev = torch.device("cuda:0")
    lanes = tuple(int(x) for x in args.lanes.split(",") if x) + (None,)
    srv = serve.Server(0, iters_per_step=args.iters_per_step, lanes=lanes)
    # warm up kernels and tables on a tiny stream
    for f in [srv.submit(inputs.kms_device(n, 0.7, dev), 1e-6, 1e-8, leaf=64) for n in (512, 1024)]:
        f.result()
    futures = [None] * len(reqs)
    done = [0]
    t0 = time.perf_counter()

    def on_done(f):
        # keep the timing and status; drop Y, Z so finished outputs do not pile up in HBM
        if f.exception() is None:
            res = f.result()
            res.Y = res.Z = None
        done[0] += 1
        if done[0] % 100 == 0 or done[0] == len(reqs):
            print(f"served {done[0]}/{len(reqs)} at {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)

    def client():
        # inputs are materialised on the device at arrival; when the queue of
        # unadmitted requests is deep (offered load above capacity) the client
        # holds back so queued inputs cannot exhaust HBM.  Latency is measured
        # from the scheduled arrival, so holding back never hides queueing.
        for i, r in enumerate(reqs):
            delay = r["t"] - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            while True:
                cnt, nbytes = srv.backlog()
                if cnt < 32 and nbytes < (16 << 30):
                    break
                time.sleep(0.0005)
            s = inputs.build_spec_device(r, dev)
            f = srv.submit(s, r["tau"], 1e-8, maxit=40, leaf=64, prec="f64", tau_s=0.01 * r["tau"],
                           stagnation_stop=True)
            f.add_done_callback(on_done)
            futures[i] = f
            del s

    err = []

    def client_guarded():
        try:
            client()
        except BaseException as e:
            err.append(e)

    th = threading.Thread(target=client_guarded)
    th.start()
    th.join()
    if err:
        srv.close()
        raise err[0]
    results, failed = [], 0
    for f, r in zip(futures, reqs):
        try:
            results.append((f.result(timeout=600), r))
        except Exception as e:
            failed += 1
            print(f"request n={r['n']} failed: {e}", file=sys.stderr, flush=True)
    t_end = time.perf_counter() - t0
    stats = dict(srv.stats)
    srv.close()
    lat = np.array([res.t_done - (t0 + r["t"]) for res, r in results])
    statuses = [res.info["status"] for res, _ in results]
    # a request whose solve diverged is answered (with its status) but is not a solve
    nvalid = sum(1 for st in statuses if st >= 0)
    div_by = {}
    for (res, r) in results:
        if res.info["status"] < 0:
            key = f'{r["kind"]} tau={r["tau"]:g}'
            div_by[key] = div_by.get(key, 0) + 1
    line = {
        "metric": "NS sqrt serving: solves/sec and p50/p99 latency under Poisson arrivals",
        "value": nvalid / t_end, "unit": "solves/s", "n_gpus": 1, "steps": len(results), "warmup": 2,
        "ms_per_step": t_end * 1e3 / len(results), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {
            "workload": f"serving_poisson_{args.rate:g}rps_{args.duration:g}s_n512-{args.nmax}",
            "requests": len(reqs), "failed": failed, "valid_solves": nvalid, "diverged_by": div_by,
            "answered_per_s": len(results) / t_end, "offered_rate": args.rate, "duration_s": args.duration,
            "makespan_s": t_end, "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)), "mean_latency_s": float(lat.mean()),
            "tol": 1e-8, "tau_s": "0.01 tau", "stop": "stagnation", "iters_per_step": args.iters_per_step,
            "lanes": [x if x is not None else "rest" for x in lanes],
            "sizes_n": [int(min(r["n"] for r in reqs)), int(max(r["n"] for r in reqs))],
            "statuses": {str(k): statuses.count(k) for k in sorted(set(statuses))},
            "useful_tflops": sum(res.info["flops_total"] for res, _ in results) / t_end / 1e12,
            "engine": stats,
        },
    }
    print(json.dumps(line), flush=True)


ORACLE_FULL_MAX_N = 8192  # device-built inputs up to this n: the oracle solves them whole


def cpu_baseline_full(s, leaf, args, mu_rel, stag, info, Y, Z):
    """The oracle's whole solve of the same input and options (FP64 leaves
    whatever the GPU precision), timed, with its agreement with the GPU
    outputs beside it."""
    import oracle
    a = s.cpu().numpy()
    tc = time.perf_counter()
    ores = oracle.ns_sqrt(a, leaf, args.tau, args.tol, args.maxit, tau_s=args.tau_s, mu_rel=mu_rel,
                          stagnation_stop=stag, damped=args.damped)
    sec = time.perf_counter() - tc
    Yh, Zh = Y.cpu().numpy(), Z.cpu().numpy()
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": 1.0 / sec, "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": f"the whole solve (n = {a.shape[0]}, FP64 leaves): {sec:.1f} s",
            "agreement": {"status": [info["status"], int(ores["status"])],
                          "iterations": [info["iterations"], int(ores["iterations"])],
                          "rel_Y": float(np.linalg.norm(Yh - ores["Y"]) / np.linalg.norm(ores["Y"])),
                          "rel_Z": float(np.linalg.norm(Zh - ores["Z"]) / np.linalg.norm(ores["Z"]))}}


def cpu_baseline_sampled_tiles(s, mu_rel, leaf, tau, info):
    """The oracle on a bounded sample of a problem too large for it whole: the
    pyramid of the regularised, scaled operand s' (all of it) and a sample of
    output tiles of the first product s' (x)_tau s', timed and scaled to the
    solve by retained triples (pyramid time counted once per product)."""
    import oracle
    import torch
    c0 = float(s.abs().sum(1).max())
    sm = s.clone()
    sm.diagonal().add_(mu_rel * c0)
    sm /= float(sm.abs().sum(1).max())
    a = sm.cpu().numpy()
    del sm
    nb = -(-a.shape[0] // leaf)
    rng = np.random.default_rng(0)
    # output tiles on and near the diagonal, where the retained triples are
    tiles = [(int(i), int(min(nb - 1, max(0, i + d)))) for i, d in
             zip(rng.integers(0, nb, 3000), rng.integers(-6, 7, 3000))]
    tc = time.perf_counter()
    oracle.norms(a, leaf)
    t_pyr = time.perf_counter() - tc
    tc = time.perf_counter()
    oracle.spamm_tiles(a, a, leaf, tau, [])   # set-up alone: copies and both pyramids
    t_setup = time.perf_counter() - tc
    tc = time.perf_counter()
    _, counts = oracle.spamm_tiles(a, a, leaf, tau, tiles)
    t_tiles = max(time.perf_counter() - tc - t_setup, 1e-9)
    sample = int(np.sum(counts))
    products = 3 * info["iterations"] + 1
    sec = t_pyr * products + t_tiles * info["triples_total"] / max(sample, 1)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": 1.0 / sec, "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": (f"pyramid of s' ({t_pyr:.1f} s, counted once per product x {products}) + {len(tiles)} "
                       f"output tiles of s' (x) s' near the diagonal ({sample} triples, {t_tiles:.2f} s net of "
                       f"set-up) scaled to the solve's {info['triples_total']} triples")}


def run_product(args):
    """One SpAMM product alone: y (x)_tau z of the n = 4096 Gaussian solve at
    its tau floor (the operands of its last x product, from an untimed FP64
    solve, so every leaf precision multiplies the same operands), timed over K
    launches with HIP events on the library's stream."""
    import torch

    from paper_1508_05856_amd import inputs, spamm
    cfg = inputs.config_c2(args.tau)
    ctx = spamm.Context(0)
    s = torch.from_numpy(cfg["s"]).cuda()
    Y, Z, _ = ctx.ns_sqrt(s, args.tau, args.tol, args.maxit, leaf=cfg["leaf"], prec="f64",
                          stagnation_stop=True, raise_on_error=False)
    c = _scale_of(s)
    y, z = Y / c ** 0.5, Z * c ** 0.5  # the scaled iterates the solve multiplies
    for _ in range(args.warmup):
        ctx.spamm_multiply(y, z, args.tau, cfg["leaf"], prec=args.prec)
    ctx.profile(True)
    ctx.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, st, _ = ctx.spamm_multiply(y, z, args.tau, cfg["leaf"], prec=args.prec)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    g = ctx.profile_read(spamm.KIND_GEMM)
    ctx.profile(False)
    achieved = st["flops"] / (float(np.mean(g)) * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.prec]
    if args.prec == "bf16x3":
        achieved *= 3.0
    print(json.dumps({"metric": "SpAMM product y (x)_tau z at the n=4096 Gaussian solve's tau floor",
                      "value": st["flops"] / dt / 1e12, "unit": "useful TFLOP/s (whole product)", "n_gpus": 1,
                      "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
                      "higher_is_better": True, "dtype": args.prec, "data": "synthetic",
                      "config": {"workload": f"product_{cfg['name']}", "retained": st["retained"],
                                 "possible": st["possible"], "flops": st["flops"]},
                      "roofline": {"bound": "mfma",
                                   "kernel": _gemm_kernel(args.prec, cfg["leaf"]),
                                   "achieved": achieved, "peak": peak,
                                   "unit": "TFLOP/s", "frac": achieved / peak, "traffic": None,
                                   "avg_launch_ms": float(np.mean(g))}}), flush=True)
    ctx.close()


def _gemm_kernel(prec, leaf):
    """Name of the leaf-product kernel a precision and leaf size run."""
    if prec == "bf16x3":
        return "k_leaf_gemm_bf3_quad" if leaf == 64 else "k_leaf_gemm_bf3"
    return "k_leaf_gemm"


def _scale_of(s):
    """Gershgorin bound max_j sum_i |s_ij| (the scale the solve divides by)."""
    return float(s.abs().sum(0).max())


def run_norms(args):
    """The norm pass alone: spamm_norms of the n = 32768 Gaussian Gramian
    (8 GiB FP64, leaf 64), HBM-bound; algorithmic bytes = one read of s."""
    import torch

    from paper_1508_05856_amd import inputs, spamm
    cfg = inputs.config_c3_spec()
    n = cfg["n"]
    s = inputs.gramian_device(inputs.gauss_positions(cfg["m"], cfg["h"], 0.1, 0, n), "cuda")
    ctx = spamm.Context(0)
    for _ in range(args.warmup):
        ctx.spamm_norms(s, cfg["leaf"], want_root=False)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[2 * k].record()
        ctx.spamm_norms(s, cfg["leaf"], want_root=False)
        ev[2 * k + 1].record()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    ms = float(np.mean([ev[2 * k].elapsed_time(ev[2 * k + 1]) for k in range(args.steps)]))
    nbytes = float(n) * n * 8
    gbs = nbytes / (ms * 1e-3) / 1e9
    print(json.dumps({"metric": "norm pyramid of one operand (the norm pass)", "value": nbytes / dt / 1e9,
                      "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                      "ms_per_step": dt * 1e3, "higher_is_better": True, "dtype": "f64", "data": "synthetic",
                      "config": {"workload": f"norms_{cfg['name']}", "n": n, "leaf": cfg["leaf"]},
                      "roofline": {"bound": "hbm", "kernel": "k_leaf_norms", "achieved": gbs, "peak": 8000.0,
                                   "unit": "GB/s", "frac": gbs / 8000.0, "traffic": None,
                                   "avg_call_ms": ms}}), flush=True)
    ctx.close()


def run_copy(args):
    """A plain elementwise device copy of known size (y = -x over FP64), the
    reference that scales hardware read/write byte counters to bytes."""
    import torch
    n = args.copy_bytes // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(args.warmup):
        torch.neg(x, out=y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        torch.neg(x, out=y)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    print(json.dumps({"metric": "device copy bandwidth (read + write)", "value": 2 * n * 8 / dt / 1e9,
                      "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                      "ms_per_step": dt * 1e3, "higher_is_better": True, "dtype": "f64", "data": "synthetic",
                      "config": {"workload": "copy", "bytes_read_per_launch": n * 8,
                                 "bytes_written_per_launch": n * 8}}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU sharding is design-only",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.workload == "batched":
        run_batched(args)
        return
    if args.workload == "serving":
        run_serving(args)
        return
    if args.workload == "copy":
        run_copy(args)
        return
    if args.workload == "product":
        run_product(args)
        return
    if args.workload == "norms":
        run_norms(args)
        return

    import torch

    from paper_1508_05856_amd import inputs, spamm

    dev = torch.device("cuda:0")
    stag = not args.literal_stop
    mu_rel = 0.0
    if args.workload == "c3":
        # n = 32768 ill-conditioned Gramian, built on the device (8 GiB in FP64)
        cfg = inputs.config_c3_spec(args.m)
        n, leaf = cfg["n"], cfg["leaf"]
        s_host = None
        s = inputs.gramian_device(inputs.gauss_positions(cfg["m"], cfg["h"], 0.1, 0, n), dev)
        mu_rel = cfg["mu_rel"]
        if args.tau_cli is None:
            args.tau = cfg["tau"]
        if args.tol_cli is None:
            args.tol = cfg["tol"]
        if args.tau_s < 0:
            args.tau_s = cfg["tau_s_rel"] * args.tau
        args.damped = args.damped or cfg["damped"]
    elif args.workload == "c1":
        # KMS rho = 0.7, n = 512, leaf 32, stop at tol 1e-10 or 40 updates (the
        # literal rule unless --stagnation is given): launch-latency bound
        cfg = inputs.config_c1()
        s_host = cfg["s"]
        n, leaf = s_host.shape[0], cfg["leaf"]
        s = torch.from_numpy(s_host).to(dev)
        if args.tau_cli is None:
            args.tau = cfg["tau"]
        if args.tol_cli is None:
            args.tol = cfg["tol"]
        stag = args.stagnation
    else:
        cfg = inputs.config_c2(args.tau)
        s_host = cfg["s"]
        n, leaf = s_host.shape[0], cfg["leaf"]
        s = torch.from_numpy(s_host).to(dev)
    Y = torch.empty_like(s)
    Z = torch.empty_like(s)
    ctx = spamm.Context(0)

    def step(prec=args.prec, Yo=Y, Zo=Z):
        return ctx.ns_sqrt(s, args.tau, args.tol, args.maxit, leaf=leaf, prec=prec, tau_s=args.tau_s,
                           mu_rel=mu_rel, stagnation_stop=stag, damped=args.damped, Y=Yo, Z=Zo,
                           raise_on_error=False)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # timed steps: the product path as it runs in use (iterations replayed
    # from captured graphs, no launch timing)
    infos, step_ms = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        _, _, info = step()  # a solve ends with its outputs written and its stream synchronised
        step_ms.append((time.perf_counter() - ts) * 1e3)
        infos.append(info)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    info = infos[-1]

    # a separate profiled pass (plain launches, HIP events on the library's
    # stream around every launch) for the kernel durations of the roofline
    gemm_ms, gemm_flops, cull_ms, pyr_ms = [], [], [], []
    ctx.profile(True)
    torch.cuda.synchronize()
    tp0 = time.perf_counter()
    for _ in range(max(1, min(args.steps, 2))):
        ctx.profile_reset()
        step()
        # the solve has synchronised its stream; read this step's launch records
        r, t, nR = ctx.ns_history()
        g = ctx.profile_read(spamm.KIND_GEMM)
        # launches alternate x product / (y, z) update per enqueued iteration;
        # those after the solve stopped do no work (and still count as time)
        kfin = len(nR) - 1
        fl = []
        for L in range(len(g)):
            it, upd = divmod(L, 2)
            if upd == 0:
                fl.append(2.0 * leaf ** 3 * nR[it, 0] if it <= kfin else 0.0)
            else:
                fl.append(2.0 * leaf ** 3 * (nR[it, 1] + nR[it, 2]) if it < kfin else 0.0)
        gemm_ms.extend(g.tolist())
        gemm_flops.extend(fl)
        cull_ms.extend(ctx.profile_read(spamm.KIND_CULL).tolist())
        pyr_ms.extend(ctx.profile_read(spamm.KIND_PYRAMID).tolist())
    torch.cuda.synchronize()
    prof_steps = max(1, min(args.steps, 2))
    ms_per_step_profiled = (time.perf_counter() - tp0) * 1e3 / prof_steps
    ctx.profile(False)

    rel_vs_f64 = None
    if args.compare_f64 and args.prec != "f64":
        Y64, Z64 = torch.empty_like(s), torch.empty_like(s)
        step("f64", Y64, Z64)
        rel_vs_f64 = dict(Y=float(torch.linalg.norm(Y - Y64) / torch.linalg.norm(Y64)),
                          Z=float(torch.linalg.norm(Z - Z64) / torch.linalg.norm(Z64)))
        del Y64, Z64

    # exact ||I - Y Z||_F with a dense FP64 product through the library (tau = 0)
    C, _, _ = ctx.spamm_multiply(Y, Z, 0.0, leaf)
    C.diagonal().sub_(1.0)
    resid_exact = float(torch.linalg.norm(C))
    del C

    if args.dump_launches:
        with open(args.dump_launches, "w") as f:
            json.dump(dict(gemm_ms=gemm_ms, gemm_flops=gemm_flops, cull_ms=cull_ms, pyramid_ms=pyr_ms), f)
    useful = sum(gemm_flops) / (sum(gemm_ms) * 1e-3) / 1e12
    # BF16x3 executes three bf16 products per useful one: its roofline is the
    # executed rate against the bf16 peak (the useful rate is reported beside it)
    achieved = 3.0 * useful if args.prec == "bf16x3" else useful
    peak = PEAK_TFLOPS[args.prec]
    line = {
        "metric": "NS sqrt solves/sec at stated ||I-YZ||_F (culled-leaf TFLOP/s vs MFMA peak in roofline)",
        "value": 1e3 / ms_per_step,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "ms_per_step_median": float(np.median(step_ms)),
        "ms_per_step_p99": float(np.percentile(step_ms, 99)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": {
            "workload": cfg["name"], "n": n, "leaf": leaf, "tau": args.tau,
            "tau_s": args.tau if args.tau_s < 0 else args.tau_s, "tol": args.tol, "maxit": args.maxit,
            "stop": "literal" if not stag else "stagnation", "precision": args.prec,
            "map": "damped" if args.damped else "plain",
            "status": spamm.STATUS_NAMES.get(info["status"], info["status"]),
            "iterations": info["iterations"], "resid_inloop": info["resid"], "resid_exact": resid_exact,
            "us_per_update": ms_per_step * 1e3 / max(info["iterations"], 1),
            "trace_err": info["trace_err"], "triples_per_solve": info["triples_total"],
            "flops_per_solve": info["flops_total"], "mu_rel": mu_rel, "rel_vs_f64": rel_vs_f64,
        },
        "roofline": {
            "bound": "mfma", "kernel": _gemm_kernel(args.prec, leaf), "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": committed_traffic(cfg["name"], args.prec),
            "traffic_unit": "bytes per launch", "useful_tflops": useful,
            "launches": len(gemm_ms), "avg_launch_ms": float(np.mean(gemm_ms)),
            "gemm_ms_per_step": sum(gemm_ms) / prof_steps,
            "cull_ms_per_step": sum(cull_ms) / prof_steps, "pyramid_ms_per_step": sum(pyr_ms) / prof_steps,
            "timing": "value: graph-replayed solves; kernel durations: a separate profiled pass of plain launches",
            "ms_per_step_profiled_pass": ms_per_step_profiled,
        },
    }

    if not args.no_cpu_baseline and s_host is None and n <= ORACLE_FULL_MAX_N:
        line["cpu_baseline"] = cpu_baseline_full(s, leaf, args, mu_rel, stag, info, Y, Z)
    elif not args.no_cpu_baseline and s_host is None:
        line["cpu_baseline"] = cpu_baseline_sampled_tiles(s, mu_rel, leaf, args.tau, info)
    elif not args.no_cpu_baseline:
        import oracle
        m = args.cpu_sample_iters
        tc = time.perf_counter()
        ores = oracle.ns_sqrt(s_host, leaf, args.tau, args.tol, m, tau_s=args.tau_s, stagnation_stop=stag)
        tcpu = time.perf_counter() - tc
        sample_triples = int(ores["nR"].sum())
        sec_per_solve = tcpu * info["triples_total"] / max(sample_triples, 1)
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        line["cpu_baseline"] = {
            "value": 1.0 / sec_per_solve, "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": (f"first {m} updates ({sample_triples} retained leaf triples) of the same solve took "
                       f"{tcpu:.1f} s; scaled to the full solve's {info['triples_total']} triples"),
        }
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
