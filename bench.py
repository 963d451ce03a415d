"""Benchmark: Newton-Schulz square-root solves per second on one MI355X.

Default workload: the ill-conditioned Gaussian overlap Gramian on 32^3 = 32768
Morton-ordered jittered lattice sites (h = 0.6, jitter 0.1, seed 0), shifted
by mu = 1e-4 c0 (Sec. 6), leaf 64, tau = 1e-9 with the damped map and
tau_s = 0.01 tau, stagnation stop, FP64 leaves (the paper's arithmetic), with
the input already resident in HBM.  One step = one Newton-Schulz iteration of
a stream of such solves (x product with its stop test, then the y and z
update while the solve goes on); each solve is begun (ingest, pyramids) and
finished (egress) inside the timed region.  value = solves/s of the first
solve that runs whole inside the timed region.  Prints one JSON line.

The leaf-product kernel is timed live with HIP events that the library records
on its own stream around every leaf-product launch of the timed region; its
algorithmic rate is 2 b^3 |R| per launch over the measured launch time.  The
CPU baseline times the FP64 oracle on a bounded sample (the pyramid and a
sample of output tiles of the first product) scaled by retained triples.

--workload c2 is the n = 4096 Gaussian Gramian (whole-solve steps; its CPU
baseline is the oracle's whole solve with its agreement with the GPU).
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

PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16x3": 2500.0, "bf16x6": 2500.0}
# bf16 products executed per useful product by the split-bf16 modes
EXEC_PER_USEFUL = {"f64": 1.0, "f32": 1.0, "bf16x3": 3.0, "bf16x6": 6.0}
CSRC = os.path.join(ROOT, "paper_1508_05856_amd", "csrc")
PROFILES = os.path.join(ROOT, "profiles")


def committed_traffic(workload: str, prec: str):
    """HBM bytes per leaf-product launch (FETCH_SIZE + WRITE_SIZE, each
    scaled by the same counter on a plain copy of known size) from a committed
    counter profile of this workload and precision, or None when there is
    none or the leaf-product or job-order source (leaf_gemm.hip, kernels.hip)
    has changed since it was taken."""
    import glob
    import hashlib
    import re
    sha = {name: hashlib.sha256(open(os.path.join(CSRC, name), "rb").read()).hexdigest()
           for name in ("leaf_gemm.hip", "kernels.hip")}
    for path in sorted(glob.glob(os.path.join(PROFILES, "*.md"))):
        for block in re.findall(r"```json\n(.*?)\n```", open(path).read(), re.S):
            try:
                rec = json.loads(block)
            except ValueError:
                continue
            if (rec.get("workload") == workload and rec.get("prec") == prec
                    and rec.get("leaf_gemm_sha256") == sha["leaf_gemm.hip"]
                    and rec.get("kernels_sha256") == sha["kernels.hip"]):
                return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
    return None


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    # c3: a step is one iteration and a whole n = 32768 solve takes 14, so
    # the default region holds one whole solve
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--tau", type=float, default=None)
    p.add_argument("--tau-s", type=float, default=-1.0)
    p.add_argument("--prec", default="f64", choices=["f64", "f32", "bf16x3", "bf16x6"])
    p.add_argument("--tol", type=float, default=None)
    p.add_argument("--maxit", type=int, default=40)
    p.add_argument("--literal-stop", action="store_true", help="disable the stagnation stop")
    p.add_argument("--stagnation", action="store_true", help="c1: use the stagnation stop (default: literal)")
    p.add_argument("--damped", action="store_true", help="the damped map (alpha(t), eps(t) of the trace error)")
    p.add_argument("--m", type=int, default=32, help="c3: lattice side, n = m^3 (16: the n = 4096 analogue, "
                   "which the oracle solves whole for the CPU baseline)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--dump-launches", default=None, help="write per-launch (flops, ms) of the timed steps")
    p.add_argument("--compare-f64", action="store_true", help="also solve in FP64 and report the relative gap")
    p.add_argument("--copy-bytes", type=int, default=1 << 31, help="copy: bytes read (and written) per launch")
    p.add_argument("--workload", default="c3",
                   choices=["c3", "c2", "gauss4096", "c1", "batched", "serving", "copy", "product", "norms"],
                   help="c3: the n=32768 ill-conditioned Gramian, steps of one iteration (default); "
                        "c2 (= gauss4096): the n=4096 Gaussian Gramian, whole-solve steps; batched: 64 uneven "
                        "solves together; serving: a Poisson request stream through the continuous-batching server")
    p.add_argument("--rate", type=float, default=200.0, help="serving: arrivals per second")
    p.add_argument("--duration", type=float, default=60.0, help="serving: seconds of arrivals")
    p.add_argument("--nmax", type=int, default=16384, help="serving: largest n (log-uniform from 512)")
    p.add_argument("--iters-per-step", default="4", help="batched: iterations per synchronisation; serving: "
                   "one value or one per lane, comma-separated")
    p.add_argument("--check", choices=("replay", "server"), default="replay",
                   help="serving: exact residuals from the one-at-a-time replay (outside both timings), or "
                        "computed by the server for every answer (inside the served time; no replay)")
    p.add_argument("--count-below", type=float, default=1e-2,
                   help="batched, serving: solves/s counts solves whose exact ||I - YZ||_F is at most this")
    p.add_argument("--pool-share", type=float, default=0.2,
                   help="serving: fraction of the admission budget each lane may keep pooled")
    p.add_argument("--lanes", default="2048,8192", help="serving: comma-separated largest n of each engine lane "
                   "but the last (each lane has its own stream); empty = one lane")
    a = p.parse_args()
    if a.workload == "gauss4096":
        a.workload = "c2"
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
    tables = {tau: autotune.load(prec, tau) for tau in sorted({sp["tau"] for sp in specs})}
    leaves = [autotune.choose_leaf(tables[sp["tau"]], sp["kind"], sp["n"]) for sp in specs]
    mats = [torch.from_numpy(inputs.build_spec(sp)).cuda() for sp in specs]
    outs = [(torch.empty_like(m), torch.empty_like(m)) for m in mats]
    ctx = spamm.Context(0)

    def batched():
        solves = [ctx.solve_begin(m, sp["tau"], tol, maxit, leaf=lf, prec=prec, tau_s=tsr * sp["tau"],
                                  stagnation_stop=True)
                  for m, sp, lf in zip(mats, specs, leaves)]
        while ctx.solve_step(solves, int(args.iters_per_step)) > 0:
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
    # solves/s counts solves that end with status >= 0 and exact residual at most --count-below
    counted = [i["status"] >= 0 and r <= args.count_below for r, i in zip(resid, infos)]
    nvalid = sum(counted)
    diverged = [dict(kind=sp["kind"], n=sp["n"], tau=sp["tau"]) for sp, i in zip(specs, infos) if i["status"] < 0]
    cpu = None if args.no_cpu_baseline else batched_cpu_baseline(specs, leaves, infos, nvalid, tol, maxit, tsr)
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
            "iters_per_step": int(args.iters_per_step), "graphs": True,
            "counted": f"solves with status >= 0 and exact ||I - YZ||_F <= {args.count_below:g}",
            "count_below": args.count_below, "counted_solves": nvalid,
            "status_ge0": sum(1 for i in infos if i["status"] >= 0), "diverged": diverged,
            "resid_exact_by_tau": {f"tau={tau:g}": sorted(round(r, 6) for r, i, sp in zip(resid, infos, specs)
                                                          if sp["tau"] == tau and i["status"] >= 0)
                                   for tau in sorted({sp["tau"] for sp in specs})},
            "one_at_a_time_solves_per_s": nvalid / t_single, "speedup_vs_one_at_a_time": t_single / t_batched,
            "statuses": {str(k): [i["status"] for i in infos].count(k) for k in sorted({i["status"] for i in infos})},
            "iterations_max": max(i["iterations"] for i in infos),
            "resid_exact_max_valid": max(r for r, i in zip(resid, infos) if i["status"] >= 0),
            "resid_exact_median_valid": float(np.median([r for r, i in zip(resid, infos) if i["status"] >= 0])),
            "same_iterations_as_one_at_a_time": all(a["iterations"] == b["iterations"]
                                                    for a, b in zip(infos, single_infos)),
        },
        "roofline": {"bound": "mfma", "kernel": "k_leaf_gemm", "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": committed_traffic("batched_64_kms_gauss_n256-4096", prec),
                     "traffic_unit": "bytes per launch (mean over the profiled pass)",
                     "launches": int(len(gemm_ms)), "avg_launch_ms": float(np.mean(gemm_ms)),
                     "timing": "separate profiled pass with plain launches"},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def batched_cpu_baseline(specs, leaves, infos, counted, tol, maxit, tsr, budget_s=20.0):
    """The oracle (FP64 leaves) on a sample of the batched instances: every
    8th by size, smallest first, until about budget_s of CPU time.  Its flop
    rate on the sample scales the whole batch's retained leaf products (the
    GPU run's) to an estimated batch time."""
    import oracle

    from paper_1508_05856_amd import inputs
    order = sorted(range(len(specs)), key=lambda i: specs[i]["n"])
    secs, flops, used = 0.0, 0.0, []
    for i in order[::8]:
        if secs > budget_s:
            break
        sp = specs[i]
        a = inputs.build_spec(sp)
        t0 = time.perf_counter()
        o = oracle.ns_sqrt(a, leaves[i], sp["tau"], tol, maxit, tau_s=tsr * sp["tau"], stagnation_stop=True)
        secs += time.perf_counter() - t0
        flops += 2.0 * leaves[i] ** 3 * float(o["nR"].sum())
        used.append(sp["n"])
    rate = flops / secs
    total = float(sum(i["flops_total"] for i in infos))
    est = total / rate
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": counted / est, "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": (f"the oracle's whole solves of {len(used)} of the {len(specs)} instances (n = "
                       f"{', '.join(map(str, used))}): {secs:.1f} s at {rate / 1e9:.2f} GFLOP/s of retained leaf "
                       f"products; the batch's {total / 1e12:.2f} TFLOP at that rate take {est:.0f} s for its "
                       f"{counted} counted solves")}


def serving_cpu_baseline(reqs, results, counted, t_end, budget_s=20.0):
    """The oracle (FP64 leaves, the same options) on a sample of the served
    requests: every 25th by size, smallest first, until about budget_s of
    CPU time.  Its flop rate on the sample scales the stream's retained leaf
    products (the served run's) to an estimated one-at-a-time CPU time."""
    import oracle

    from paper_1508_05856_amd import inputs
    order = sorted(range(len(reqs)), key=lambda i: reqs[i]["n"])
    secs, flops, used = 0.0, 0.0, []
    for i in order[::25]:
        if secs > budget_s:
            break
        r = reqs[i]
        a = inputs.build_spec(r)
        t0 = time.perf_counter()
        o = oracle.ns_sqrt(a, 64, r["tau"], 1e-8, 40, tau_s=0.01 * r["tau"], stagnation_stop=True)
        secs += time.perf_counter() - t0
        flops += 2.0 * 64 ** 3 * float(o["nR"].sum())
        used.append(r["n"])
    rate = flops / secs
    total = float(sum(res.info["flops_total"] for res, _, _ in results))
    est = total / rate
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": counted / est, "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": (f"the oracle's whole solves of {len(used)} of the {len(reqs)} requests (n = "
                       f"{', '.join(map(str, used))}): {secs:.1f} s at {rate / 1e9:.2f} GFLOP/s of retained leaf "
                       f"products; the stream's {total / 1e12:.1f} TFLOP at that rate take {est:.0f} s for its "
                       f"{counted} counted solves (the GPU served them in {t_end:.0f} s); the sample holds the "
                       f"smallest requests, on which the oracle's rate may be lower than on the large ones")}


def run_serving(args):
    """Poisson arrivals of sqrt / inverse-sqrt requests (n log-uniform in
    [512, nmax], KMS and Gaussian, tau in {1e-4, 1e-6, 1e-8}, tol 1e-8, FP64)
    submitted in real time to the continuous-batching server; latency is
    arrival to result on the device.  The same request stream is then served
    one request at a time (ns_sqrt after ns_sqrt in arrival order, each
    request's service time measured, first-come first-served from its
    arrival), the plain path the server is compared with; results are bitwise
    the same either way (checked by checksums of every answer), so both run
    at the same accuracy.  The replay also computes each answer's exact
    ||I - Y Z||_F (a dense product, outside both timings), and solves/s counts
    the answers at or below --count-below.  With --check server the server
    computes every answer's exact residual itself, inside the served time,
    and no replay runs."""
    import threading

    import torch

    from paper_1508_05856_amd import inputs, serve, spamm

    reqs = inputs.serving_requests(args.rate, args.duration, seed=0, nmin=512, nmax=args.nmax)
    dev = torch.device("cuda:0")
    lanes = tuple(int(x) for x in args.lanes.split(",") if x) + (None,)
    opts = dict(maxit=40, leaf=64, prec="f64", stagnation_stop=True)
    its = [int(x) for x in str(args.iters_per_step).split(",")]
    srv = serve.Server(0, iters_per_step=its if len(its) > 1 else its[0], lanes=lanes, pool_share=args.pool_share)
    # warm up kernels and tables on a tiny stream
    for f in [srv.submit(inputs.kms_device(n, 0.7, dev), 1e-6, 1e-8, leaf=64) for n in (512, 1024)]:
        f.result()
    in_server = args.check == "server"
    futures = [None] * len(reqs)
    sums = [None] * len(reqs)
    done = [0]
    t0 = time.perf_counter()

    def make_cb(i):
        def on_done(f):
            # keep the timing, status and a checksum of the answer; drop Y, Z so
            # finished outputs do not pile up in HBM
            if f.exception() is None:
                res = f.result()
                sums[i] = (float(res.Y.sum()), float(res.Z.sum()))
                res.Y = res.Z = None
            done[0] += 1
            if done[0] % 100 == 0 or done[0] == len(reqs):
                print(f"served {done[0]}/{len(reqs)} at {time.perf_counter() - t0:.1f} s", file=sys.stderr,
                      flush=True)
        return on_done

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
            f = srv.submit(s, r["tau"], 1e-8, tau_s=0.01 * r["tau"], verify=in_server, **opts)
            f.add_done_callback(make_cb(i))
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
    for i, (f, r) in enumerate(zip(futures, reqs)):
        try:
            results.append((f.result(timeout=600), r, i))
        except Exception as e:
            failed += 1
            print(f"request n={r['n']} failed: {e}", file=sys.stderr, flush=True)
    t_end = time.perf_counter() - t0
    stats = dict(srv.stats)
    srv.close()
    lat = np.array([res.t_done - (t0 + r["t"]) for res, r, _ in results])
    statuses = [res.info["status"] for res, _, _ in results]

    # The same stream one request at a time: each request's service time (its
    # input built on the device, as the served run's client does at arrival,
    # then its solve), then first-come first-served from its arrival.  After
    # each timed solve, outside its service time, the answer's exact
    # ||I - Y Z||_F (a dense product) and its checksum: every answer is
    # bitwise the one served (equal checksums), so these residuals are the
    # served answers' residuals.
    ex1, sums1, service = [None] * len(reqs), [None] * len(reqs), []
    if not in_server:
        ctx = spamm.Context(0)
        for k, r in enumerate(reqs):
            torch.cuda.synchronize()
            ts = time.perf_counter()
            s = inputs.build_spec_device(r, dev)
            Y, Z, info = ctx.ns_sqrt(s, r["tau"], 1e-8, tau_s=0.01 * r["tau"], raise_on_error=False, **opts)
            torch.cuda.synchronize()
            service.append(time.perf_counter() - ts)
            if info["status"] >= 0:
                ex1[k] = serve.exact_residual(ctx, Y, Z)
                sums1[k] = (float(Y.sum()), float(Z.sum()))
            del s, Y, Z
            if len(service) % 200 == 0 or len(service) == len(reqs):
                print(f"one at a time: {len(service)}/{len(reqs)}, busy {sum(service):.1f} s", file=sys.stderr,
                      flush=True)
        ctx.close()
        t_free, lat1 = 0.0, []
        for r, sv in zip(reqs, service):
            start = max(r["t"], t_free)
            t_free = start + sv
            lat1.append(t_free - r["t"])

    # counted: answered solves whose exact ||I - Y Z||_F is at most
    # --count-below; diverged ones (status < 0) are answered but never counted
    if in_server:
        ex = [res.info.get("resid_exact") for res, _, _ in results]
    else:
        ex = [ex1[i] for _, _, i in results]
        same = all(sums1[i] == sums[i] for res, _, i in results if res.info["status"] >= 0)
    counted = [e is not None and e <= args.count_below for e in ex]
    nvalid = sum(counted)
    div_by = {}
    for res, r, _ in results:
        if res.info["status"] < 0:
            key = f'{r["kind"]} tau={r["tau"]:g}'
            div_by[key] = div_by.get(key, 0) + 1

    def pct(v):
        v = np.asarray(v, dtype=float)
        return None if v.size == 0 else {q: float(np.percentile(v, int(q[1:]))) for q in ("p0", "p50", "p90", "p100")}

    thresholds = (1e-8, 1e-6, 1e-4, 1e-2, 1e-1)
    accuracy = {}
    for tau in sorted({r["tau"] for r in reqs}):
        rex = [e for e, (_, r, _) in zip(ex, results) if e is not None and r["tau"] == tau]
        rin = [res.info["resid"] for e, (res, r, _) in zip(ex, results) if e is not None and r["tau"] == tau]
        accuracy[f"tau={tau:g}"] = {"answered_status_ge0": len(rex), "resid_exact": pct(rex),
                                    "resid_inloop": pct(rin),
                                    "at_or_below": {f"{x:g}": sum(1 for e in rex if e <= x) for x in thresholds}}
    one = None if in_server else {
        "solves_per_s": nvalid / t_free, "makespan_s": t_free, "busy_s": float(sum(service)),
        "capacity_solves_per_s": nvalid / float(sum(service)),
        "p50_latency_s": float(np.percentile(lat1, 50)), "p99_latency_s": float(np.percentile(lat1, 99)),
        "mean_latency_s": float(np.mean(lat1)), "same_answers_as_served": same}
    line = {
        "metric": "NS sqrt serving: solves/sec and p50/p99 latency under Poisson arrivals",
        "value": nvalid / t_end, "unit": "solves/s", "n_gpus": 1, "steps": len(results), "warmup": 2,
        "ms_per_step": t_end * 1e3 / len(results), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {
            "workload": f"serving_poisson_{args.rate:g}rps_{args.duration:g}s_n512-{args.nmax}",
            "counted": f"answered solves with exact ||I - YZ||_F <= {args.count_below:g} (status >= 0)",
            "count_below": args.count_below,
            "solves_per_s_at_or_below": {f"{x:g}": sum(1 for e in ex if e is not None and e <= x) / t_end
                                         for x in thresholds},
            "requests": len(reqs), "failed": failed, "counted_solves": nvalid, "diverged_by": div_by,
            "answered_per_s": len(results) / t_end, "offered_rate": args.rate, "duration_s": args.duration,
            "makespan_s": t_end, "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)), "mean_latency_s": float(lat.mean()),
            "tol": 1e-8, "tau_s": "0.01 tau", "stop": "stagnation", "iters_per_step": its,
            "lanes": [x if x is not None else "rest" for x in lanes],
            "sizes_n": [int(min(r["n"] for r in reqs)), int(max(r["n"] for r in reqs))],
            "statuses": {str(k): statuses.count(k) for k in sorted(set(statuses))},
            "accuracy_by_tau": accuracy,
            "one_at_a_time": one,
            "residuals_from": ("the server, for every answer (inside the served time)" if in_server else
                               "the one-at-a-time replay, checksum-equal answers (outside both timings)"),
            "speedup_vs_one_at_a_time": one["makespan_s"] / t_end if one else None,
            "useful_tflops": sum(res.info["flops_total"] for res, _, _ in results) / t_end / 1e12,
            "engine": stats,
        },
        "cpu_baseline": None if args.no_cpu_baseline else serving_cpu_baseline(reqs, results, nvalid, t_end),
    }
    print(json.dumps(line), flush=True)


ORACLE_FULL_MAX_N = 8192  # device-built inputs up to this n: the oracle solves them whole


def cpu_baseline_full(s, leaf, args, mu_rel, stag, info, Y, Z):
    """The oracle's whole solve of the same input and options (FP64 leaves
    whatever the GPU precision), timed (the median of up to three runs, as
    many as fit in about a minute), with its agreement with the GPU outputs
    beside it."""
    import oracle
    a = s.cpu().numpy()
    secs = []
    while len(secs) < 3 and sum(secs) < 40.0:
        tc = time.perf_counter()
        ores = oracle.ns_sqrt(a, leaf, args.tau, args.tol, args.maxit, tau_s=args.tau_s, mu_rel=mu_rel,
                              stagnation_stop=stag, damped=args.damped)
        secs.append(time.perf_counter() - tc)
    sec = float(np.median(secs))
    Yh, Zh = Y.cpu().numpy(), Z.cpu().numpy()
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": 1.0 / sec, "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": (f"the whole solve (n = {a.shape[0]}, FP64 leaves), median of {len(secs)} run(s): "
                       f"{', '.join(f'{x:.1f}' for x in secs)} s"),
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


def run_c3(args):
    """The n = m^3 ill-conditioned Gramian (default m = 32, n = 32768), one
    step = one Newton-Schulz iteration of a stream of solves.  W warm-up
    iterations run on a solve that is then dropped; the timed region then
    begins a solve (ingest), steps it iteration by iteration, finishes it
    (egress) when its stop test fires and begins the next, until exactly K
    iterations have run.  Leaf-product launches of the timed region are timed
    with HIP events on the library's stream (plain launches; at this size a
    launch lasts milliseconds, so replaying graphs would change nothing)."""
    import torch

    from paper_1508_05856_amd import inputs, spamm

    cfg = inputs.config_c3_spec(args.m)
    n, leaf, mu_rel = cfg["n"], cfg["leaf"], cfg["mu_rel"]
    tau = cfg["tau"] if args.tau_cli is None else args.tau
    tol = cfg["tol"] if args.tol_cli is None else args.tol
    tau_s = cfg["tau_s_rel"] * tau if args.tau_s < 0 else args.tau_s
    stag = not args.literal_stop
    damped = True
    dev = torch.device("cuda:0")
    s = inputs.gramian_device(inputs.gauss_positions(cfg["m"], cfg["h"], 0.1, 0, n), dev)
    Y, Z = torch.empty_like(s), torch.empty_like(s)
    ctx = spamm.Context(0)
    opts = dict(leaf=leaf, prec=args.prec, tau_s=tau_s, mu_rel=mu_rel, stagnation_stop=stag, damped=damped)

    def history_flops(it_from, it_to):
        """Useful flops of the leaf-product launches of iterations
        [it_from, it_to) of the solve just finished (x product, then the y and
        z update unless the solve stopped at that iteration)."""
        r, t, nR = ctx.ns_history()
        kfin = len(nR) - 1
        fl = 0.0
        for it in range(it_from, min(it_to, kfin + 1)):
            fl += 2.0 * leaf ** 3 * nR[it, 0]
            if it < kfin:
                fl += 2.0 * leaf ** 3 * (nR[it, 1] + nR[it, 2])
        return fl

    sv = ctx.solve_begin(s, tau, tol, args.maxit, **opts)
    for _ in range(args.warmup):
        if ctx.solve_step([sv], 1) == 0:
            break
    sv.finish(want_outputs=False)

    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done, flops, k, sv, its, tb = [], 0.0, 0, None, 0, 0.0
    while k < args.steps:
        if sv is None:
            tb = time.perf_counter()
            sv = ctx.solve_begin(s, tau, tol, args.maxit, **opts)
            its = 0
        running = ctx.solve_step([sv], 1)
        k += 1
        its += 1
        if running == 0:
            _, _, info = sv.finish(Y, Z)
            done.append(dict(seconds=time.perf_counter() - tb, info=info))
            flops += history_flops(0, its)
            sv = None
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gemm_ms = ctx.profile_read(spamm.KIND_GEMM)
    cull_ms = ctx.profile_read(spamm.KIND_CULL)
    pyr_ms = ctx.profile_read(spamm.KIND_PYRAMID)
    ctx.profile(False)
    if sv is not None:  # the partial solve the region ended in: its launches were timed too
        sv.finish(want_outputs=False)
        flops += history_flops(0, its)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    if done:
        info = done[0]["info"]
        sec_per_solve = done[0]["seconds"]
        how = "the first solve run whole inside the timed region, ingest to egress"
    else:
        info = None
        sec_per_solve = None
        how = None
        print(f"no solve ran whole inside the {args.steps} timed iterations: value needs --steps at least "
              f"the iterations of one solve (14 at n = 32768)", file=sys.stderr, flush=True)

    useful = flops / (float(np.sum(gemm_ms)) * 1e-3) / 1e12
    achieved = EXEC_PER_USEFUL[args.prec] * useful
    peak = PEAK_TFLOPS[args.prec]
    resid_exact = None
    if info is not None:
        C, _, _ = ctx.spamm_multiply(Y, Z, 0.0, leaf)
        C.diagonal().sub_(1.0)
        resid_exact = float(torch.linalg.norm(C))
        del C
    line = {
        "metric": "NS sqrt solves/sec at stated ||I-YZ||_F (culled-leaf TFLOP/s vs MFMA peak in roofline)",
        "value": (1.0 / sec_per_solve) if sec_per_solve else None,
        "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.prec, "data": "synthetic",
        "config": {
            "workload": cfg["name"] + ("" if args.prec == "f64" else f"_{args.prec}"), "n": n, "leaf": leaf,
            "tau": tau, "tau_s": tau_s, "tol": tol, "maxit": args.maxit, "mu_rel": mu_rel,
            "stop": "stagnation" if stag else "literal", "precision": args.prec, "map": "damped",
            "step": "one Newton-Schulz iteration (x product and stop test, then the y and z update)",
            "value_from": how,
            "solves_completed_in_timed_region": len(done),
            "status": spamm.STATUS_NAMES.get(info["status"], info["status"]) if info else None,
            "iterations": info["iterations"] if info else None,
            "resid_inloop": info["resid"] if info else None, "resid_exact": resid_exact,
            "trace_err": info["trace_err"] if info else None,
            "triples_per_solve": info["triples_total"] if info else None,
            "flops_per_solve": info["flops_total"] if info else None,
            "seconds_per_solve": sec_per_solve,
        },
        "roofline": {
            "bound": "mfma", "kernel": _gemm_kernel(args.prec, leaf), "achieved": achieved, "peak": peak,
            "unit": "TFLOP/s", "frac": achieved / peak,
            "traffic": committed_traffic(cfg["name"], args.prec), "traffic_unit": "bytes per launch",
            "useful_tflops": useful, "launches": int(len(gemm_ms)), "avg_launch_ms": float(np.mean(gemm_ms)),
            "gemm_ms_in_region": float(np.sum(gemm_ms)), "cull_ms_in_region": float(np.sum(cull_ms)),
            "pyramid_ms_in_region": float(np.sum(pyr_ms)), "region_ms": (t1 - t0) * 1e3,
            "timing": "HIP events on the library's stream around every leaf-product launch of the timed region",
        },
    }
    if not args.no_cpu_baseline and info is not None:
        if n <= ORACLE_FULL_MAX_N:
            args.tau, args.tol, args.tau_s, args.damped = tau, tol, tau_s, damped
            line["cpu_baseline"] = cpu_baseline_full(s, leaf, args, mu_rel, stag, info, Y, Z)
        else:
            line["cpu_baseline"] = cpu_baseline_sampled_tiles(s, mu_rel, leaf, tau, info)
    ctx.close()
    print(json.dumps(line), flush=True)


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
    achieved = EXEC_PER_USEFUL[args.prec] * st["flops"] / (float(np.mean(g)) * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.prec]
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
    if prec == "bf16x6":
        return "k_leaf_gemm_bf3"
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
        print(json.dumps({"error": "bench.py runs on one GPU; sharding across GPUs is not implemented",
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
    if args.workload == "c3":
        run_c3(args)
        return

    import torch

    from paper_1508_05856_amd import inputs, spamm

    dev = torch.device("cuda:0")
    stag = not args.literal_stop
    mu_rel = 0.0
    if args.workload == "c1":
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
    # the split-bf16 modes execute three or six bf16 products per useful one:
    # their roofline is the executed rate against the bf16 peak (the useful
    # rate is reported beside it)
    achieved = EXEC_PER_USEFUL[args.prec] * useful
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

    # the same workload under the other stop rule (the literal rule of tol or
    # maxit beside the stagnation stop, or the reverse), timed over 3 solves
    stag_other = not stag
    Yo, Zo = torch.empty_like(s), torch.empty_like(s)
    torch.cuda.synchronize()
    to0 = time.perf_counter()
    for _ in range(3):
        _, _, oinfo = ctx.ns_sqrt(s, args.tau, args.tol, args.maxit, leaf=leaf, prec=args.prec, tau_s=args.tau_s,
                                  mu_rel=mu_rel, stagnation_stop=stag_other, damped=args.damped, Y=Yo, Z=Zo,
                                  raise_on_error=False)
    torch.cuda.synchronize()
    line["config"]["other_stop"] = {
        "stop": "stagnation" if stag_other else "literal", "solves_per_s": 3.0 / (time.perf_counter() - to0),
        "status": spamm.STATUS_NAMES.get(oinfo["status"], oinfo["status"]), "iterations": oinfo["iterations"],
        "resid_inloop": oinfo["resid"]}
    del Yo, Zo

    if not args.no_cpu_baseline and n <= ORACLE_FULL_MAX_N:
        line["cpu_baseline"] = cpu_baseline_full(s, leaf, args, mu_rel, stag, info, Y, Z)
    elif not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_sampled_tiles(s, mu_rel, leaf, args.tau, info)
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
