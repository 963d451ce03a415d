"""GPU tests of the step API: batched solves of uneven n sharing launches, and
continuous batching (solves joining and leaving between steps).

Every solve advances through the same kernels whether it runs alone or in a
mix, one workgroup per output tile with fixed-order reductions, so its result
must be bitwise identical alone and in any mix; against the FP64 oracle the
FP64 results must agree to 1e-12 (relative Frobenius) with the same iteration
count and retained-triple history.
"""
import numpy as np
import pytest

import oracle
from paper_1508_05856_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_1508_05856_amd import spamm
    c = spamm.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.cpu().numpy()


def rel(x, ref):
    return np.linalg.norm(x - ref) / np.linalg.norm(ref)


# (kind, n, param, seed, leaf, tau) -- uneven n, both leaf sizes, ragged n
CASES = [
    ("kms", 256, 0.7, 0, 32, 1e-8),
    ("gauss", 300, 1.1, 1, 32, 1e-6),
    ("kms", 448, 0.85, 2, 64, 1e-6),
    ("gauss", 700, 1.0, 3, 64, 1e-8),
    ("kms", 96, 0.6, 4, 32, 1e-4),
    ("gauss", 1000, 1.2, 5, 64, 1e-6),
]


def make(kind, n, param, seed):
    spec = dict(kind=kind, n=n, seed=seed, rho=param, h=param)
    return inputs.build_spec(spec)


def solo(ctx, s, leaf, tau, prec="f64"):
    Y, Z, info = ctx.ns_sqrt(dev(s), tau, 1e-10, 30, leaf=leaf, prec=prec, stagnation_stop=True,
                             raise_on_error=False)
    return host(Y), host(Z), info


def test_step_api_equals_ns_sqrt(ctx):
    s = inputs.kms(384, 0.8)
    Y0, Z0, info0 = solo(ctx, s, 32, 1e-8)
    sv = ctx.solve_begin(dev(s), 1e-8, 1e-10, 30, leaf=32, stagnation_stop=True)
    while ctx.solve_step([sv], 1) > 0:
        pass
    Y, Z, info = sv.finish()
    assert info["status"] == info0["status"] and info["iterations"] == info0["iterations"]
    np.testing.assert_array_equal(host(Y), Y0)
    np.testing.assert_array_equal(host(Z), Z0)


def test_batched_uneven_solves_match_oracle_and_solo(ctx):
    mats = [make(k, n, p, sd) for (k, n, p, sd, _, _) in CASES]
    solos = [solo(ctx, s, leaf, tau) for s, (_, _, _, _, leaf, tau) in zip(mats, CASES)]
    solves = [ctx.solve_begin(dev(s), tau, 1e-10, 30, leaf=leaf, stagnation_stop=True)
              for s, (_, _, _, _, leaf, tau) in zip(mats, CASES)]
    steps = 0
    while ctx.solve_step(solves, 3) > 0:
        steps += 1
        assert steps < 40
    for sv, s, (Ys, Zs, infos), (_, n, _, _, leaf, tau) in zip(solves, mats, solos, CASES):
        Y, Z, info = sv.finish()
        Y, Z = host(Y), host(Z)
        assert info["status"] == infos["status"] and info["iterations"] == infos["iterations"]
        np.testing.assert_array_equal(Y, Ys)     # alone == in the mix, bitwise
        np.testing.assert_array_equal(Z, Zs)
        ores = oracle.ns_sqrt(s, leaf, tau, 1e-10, 30, stagnation_stop=True)
        r, t, nR = ctx.ns_history()
        assert info["status"] == ores["status"] and info["iterations"] == ores["iterations"]
        assert rel(Y, ores["Y"]) <= 1e-12 and rel(Z, ores["Z"]) <= 1e-12


def test_batched_large_tables_match_solo(ctx):
    """Tables of more than 1024 tiles take the parallel cull, the multi-block
    longest-first sort and the job expansion (smaller ones take the one-launch
    front): four solves at leaf 32, three with more than 1024 tiles each (and
    one small one in the same tables), at different tau so that they stop at
    different steps, must match their solo runs bitwise."""
    specs = [("kms", 1100, 0.8, 0, 1e-8), ("gauss", 1200, 1.0, 1, 1e-6), ("kms", 1056, 0.6, 2, 1e-4),
             ("kms", 200, 0.7, 3, 1e-6)]
    mats = [make(k, n, p, sd) for (k, n, p, sd, _) in specs]
    solos = [solo(ctx, s, 32, tau) for s, (_, _, _, _, tau) in zip(mats, specs)]
    solves = [ctx.solve_begin(dev(s), tau, 1e-10, 30, leaf=32, stagnation_stop=True)
              for s, (_, _, _, _, tau) in zip(mats, specs)]
    steps = 0
    while ctx.solve_step(solves, 3) > 0:
        steps += 1
        assert steps < 40
    its = set()
    for sv, (Ys, Zs, infos) in zip(solves, solos):
        Y, Z, info = sv.finish()
        assert info["status"] == infos["status"] and info["iterations"] == infos["iterations"]
        np.testing.assert_array_equal(host(Y), Ys)
        np.testing.assert_array_equal(host(Z), Zs)
        its.add(info["iterations"])
    assert len(its) > 1  # the solves left the shared launches at different steps


def test_batched_multiblock_sort_matches_solo(ctx):
    """Tables of more than 16384 tiles are ordered by the multi-block sort
    (per-block histograms, a scan, a scatter): a 132 x 132-tile solve and a
    small one share such tables, and both must match their solo runs bitwise
    (the small one runs alone on the one-launch front)."""
    specs = [("kms", 4200, 0.8, 0, 1e-8), ("kms", 200, 0.7, 3, 1e-6)]
    mats = [make(k, n, p, sd) for (k, n, p, sd, _) in specs]
    solos = [solo(ctx, s, 32, tau) for s, (_, _, _, _, tau) in zip(mats, specs)]
    solves = [ctx.solve_begin(dev(s), tau, 1e-10, 30, leaf=32, stagnation_stop=True)
              for s, (_, _, _, _, tau) in zip(mats, specs)]
    steps = 0
    while ctx.solve_step(solves, 3) > 0:
        steps += 1
        assert steps < 40
    for sv, (Ys, Zs, infos) in zip(solves, solos):
        Y, Z, info = sv.finish()
        assert info["status"] == infos["status"] and info["iterations"] == infos["iterations"]
        np.testing.assert_array_equal(host(Y), Ys)
        np.testing.assert_array_equal(host(Z), Zs)


def test_batched_mixed_cull_kernels_match_solo(ctx):
    """A 257 x 257-tile solve (the blocked cull, with ragged blocks at the
    edge) shares its tables with two that take the per-tile cull; each kernel
    covers only its own products.  All three must match their solo runs
    bitwise."""
    specs = [("kms", 8200, 0.8, 0, 1e-8), ("kms", 1100, 0.7, 1, 1e-8), ("kms", 300, 0.6, 2, 1e-6)]
    mats = [make(k, n, p, sd) for (k, n, p, sd, _) in specs]
    solos = [solo(ctx, s, 32, tau) for s, (_, _, _, _, tau) in zip(mats, specs)]
    solves = [ctx.solve_begin(dev(s), tau, 1e-10, 30, leaf=32, stagnation_stop=True)
              for s, (_, _, _, _, tau) in zip(mats, specs)]
    steps = 0
    while ctx.solve_step(solves, 3) > 0:
        steps += 1
        assert steps < 40
    for sv, (Ys, Zs, infos) in zip(solves, solos):
        Y, Z, info = sv.finish()
        assert info["status"] == infos["status"] and info["iterations"] == infos["iterations"]
        np.testing.assert_array_equal(host(Y), Ys)
        np.testing.assert_array_equal(host(Z), Zs)


def test_continuous_batching_join_and_leave(ctx):
    mats = [make(k, n, p, sd) for (k, n, p, sd, _, _) in CASES]
    solos = [solo(ctx, s, leaf, tau) for s, (_, _, _, _, leaf, tau) in zip(mats, CASES)]
    pending = list(range(len(CASES)))
    active = {}
    results = {}
    tick = 0
    while pending or active:
        # admit up to two new solves every other tick
        if pending and tick % 2 == 0:
            for _ in range(2):
                if pending:
                    i = pending.pop(0)
                    _, _, _, _, leaf, tau = CASES[i]
                    active[i] = ctx.solve_begin(dev(mats[i]), tau, 1e-10, 30, leaf=leaf, stagnation_stop=True)
        order = sorted(active)
        ctx.solve_step([active[i] for i in order], 1)
        for i in order:
            if active[i].poll()["done"]:
                Y, Z, info = active.pop(i).finish()
                results[i] = (host(Y), host(Z), info)
        tick += 1
        assert tick < 200
    for i, (Ys, Zs, infos) in enumerate(solos):
        Y, Z, info = results[i]
        assert info["iterations"] == infos["iterations"]
        np.testing.assert_array_equal(Y, Ys)
        np.testing.assert_array_equal(Z, Zs)


@pytest.mark.parametrize("prec", ["f32", "bf16x3", "bf16x6"])
def test_batched_reduced_precision_matches_solo(ctx, prec):
    mats = [inputs.kms(256, 0.7), inputs.gauss_gramian(6, 1.2), inputs.kms(640, 0.6)]
    solos = [solo(ctx, s, 64, 1e-6, prec=prec) for s in mats]
    solves = [ctx.solve_begin(dev(s), 1e-6, 1e-10, 30, leaf=64, prec=prec, stagnation_stop=True) for s in mats]
    while ctx.solve_step(solves, 4) > 0:
        pass
    for sv, (Ys, Zs, infos), s in zip(solves, solos, mats):
        Y, Z, info = sv.finish()
        np.testing.assert_array_equal(host(Y), Ys)
        w, V = np.linalg.eigh(s)
        assert rel(host(Y), (V * np.sqrt(w)) @ V.T) < 1e-3


def test_bf16x6_quads_in_a_shared_table_match_one_tile_solo(ctx):
    """BF16x6 products of tables past 1024 tiles run on the quad kernel,
    smaller tables one tile per workgroup, and the two give bitwise the same
    tiles: three solves of 576-625 tiles each (alone: one tile per
    workgroup) stepped together (1826 tiles: quads, the last quad row and
    column of each product past its edge) must match their solo runs bit for
    bit."""
    mats = [inputs.kms(1600, 0.8), inputs.gauss_gramian(12, 1.0, n=1600), inputs.kms(1500, 0.6)]
    solos = [solo(ctx, s, 64, 1e-8, prec="bf16x6") for s in mats]
    solves = [ctx.solve_begin(dev(s), 1e-8, 1e-10, 30, leaf=64, prec="bf16x6", stagnation_stop=True) for s in mats]
    while ctx.solve_step(solves, 4) > 0:
        pass
    for sv, (Ys, Zs, infos) in zip(solves, solos):
        Y, Z, info = sv.finish()
        assert info["status"] == infos["status"] and info["iterations"] == infos["iterations"]
        np.testing.assert_array_equal(host(Y), Ys)
        np.testing.assert_array_equal(host(Z), Zs)


def test_footprint_and_errors(ctx):
    from paper_1508_05856_amd import spamm
    fp64 = ctx.footprint(4096, 64, "f64", 40)
    fp32 = ctx.footprint(4096, 64, "f32", 40)
    assert fp64 > 5 * 4096 * 4096 * 8 and fp32 > 5 * 4096 * 4096 * 4 and fp32 < fp64
    assert ctx.footprint(0, 64, "f64", 40) == 0
    s = inputs.kms(128, 0.5)
    sv = ctx.solve_begin(dev(s), 1e-6, 1e-10, 10, leaf=32)
    with pytest.raises(spamm.SpammError):
        ctx.solve_step([sv, sv], 1)          # a solve may appear once per step
    with pytest.raises(spamm.SpammError):
        ctx.solve_step([sv], 0)
    while ctx.solve_step([sv], 2) > 0:
        pass
    assert ctx.solve_step([sv], 1) == 0      # finished solves are skipped
    _, _, info = sv.finish()
    assert info["status"] in (0, 1, 2)


def test_graph_replays_equal_plain_launches(ctx):
    """Each step replays a captured iteration several times, with the engine's
    own eager read-back between steps; every result must equal the plain-launch
    result bitwise."""
    mats = [make(k, n, p, sd) for (k, n, p, sd, _, _) in CASES[:4]]

    def run(graphs):
        ctx.set_graphs(graphs)
        solves = [ctx.solve_begin(dev(s), tau, 1e-10, 30, leaf=leaf, stagnation_stop=True)
                  for s, (_, _, _, _, leaf, tau) in zip(mats, CASES[:4])]
        while ctx.solve_step(solves, 2) > 0:
            pass
        out = []
        for sv in solves:
            Y, Z, info = sv.finish()
            out.append((host(Y), host(Z), info["iterations"]))
        return out

    try:
        a = run(True)
        b = run(False)
        c = run(True)
    finally:
        ctx.set_graphs(True)
    for (ya, za, ka), (yb, zb, kb), (yc, zc, kc) in zip(a, b, c):
        assert ka == kb == kc
        np.testing.assert_array_equal(ya, yb)
        np.testing.assert_array_equal(za, zb)
        np.testing.assert_array_equal(ya, yc)


def test_step_with_more_groups_than_the_plan_cache(ctx):
    """One step over solves of 12 distinct (precision, leaf, channel) groups,
    more than the context caches plans for: every group's plan stays alive
    until the step has synchronised, and each solve equals its solo run bit
    for bit."""
    groups = [(p, lf, sg) for p in ("f64", "f32", "bf16x3", "bf16x6") for lf in (32, 64) for sg in (False, True)
              if not (p == "f32" and lf == 64)]
    assert len(groups) == 14
    mats = [inputs.kms(128 + 16 * i, 0.5 + 0.02 * i) for i in range(len(groups))]
    solo_out = [ctx.ns_sqrt(dev(s), 1e-8, 1e-8, 12, leaf=lf, prec=p, single=sg, stagnation_stop=True)
                for s, (p, lf, sg) in zip(mats, groups)]
    solves = [ctx.solve_begin(dev(s), 1e-8, 1e-8, 12, leaf=lf, prec=p, single=sg, stagnation_stop=True)
              for s, (p, lf, sg) in zip(mats, groups)]
    while ctx.solve_step(solves, 3) > 0:
        pass
    for sv, (Ys, Zs, infos), g in zip(solves, solo_out, groups):
        Y, Z, info = sv.finish()
        assert info["iterations"] == infos["iterations"], g
        assert torch.equal(Y, Ys) and torch.equal(Z, Zs), g


def test_warm_context_steps_and_finishes_without_allocating():
    """Solve memory and tables are pooled, not freed: once a set of solves has
    run, the same set begun again allocates nothing, and on a warm context a
    solve joining a running set (its begin reserves the group's tables) and
    a solve leaving it are stepped and finished without any allocation."""
    from paper_1508_05856_amd import spamm
    c = spamm.Context(0)
    try:
        mats = [inputs.kms(300, 0.7), inputs.gauss_gramian(7, 1.0), inputs.kms(500, 0.6)]

        def run_all():
            a0 = c.alloc_count()
            svs = [c.solve_begin(dev(m), 1e-8, 1e-9, 20, leaf=32, stagnation_stop=True) for m in mats]
            a1 = c.alloc_count()
            while c.solve_step(svs, 2) > 0:
                pass
            outs = [sv.finish() for sv in svs]
            return a0, a1, c.alloc_count(), outs

        _, _, _, first = run_all()
        a0, a1, a2, second = run_all()
        assert a2 == a1 == a0, (a0, a1, a2)
        for (Y1, Z1, i1), (Y2, Z2, i2) in zip(first, second):
            assert torch.equal(Y1, Y2) and torch.equal(Z1, Z2) and i1["iterations"] == i2["iterations"]
        # join and leave on the warm context
        A = c.solve_begin(dev(mats[0]), 1e-8, 1e-9, 20, leaf=32, stagnation_stop=True)
        c.solve_step([A], 1)
        B = c.solve_begin(dev(mats[2]), 1e-8, 1e-9, 20, leaf=32, stagnation_stop=True)
        b0 = c.alloc_count()
        c.solve_step([A, B], 1)
        A.finish()  # leaves after two iterations
        while c.solve_step([B], 2) > 0:
            pass
        YB, ZB, _ = B.finish()
        assert c.alloc_count() == b0
        # B joined a running solve and saw it leave: still bitwise its run with the others
        assert torch.equal(YB, first[2][0]) and torch.equal(ZB, first[2][1])
    finally:
        c.close()


def test_pool_limit_frees_returned_memory():
    """With a pool limit of zero a finished solve's memory is freed at once,
    so the next solve allocates again; with the default (no limit) it is
    reused.  Results are the same either way."""
    from paper_1508_05856_amd import spamm
    c = spamm.Context(0)
    try:
        s = dev(inputs.kms(400, 0.7))
        Y0, Z0, _ = c.ns_sqrt(s, 1e-8, 1e-9, 20, leaf=32, stagnation_stop=True)
        a = c.alloc_count()
        Y1, Z1, _ = c.ns_sqrt(s, 1e-8, 1e-9, 20, leaf=32, stagnation_stop=True)
        assert c.alloc_count() == a
        c.set_pool_limit(0)
        Y2, Z2, _ = c.ns_sqrt(s, 1e-8, 1e-9, 20, leaf=32, stagnation_stop=True)
        assert c.alloc_count() > a
        assert torch.equal(Y0, Y1) and torch.equal(Y0, Y2) and torch.equal(Z0, Z2)
    finally:
        c.close()


def test_batched_fp32_instances_match_the_fp64_oracle():
    """The largest converging instances of the batched workload (64 uneven
    SPD matrices, FP32 leaves, tol 1e-6, tau_s = 0.01 tau, stagnation stop,
    autotuned leaf): the largest KMS (n = 3904, rho = 0.70) and the largest
    Gaussian Gramian at tau = 1e-6 (n = 3968, h = 0.90), solved together
    through the step API and each compared with the oracle's FP64 solve of the
    same instance and options, with the oracle's status and a stop within one
    update of its.  FP32 leaves accumulate each tile's whole retained k list
    in one FP32 running sum, whose rounding grows with the list and which the
    inverse root amplifies by up to sqrt(kappa): measured Y, Z 3.6e-7, 8.8e-7 on the KMS
    matrix (kappa 5.6) and 3.0e-3, 3.3e-3 on the Gramian (kappa 2.2e5, at
    its tau floor), both held to sqrt(kappa) 2^-16."""
    from paper_1508_05856_amd import autotune, spamm
    specs = inputs.batch_specs(64, seed=0)
    picks = [specs[14], specs[36]]
    assert picks[0]["kind"] == "kms" and picks[1]["kind"] == "gauss"
    mats = [inputs.build_spec(sp) for sp in picks]
    leaves = [autotune.choose_leaf(autotune.load("f32", sp["tau"]), sp["kind"], sp["n"]) for sp in picks]
    c = spamm.Context(0)
    try:
        solves = [c.solve_begin(dev(m), sp["tau"], 1e-6, 40, leaf=lf, prec="f32", tau_s=0.01 * sp["tau"],
                                stagnation_stop=True) for m, sp, lf in zip(mats, picks, leaves)]
        while c.solve_step(solves, 4) > 0:
            pass
        outs = [sv.finish() for sv in solves]
    finally:
        c.close()
    for m, sp, lf, (Y, Z, info) in zip(mats, picks, leaves, outs):
        o = oracle.ns_sqrt(m, lf, sp["tau"], 1e-6, 40, tau_s=0.01 * sp["tau"], stagnation_stop=True)
        w = np.linalg.eigvalsh(m)
        bound = np.sqrt(w[-1] / w[0]) * 2.0 ** -16
        ey, ez = rel(host(Y), o["Y"]), rel(host(Z), o["Z"])
        print(f"batched FP32 {sp['kind']} n={sp['n']} leaf {lf}: relY {ey:.2e} relZ {ez:.2e} (bound {bound:.2e}); "
              f"status {info['status']} vs {o['status']}, updates {info['iterations']} vs {o['iterations']}")
        assert info["status"] == o["status"] and abs(info["iterations"] - o["iterations"]) <= 1
        assert ey <= bound and ez <= bound
