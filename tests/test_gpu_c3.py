"""Full-size ill-conditioned case: the n = 32768 Gaussian lattice Gramian
(m = 32, h = 0.6), shifted by mu = 1e-4 c0 and scaled to s' = (s + mu I)/c,
leaf 64 (nb = 512), tau = 1e-6.  The oracle cannot run the whole solve at this
size, so the product is checked on sampled output tiles (recomputed by the
oracle's recursion one by one) and on its whole retained set (counted from
the oracle's norm pyramid), and the BF16x3 solve is checked against the FP64
solve by the perturbation bound sqrt(kappa) 2^-16, with
kappa(s + mu I) <= (c0 + mu)/mu = 1 + 1e4.  At this n the solve diverges for
tau = 1e-6 (both maps, every leaf precision); it is run at tau = 1e-9 with
the damped map and tau_s = 0.01 tau, where it reaches its floor.
"""
import numpy as np
import pytest

import oracle
from paper_1508_05856_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TAU, LEAF, MU_REL = 1e-6, 64, 1e-4


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_1508_05856_amd import spamm
    c = spamm.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def raw():
    cfg = inputs.config_c3_spec()
    print(f"building the n={cfg['n']} Gramian on the device", flush=True)
    return inputs.gramian_device(inputs.gauss_positions(cfg["m"], cfg["h"], 0.1, 0, cfg["n"]), "cuda")


@pytest.fixture(scope="module")
def scaled(raw):
    """s' = (s + mu I)/c in FP64, by Gershgorin row sums (test-side plumbing)."""
    s = raw.clone()
    c0 = float(s.abs().sum(1).max())
    s.diagonal().add_(MU_REL * c0)
    s /= float(s.abs().sum(1).max())
    return s


def sample_tiles(nb, seed=0):
    rng = np.random.default_rng(seed)
    diag = [(int(i), int(i)) for i in rng.integers(0, nb, 4)]
    near = [(int(i), int(min(nb - 1, max(0, i + d)))) for i, d in zip(rng.integers(0, nb, 6),
                                                                        rng.integers(-4, 5, 6))]
    far = [(int(i), int(j)) for i, j in rng.integers(0, nb, (4, 2))]
    return diag + near + far + [(0, 0), (nb - 1, nb - 1)]


def flat_count(levels, nb, tau):
    """|R| = #{(i,j,k): ||A_ik|| ||A_kj|| >= tau ||A||^2} from the oracle's
    pyramid (the flat set equals the recursive one), and the near-ties."""
    na = levels[0][:nb, :nb]
    root = levels[-1][0, 0]
    thr = tau * (root * root)
    count = ties = 0
    for i in range(nb):
        prod = na[i][:, None] * na            # [k, j] = ||A_ik|| ||A_kj||
        count += int(np.count_nonzero(prod >= thr))
        ties += int(np.count_nonzero(np.abs(prod - thr) <= 1e-12 * thr))
    return count, ties


@pytest.mark.parametrize("prec", ["f64", "bf16x3"])
def test_c3_product_sampled_tiles_and_retained_set(ctx, scaled, prec):
    # the FP32-stored operand for the reduced-precision leaves (the cull sees those values)
    A = scaled if prec == "f64" else scaled.float().double()
    n = A.shape[0]
    nb = n // LEAF
    print(f"C3 product {prec}: n={n} leaf={LEAF} tau={TAU}", flush=True)
    C, st, trip = ctx.spamm_multiply(A, A, TAU, LEAF, prec=prec, triples=True, cap=8_000_000)
    a = A.cpu().numpy()
    count, ties = flat_count(oracle.norms(a, LEAF), nb, TAU)
    assert abs(st["retained"] - count) <= ties
    tiles = sample_tiles(nb)
    out, counts = oracle.spamm_tiles(a, a, LEAF, TAU, tiles)
    trip = trip.cpu().numpy()
    key = trip[:, 0].astype(np.int64) * nb + trip[:, 1]
    for (i, j), o, cnt in zip(tiles, out, counts):
        got = C[i * LEAF:(i + 1) * LEAF, j * LEAF:(j + 1) * LEAF].cpu().numpy()
        assert np.count_nonzero(key == i * nb + j) == cnt
        # every entry of s' is positive, so sum_R |A_ik||A_kj| is the oracle's tile itself
        if prec == "f64":
            assert np.all(np.abs(got - o) <= 1e-12 * o + 1e-300)
        else:
            assert np.all(np.abs(got - o) <= 2.0 ** -13 * o + 1e-300)
    del C


def test_c3_ns_bf16x3_against_fp64(ctx, raw):
    n = raw.shape[0]
    cfg = inputs.config_c3_spec()
    tau = cfg["tau"]
    res = {}
    for prec in ("f64", "bf16x3"):
        print(f"C3 solve {prec} tau={tau} damped", flush=True)
        Y, Z, info = ctx.ns_sqrt(raw, tau, cfg["tol"], cfg["maxit"], leaf=LEAF, prec=prec, mu_rel=MU_REL,
                                 tau_s=cfg["tau_s_rel"] * tau, stagnation_stop=True, damped=True,
                                 raise_on_error=False)
        print(f"  status {info['status']} iterations {info['iterations']} r {info['resid']:.3e} "
              f"t {info['trace_err']:.3e}", flush=True)
        assert info["status"] in (0, 2)
        res[prec] = (Y, Z, info)
    Y64, Z64, i64 = res["f64"]
    Y3, Z3, i3 = res["bf16x3"]
    # the iteration has left its slow start: trace error far below its start near 1
    assert abs(i64["trace_err"]) < 1e-3
    bound = np.sqrt(1.0 + 1.0 / MU_REL) * 2.0 ** -16
    ey = float(torch.linalg.norm(Y3 - Y64) / torch.linalg.norm(Y64))
    ez = float(torch.linalg.norm(Z3 - Z64) / torch.linalg.norm(Z64))
    print(f"  bf16x3 vs f64: relY {ey:.2e} relZ {ez:.2e} (bound {bound:.2e})", flush=True)
    assert ey <= bound and ez <= bound
    # sampled columns of Y Z - I with an independent FP64 GEMM
    cols = torch.arange(0, n, n // 64, device=Y64.device)
    E = Y64 @ Z64[:, cols]
    E[cols, torch.arange(len(cols), device=E.device)] -= 1.0
    col_rms = float(torch.linalg.norm(E)) / np.sqrt(len(cols))
    print(f"  sampled columns of YZ - I: rms {col_rms:.2e}, in-loop r/sqrt(n) {i64['resid'] / np.sqrt(n):.2e}")
    # the exact residual of the sampled columns agrees with the in-loop one
    assert col_rms < 3.0 * i64["resid"] / np.sqrt(n)


@pytest.mark.parametrize("prec", ["f64", "bf16x3"])
def test_c3_analogue_whole_solve_vs_oracle(ctx, prec):
    """The same configuration (mu = 1e-4 c0, tau = 1e-9, tau_s = 0.01 tau,
    damped map, stagnation stop, leaf 64) on the m = 12 lattice (n = 1728),
    where the oracle runs the whole solve.  FP64 leaves: same status, update
    count and residual history as the oracle, Y and Z to 1e-12.  BF16x3 leaves:
    Y and Z within sqrt(kappa) 2^-16 of the oracle's FP64 roots (kappa <= 1 +
    1/mu_rel), and a valid stop at a floor well below the stagnation guard's
    1/2."""
    cfg = inputs.config_c3_spec(12)
    s = inputs.gauss_gramian(12, cfg["h"], 0.1, 0)
    tau, tau_s = cfg["tau"], cfg["tau_s_rel"] * cfg["tau"]
    print(f"n={s.shape[0]} tau={tau} damped mu_rel={cfg['mu_rel']} prec={prec}", flush=True)
    Y, Z, info = ctx.ns_sqrt(torch.from_numpy(s).cuda(), tau, cfg["tol"], cfg["maxit"], leaf=cfg["leaf"], prec=prec,
                             tau_s=tau_s, mu_rel=cfg["mu_rel"], stagnation_stop=True, damped=True,
                             raise_on_error=False)
    ores = oracle.ns_sqrt(s, cfg["leaf"], tau, cfg["tol"], cfg["maxit"], tau_s=tau_s, mu_rel=cfg["mu_rel"],
                          stagnation_stop=True, damped=True)
    Yh, Zh = Y.cpu().numpy(), Z.cpu().numpy()
    ey = np.linalg.norm(Yh - ores["Y"]) / np.linalg.norm(ores["Y"])
    ez = np.linalg.norm(Zh - ores["Z"]) / np.linalg.norm(ores["Z"])
    print(f"status {info['status']} vs {ores['status']}, updates {info['iterations']} vs {ores['iterations']}, "
          f"relY {ey:.2e} relZ {ez:.2e}")
    if prec == "f64":
        assert info["status"] == ores["status"] and info["iterations"] == ores["iterations"]
        r, _, _ = ctx.ns_history()
        k = ores["iterations"]
        np.testing.assert_allclose(r[:k + 1], ores["r"][:k + 1], rtol=1e-9)
        assert ey <= 1e-12 and ez <= 1e-12
    else:
        bound = np.sqrt(1.0 + 1.0 / cfg["mu_rel"]) * 2.0 ** -16
        assert info["status"] in (0, 2)
        assert ey <= bound and ez <= bound
        assert info["resid"] < 0.05
