"""GPU parity of the single-channel instance (z_{k+1} = z_k h[x_k],
x_k = z_k^T s z_k with the implicit y channel y_k = s' (x)_{tau_s} z_k)
against the FP64 oracle: same status and update count, identical
retained-triple histories, residual histories to 1e-9 and iterates to 1e-12
relative; single and dual solves sharing a step equal to their solo results
bit for bit; BF16x3 leaves within the sqrt(kappa) 2^-16 bound."""
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


def rel(x, ref):
    return np.linalg.norm(x - ref) / np.linalg.norm(ref)


CASES = [
    # (name, builder, leaf, tau, tau_s, mu_rel, damped)
    ("kms384", lambda: inputs.kms(384, 0.8), 32, 1e-8, -1.0, 0.0, False),
    ("gauss512_exact", lambda: inputs.gauss_gramian(8, 0.8), 32, 0.0, -1.0, 0.0, False),
    ("gauss700_ragged", lambda: inputs.gauss_gramian(9, 1.0, n=700), 64, 1e-8, 1e-10, 0.0, False),
    ("gauss1000_mu_damped", lambda: inputs.gauss_gramian(10, 0.6), 32, 1e-6, 1e-8, 1e-4, True),
    ("kms200_leaf16", lambda: inputs.kms(200, 0.6), 16, 1e-6, -1.0, 0.0, False),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_single_channel_matches_oracle(ctx, case):
    name, build, leaf, tau, tau_s, mu, damped = case
    s = build()
    Y, Z, info = ctx.ns_sqrt(dev(s), tau, 1e-10, 40, leaf=leaf, tau_s=tau_s, mu_rel=mu, stagnation_stop=True,
                             damped=damped, single=True, raise_on_error=False)
    r, t, nR = ctx.ns_history()
    o = oracle.ns_sqrt(s, leaf, tau, 1e-10, 40, tau_s=tau_s, mu_rel=mu, stagnation_stop=True, damped=damped,
                       single=True)
    print(f"{name}: status {info['status']} / {o['status']}, updates {info['iterations']} / {o['iterations']}")
    assert info["status"] == o["status"] and info["iterations"] == o["iterations"]
    np.testing.assert_array_equal(nR, o["nR"])
    # x_k = z_k^T s' z_k carries sqrt(kappa(s')) into the rounding of every
    # entry: residuals agree to 1e-9 relative above a floor of u n sqrt(kappa)
    w = np.linalg.eigvalsh(s)
    floor = 2.2e-16 * s.shape[0] * np.sqrt(w[-1] / w[0])
    np.testing.assert_allclose(r, o["r"], rtol=1e-9, atol=floor)
    assert rel(Y.cpu().numpy(), o["Y"]) <= 1e-12 and rel(Z.cpu().numpy(), o["Z"]) <= 1e-12


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3", "bf16x6"])
def test_single_and_dual_in_one_step_match_solo(ctx, prec):
    mats = [inputs.kms(300, 0.7), inputs.gauss_gramian(8, 1.0), inputs.kms(500, 0.85), inputs.gauss_gramian(6, 1.2)]
    single = [True, False, True, False]
    solo = [ctx.ns_sqrt(dev(s), 1e-7, 1e-10, 30, leaf=64, prec=prec, stagnation_stop=True, single=sg,
                        raise_on_error=False) for s, sg in zip(mats, single)]
    solves = [ctx.solve_begin(dev(s), 1e-7, 1e-10, 30, leaf=64, prec=prec, stagnation_stop=True, single=sg)
              for s, sg in zip(mats, single)]
    while ctx.solve_step(solves, 2) > 0:
        pass
    for sv, (Ys, Zs, infos) in zip(solves, solo):
        Y, Z, info = sv.finish()
        assert info["iterations"] == infos["iterations"]
        assert torch.equal(Y, Ys) and torch.equal(Z, Zs)


@pytest.mark.parametrize("leaf", [32, 64])
def test_single_channel_bf16x3_error(ctx, leaf):
    """Leaf 32 runs the one-tile BF16x3 kernel, leaf 64 the quad kernel."""
    s = inputs.kms(512, 0.7)
    w = np.linalg.eigvalsh(s)
    bound = np.sqrt(w[-1] / w[0]) * 2.0 ** -16
    Y, Z, info = ctx.ns_sqrt(dev(s), 1e-8, 1e-5, 40, leaf=leaf, prec="bf16x3", stagnation_stop=True, single=True)
    o = oracle.ns_sqrt(s, leaf, 1e-8, 1e-5, 40, stagnation_stop=True, single=True)
    ey, ez = rel(Y.cpu().numpy(), o["Y"]), rel(Z.cpu().numpy(), o["Z"])
    print(f"single bf16x3: relY {ey:.2e} relZ {ez:.2e} (bound {bound:.2e})")
    assert ey <= bound and ez <= bound


def test_single_footprint_holds_the_transpose(ctx):
    dual = ctx.footprint(2048, 64, "f64", 40)
    single = ctx.footprint(2048, 64, "f64", 40, single=True)
    assert single - dual >= 2048 * 2048 * 8


@pytest.mark.parametrize("leaf", [32, 64])
def test_single_channel_bf16x6_error(ctx, leaf):
    """The single-channel instance with BF16x6 leaves (the one-tile split
    kernel at both leaf sizes) against the FP64 oracle: Y and Z within 5e-6
    on the KMS matrix (kappa 32)."""
    s = inputs.kms(512, 0.7)
    Y, Z, info = ctx.ns_sqrt(dev(s), 1e-8, 1e-5, 40, leaf=leaf, prec="bf16x6", stagnation_stop=True, single=True)
    o = oracle.ns_sqrt(s, leaf, 1e-8, 1e-5, 40, stagnation_stop=True, single=True)
    ey, ez = rel(Y.cpu().numpy(), o["Y"]), rel(Z.cpu().numpy(), o["Z"])
    print(f"single bf16x6 leaf {leaf}: relY {ey:.2e} relZ {ez:.2e}")
    assert ey <= 5e-6 and ez <= 5e-6


def test_single_channel_bf16x6_quads_error():
    """A single-channel solve whose tables pass 1024 tiles (n = 2100, 33 x 33
    tiles of 64, the last quad row and column past the edge), so the BF16x6
    products, the transposed z^T included, run on the quad kernel: Y and Z
    within 5e-6 of the FP64 oracle on the KMS matrix (kappa 32)."""
    from paper_1508_05856_amd import spamm
    ctx = spamm.Context(0)
    s = inputs.kms(2100, 0.7)
    Y, Z, info = ctx.ns_sqrt(dev(s), 1e-8, 1e-5, 40, leaf=64, prec="bf16x6", stagnation_stop=True, single=True)
    ctx.close()
    o = oracle.ns_sqrt(s, 64, 1e-8, 1e-5, 40, stagnation_stop=True, single=True)
    ey, ez = rel(Y.cpu().numpy(), o["Y"]), rel(Z.cpu().numpy(), o["Z"])
    print(f"single bf16x6 quads n=2100: relY {ey:.2e} relZ {ez:.2e}; updates {info['iterations']} vs {o['iterations']}")
    assert info["status"] == o["status"]
    assert ey <= 5e-6 and ez <= 5e-6
