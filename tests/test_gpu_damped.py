"""GPU parity of the damped map (scaling alpha(t), stabilisation eps(t) of the
trace error, switched off once t_k < 0.1) against the FP64 oracle: same
status and update count, iterates to 1e-12 relative, residual histories to
1e-9; the switched-off map equal to the plain map bit for bit; damped and
plain solves sharing launches equal to their solo results bit for bit."""
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
    # (name, matrix builder, leaf, tau, tau_s, mu_rel)
    ("kms384", lambda: inputs.kms(384, 0.8), 32, 1e-8, -1.0, 0.0),
    ("gauss512_exact", lambda: inputs.gauss_gramian(8, 0.8), 32, 0.0, -1.0, 0.0),
    ("gauss512_tau", lambda: inputs.gauss_gramian(8, 0.8), 64, 1e-6, 1e-8, 0.0),
    ("gauss1000_mu", lambda: inputs.gauss_gramian(10, 0.6), 32, 1e-6, 1e-8, 1e-4),
    ("gauss700_ragged", lambda: inputs.gauss_gramian(9, 1.0, n=700), 64, 1e-8, -1.0, 0.0),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_damped_ns_matches_oracle(ctx, case):
    name, build, leaf, tau, tau_s, mu = case
    s = build()
    Y, Z, info = ctx.ns_sqrt(dev(s), tau, 1e-10, 40, leaf=leaf, tau_s=tau_s, mu_rel=mu, stagnation_stop=True,
                             damped=True, raise_on_error=False)
    r, t, nR = ctx.ns_history()
    o = oracle.ns_sqrt(s, leaf, tau, 1e-10, 40, tau_s=tau_s, mu_rel=mu, stagnation_stop=True, damped=True)
    print(f"{name}: status {info['status']} / {o['status']}, updates {info['iterations']} / {o['iterations']}")
    assert info["status"] == o["status"] and info["iterations"] == o["iterations"]
    np.testing.assert_allclose(r, o["r"], rtol=1e-9, atol=1e-13)
    np.testing.assert_array_equal(nR, o["nR"])
    assert rel(Y.cpu().numpy(), o["Y"]) <= 1e-12 and rel(Z.cpu().numpy(), o["Z"]) <= 1e-12


def test_damped_switched_off_equals_plain(ctx):
    s = dev(inputs.kms(256, 0.03))
    Yp, Zp, ip = ctx.ns_sqrt(s, 1e-8, 1e-12, 30, leaf=32, stagnation_stop=True)
    Yd, Zd, idm = ctx.ns_sqrt(s, 1e-8, 1e-12, 30, leaf=32, stagnation_stop=True, damped=True)
    assert ip["iterations"] == idm["iterations"]
    assert torch.equal(Yp, Yd) and torch.equal(Zp, Zd)


@pytest.mark.parametrize("prec", ["f64", "bf16x3"])
def test_damped_and_plain_in_one_batch_match_solo(ctx, prec):
    mats = [inputs.gauss_gramian(8, 0.8), inputs.kms(300, 0.7), inputs.gauss_gramian(7, 1.0, n=300)]
    flags = [True, False, True]
    solo = [ctx.ns_sqrt(dev(s), 1e-6, 1e-10, 30, leaf=64, prec=prec, tau_s=1e-8, stagnation_stop=True,
                        damped=d, raise_on_error=False) for s, d in zip(mats, flags)]
    solves = [ctx.solve_begin(dev(s), 1e-6, 1e-10, 30, leaf=64, prec=prec, tau_s=1e-8, stagnation_stop=True,
                              damped=d) for s, d in zip(mats, flags)]
    while ctx.solve_step(solves, 3) > 0:
        pass
    for sv, (Ys, Zs, infos) in zip(solves, solo):
        Y, Z, info = sv.finish()
        assert info["iterations"] == infos["iterations"]
        assert torch.equal(Y, Ys) and torch.equal(Z, Zs)
