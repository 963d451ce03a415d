"""GPU parity of the product representation (Secs. 6.1, 6.3) against the FP64
oracle: the same per-slice statuses and update counts and the factor to
1e-10 relative; at tau = 0 the factor is (s + mu c0 I)^{-1/2}."""
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


def rel(x, ref):
    return np.linalg.norm(x - ref) / np.linalg.norm(ref)


@pytest.mark.parametrize("case", [
    ("gauss512_4slices", lambda: inputs.gauss_gramian(8, 0.8), [1e-1, 1e-2, 1e-3, 1e-4], 1e-4, 1e-8, 32),
    ("gauss343_exact", lambda: inputs.gauss_gramian(7, 0.8), [1e-2, 1e-3, 1e-4], 0.0, 0.0, 32),
    ("gauss700_ragged", lambda: inputs.gauss_gramian(9, 0.9, n=700), [1e-1, 1e-2, 1e-3], 1e-5, 1e-9, 64),
], ids=lambda c: c[0])
def test_product_rep_matches_oracle(ctx, case):
    name, build, mus, ts, tr, leaf = case
    s = build()
    W, info = ctx.product_rep(torch.from_numpy(s).cuda(), mus, ts, tr, 1e-10, 40, leaf=leaf, tau_s_slice=0.01 * ts,
                              damped=True)
    o = oracle.product_rep(s, leaf, mus, ts, tr, 1e-10, 40, tau_s_slice=0.01 * ts, damped=True)
    print(f"{name}: statuses {info['statuses']} / {o['statuses']}, updates {info['iterations']} / {o['iterations']}")
    assert info["statuses"] == o["statuses"] and info["iterations"] == o["iterations"]
    assert rel(W.cpu().numpy(), o["W"]) <= 1e-10


def test_product_rep_errors(ctx):
    from paper_1508_05856_amd import spamm
    s = torch.from_numpy(inputs.kms(128, 0.5)).cuda()
    with pytest.raises(spamm.SpammError):
        ctx.product_rep(s, [], 1e-4, 1e-8, 1e-10, 40)
    with pytest.raises(spamm.SpammError):
        ctx.product_rep(s, [1e-2, -1.0], 1e-4, 1e-8, 1e-10, 40)
