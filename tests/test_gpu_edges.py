"""GPU edge cases against the oracle: orders below one leaf (n = 1, 3, 5, 17),
the identity (zero updates), the zero matrix and other invalid inputs, and the
largest blocked order the library accepts."""
import ctypes

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


@pytest.mark.parametrize("n,leaf", [(1, 16), (3, 16), (17, 32), (5, 64), (1, 64)])
@pytest.mark.parametrize("single", [False, True])
def test_orders_below_one_leaf(ctx, n, leaf, single):
    s = inputs.kms(n, 0.5) + 0.5 * np.eye(n)
    Y, Z, info = ctx.ns_sqrt(dev(s), 1e-8, 1e-12, 20, leaf=leaf, stagnation_stop=True, single=single)
    o = oracle.ns_sqrt(s, leaf, 1e-8, 1e-12, 20, stagnation_stop=True, single=single)
    assert info["status"] == o["status"] and info["iterations"] == o["iterations"]
    np.testing.assert_allclose(Y.cpu().numpy(), o["Y"], rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(Z.cpu().numpy(), o["Z"], rtol=1e-13, atol=1e-15)
    a = np.random.default_rng(n).standard_normal((n, n))
    C, st, trip = ctx.spamm_multiply(dev(a), dev(a), 1e-6, leaf, triples=True)
    Co, Ro, cnt = oracle.spamm(a, a, leaf, 1e-6, want_triples=True)
    assert st["retained"] == cnt == 1
    np.testing.assert_allclose(C.cpu().numpy(), Co, rtol=0, atol=1e-13 * np.linalg.norm(a) ** 2)


def test_identity_needs_no_update(ctx):
    for single in (False, True):
        Y, Z, info = ctx.ns_sqrt(dev(np.eye(200)), 1e-8, 1e-10, 20, leaf=32, single=single)
        assert info["status"] == 0 and info["iterations"] == 0 and info["resid"] == 0.0
        assert torch.equal(Y, torch.eye(200, dtype=torch.float64, device="cuda"))
        assert torch.equal(Z, torch.eye(200, dtype=torch.float64, device="cuda"))


def test_invalid_inputs(ctx):
    from paper_1508_05856_amd import spamm
    with pytest.raises(spamm.SpammError) as e:
        ctx.ns_sqrt(dev(np.zeros((8, 8))), 1e-8, 1e-10, 20, leaf=16)
    assert e.value.status == spamm.EINVAL                       # zero Gershgorin bound
    with pytest.raises(spamm.SpammError) as e:
        ctx.ns_sqrt(torch.zeros((0, 0), dtype=torch.float64, device="cuda"), 1e-8, 1e-10, 20)
    assert e.value.status == spamm.EINVAL                       # empty
    # more than 1024 leaf blocks per side: rejected from the sizes alone,
    # before the (small, real) buffers are touched
    buf = torch.zeros(16, dtype=torch.float64, device="cuda")
    n = 1025 * 16
    opts = spamm.NsOpts(16, 0, -1.0, 0.0, 0, 0, 0)
    res = spamm.NsResult()
    st = ctx.lib.ns_sqrt(ctx.handle, buf.data_ptr(), buf.data_ptr(), buf.data_ptr(), n, n, 1e-8, 1e-10, 20,
                         ctypes.byref(opts), ctypes.byref(res), None)
    assert st == spamm.EINVAL and b"blocks per side" in ctx.lib.spamm_last_error()
    with pytest.raises(spamm.SpammError) as e:
        ctx.solve_begin(dev(inputs.kms(64, 0.5)), 1e-8, 1e-10, 20, leaf=16, prec="bf16x3")
    assert e.value.status == spamm.EINVAL                       # BF16x3 needs leaf 32 or 64
