"""GPU: the retained triples a solve exports per product (the ijk volumes of
Secs. 5.4, 6.2 and 7.2) against the oracle and the solve's own history, and
the lensing the paper describes: towards convergence the y-product volume
h (x) y collapses onto the plane diagonal i = k as h tends to I."""
import numpy as np
import pytest

import oracle
from paper_1508_05856_amd import inputs, lensing

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_1508_05856_amd import spamm
    c = spamm.Context(0)
    yield c
    c.close()


def test_first_x_product_triples_match_the_oracle(ctx):
    """x_0 = s' (x)_tau I: its retained set is the oracle's for s' and I
    (triples within 1e-12 of the threshold excluded)."""
    n, leaf, tau = 512, 32, 1e-8
    s = inputs.kms(n, 0.7)
    sv = ctx.solve_begin(torch.from_numpy(s).cuda(), tau, 1e-10, 40, leaf=leaf)
    ctx.solve_step([sv], 1)
    got = sv.triples(0).cpu().numpy()
    sv.finish(want_outputs=False)
    sp = s / np.abs(s).sum(axis=0).max()
    _, ro, cnt = oracle.spamm(sp, np.eye(n), leaf, tau, want_triples=True)
    la, lb = oracle.norms(sp, leaf), oracle.norms(np.eye(n), leaf)
    nb = n // leaf
    thr = tau * (la[-1][0, 0] * lb[-1][0, 0])
    prod = la[0][:nb, :nb][:, None, :] * lb[0][:nb, :nb].T[None, :, :]
    ties = np.abs(prod - thr) <= 1e-12 * thr
    g = {tuple(t) for t in got.tolist() if not ties[t[0], t[1], t[2]]}
    e = {tuple(t) for t in np.asarray(ro).tolist() if not ties[t[0], t[1], t[2]]}
    assert g == e and len(got) == cnt


def test_volumes_match_history_and_lens(ctx):
    n, leaf, tau = 512, 32, 1e-8
    s = torch.from_numpy(inputs.kms(n, 0.7)).cuda()
    recs = lensing.trace_solve(ctx, s, tau, 1e-10, 40, leaf=leaf, stagnation_stop=True)
    r, t, nR = ctx.ns_history()
    assert recs[-1]["stopped"] and recs[-1]["k"] == len(nR) - 1
    for rec in recs:
        k = rec["k"]
        kx = k if rec["stopped"] else k - 1
        assert rec["x"]["count"] == nR[kx, 0]
        if k > 0:
            assert rec["y"]["count"] == nR[k - 1, 1] and rec["z"]["count"] == nR[k - 1, 2]
    first = next(rc for rc in recs if rc["k"] > 0)
    last = [rc for rc in recs if rc["k"] > 0][-1]
    print("y-product share on i = k:", first["y"]["ik"], "->", last["y"]["ik"])
    assert last["y"]["ik"] > first["y"]["ik"] + 0.1
