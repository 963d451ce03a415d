"""GPU tests of the continuous-batching server.

Requests submitted while others are on the device join them at a step
boundary and share their launches; each result must be bitwise the one the
same request gets when solved alone (same kernels, one workgroup per output
tile, fixed-order reductions), and admission must respect the memory budget.
"""
import threading
import time

import numpy as np
import pytest

from paper_1508_05856_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# (kind, n, param, seed, leaf, tau)
REQS = [
    ("kms", 320, 0.7, 0, 32, 1e-8),
    ("gauss", 500, 1.0, 1, 64, 1e-6),
    ("kms", 777, 0.85, 2, 64, 1e-4),
    ("gauss", 216, 1.2, 3, 32, 1e-8),
    ("gauss", 900, 0.9, 4, 64, 1e-8),
    ("kms", 130, 0.5, 5, 32, 1e-6),
    ("gauss", 1331, 1.1, 6, 64, 1e-6),
    ("kms", 1024, 0.9, 7, 64, 1e-8),
]


def mat(kind, n, param, seed):
    return torch.from_numpy(inputs.build_spec(dict(kind=kind, n=n, seed=seed, rho=param, h=param))).cuda()


@pytest.fixture(scope="module")
def solo_results():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_1508_05856_amd import spamm
    ctx = spamm.Context(0)
    out = []
    for kind, n, p, sd, leaf, tau in REQS:
        Y, Z, info = ctx.ns_sqrt(mat(kind, n, p, sd), tau, 1e-8, 40, leaf=leaf, stagnation_stop=True,
                                 raise_on_error=False)
        out.append((Y.cpu().numpy(), Z.cpu().numpy(), info))
    ctx.close()
    return out


@pytest.mark.parametrize("lanes", [(None,), (700, None)])
def test_requests_joining_a_running_mix_match_solo(solo_results, lanes):
    """One lane, and two lanes (n <= 700 and the rest) on their own streams."""
    from paper_1508_05856_amd import serve
    srv = serve.Server(0, iters_per_step=1, autostart=False, lanes=lanes)
    futs = {}
    for i in range(3):  # queued before the engine starts: admitted together
        kind, n, p, sd, leaf, tau = REQS[i]
        futs[i] = srv.submit(mat(kind, n, p, sd), tau, 1e-8, maxit=40, leaf=leaf, stagnation_stop=True)
    srv.start()

    def client():
        while srv.stats["steps"] < 2:   # the rest arrive while the first ones are on the device
            time.sleep(0.001)
        for i in range(3, len(REQS)):
            kind, n, p, sd, leaf, tau = REQS[i]
            futs[i] = srv.submit(mat(kind, n, p, sd), tau, 1e-8, maxit=40, leaf=leaf, stagnation_stop=True)
            time.sleep(0.002)

    th = threading.Thread(target=client)
    th.start()
    th.join()
    results = {i: f.result(timeout=120) for i, f in futs.items()}
    stats = dict(srv.stats)
    srv.close()
    assert stats["completed"] == len(REQS) and stats["max_active"] >= 3
    for i, (Ys, Zs, infos) in enumerate(solo_results):
        r = results[i]
        assert r.info["status"] == infos["status"] and r.info["iterations"] == infos["iterations"], i
        np.testing.assert_array_equal(r.Y.cpu().numpy(), Ys)
        np.testing.assert_array_equal(r.Z.cpu().numpy(), Zs)
        assert r.latency_s >= r.queued_s >= 0.0


def test_admission_by_footprint(solo_results):
    from paper_1508_05856_amd import serve
    probe = serve.Server(0, autostart=False)
    fp = [probe.reservation(REQS[i][1], REQS[i][4], "f64", 40) for i in (4, 6)]
    probe.close()
    # room for either request alone but not both: they must run one after the other
    srv = serve.Server(0, hbm_budget=max(fp) + min(fp) // 2, iters_per_step=2, autostart=False)
    futs = []
    for i in (4, 6):
        kind, n, p, sd, leaf, tau = REQS[i]
        futs.append(srv.submit(mat(kind, n, p, sd), tau, 1e-8, maxit=40, leaf=leaf, stagnation_stop=True))
    too_big = srv.submit(mat("kms", 4096, 0.7, 0), 1e-6, 1e-8, leaf=64)
    srv.start()
    res = [f.result(timeout=120) for f in futs]
    stats = dict(srv.stats)
    srv.close()
    with pytest.raises(ValueError):
        too_big.result(timeout=1)
    assert stats["max_active"] == 1 and stats["completed"] == 2
    assert stats["peak_bytes"] <= max(fp) + min(fp) // 2
    for r, i in zip(res, (4, 6)):
        np.testing.assert_array_equal(r.Y.cpu().numpy(), solo_results[i][0])
        np.testing.assert_array_equal(r.Z.cpu().numpy(), solo_results[i][1])


def test_submit_after_close_fails():
    from paper_1508_05856_amd import serve
    srv = serve.Server(0, iters_per_step=2)
    f = srv.submit(mat("kms", 128, 0.7, 0), 1e-6, 1e-8, leaf=32)
    assert f.result(timeout=60).info["status"] >= 0
    srv.close()
    late = srv.submit(mat("kms", 128, 0.7, 0), 1e-6, 1e-8, leaf=32)
    with pytest.raises(RuntimeError):
        late.result(timeout=1)


def test_invalid_request_fails_alone(solo_results):
    """An input the library rejects (not symmetric) fails its own future only."""
    from paper_1508_05856_amd import serve, spamm
    srv = serve.Server(0, iters_per_step=2, autostart=False, lanes=(700, None))
    good = {}
    for i in (0, 2):
        kind, n, p, sd, leaf, tau = REQS[i]
        good[i] = srv.submit(mat(kind, n, p, sd), tau, 1e-8, maxit=40, leaf=leaf, stagnation_stop=True)
    bad = mat("kms", 320, 0.7, 0)
    bad[0, 5] += 1.0
    bad_f = srv.submit(bad, 1e-8, 1e-8, maxit=40, leaf=32, stagnation_stop=True)
    srv.start()
    res = {i: f.result(timeout=120) for i, f in good.items()}
    with pytest.raises(spamm.SpammError):
        bad_f.result(timeout=120)
    stats = dict(srv.stats)
    srv.close()
    assert stats["completed"] == 2
    for i, r in res.items():
        np.testing.assert_array_equal(r.Y.cpu().numpy(), solo_results[i][0])
        np.testing.assert_array_equal(r.Z.cpu().numpy(), solo_results[i][1])


def test_served_results_match_the_fp64_oracle():
    """Served results against the oracle itself, not only against solo runs:
    small requests of each kind sharing the server, FP64 leaves, Y and Z to
    1e-12 (relative Frobenius) with the oracle's status and update count."""
    import oracle
    from paper_1508_05856_amd import serve
    picks = [REQS[0], REQS[3], REQS[5], REQS[1]]
    srv = serve.Server(0, iters_per_step=2)
    futs = [srv.submit(mat(kind, n, p, sd), tau, 1e-8, maxit=40, leaf=leaf, stagnation_stop=True)
            for kind, n, p, sd, leaf, tau in picks]
    results = [f.result(timeout=120) for f in futs]
    srv.close()
    for (kind, n, p, sd, leaf, tau), r in zip(picks, results):
        s = inputs.build_spec(dict(kind=kind, n=n, seed=sd, rho=p, h=p))
        o = oracle.ns_sqrt(s, leaf, tau, 1e-8, 40, stagnation_stop=True)
        assert r.info["status"] == o["status"] and r.info["iterations"] == o["iterations"], (kind, n)
        Y, Z = r.Y.cpu().numpy(), r.Z.cpu().numpy()
        assert np.linalg.norm(Y - o["Y"]) <= 1e-12 * np.linalg.norm(o["Y"]), (kind, n)
        assert np.linalg.norm(Z - o["Z"]) <= 1e-12 * np.linalg.norm(o["Z"]), (kind, n)


def test_verified_answers_carry_the_exact_residual(solo_results):
    """verify=True returns ||I - Y Z||_F of the answer, computed by the
    server: equal to the residual of the solo result computed in FP64 on the
    host, within the rounding bound of two dense products of length n
    (2 n 2^-53 ||Y||_F ||Z||_F), and None for a diverged solve."""
    from paper_1508_05856_amd import serve
    srv = serve.Server(0, iters_per_step=2)
    futs = [srv.submit(mat(kind, n, p, sd), tau, 1e-8, maxit=40, leaf=leaf, stagnation_stop=True, verify=True)
            for kind, n, p, sd, leaf, tau in REQS]
    results = [f.result(timeout=120) for f in futs]
    srv.close()
    for (kind, n, *_), r, (Y, Z, info) in zip(REQS, results, solo_results):
        if info["status"] < 0:
            assert r.info["resid_exact"] is None
            continue
        ref = np.linalg.norm(np.eye(n) - Y @ Z)
        bound = 2 * n * 2.0 ** -53 * np.linalg.norm(Y) * np.linalg.norm(Z)
        assert abs(r.info["resid_exact"] - ref) <= bound, (kind, n, r.info["resid_exact"], ref, bound)
