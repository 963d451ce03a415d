"""Server configuration checks that need no GPU (they fail before any device call)."""
import pytest

pytest.importorskip("torch")


@pytest.mark.parametrize("lanes", [(), (4096,), (None, 4096), (4096, 2048, None), (4096, 4096, None)])
def test_lane_bounds_are_validated(lanes):
    from paper_1508_05856_amd import serve
    with pytest.raises(ValueError):
        serve.Server(0, lanes=lanes)


@pytest.mark.parametrize("iters", [0, (4, 4), (4, 0, 4), [2, 4, 8, 1]])
def test_iterations_per_step_are_validated(iters):
    """One value, or one value >= 1 per lane (three lanes here)."""
    from paper_1508_05856_amd import serve
    with pytest.raises(ValueError):
        serve.Server(0, hbm_budget=1 << 30, iters_per_step=iters, lanes=(2048, 8192, None))
