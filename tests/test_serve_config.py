"""Server configuration checks that need no GPU (they fail before any device call)."""
import pytest

pytest.importorskip("torch")


@pytest.mark.parametrize("lanes", [(), (4096,), (None, 4096), (4096, 2048, None), (4096, 4096, None)])
def test_lane_bounds_are_validated(lanes):
    from paper_1508_05856_amd import serve
    with pytest.raises(ValueError):
        serve.Server(0, lanes=lanes)
