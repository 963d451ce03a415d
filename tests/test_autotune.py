"""The autotuner's choice rule (CPU, no GPU): the fastest leaf among the
candidates that end with status >= 0 and an exact residual within the
accuracy factor of the best one."""
import math

from paper_1508_05856_amd import autotune


def test_fastest_among_accurate_candidates():
    c = {32: dict(ms=5.0, status=2, resid=1e-3), 64: dict(ms=3.0, status=2, resid=1e-1),
         16: dict(ms=4.0, status=0, resid=1.5e-3)}
    # 64 is fastest but 100x less accurate; 16 is within the factor of 32 and faster
    assert autotune.choose(c) == 16


def test_diverged_candidates_never_chosen():
    c = {32: dict(ms=9.0, status=2, resid=1e-2), 64: dict(ms=1.0, status=-3, resid=math.inf)}
    assert autotune.choose(c) == 32
    assert autotune.choose({64: dict(ms=1.0, status=-3, resid=math.inf)}) is None


def test_candidate_leaves_per_precision():
    assert autotune.candidate_leaves("f32") == (16, 32, 64)
    assert autotune.candidate_leaves("bf16x6") == (32, 64)
