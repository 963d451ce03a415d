"""The allocation-free product (spamm_multiply_noalloc, static device
scratch) against spamm_multiply, through the C ABI: two calls in a row, the
second on a smaller input, each bitwise equal to the allocating entry point
(same kernels, same arithmetic); sizes beyond the static array are rejected."""
import numpy as np
import pytest
import torch

from paper_1508_05856_amd import inputs, spamm

pytestmark = pytest.mark.gpu

# (matrix, leaf, precision, tau): the second is smaller than the first and
# ragged (n not a multiple of the leaf), so the second call runs on a scratch
# array holding the first call's larger buffers
CASES = [
    (lambda: inputs.kms(1000, 0.7), 32, "f64", 1e-6),
    (lambda: inputs.gauss_gramian(7, 1.0, 0.1, 0), 16, "f32", 1e-4),
]


@pytest.fixture(scope="module")
def ctx():
    c = spamm.Context(0)
    yield c
    c.close()


def test_noalloc_equals_multiply_on_two_calls(ctx):
    for make, leaf, prec, tau in CASES:
        s = torch.from_numpy(make()).cuda()
        a = s
        b = (s @ s).contiguous() / s.shape[0]
        print(f"noalloc n={s.shape[0]} leaf={leaf} prec={prec} tau={tau}", flush=True)
        ref, stats, _ = ctx.spamm_multiply(a, b, tau, leaf, prec)
        C = torch.full_like(a, float("nan"))
        ctx.spamm_multiply_noalloc(a, b, tau, leaf, prec, C=C)
        torch.cuda.synchronize()
        assert 0 < stats["retained"] <= stats["possible"]
        assert torch.equal(C, ref), float((C - ref).abs().max())


def test_noalloc_repeat_after_larger_call_and_rejects_oversize(ctx):
    small = torch.from_numpy(inputs.kms(200, 0.6)).cuda()
    ref, _, _ = ctx.spamm_multiply(small, small, 1e-8, 64, "bf16x3")
    for _ in range(2):
        C = torch.full_like(small, float("nan"))
        ctx.spamm_multiply_noalloc(small, small, 1e-8, 64, "bf16x3", C=C)
        torch.cuda.synchronize()
        assert torch.equal(C, ref)
    big = torch.zeros((2048, 2048), dtype=torch.float64, device="cuda")
    with pytest.raises(spamm.SpammError) as e:
        ctx.spamm_multiply_noalloc(big, big, 1e-8, 64, "f64")
    assert e.value.status == spamm.EINVAL and "scratch" in str(e.value)
