"""What the gfx950 bf16 matrix core does with the low bits of a block product
(tests/gpu_probes/mfma_round.hip, built by build()).

Measured: the 32 products of one 16x16x32 bf16 MFMA are summed keeping about
FP32's 24 bits below the largest product and dropping the rest (a
cancellation 1 - 1 + 2^-30 gives 0; 1 + 0.75 ulp gives 1, also for negative
sums: toward zero), and that sum is then added to the accumulator input with
round to nearest even.  The dropped bits are a biased error of up to an FP32
unit of the largest product per instruction, which is why the split-bf16
leaves land above what round-to-nearest arithmetic predicts on the
ill-conditioned analogue."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

PROBE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "gpu_probes", "mfma_round")


def test_bf16_mfma_truncates_below_its_largest_product():
    if not os.path.exists(PROBE):
        pytest.fail(f"{PROBE} is missing: run __graft_entry__.build()")
    out = subprocess.run([PROBE], capture_output=True, text=True, timeout=60).stdout
    print(out)
    lines = {ln.split(" got ")[0].strip(): ln for ln in out.splitlines() if " got " in ln}
    assert len(lines) == 8, out
    # the accumulator input is added with round to nearest even
    assert lines["C = 1 plus 2^-24 + 2^-25"].endswith("= RNE")
    # bits more than ~24 below the largest product are dropped, toward zero
    assert "got 1 (0x3f800000)" in lines["1 + 2^-24 + 2^-25 (0.75 ulp above 1)"]
    assert "got -1 (0xbf800000)" in lines["-(1 + 2^-24 + 2^-25)"]
    assert "got 0 (0x00000000)" in lines["1 - 1 + 2^-30 (cancellation)"]
