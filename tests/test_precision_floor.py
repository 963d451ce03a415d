"""What FP32 storage alone costs the inverse square root (CPU, no GPU).

The reduced-precision leaf modes store every operand in FP32.  Rounding the
scaled input s' alone to FP32 perturbs s' by half an FP32 unit per entry,
and s'^{-1/2} amplifies that by up to the condition number: on the Gaussian
Gramians of the tests (kappa ~ 1e4) the eigendecomposition roots of fl32(s')
and s' differ by more than 5e-6 (relative Frobenius) in s'^{-1/2}, while
s'^{1/2} moves far less.  So no leaf arithmetic on FP32-stored operands can
bring Z within 5e-6 of the FP64 oracle there; the GPU tests hold Y to 5e-6
and Z to a multiple of this floor."""
import numpy as np

from paper_1508_05856_amd import inputs


def _roots(a):
    w, v = np.linalg.eigh(a)
    return (v * np.sqrt(w)) @ v.T, (v / np.sqrt(w)) @ v.T


def _floors(s, mu_rel=0.0):
    c0 = np.abs(s).sum(0).max()
    sm = s + mu_rel * c0 * np.eye(s.shape[0])
    sp = sm / np.abs(sm).sum(0).max()
    y, z = _roots(sp)
    y32, z32 = _roots(sp.astype(np.float32).astype(np.float64))
    rel = lambda x, r: np.linalg.norm(x - r) / np.linalg.norm(r)
    return rel(y32, y), rel(z32, z)


def test_fp32_storage_floor_of_the_inverse_root():
    fy, fz = _floors(inputs.gauss_gramian(8, 1.0))
    assert fz > 5e-6 and fy < 5e-7
    fy, fz = _floors(inputs.gauss_gramian(12, 0.6, 0.1, 0), 1e-4)
    assert fz > 5e-6 and fy < 5e-7
    # a well-conditioned Kac-Murdock-Szego matrix (kappa 32) loses only ~u32
    fy, fz = _floors(inputs.kms(512, 0.7))
    assert fz < 2e-7 and fy < 2e-7
