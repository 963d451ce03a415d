"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds only input construction: it performs none of the method's
arithmetic (no scaling, no norms, no products, no iteration).  Every matrix is
built in FP64 on the host with NumPy, so the oracle and the GPU path see the
same bits.

Workloads (symmetric positive-definite stand-ins for the paper's overlap
matrices, Sec. "Data"; none of the paper's data sets is available):

* Kac-Murdock-Szego matrices, s_ij = rho^|i-j|: one-dimensional exponential
  decay, a quasi-1-D analogue of the nanotube overlaps.
* Gramians of equal-exponent s-type Gaussians on a jittered cubic lattice,
  s_ij = exp(-r_ij^2 / 2), with the sites ordered along a Morton (Z-order)
  space-filling curve.  The ordering gives the block-by-magnitude structure the
  paper attributes to space-filling-curve orderings of local bases (Sec. 1,
  Sec. "Spatial and metric locality").
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "kms",
    "morton_sites",
    "gauss_positions",
    "gramian_from_positions",
    "gauss_gramian",
    "config_c1",
    "config_c2",
    "config_c3",
    "batch_specs",
    "serving_requests",
]


def kms(n: int, rho: float) -> np.ndarray:
    """Kac-Murdock-Szego matrix s_ij = rho^|i-j| (FP64, exactly symmetric)."""
    idx = np.arange(n)
    return np.power(float(rho), np.abs(idx[:, None] - idx[None, :]).astype(np.float64))


def _morton_key(ix: np.ndarray, iy: np.ndarray, iz: np.ndarray, bits: int) -> np.ndarray:
    """Bit-interleaved Morton code; x takes the most significant bit of each triple."""
    key = np.zeros(ix.shape, dtype=np.int64)
    for bit in range(bits - 1, -1, -1):
        key = (key << 3) | (((ix >> bit) & 1) << 2) | (((iy >> bit) & 1) << 1) | ((iz >> bit) & 1)
    return key


def morton_sites(m: int) -> np.ndarray:
    """Integer lattice sites of [0, m)^3 sorted along the Morton curve, shape (m^3, 3)."""
    g = np.arange(m, dtype=np.int64)
    ix, iy, iz = np.meshgrid(g, g, g, indexing="ij")
    ix, iy, iz = ix.ravel(), iy.ravel(), iz.ravel()
    bits = max(1, int(math.ceil(math.log2(max(m, 2)))))
    order = np.argsort(_morton_key(ix, iy, iz, bits), kind="stable")
    return np.stack([ix[order], iy[order], iz[order]], axis=1)


def gauss_positions(m: int, h: float, jitter: float = 0.1, seed: int = 0, n: int | None = None) -> np.ndarray:
    """Jittered, Morton-ordered lattice positions.

    positions = h * site + U(-jitter, jitter), the jitter drawn with
    ``numpy.random.default_rng(seed)`` in Morton order for all m^3 sites.  For
    n < m^3 the first n sites along the curve are kept.
    """
    sites = morton_sites(m).astype(np.float64)
    rng = np.random.default_rng(seed)
    jit = rng.uniform(-jitter, jitter, size=(m ** 3, 3))
    pos = h * sites + jit
    if n is not None:
        if n > m ** 3:
            raise ValueError("n exceeds the lattice size")
        pos = pos[:n]
    return np.ascontiguousarray(pos)


def gramian_from_positions(pos: np.ndarray, out: np.ndarray | None = None, rows_per_chunk: int = 512) -> np.ndarray:
    """s_ij = exp(-0.5 * |p_i - p_j|^2) in FP64, built in row chunks.

    The squared distance is summed x, y, z in that order from exact negated
    differences, so the result is exactly symmetric.
    """
    n = pos.shape[0]
    if out is None:
        out = np.empty((n, n), dtype=np.float64)
    px, py, pz = pos[:, 0], pos[:, 1], pos[:, 2]
    for r0 in range(0, n, rows_per_chunk):
        r1 = min(n, r0 + rows_per_chunk)
        dx = px[r0:r1, None] - px[None, :]
        dy = py[r0:r1, None] - py[None, :]
        dz = pz[r0:r1, None] - pz[None, :]
        d2 = dx * dx
        d2 += dy * dy
        d2 += dz * dz
        d2 *= -0.5
        np.exp(d2, out=out[r0:r1])
    return out


def gauss_gramian(m: int, h: float, jitter: float = 0.1, seed: int = 0, n: int | None = None) -> np.ndarray:
    """Gaussian overlap Gramian on m^3 (or the first n Morton) jittered lattice sites."""
    if n is not None and m is None:
        m = int(math.ceil(round(n ** (1.0 / 3.0), 9)))
        while m ** 3 < n:
            m += 1
    return gramian_from_positions(gauss_positions(m, h, jitter, seed, n))


def smallest_cube(n: int) -> int:
    m = max(1, int(round(n ** (1.0 / 3.0))))
    while m ** 3 < n:
        m += 1
    while m > 1 and (m - 1) ** 3 >= n:
        m -= 1
    return m


# ---------------------------------------------------------------------------
# The five workloads.  Sizes, thresholds and tolerances are the workload's own;
# see the design notes for how unstated parameters were fixed.
# ---------------------------------------------------------------------------

def config_c1() -> dict:
    """Plain FP64: KMS rho=0.7, n=512, leaf 32, tau=1e-8, tol 1e-10, maxit 40."""
    return dict(name="kms_n512_rho0.7_b32", s=kms(512, 0.7), leaf=32, tau=1e-8, tol=1e-10, maxit=40)


def config_c2(tau: float = 1e-6) -> dict:
    """Gaussian Gramian 16^3 = 4096 sites, h=1.0, jitter 0.1, seed 0, leaf 64."""
    return dict(name=f"gauss_m16_h1.0_b64_tau{tau:g}", s=gauss_gramian(16, 1.0, 0.1, 0), leaf=64,
                tau=tau, tol=1e-10, maxit=40)


def config_c3(m: int = 32) -> dict:
    """Ill-conditioned Gramian: m^3 sites (m=32 gives n=32768), h=0.6, mu = 1e-4 * c0, tau=1e-6."""
    return dict(name=f"gauss_m{m}_h0.6_mu1e-4_b64", s=gauss_gramian(m, 0.6, 0.1, 0), leaf=64,
                tau=1e-6, tol=1e-8, maxit=40, mu_rel=1e-4)


def config_c3_spec(m: int = 32) -> dict:
    """The ill-conditioned case without materialising s (n = m^3 = 32768 is
    8 GiB in FP64): h = 0.6, mu = 1e-4 c0, leaf 64.  At this n the iteration
    diverges for tau = 1e-6 and 1e-7 (plain and damped map, FP64 and BF16x3
    alike); tau = 1e-9 with the damped map and tau_s = 0.01 tau reaches its
    floor, so that is the solve measured."""
    return dict(name=f"gauss_m{m}_h0.6_mu1e-4_b64_tau1e-9_damped", m=m, n=m ** 3, h=0.6, leaf=64, tau=1e-9,
                tau_s_rel=0.01, damped=True, tol=1e-8, maxit=40, mu_rel=1e-4)


def batch_specs(count: int = 64, seed: int = 0, nmin_blocks: int = 4, nmax_blocks: int = 64) -> list[dict]:
    """Batched workload: n = 64*U{4..64}; half KMS (rho ~ U[0.5,0.9]), half Gaussian
    (h ~ U[0.8,1.2], first n Morton sites of the smallest cube); tau in {1e-4, 1e-6}."""
    rng = np.random.default_rng(seed)
    kinds = np.array(["kms"] * (count // 2) + ["gauss"] * (count - count // 2))
    rng.shuffle(kinds)
    specs = []
    for i, kind in enumerate(kinds):
        n = 64 * int(rng.integers(nmin_blocks, nmax_blocks + 1))
        tau = float(rng.choice([1e-4, 1e-6]))
        if kind == "kms":
            rho = float(rng.uniform(0.5, 0.9))
            specs.append(dict(kind="kms", n=n, rho=rho, tau=tau, seed=seed * 1000 + i))
        else:
            h = float(rng.uniform(0.8, 1.2))
            specs.append(dict(kind="gauss", n=n, h=h, tau=tau, seed=seed * 1000 + i))
    return specs


def build_spec(spec: dict) -> np.ndarray:
    """Materialise one batched/serving instance."""
    if spec["kind"] == "kms":
        return kms(spec["n"], spec["rho"])
    m = smallest_cube(spec["n"])
    return gramian_from_positions(gauss_positions(m, spec["h"], 0.1, spec["seed"], spec["n"]))


def serving_requests(rate: float = 200.0, duration: float = 60.0, seed: int = 0,
                     nmin: int = 512, nmax: int = 16384) -> list[dict]:
    """Poisson arrivals; n = round(exp(U[ln nmin, ln nmax])); KMS/Gaussian 50/50;
    tau in {1e-4, 1e-6, 1e-8}."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    i = 0
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration:
            break
        n = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        tau = float(rng.choice([1e-4, 1e-6, 1e-8]))
        if rng.uniform() < 0.5:
            reqs.append(dict(t=t, kind="kms", n=n, rho=float(rng.uniform(0.5, 0.9)), tau=tau, seed=i))
        else:
            reqs.append(dict(t=t, kind="gauss", n=n, h=float(rng.uniform(0.8, 1.2)), tau=tau, seed=i))
        i += 1
    return reqs


# ---------------------------------------------------------------------------
# Device-side construction for serving-scale inputs (n up to 16384, where
# building on the host would dominate).  Same seeded positions; the Gramian is
# formed on the GPU in row chunks, exactly symmetric.
# ---------------------------------------------------------------------------

def kms_device(n: int, rho: float, device):
    import torch
    idx = torch.arange(n, device=device, dtype=torch.float64)
    return torch.pow(torch.tensor(float(rho), dtype=torch.float64, device=device),
                     (idx[:, None] - idx[None, :]).abs())


def gramian_device(pos: np.ndarray, device, rows_per_chunk: int = 2048):
    import torch
    p = torch.from_numpy(np.ascontiguousarray(pos)).to(device)
    n = p.shape[0]
    out = torch.empty((n, n), dtype=torch.float64, device=device)
    for r0 in range(0, n, rows_per_chunk):
        r1 = min(n, r0 + rows_per_chunk)
        dx = p[r0:r1, 0:1] - p[None, :, 0]
        dy = p[r0:r1, 1:2] - p[None, :, 1]
        dz = p[r0:r1, 2:3] - p[None, :, 2]
        d2 = dx * dx
        d2 += dy * dy
        d2 += dz * dz
        d2 *= -0.5
        torch.exp(d2, out=out[r0:r1])
    return out


def build_spec_device(spec: dict, device):
    """Materialise one batched/serving instance directly on the device."""
    if spec["kind"] == "kms":
        return kms_device(spec["n"], spec["rho"], device)
    m = smallest_cube(spec["n"])
    return gramian_device(gauss_positions(m, spec["h"], 0.1, spec["seed"], spec["n"]), device)
