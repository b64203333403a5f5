"""Seeded synthetic inputs for dynamic-OT solves on the staggered grid.

This module is shared by the oracle, the tests and the benchmark. It holds no
arithmetic of the solution method: it only produces node masses rho0, rho1
(arrays over the spatial nodes x_i = i*h, summing to one) and optional obstacle
masks, with the shapes and value distributions of the workloads the paper
measures (Gaussian bumps with and without a density floor, mixtures with
near-zero-mass regions, rectangular obstacles).

Sampling convention: a density is evaluated at the spatial nodes of the
centred grid, optionally raised by a floor, zeroed on obstacle nodes and
divided by its sum, so each array is a vector of node masses of total one
(the paper normalises the discrete densities to unit sum in its flat-domain
examples, Sec. 5.4.1).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "Instance",
    "gaussian_pdf_nodes",
    "mixture_nodes",
    "rect_mask",
    "normalise",
    "config1_instance",
    "config2_instance",
    "config3_instance",
    "config4_instances",
    "serving_3d_instance",
    "image_like_instance",
    "serving_request",
    "tiny_instance",
]


@dataclasses.dataclass
class Instance:
    """One synthetic problem: spatial dimension D, segment counts n = (n0, n1..nD),
    node masses rho0/rho1 of shape (n1+1, ..., nD+1), optional uint8 mask of the
    same shape (1 = obstacle)."""

    D: int
    n: Tuple[int, ...]
    rho0: np.ndarray
    rho1: np.ndarray
    mask: Optional[np.ndarray] = None
    seed: int = 0
    label: str = ""

    @property
    def spatial_shape(self) -> Tuple[int, ...]:
        return tuple(k + 1 for k in self.n[1:])


def _node_coords(n_spatial: Sequence[int]) -> List[np.ndarray]:
    """Open-mesh coordinates x_d = i/n_d for i = 0..n_d on each spatial axis."""
    D = len(n_spatial)
    axes = []
    for d, nd in enumerate(n_spatial):
        shape = [1] * D
        shape[d] = nd + 1
        axes.append((np.arange(nd + 1, dtype=np.float64) / nd).reshape(shape))
    return axes


def gaussian_pdf_nodes(n_spatial: Sequence[int], mean: Sequence[float], sd: float) -> np.ndarray:
    """Isotropic normal pdf N(mean, sd^2 I) evaluated at the spatial nodes."""
    axes = _node_coords(n_spatial)
    D = len(axes)
    r2 = sum((axes[d] - mean[d]) ** 2 for d in range(D))
    return np.exp(-0.5 * r2 / sd ** 2) / ((2.0 * math.pi) ** (D / 2) * sd ** D)


def mixture_nodes(n_spatial: Sequence[int], rng: np.random.Generator, n_comp: int,
                  mean_lo: float = 0.2, mean_hi: float = 0.8,
                  sd_lo: float = 0.04, sd_hi: float = 0.12) -> np.ndarray:
    """Mixture of n_comp isotropic Gaussians: means U[mean_lo, mean_hi]^D,
    standard deviations U[sd_lo, sd_hi], weights Dirichlet(1, ..., 1)."""
    D = len(n_spatial)
    w = rng.dirichlet(np.ones(n_comp))
    out = np.zeros(tuple(k + 1 for k in n_spatial))
    for c in range(n_comp):
        mu = rng.uniform(mean_lo, mean_hi, size=D)
        sd = rng.uniform(sd_lo, sd_hi)
        out += w[c] * gaussian_pdf_nodes(n_spatial, mu, sd)
    return out


def rect_mask(n_spatial: Sequence[int], rng: np.random.Generator,
              n_rect_range: Tuple[int, int] = (1, 3),
              area_range: Tuple[float, float] = (0.10, 0.25),
              max_tries: int = 1000) -> np.ndarray:
    """1-3 random axis-aligned rectangles whose union covers a fraction of the
    nodes inside area_range; rejection-sampled so that the free nodes stay
    connected (4-/6-neighbour connectivity) and no rectangle touches the whole
    width of an axis."""
    shape = tuple(k + 1 for k in n_spatial)
    D = len(shape)
    for _ in range(max_tries):
        m = np.zeros(shape, dtype=np.uint8)
        k = int(rng.integers(n_rect_range[0], n_rect_range[1] + 1))
        for _r in range(k):
            sl = []
            for d in range(D):
                L = shape[d]
                w = int(rng.integers(max(2, L // 8), max(3, L // 2)))
                a = int(rng.integers(1, max(2, L - w - 1)))
                sl.append(slice(a, min(L - 1, a + w)))
            m[tuple(sl)] = 1
        frac = m.mean()
        if not (area_range[0] <= frac <= area_range[1]):
            continue
        if _free_connected(m):
            return m
    raise RuntimeError("could not sample a connected obstacle mask")


def _free_connected(mask: np.ndarray) -> bool:
    free = mask == 0
    if not free.any():
        return False
    seen = np.zeros_like(free)
    start = tuple(np.argwhere(free)[0])
    stack = [start]
    seen[start] = True
    D = mask.ndim
    while stack:
        p = stack.pop()
        for d in range(D):
            for s in (-1, 1):
                qq = list(p)
                qq[d] += s
                if 0 <= qq[d] < mask.shape[d]:
                    t = tuple(qq)
                    if free[t] and not seen[t]:
                        seen[t] = True
                        stack.append(t)
    return bool(seen.sum() == free.sum())


def normalise(rho: np.ndarray, floor: float = 0.0, mask: Optional[np.ndarray] = None) -> np.ndarray:
    """Add a floor, zero obstacle nodes, divide by the sum (unit total mass)."""
    r = np.asarray(rho, dtype=np.float64) + floor
    if mask is not None:
        r = np.where(mask != 0, 0.0, r)
    s = r.sum()
    if not s > 0:
        raise ValueError("density has no mass")
    return r / s


def config1_instance(n1: int = 32, n0: int = 16, floor: float = 1e-3, seed: int = 1000) -> Instance:
    """1D: rho0 = N(0.3, 0.05^2), rho1 = N(0.7, 0.08^2) at the nodes, +floor, unit mass."""
    r0 = normalise(gaussian_pdf_nodes([n1], [0.3], 0.05), floor)
    r1 = normalise(gaussian_pdf_nodes([n1], [0.7], 0.08), floor)
    return Instance(1, (n0, n1), r0, r1, None, seed, f"1d-{n0}x{n1}")


def _mixture_pair(D, n, seed, n_comp, mask=None) -> Instance:
    rng = np.random.default_rng(seed)
    sp = list(n[1:])
    r0 = normalise(mixture_nodes(sp, rng, n_comp), 0.0, mask)
    r1 = normalise(mixture_nodes(sp, rng, n_comp), 0.0, mask)
    return Instance(D, tuple(n), r0, r1, mask, seed, f"{D}d-" + "x".join(map(str, n)))


def config2_instance(seed: int = 2000, n0: int = 32, n1: int = 64) -> Instance:
    """2D, 64x64 segments, 32 time steps, 3-component mixtures, no floor."""
    return _mixture_pair(2, (n0, n1, n1), seed, 3)


def config3_instance(seed: int = 3000, n0: int = 64, n1: int = 256) -> Instance:
    """2D, 256x256 segments, 64 time steps, 5-component mixtures, no floor."""
    return _mixture_pair(2, (n0, n1, n1), seed, 5)


def serving_3d_instance(seed: int = 5003) -> Instance:
    """The 3D request shape of the serving stream: 64^3 segments, 32 time
    steps, 3-component mixtures in [0,1]^3, no floor."""
    return _mixture_pair(3, (32, 64, 64, 64), seed, 3)


def image_like_instance(n: Sequence[int] = (32, 1024, 1024), seed: int = 6000, n_comp: int = 16) -> Instance:
    """Large 2D instance standing in for the paper's 1024^2 image pair (the
    images are not available): mixtures of n_comp narrow isotropic Gaussians
    (standard deviations U[0.015, 0.06], means U[0.1, 0.9]^2, Dirichlet(1)
    weights), no floor."""
    rng = np.random.default_rng(seed)
    sp = list(n[1:])
    r0 = normalise(mixture_nodes(sp, rng, n_comp, 0.1, 0.9, 0.015, 0.06))
    r1 = normalise(mixture_nodes(sp, rng, n_comp, 0.1, 0.9, 0.015, 0.06))
    return Instance(len(sp), tuple(n), r0, r1, None, seed, "image-like-" + "x".join(map(str, n)))


def config4_instances(count: int = 64, seed: int = 4000,
                      sides: Sequence[int] = (32, 48, 64, 96, 128),
                      times: Sequence[int] = (16, 32, 64)) -> List[Instance]:
    """Heterogeneous batch: grid sides drawn from `sides` per axis, n0 from
    `times`, 3-component mixtures; every second instance carries a rectangle
    obstacle mask (densities are zero on the mask)."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed + i)
        n1 = int(rng.choice(sides))
        n2 = int(rng.choice(sides))
        n0 = int(rng.choice(times))
        mask = rect_mask([n1, n2], rng) if i % 2 == 1 else None
        inst = _mixture_pair(2, (n0, n1, n2), seed + 7919 * (i + 1), 3, mask)
        inst.seed = seed + i
        inst.label = f"b{i}-{n0}x{n1}x{n2}" + ("-mask" if mask is not None else "")
        out.append(inst)
    return out


def serving_request(index: int, seed: int = 5000, frac_3d: float = 0.1) -> Instance:
    """One request of the serving stream: 2D with log-uniform sides in [32, 256]
    (mask on every second 2D request), or with probability frac_3d a 3D solve
    of 64^3 cells with 32 time steps and 3-component mixtures."""
    rng = np.random.default_rng(seed + index)
    if rng.uniform() < frac_3d:
        return _mixture_pair(3, (32, 64, 64, 64), seed + 104729 * (index + 1), 3)
    n1 = int(round(math.exp(rng.uniform(math.log(32), math.log(256)))))
    n2 = int(round(math.exp(rng.uniform(math.log(32), math.log(256)))))
    n0 = int(rng.choice((16, 32, 64)))
    mask = rect_mask([n1, n2], rng) if index % 2 == 1 else None
    return _mixture_pair(2, (n0, n1, n2), seed + 104729 * (index + 1), 3, mask)


def tiny_instance(D: int, n: Sequence[int], seed: int = 7, floor: float = 0.05,
                  n_comp: int = 2, masked: bool = False) -> Instance:
    """Small random instance with a floor (strictly positive densities), used
    for brute-force and parity cases that must run in seconds."""
    rng = np.random.default_rng(seed)
    sp = list(n[1:])
    mask = None
    if masked:
        shape = tuple(k + 1 for k in sp)
        mask = np.zeros(shape, dtype=np.uint8)
        sl = tuple(slice(max(1, s // 3), max(2, (2 * s) // 3)) for s in shape)
        mask[sl] = 1
    r0 = normalise(mixture_nodes(sp, rng, n_comp, sd_lo=0.1, sd_hi=0.25), floor, mask)
    r1 = normalise(mixture_nodes(sp, rng, n_comp, sd_lo=0.1, sd_hi=0.25), floor, mask)
    return Instance(D, tuple(n), r0, r1, mask, seed, f"tiny{D}d-" + "x".join(map(str, n)))
