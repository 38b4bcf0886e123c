"""Seeded synthetic densities on the unit-box unigrid.

This module is the only code shared by the HIP path and the CPU oracle: it
draws input densities and holds none of the solver's arithmetic.

Every density is sampled point-wise at cell centres x = (i + 1/2)/n of the
unit box [0, 1]^3, C order (the last index is fastest), float64.  Nothing is
renormalised: mass of a profile that falls outside the box, or between
sample points, is simply absent.

Plummer sphere of mass M, scale radius a, centre c:
    rho(x) = 3 M / (4 pi a^3) * (1 + |x - c|^2 / a^2)^(-5/2)
Its potential (G = 1) is  phi(x) = -M / sqrt(|x - c|^2 + a^2).

The multi-Plummer recipe draws, from numpy.random.default_rng(seed), in this
order: K centres ~ U[0.2, 0.8]^3, K scale radii a = exp(U[ln 0.005, ln 0.05]),
K masses M = exp(U[ln 1e-2, ln 1]).  These fields stand in for the paper's
particle-built test densities (point charges, uniform spheres, NFW halos),
whose particle data are not available.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "PlummerSet", "multi_plummer_params", "plummer_density", "cell_centres",
    "single_plummer", "uniform_sphere_density", "batch_sizes",
    "fd_cells", "batch_field_params",
]


@dataclass(frozen=True)
class PlummerSet:
    centres: np.ndarray  # (K, 3)
    radii: np.ndarray    # (K,)
    masses: np.ndarray   # (K,)


def _plummer_draws(rng, k: int) -> PlummerSet:
    centres = rng.uniform(0.2, 0.8, size=(k, 3))
    radii = np.exp(rng.uniform(math.log(0.005), math.log(0.05), size=k))
    masses = np.exp(rng.uniform(math.log(1e-2), math.log(1.0), size=k))
    return PlummerSet(centres, radii, masses)


def multi_plummer_params(k: int, seed: int) -> PlummerSet:
    """K spheres from default_rng(seed): centres, then radii, then masses."""
    return _plummer_draws(np.random.default_rng(seed), k)


def batch_field_params(f: int) -> PlummerSet:
    """Field f of the uneven batch: K = integers(8, 65) drawn first from
    default_rng(4000 + f), then the K spheres from the same generator."""
    rng = np.random.default_rng(4000 + f)
    k = int(rng.integers(8, 65))
    return _plummer_draws(rng, k)


def single_plummer(mass: float = 1.0, radius: float = 0.1,
                   centre=(0.5, 0.5, 0.5)) -> PlummerSet:
    return PlummerSet(np.asarray([centre], dtype=np.float64),
                      np.asarray([radius], dtype=np.float64),
                      np.asarray([mass], dtype=np.float64))


def cell_centres(n: int) -> np.ndarray:
    """1-D array of the n cell-centre coordinates (i + 1/2)/n."""
    return (np.arange(n, dtype=np.float64) + 0.5) / n


def plummer_density(n: int, ps: PlummerSet, device: str | None = None):
    """Sampled density on an n^3 grid, float64, shape (n, n, n).

    With ``device`` None a numpy array is returned.  With a torch device
    string ("cpu", "cuda", "cuda:0") the same values are evaluated with torch
    in float64 on that device and a torch tensor is returned; this is only a
    faster way to draw large inputs and is not part of either solver.
    """
    if device is None:
        x = cell_centres(n)
        out = np.zeros((n, n, n), dtype=np.float64)
        for c, a, m in zip(ps.centres, ps.radii, ps.masses):
            dx2 = (x - c[0]) ** 2
            dy2 = (x - c[1]) ** 2
            dz2 = (x - c[2]) ** 2
            r2 = dx2[:, None, None] + dy2[None, :, None] + dz2[None, None, :]
            out += (3.0 * m / (4.0 * math.pi * a ** 3)) * (1.0 + r2 / (a * a)) ** -2.5
        return out
    import torch
    x = (torch.arange(n, dtype=torch.float64, device=device) + 0.5) / n
    out = torch.zeros((n, n, n), dtype=torch.float64, device=device)
    for c, a, m in zip(ps.centres, ps.radii, ps.masses):
        dx2 = (x - float(c[0])) ** 2
        dy2 = (x - float(c[1])) ** 2
        dz2 = (x - float(c[2])) ** 2
        r2 = dx2[:, None, None] + dy2[None, :, None] + dz2[None, None, :]
        out += (3.0 * float(m) / (4.0 * math.pi * float(a) ** 3)) * (1.0 + r2 / float(a) ** 2) ** -2.5
    return out


def uniform_sphere_density(n: int, centre, radius: float, value: float = 1.0) -> np.ndarray:
    """rho = value inside the sphere (cell centre within radius), 0 outside."""
    x = cell_centres(n)
    r2 = ((x - centre[0]) ** 2)[:, None, None] + ((x - centre[1]) ** 2)[None, :, None] \
        + ((x - centre[2]) ** 2)[None, None, :]
    return np.where(r2 <= radius * radius, value, 0.0).astype(np.float64)


def point_charge_cic(n: int, mass: float = 1.0) -> np.ndarray:
    """Density of a point mass at the centre of the unit box deposited by
    cloud-in-cell: the point sits on the common corner of the 8 central cells,
    so each receives mass / 8 (density mass / 8 / dx^3)."""
    rho = np.zeros((n, n, n))
    h = n // 2
    rho[h - 1:h + 1, h - 1:h + 1, h - 1:h + 1] = mass / 8.0 * n ** 3
    return rho


# The paper's two uniform-density spheres (Sec. 3: radii 0.1 and 0.2 at
# x = 0.7 and 1.2 on the axis y = z = 1 of a box of size 2), scaled to the
# unit box: radii 0.05 and 0.1, density 1.
TWO_SPHERES = (((0.35, 0.5, 0.5), 0.05), ((0.6, 0.5, 0.5), 0.1))


def two_spheres_particles(count: int, seed: int = 11):
    """Particles spread uniformly through the two spheres, count in
    proportion to their volumes, each sphere's particles sharing its mass
    4/3 pi R^3.  Returns pos (k, 3), mass (k,) as float64 arrays."""
    rng = np.random.default_rng(seed)
    vols = [r ** 3 for _, r in TWO_SPHERES]
    pos, mass = [], []
    for (c, r), v in zip(TWO_SPHERES, vols):
        k = int(round(count * v / sum(vols)))
        d = rng.standard_normal((k, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        d *= r * rng.uniform(0, 1, (k, 1)) ** (1.0 / 3.0)
        pos.append(np.asarray(c) + d)
        mass.append(np.full(k, 4.0 / 3.0 * math.pi * r ** 3 / k))
    return np.concatenate(pos), np.concatenate(mass)


def two_spheres_potential(points) -> np.ndarray:
    """Exact potential (G = 1) of the two uniform spheres at points (k, 3):
    -M/r outside a sphere, -M (3 R^2 - r^2) / (2 R^3) inside."""
    points = np.asarray(points, dtype=np.float64)
    phi = np.zeros(len(points))
    for c, r in TWO_SPHERES:
        m = 4.0 / 3.0 * math.pi * r ** 3
        d = np.linalg.norm(points - np.asarray(c), axis=1)
        phi += np.where(d >= r, -m / np.maximum(d, 1e-300), -m * (3 * r * r - d * d) / (2 * r ** 3))
    return phi


def cell_order(pos, n: int) -> np.ndarray:
    """Permutation that puts particles in cell order on an n^3 grid (by the
    cell below-left of each, C order, for particles inside the box), the
    order AMR codes keep them in."""
    lo = np.floor(np.asarray(pos) * n - 0.5).astype(np.int64) + 1
    key = (lo[:, 0] * (n + 2) + lo[:, 1]) * (n + 2) + lo[:, 2]
    return np.argsort(key, kind="stable")


def two_spheres_force(points) -> np.ndarray:
    """Exact acceleration (G = 1) of the two uniform spheres at points (k, 3):
    -M d / r^3 outside a sphere, -M d / R^3 inside (d = x - centre); (3, k)."""
    points = np.asarray(points, dtype=np.float64)
    g = np.zeros((3, len(points)))
    for c, r in TWO_SPHERES:
        m = 4.0 / 3.0 * math.pi * r ** 3
        d = points - np.asarray(c)
        dist = np.linalg.norm(d, axis=1)
        scale = np.where(dist >= r, m / np.maximum(dist, 1e-300) ** 3, m / r ** 3)
        g -= (d * scale[:, None]).T
    return g


def batch_sizes(count: int = 96, seed: int = 4) -> list[int]:
    """Grid sizes of the uneven batch: 32^3, 64^3, 128^3 in ratio 4:2:1.

    96 fields cannot split 4:2:1 exactly; largest-remainder rounding gives
    55 x 32, 27 x 64, 14 x 128, shuffled with default_rng(seed).
    """
    w = np.array([4, 2, 1], dtype=np.float64)
    raw = count * w / w.sum()
    base = np.floor(raw).astype(int)
    rem = count - base.sum()
    order = np.argsort(-(raw - base), kind="stable")
    base[order[:rem]] += 1
    sizes = [32] * base[0] + [64] * base[1] + [128] * base[2]
    perm = np.random.default_rng(seed).permutation(len(sizes))
    return [sizes[i] for i in perm]


def fd_cells(n: int, count: int = 64, seed: int = 5003) -> np.ndarray:
    """Seeded distinct flat cell indices used by finite-difference checks."""
    return np.random.default_rng(seed).choice(n ** 3, size=count, replace=False)
