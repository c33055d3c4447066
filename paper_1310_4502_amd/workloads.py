"""Seeded synthetic particle sets for the force-evaluation path.

This module only draws inputs (positions, masses, velocities, cotangents).
It holds none of the force method's arithmetic, so both the GPU path and the
CPU oracle can be fed from it without sharing any computation.

The paper runs on cosmological initial conditions and simulations that are
not available here; these generators are synthetic stand-ins with the shapes
and structure of its workloads (Section "Error Analysis" uses a uniform cube;
the cosmological runs are near-uniform perturbed grids and clustered halos):

* ``uniform``   -- N points uniform in the unit cube.
* ``plummer``   -- a Plummer sphere, truncated by rejection at ``rmax``.
* ``clustered`` -- half the mass in Plummer halos with log-uniform weights,
                   half uniform (a stand-in for an evolved, clustered field).
* ``zeldovich`` -- a grid displaced by a Gaussian random field whose density
                   power spectrum is proportional to k^-2 (a stand-in for
                   early-time, near-uniform cosmological initial conditions).

Every array is float64; masses are 1/N (total mass 1, G = 1).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np


def uniform(n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.random((n, 3))


def _plummer_radii(rng, m, a, rmax):
    """Inverse-CDF radii of a Plummer profile, truncated at rmax by rejection."""
    out = np.empty(0)
    while out.size < m:
        want = int((m - out.size) * 1.1) + 16
        u = rng.random(want)
        u = u[u > 0]
        r = a / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
        r = r[r <= rmax]
        out = np.concatenate([out, r])
    return out[:m]


def _directions(rng, m):
    v = rng.standard_normal((m, 3))
    nrm = np.linalg.norm(v, axis=1)
    bad = nrm == 0
    while bad.any():
        v[bad] = rng.standard_normal((int(bad.sum()), 3))
        nrm = np.linalg.norm(v, axis=1)
        bad = nrm == 0
    return v / nrm[:, None]


def plummer(n: int, seed: int, a: float = 1.0 / 16, centre=(0.5, 0.5, 0.5),
            rmax: float = 0.5) -> np.ndarray:
    rng = np.random.default_rng(seed)
    r = _plummer_radii(rng, n, a, rmax)
    return np.asarray(centre, dtype=np.float64) + r[:, None] * _directions(rng, n)


def plummer_velocities(pos: np.ndarray, seed: int, a: float = 1.0 / 16,
                       centre=(0.5, 0.5, 0.5)) -> np.ndarray:
    """Isotropic Gaussian velocities with the Plummer Jeans dispersion
    sigma^2(r) = 1 / (6 sqrt(r^2 + a^2)) (total mass 1, G = 1)."""
    rng = np.random.default_rng(seed)
    r = np.linalg.norm(pos - np.asarray(centre), axis=1)
    sig = np.sqrt(1.0 / (6.0 * np.sqrt(r * r + a * a)))
    return rng.standard_normal(pos.shape) * sig[:, None]


def clustered(n: int, seed: int, n_halos: int = 512, halo_fraction: float = 0.5,
              rs_range=(0.002, 0.02), trunc: float = 10.0) -> np.ndarray:
    """Half the particles in Plummer halos, half uniform in the unit cube.

    Halo weights are 10^U(0,2); halo particle counts follow the weights by
    largest-remainder rounding; scale radii are log-uniform in rs_range,
    independent of mass; centres uniform in the unit cube; every halo is
    truncated at ``trunc`` scale radii by rejection.
    """
    rng = np.random.default_rng(seed)
    n_h = int(round(n * halo_fraction))
    w = 10.0 ** rng.uniform(0.0, 2.0, n_halos)
    share = n_h * w / w.sum()
    cnt = np.floor(share).astype(np.int64)
    rem = n_h - int(cnt.sum())
    order = np.argsort(-(share - cnt), kind="stable")
    cnt[order[:rem]] += 1
    rs = np.exp(rng.uniform(np.log(rs_range[0]), np.log(rs_range[1]), n_halos))
    centres = rng.random((n_halos, 3))
    parts = []
    for h in range(n_halos):
        m = int(cnt[h])
        if m == 0:
            continue
        r = _plummer_radii(rng, m, rs[h], trunc * rs[h])
        parts.append(centres[h] + r[:, None] * _directions(rng, m))
    parts.append(rng.random((n - n_h, 3)))
    pos = np.concatenate(parts, axis=0)
    return pos


def zeldovich(ngrid: int, seed: int, rms_disp_cells: float = 0.3) -> np.ndarray:
    """ngrid^3 grid points at ((i+1/2)/ngrid, ...) displaced by a curl-free
    Gaussian field derived from a density field with P(k) ~ k^-2; the
    displacement is rescaled to an RMS length of rms_disp_cells grid
    spacings. Not wrapped (isolated boundaries)."""
    rng = np.random.default_rng(seed)
    g = ngrid
    white = rng.standard_normal((g, g, g))
    dk = np.fft.rfftn(white)
    kx = np.fft.fftfreq(g)[:, None, None]
    ky = np.fft.fftfreq(g)[None, :, None]
    kz = np.fft.rfftfreq(g)[None, None, :]
    k2 = kx * kx + ky * ky + kz * kz
    k2[0, 0, 0] = 1.0
    dk = dk / np.sqrt(k2)          # amplitude ~ sqrt(P) = 1/k
    dk[0, 0, 0] = 0.0
    disp = np.empty((g, g, g, 3))
    for d, kd in enumerate((kx, ky, kz)):
        disp[..., d] = np.fft.irfftn(1j * kd * dk / k2, s=(g, g, g), axes=(0, 1, 2))
    del dk
    rms = np.sqrt(np.mean(np.sum(disp * disp, axis=-1)))
    disp *= (rms_disp_cells / g) / rms
    idx = (np.arange(g, dtype=np.float64) + 0.5) / g
    grid = np.stack(np.meshgrid(idx, idx, idx, indexing="ij"), axis=-1)
    return (grid + disp).reshape(-1, 3)


@dataclass
class Workload:
    name: str
    pos: np.ndarray
    mass: np.ndarray
    eps: float
    theta: float
    p: int
    box: Optional[tuple] = None          # (lo_x, lo_y, lo_z, side) or None
    n_leaf: int = 16
    n_group: int = 64
    direct_max: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.pos.shape[0]


def make(name: str, seed: Optional[int] = None, n: Optional[int] = None) -> Workload:
    """Named workloads. ``n`` overrides the particle count (same recipe)."""
    if name == "uniform4k":
        n = n or 4096
        pos = uniform(n, 1 if seed is None else seed)
        return Workload(name, pos, np.full(n, 1.0 / n), 1e-3, 0.5, 2,
                        box=(0.0, 0.0, 0.0, 1.0))
    if name == "plummer1m":
        n = n or (1 << 20)
        pos = plummer(n, 2 if seed is None else seed)
        return Workload(name, pos, np.full(n, 1.0 / n), 1e-4, 0.6, 4,
                        box=(0.0, 0.0, 0.0, 1.0))
    if name in ("clustered4m", "clustered16m"):
        n = n or (1 << 22 if name == "clustered4m" else 1 << 24)
        s = seed if seed is not None else (3 if name == "clustered4m" else 33)
        pos = clustered(n, s)
        return Workload(name, pos, np.full(n, 1.0 / n), 5e-5, 0.5, 6)
    if name == "zeldovich16m":
        g = 256 if n is None else int(round(n ** (1.0 / 3.0)))
        pos = zeldovich(g, 4 if seed is None else seed)
        n = pos.shape[0]
        return Workload(name, pos, np.full(n, 1.0 / n), 2e-5, 0.5, 8)
    if name == "plummer256k":
        n = n or (1 << 18)
        s = 5 if seed is None else seed
        pos = plummer(n, s)
        vel = plummer_velocities(pos, s + 500)
        return Workload(name, pos, np.full(n, 1.0 / n), 1e-4, 0.6, 4,
                        extra={"vel": vel})
    raise KeyError(name)


def cotangent(n: int, seed: int) -> np.ndarray:
    """A random cotangent for the acceleration output, unit Frobenius norm."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((n, 3))
    return a / np.linalg.norm(a)


def sample_indices(n: int, k: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    if k >= n:
        return np.arange(n, dtype=np.int64)
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)
