"""Seeded FCC Lennard-Jones workloads (the paper's miniMD-style benchmark setup).

The evaluation setup (Sec. 6, first paragraphs) places atoms on an FCC lattice
with four particles per unit cell, uses epsilon = sigma = 1, cutoff 2.5 and a
Verlet buffer of 0.3; density and temperature follow miniMD's defaults
(reduced density 0.8442, T = 1.44).  The paper does not state how initial
velocities are drawn, so the recipe below is this project's reading:

* random stream: SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) in its
  published form (golden-gamma increment, two xor-shift-multiply rounds and a
  final xor-shift); a double in [0, 1) is ``(z >> 11) * 2**-53``;
* FCC basis (0,0,0), (1/2,1/2,0), (1/2,0,1/2), (0,1/2,1/2); atom id
  ``((iz*n + iy)*n + ix)*4 + b``; position ``(i + b) * a`` with
  ``a = (4 / rho) ** (1/3)``;
* draw order per system: jitter (3N draws, atom-major x,y,z) when requested,
  then velocities (3N draws, atom-major);
* jitter: ``x += width * (u - 0.5)`` then wrap into [0, L);
* velocities: ``u - 0.5`` per component, subtract the mean, scale so that
  ``m * sum |v|^2 / (3N - 3) == T``.

Nothing here evaluates a distance, a force or an integration step.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_MIX1 = np.uint64(0xBF58476D1CE4E5B9)
_MIX2 = np.uint64(0x94D049BB133111EB)
_MASK64 = (1 << 64) - 1


def _mix(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _MIX1
    z = (z ^ (z >> np.uint64(27))) * _MIX2
    return z ^ (z >> np.uint64(31))


class SplitMix64:
    """Counter form of SplitMix64: output k is mix(seed + (k+1)*gamma)."""

    def __init__(self, seed: int):
        self.state = int(seed) & _MASK64
        self.count = 0

    def next_u64(self, n: int) -> np.ndarray:
        k = np.arange(self.count + 1, self.count + 1 + n, dtype=np.uint64)
        with np.errstate(over="ignore"):
            z = np.uint64(self.state) + k * _GOLDEN
            out = _mix(z)
        self.count += n
        return out

    def next_double(self, n: int) -> np.ndarray:
        return (self.next_u64(n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def fcc_lattice_constant(rho: float) -> float:
    return (4.0 / rho) ** (1.0 / 3.0)


_BASIS = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]])


def fcc_positions(ncell: int, rho: float):
    """Perfect FCC lattice of ncell^3 unit cells; returns (pos[N,3], L)."""
    a = fcc_lattice_constant(rho)
    idx = np.arange(ncell, dtype=np.float64)
    iz, iy, ix = np.meshgrid(idx, idx, idx, indexing="ij")
    cells = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1)  # cell id = (iz*n+iy)*n+ix
    pos = (cells[:, None, :] + _BASIS[None, :, :]).reshape(-1, 3) * a
    return pos, ncell * a


def _wrap(p: np.ndarray, L: float) -> np.ndarray:
    p = np.where(p < 0.0, p + L, p)
    p = np.where(p >= L, p - L, p)
    return np.where(p >= L, 0.0, p)  # x + L may round up to L for tiny negative x


@dataclass
class MDInput:
    """One periodic cubic box: SoA positions/velocities (original atom order)."""

    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray
    L: float
    ncell: int
    rho: float
    T: float
    seed: int

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def pos(self) -> np.ndarray:
        return np.stack([self.x, self.y, self.z], axis=1)

    def vel(self) -> np.ndarray:
        return np.stack([self.vx, self.vy, self.vz], axis=1)


def md_system(ncell: int, rho: float = 0.8442, T: float = 1.44, seed: int = 1000,
              jitter: float = 0.0, mass: float = 1.0) -> MDInput:
    """FCC box of ncell^3 unit cells with seeded jitter (full width) and velocities."""
    pos, L = fcc_positions(ncell, rho)
    n = pos.shape[0]
    rng = SplitMix64(seed)
    if jitter > 0.0:
        u = rng.next_double(3 * n).reshape(n, 3)
        pos = _wrap(pos + jitter * (u - 0.5), L)
    u = rng.next_double(3 * n).reshape(n, 3)
    v = u - 0.5
    v = v - v.mean(axis=0)
    t_cur = mass * float(np.sum(v * v)) / (3 * n - 3)
    v = v * np.sqrt(T / t_cur)
    pos = np.ascontiguousarray(pos)
    v = np.ascontiguousarray(v)
    return MDInput(pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(),
                   v[:, 0].copy(), v[:, 1].copy(), v[:, 2].copy(),
                   float(L), ncell, rho, T, seed)


def batched_box_specs(n_boxes: int = 512, master_seed: int = 2000):
    """Per-box (ncell, rho, T, seed) from one master stream, four draws per box.

    u1 -> ncell = 4 + floor(9 u1) (4..12), u2 -> rho = 0.75 + 0.15 u2,
    u3 -> T = 0.7 + 0.8 u3, raw fourth output -> the box's own seed.
    """
    rng = SplitMix64(master_seed)
    raw = rng.next_u64(4 * n_boxes).reshape(n_boxes, 4)
    u = (raw >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    specs = []
    for b in range(n_boxes):
        specs.append((4 + int(np.floor(9.0 * u[b, 0])), 0.75 + 0.15 * float(u[b, 1]),
                      0.7 + 0.8 * float(u[b, 2]), int(raw[b, 3])))
    return specs


@dataclass
class SDInput(MDInput):
    """Spheres for the Spring-Dashpot contact model (Sec. 3.2, Eq. 3) with
    the parameters the run uses: spring constant k, dissipation gamma,
    diameter sigma, list radius cutoff + skin, time step dt."""

    k: float = 1000.0
    gamma: float = 5.0
    sigma: float = 1.0
    cutoff: float = 1.0
    skin: float = 0.3
    dt: float = 1e-3


def sd_system(ncell: int, seed: int = 4000, overlap: float = 0.02, jitter: float = 0.05, T: float = 0.5,
              k: float = 1000.0, gamma: float = 5.0, sigma: float = 1.0, dt: float = 1e-3) -> SDInput:
    """A dense packing of spheres of diameter sigma: an FCC lattice of
    ncell^3 unit cells whose nearest neighbours sit (1 - overlap) sigma
    apart, so every sphere presses on its twelve neighbours, then seeded
    jitter and velocities as in md_system (draw order jitter, velocities)."""
    a = np.sqrt(2.0) * (1.0 - overlap) * sigma
    rho = 4.0 / a ** 3
    b = md_system(ncell, rho=rho, T=T, seed=seed, jitter=jitter)
    return SDInput(b.x, b.y, b.z, b.vx, b.vy, b.vz, b.L, ncell, rho, T, seed, k=k, gamma=gamma, sigma=sigma,
                   cutoff=sigma, skin=0.3, dt=dt)


def sd_half_domain(ncell: int, sigma: float = 1.0):
    """The load-balancing geometry of Sec. 6: a periodic cube of ncell^3
    unit cells of side sigma, with one sphere at the corner of every unit
    cell on one side of the diagonal plane x + y + z = 3 L / 2 - half of the
    domain filled, half empty (ncell^3 / 2 spheres for even ncell).  The
    paper runs it with zero stiffness and damping (spheres at rest).
    Returns (pos[N, 3], L)."""
    idx = np.arange(ncell, dtype=np.float64)
    iz, iy, ix = np.meshgrid(idx, idx, idx, indexing="ij")
    p = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1) * sigma
    L = ncell * sigma
    keep = (p[:, 0] + p[:, 1] + p[:, 2]) + 1.5 * sigma < 1.5 * L
    return np.ascontiguousarray(p[keep]), float(L)
