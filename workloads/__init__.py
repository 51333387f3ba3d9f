"""Seeded synthetic inputs: ion(s) in rigid 3-site water, cubic periodic boxes.

This module holds no part of the electrostatics method: it only places atoms
and assigns charges.  Both the GPU path's tests/benchmarks and the CPU oracle
consume what it returns.  The paper's own inputs (MD snapshots of one ion and
1080 TIP3P waters) are not available; these boxes have the same density, the
same charges and geometry per molecule and the same net-charge structure.

Recipe (every number below is an input choice, not a result):
  * water: O -0.8476 e, H +0.4238 e, r_OH = 1.0 A, HOH = 109.47 deg;
    H1,2 = O + R (+-sin(theta/2), 0, cos(theta/2)) with R a uniform random
    rotation (unit quaternion from 4 standard normals);
  * sites: n_g = smallest even integer with n_g^3 >= N_w, sites at
    ((i + 1/2) b / n_g, ...); when n_g^3 > N_w the first N_w sites of a seeded
    permutation are used; each O is jittered by U(-0.3, 0.3) A per axis;
  * ions: one ion at the box centre (a cube corner of the site grid since n_g
    is even), or 8 ions at the octant centres;
  * atom order: waters (O, H, H per molecule) then ions; ``mask`` marks ions.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

Q_O = -0.8476
Q_H = 0.4238
R_OH = 1.0
THETA_HOH = 109.47
WATER_DENSITY = 0.0334  # molecules per cubic Angstrom


@dataclass
class Workload:
    name: str
    pos: np.ndarray      # (N, 3) float64, Angstrom, inside [0, b)
    q: np.ndarray        # (N,) float64, e
    mask: np.ndarray     # (N,) uint8, 1 = solute (ion)
    box: float
    levels: int
    p: int
    seed: int
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.q.shape[0])


def _random_rotations(rng, k):
    qv = rng.standard_normal((k, 4))
    qv /= np.linalg.norm(qv, axis=1, keepdims=True)
    w, x, y, z = qv.T
    R = np.empty((k, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def water_box(n_waters, box, ion_pos, ion_q, seed):
    """Positions, charges and solute mask for n_waters waters plus the given ions."""
    rng = np.random.default_rng(seed)
    ng = 2
    while ng ** 3 < n_waters:
        ng += 2
    idx = np.arange(ng ** 3)
    if ng ** 3 > n_waters:
        idx = rng.permutation(ng ** 3)[:n_waters]
    ix, iy, iz = idx // (ng * ng), (idx // ng) % ng, idx % ng
    sites = (np.stack([ix, iy, iz], 1).astype(np.float64) + 0.5) * (box / ng)
    o = sites + rng.uniform(-0.3, 0.3, size=sites.shape)
    rot = _random_rotations(rng, n_waters)
    half = math.radians(THETA_HOH) / 2.0
    local = np.array([[math.sin(half), 0.0, math.cos(half)],
                      [-math.sin(half), 0.0, math.cos(half)]]) * R_OH
    h = np.einsum("kij,hj->khi", rot, local)  # (k, 2, 3)
    wat = np.concatenate([o[:, None, :], o[:, None, :] + h], axis=1).reshape(-1, 3)
    ion_pos = np.asarray(ion_pos, dtype=np.float64).reshape(-1, 3)
    ion_q = np.asarray(ion_q, dtype=np.float64).reshape(-1)
    pos = np.concatenate([wat, ion_pos], 0)
    pos = pos - box * np.floor(pos / box)
    pos[pos >= box] = 0.0
    q = np.concatenate([np.tile([Q_O, Q_H, Q_H], n_waters), ion_q])
    mask = np.concatenate([np.zeros(3 * n_waters, np.uint8), np.ones(ion_q.shape[0], np.uint8)])
    return pos, q, mask


def box_for(n_waters):
    return (n_waters / WATER_DENSITY) ** (1.0 / 3.0)


def _single_ion(name, n_waters, box, z, levels, p, seed):
    pos, q, mask = water_box(n_waters, box, [[box / 2] * 3], [z], seed)
    return Workload(name, pos, q, mask, box, levels, p, seed,
                    dict(n_waters=n_waters, ion_charge=z))


OCTANT_CHARGES = (2.0, 1.0, -1.0, 2.0, -1.0, 1.0, -2.0, 1.0)


def config(name: str) -> Workload:
    """The named workloads.

    C1  216 waters + one +1 ion, b = 18.6 A, levels 2, p 8 (FP64 parity case)
    C2  10,000 waters + one +2 ion, b = 67.0 A, levels 4, p 10
    C3  333,333 waters + one -1 ion, b = 215.30 A, levels 5, p 12 (1M atoms)
    C5  1,000,000 waters + 8 ions (net +3), b = 310.52 A, levels 6
    PA  1080 waters + one +2 ion, b = 31.86 A, levels 3 (the paper's system size)
    """
    if name == "C1":
        return _single_ion("C1", 216, 18.6, 1.0, 2, 8, 1)
    if name == "C2":
        return _single_ion("C2", 10000, 67.0, 2.0, 4, 10, 2)
    if name == "C3":
        return _single_ion("C3", 333333, 215.30, -1.0, 5, 12, 3)
    if name == "PA":
        return _single_ion("PA", 1080, 31.86, 2.0, 3, 4, 6)
    if name == "C5":
        box = 310.52
        c = [[(i + 0.5) * box / 2, (j + 0.5) * box / 2, (k + 0.5) * box / 2]
             for i in range(2) for j in range(2) for k in range(2)]
        pos, q, mask = water_box(1000000, box, c, list(OCTANT_CHARGES), 5)
        return Workload("C5", pos, q, mask, box, 6, 8, 5, dict(n_waters=1000000))
    raise KeyError(name)


def batch_windows(n_boxes=32, seed=4, lo=6000, hi=48000):
    """Uneven boxes for charging windows: N ~ U{lo..hi}, ion charge lambda_w z_w."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(lo, hi + 1, size=n_boxes)
    out = []
    for w, n in enumerate(sizes):
        nw = int((int(n) - 1) // 3)
        box = box_for(nw)
        lam = w / (n_boxes - 1) if n_boxes > 1 else 1.0
        z = (2.0, 1.0, -1.0)[w % 3] * lam
        pos, q, mask = water_box(nw, box, [[box / 2] * 3], [z], 400 + w)
        out.append(Workload(f"W{w}", pos, q, mask, box, 0, 10, 400 + w,
                            dict(n_waters=nw, lam=lam, z=(2.0, 1.0, -1.0)[w % 3])))
    return out


def sample_indices(n, k, config_seed):
    """The seeded evaluation sample used where the oracle cannot do all atoms."""
    rng = np.random.default_rng(1000 + config_seed)
    return np.sort(rng.choice(n, size=min(k, n), replace=False)).astype(np.int64)


def random_charges(n, box, seed, net=None):
    """Uniform random points with random +-1-ish charges (tiny edge-case inputs)."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, box, size=(n, 3))
    q = rng.uniform(-1.0, 1.0, size=n)
    if net is not None and n > 0:
        q += (net - q.sum()) / n
    return pos, q
