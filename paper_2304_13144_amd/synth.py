"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module holds geometry and random draws only -- lattices, supercells,
species, displacements, strains and parameter draws -- and none of the
potential's arithmetic.  Every draw comes from
``numpy.random.default_rng([230413144, workload_id, purpose])`` so that both
sides of a comparison see identical bytes.

Workloads (ids 1-5):

1. one species, level 8, R_cut 5.0: BCC a = 3.30, 4x4x4 cells (128 atoms),
   sigma = 0.10, every parameter ~ N(0, 0.1^2);
2. two species, level 16, R_cut 5.0: random 50/50 FCC alloy a = 4.05,
   16x16x16 cells (16,384 atoms), sigma = 0.08, normalised teacher;
3. three species, level 20, R_cut 5.5: 512 periodic configurations with
   8..256 atoms on BCC / FCC / HCP lattices at 0.06 atoms/A^3, random
   vacancies, strain U(-0.03, 0.03), sigma = 0.15;
4. two species, level 24, R_cut 5.0: 1024 FCC alloy configurations with
   log-uniform 16..4096 atoms, >= 5 % vacancies, density 0.06, sigma = 0.08;
5. one species, level 16, R_cut 5.0: BCC a = 3.30, 64x64x128 cells
   (1,048,576 atoms), 20 snapshots with sigma_k = 0.05 + 0.35 k / 19.
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import dataclass, field

import numpy as np

SEED = 230413144
_HERE = os.path.dirname(os.path.abspath(__file__))
# seeded inputs written by the oracle-side scripts next to the tests (teacher
# scales, active sets): inputs of both the library and its checks
DATA = os.path.join(_HERE, "data")

# purposes of the random streams
P_LATTICE, P_DISPLACE, P_THETA, P_TRAIN, P_STRAIN, P_SIZES, P_VACANCY = 0, 1, 2, 3, 4, 5, 6
P_CFGMODE = 7
P_SNAPSHOT = 10


def rng(workload: int, purpose: int) -> np.random.Generator:
    return np.random.default_rng([SEED, workload, purpose])


@dataclass
class Config:
    pos: np.ndarray              # [N, 3] float64, Angstrom
    types: np.ndarray            # [N] int32
    cell: np.ndarray             # [3, 3] float64, row k = cell vector k
    pbc: tuple = (True, True, True)

    @property
    def n(self):
        return len(self.pos)


@dataclass
class Workload:
    wid: int
    level: int
    n_types: int
    r_min: float
    r_cut: float
    n_polyn: int = 8
    configs: list = field(default_factory=list)


# ---------------------------------------------------------------------------
# lattices
# ---------------------------------------------------------------------------
_BASIS = {
    "bcc": np.array([[0, 0, 0], [0.5, 0.5, 0.5]]),
    "fcc": np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]]),
    # orthorhombic 4-atom HCP cell a x sqrt(3) a x c
    "hcp": np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 5 / 6, 0.5], [0, 1 / 3, 0.5]]),
}


def unit_cell(kind: str, a: float, c_over_a: float = math.sqrt(8 / 3)):
    if kind == "hcp":
        return np.diag([a, math.sqrt(3) * a, c_over_a * a])
    return np.eye(3) * a


def lattice(kind: str, a: float, reps):
    """Perfect lattice of reps = (nx, ny, nz) unit cells; (pos, cell)."""
    uc = unit_cell(kind, a)
    b = _BASIS[kind]
    grid = np.array([[i, j, k] for i in range(reps[0]) for j in range(reps[1]) for k in range(reps[2])],
                    dtype=np.float64)
    frac = (grid[:, None, :] + b[None, :, :]).reshape(-1, 3)
    return frac @ uc, uc * np.asarray(reps, dtype=np.float64)[:, None]


def lattice_constant_for_density(kind: str, density: float):
    per_cell = len(_BASIS[kind])
    vol = per_cell / density
    if kind == "hcp":
        return (vol / (math.sqrt(3) * math.sqrt(8 / 3))) ** (1 / 3)
    return vol ** (1 / 3)


def near_cubic_reps(kind: str, n_sites_min: int):
    """Smallest near-cubic replication with at least n_sites_min sites."""
    uc = np.diag(unit_cell(kind, 1.0))
    per = len(_BASIS[kind])
    best = None
    for nx in range(1, 40):
        for ny in range(1, 40):
            for nz in range(1, 40):
                n = per * nx * ny * nz
                if n < n_sites_min:
                    continue
                L = uc * np.array([nx, ny, nz])
                score = (n, L.max() / L.min())
                if best is None or score < best[0]:
                    best = (score, (nx, ny, nz))
                break
    return best[1]


def strain_matrix(r: np.random.Generator, amp: float):
    e = r.uniform(-amp, amp, 6)
    return np.array([[e[0], e[3], e[4]], [e[3], e[1], e[5]], [e[4], e[5], e[2]]])


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------
def workload1():
    pos, cell = lattice("bcc", 3.30, (4, 4, 4))
    pos = pos + rng(1, P_DISPLACE).normal(0.0, 0.10, pos.shape)
    w = Workload(1, 8, 1, 2.0, 5.0)
    w.configs = [Config(pos, np.zeros(len(pos), np.int32), cell)]
    return w


def workload1_training(n_copies=200):
    """Seeded displaced copies of workload 1's lattice (active-set pool)."""
    base, cell = lattice("bcc", 3.30, (4, 4, 4))
    r = rng(1, P_TRAIN)
    return [Config(base + r.normal(0.0, 0.10, base.shape), np.zeros(len(base), np.int32), cell)
            for _ in range(n_copies)]


def fcc_alloy(wid, reps, purpose_species, purpose_disp, sigma=0.08, a=4.05):
    pos, cell = lattice("fcc", a, reps)
    types = (rng(wid, purpose_species).random(len(pos)) < 0.5).astype(np.int32)
    pos = pos + rng(wid, purpose_disp).normal(0.0, sigma, pos.shape)
    return Config(pos, types, cell)


def workload2(reps=(16, 16, 16)):
    w = Workload(2, 16, 2, 2.0, 5.0)
    w.configs = [fcc_alloy(2, reps, P_LATTICE, P_DISPLACE)]
    return w


def workload2_training(n_snap=8, reps=(4, 4, 4)):
    """Independently seeded alloy snapshots (active-set pool for workload 2)."""
    return [fcc_alloy(2, reps, P_SNAPSHOT + 2 * k, P_SNAPSHOT + 2 * k + 1) for k in range(n_snap)]


def _vacancy_config(r, kind, n_atoms, density, n_types, sigma, strain_amp, vac_min_frac=0.0):
    a = lattice_constant_for_density(kind, density)
    n_sites = int(math.ceil(n_atoms / (1.0 - vac_min_frac)))
    reps = near_cubic_reps(kind, n_sites)
    pos, cell = lattice(kind, a, reps)
    keep = np.sort(r.choice(len(pos), n_atoms, replace=False))
    pos = pos[keep]
    if strain_amp:
        D = np.eye(3) + strain_matrix(r, strain_amp)
        pos, cell = pos @ D.T, cell @ D.T
    pos = pos + r.normal(0.0, sigma, pos.shape)
    types = r.integers(0, n_types, n_atoms).astype(np.int32)
    return Config(pos, types, cell)


def cfg_pool(wid, n_cfg, stream=0, n_min=8, n_max=54):
    """Small periodic configurations for the configuration query mode with the
    potential of workload 1 (one species, BCC a = 3.30, sigma = 0.10) or 2
    (two species, FCC a = 4.05, sigma = 0.08): n_min..n_max atoms each on the
    smallest near-cubic cell, random vacancies, strain U(-0.03, 0.03).
    `stream` selects an independent pool."""
    r = np.random.default_rng([SEED, wid, P_CFGMODE, stream])
    if wid == 1:
        kind, a, n_types, sigma = "bcc", 3.30, 1, 0.10
    elif wid == 2:
        kind, a, n_types, sigma = "fcc", 4.05, 2, 0.08
    else:
        raise ValueError("configuration pools exist for workloads 1 and 2")
    density = len(_BASIS[kind]) / a ** 3
    sizes = r.integers(n_min, n_max + 1, n_cfg)
    return [_vacancy_config(r, kind, int(n), density, n_types, sigma, 0.03) for n in sizes]


def fcc111_slab(nx=15, ny=9, layers=6, a=3.615, box_z=40.0, sigma=0.05, stream=0):
    """FCC(111) slab, periodic along x and y only: a rectangular in-plane cell
    of d x d sqrt(3) (d = a / sqrt 2, two atoms per layer), ABC stacking at
    a / sqrt(3) per layer, nx x ny cells per layer, centred in a box of
    height box_z; displacements N(0, sigma^2).  The defaults give 1,620 atoms
    in 38.3 x 39.8 x 40 A (six layers of 270)."""
    d = a / math.sqrt(2.0)
    dy = d * math.sqrt(3.0)
    dz = a / math.sqrt(3.0)
    base = np.array([[0.0, 0.0], [0.5 * d, 0.5 * dy]])
    pos = []
    for l in range(layers):
        off = np.array([0.0, (l % 3) * dy / 3.0])   # A, B, C positions
        for i in range(nx):
            for j in range(ny):
                for b in base:
                    xy = np.array([i * d, j * dy]) + b + off
                    pos.append([xy[0], xy[1], 0.5 * box_z + (l - 0.5 * (layers - 1)) * dz])
    pos = np.array(pos)
    pos[:, 1] %= ny * dy
    cell = np.diag([nx * d, ny * dy, box_z])
    pos = pos + np.random.default_rng([SEED, 6, P_DISPLACE, stream]).normal(0.0, sigma, pos.shape)
    return Config(pos, np.zeros(len(pos), np.int32), cell, (True, True, False))


def workload3(n_cfg=512):
    w = Workload(3, 20, 3, 2.0, 5.5)
    sizes = rng(3, P_SIZES).integers(8, 257, n_cfg)
    kinds = rng(3, P_LATTICE).choice(["bcc", "fcc", "hcp"], n_cfg)
    r = rng(3, P_DISPLACE)
    w.configs = [_vacancy_config(r, k, int(n), 0.06, 3, 0.15, 0.03) for n, k in zip(sizes, kinds)]
    return w


def workload4(n_cfg=1024):
    w = Workload(4, 24, 2, 2.0, 5.0)
    sizes = np.round(np.exp(rng(4, P_SIZES).uniform(math.log(16), math.log(4096), n_cfg))).astype(int)
    r = rng(4, P_DISPLACE)
    w.configs = [_vacancy_config(r, "fcc", int(n), 0.06, 2, 0.08, 0.0, vac_min_frac=0.05) for n in sizes]
    return w


def workload5_snapshot(k, reps=(64, 64, 128), n_snap=20):
    pos, cell = lattice("bcc", 3.30, reps)
    sigma = 0.05 + 0.35 * k / (n_snap - 1)
    pos = pos + rng(5, P_SNAPSHOT + k).normal(0.0, sigma, pos.shape)
    return Config(pos, np.zeros(len(pos), np.int32), cell)


def workload5(reps=(64, 64, 128)):
    w = Workload(5, 16, 1, 2.0, 5.0)
    w.configs = [workload5_snapshot(0, reps)]
    return w


def workload5_training(n_copies=16):
    base, cell = lattice("bcc", 3.30, (4, 4, 4))
    r = rng(5, P_TRAIN)
    return [Config(base + r.normal(0.0, 0.05, base.shape), np.zeros(len(base), np.int32), cell)
            for _ in range(n_copies)]


# ---------------------------------------------------------------------------
# parameters
# ---------------------------------------------------------------------------
def dims(level_n_lin, n_rad, n_types, n_polyn=8):
    return n_types, level_n_lin, n_rad * n_types * n_types * n_polyn


def theta_normal(wid, n_types, n_lin, n_rad, n_polyn=8, std=0.1):
    """Every parameter ~ N(0, std^2) (workload 1)."""
    n = n_types + n_lin + n_rad * n_types * n_types * n_polyn
    return rng(wid, P_THETA).normal(0.0, std, n)


def theta_raw(wid, n_types, n_lin, n_rad, n_polyn=8, std=0.1):
    """Raw draws of a normalised teacher: (xi0, g, c) all ~ N(0, std^2)."""
    r = rng(wid, P_THETA)
    xi0 = r.normal(0.0, std, n_types)
    g = r.normal(0.0, std, n_lin)
    c = r.normal(0.0, std, n_rad * n_types * n_types * n_polyn)
    return xi0, g, c


def teacher_scales(wid):
    """Stored per-workload scales (s_alpha, force factor) of the teacher."""
    path = os.path.join(DATA, "teacher_scales.json")
    with open(path) as fh:
        d = json.load(fh)[str(wid)]
    return np.asarray(d["s_alpha"], dtype=np.float64), float(d["force_factor"])


def active_set(wid, mode):
    """Stored active set of a workload (rows of A): FULL over all theta columns,
    LINEAR over (onehot, B_alpha)."""
    return np.load(os.path.join(DATA, f"active_w{wid}_{mode}.npy"))


def theta_teacher(wid, n_types, n_lin, n_rad, n_polyn=8):
    """Normalised teacher: xi_alpha = force_factor * g_alpha / s_alpha."""
    xi0, g, c = theta_raw(wid, n_types, n_lin, n_rad, n_polyn)
    s, lam = teacher_scales(wid)
    return np.concatenate([xi0, lam * g / s, c])
