"""Shared test helpers: oracle-side references for seeded workloads."""
import os

import numpy as np

from oracle import mtp as om
from oracle import neighbors as onb
from paper_2304_13144_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def potential(w):
    return om.Potential(w.level, w.n_types, w.r_min, w.r_cut)


def theta_for(wid, pot):
    if wid == 1:
        return synth.theta_normal(1, pot.n_types, pot.n_lin, pot.n_rad)
    return synth.theta_teacher(wid, pot.n_types, pot.n_lin, pot.n_rad)


def active_rows(wid, mode):
    """Oracle-built active set of a workload: rows in the full theta column space
    (FULL) or (onehot, B) columns (LINEAR); written by tests/golden/make_active_sets.py
    into the package data folder."""
    return synth.active_set(wid, mode)


def oracle_pairs(cfg, rc, atoms=None):
    return onb.neighbors(cfg.pos, cfg.cell, cfg.pbc, rc, atoms=atoms)


def oracle_local_forces(pot, theta, cfg, atoms):
    """Oracle forces on the given atoms only: the energy of every neighborhood
    that holds one of them, differentiated exactly."""
    around = onb.neighbors(cfg.pos, cfg.cell, cfg.pbc, pot.r_cut, atoms=atoms)
    owners = np.unique(np.concatenate([np.asarray(atoms), around.j]))
    pairs = onb.neighbors(cfg.pos, cfg.cell, cfg.pbc, pot.r_cut, atoms=owners)
    _, F, _, V = om.energy_forces_stress(pot, theta, cfg.pos, cfg.types, cfg.cell, pairs)
    return F[np.asarray(atoms)], V[np.asarray(atoms)]


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def kappa_eq(A):
    """Condition number of A with its columns scaled to unit max-abs (column-equilibrated)."""
    A = np.asarray(A, dtype=np.float64)
    return float(np.linalg.cond(A / np.abs(A).max(axis=0)))


def fp64_gamma_tol(A):
    """FP64 bar for grades: 1e-10, relaxed to kappa(A) 1e-15 on an ill-conditioned active set."""
    return max(1e-10, kappa_eq(A) * 1e-15)
