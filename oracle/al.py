"""Extrapolation-controlled simulation pieces -- oracle side.

Test infrastructure only (see ``oracle/__init__.py``).

* ``extrapolative_neighborhood`` -- the spherical fragment around the atom of
  largest grade (Sec. III.A, the neighborhood cut used for learning on
  neighborhoods, Sec. II.F step 3 (ii)): that atom and every atom or
  periodic image closer than the cutoff, as a non-periodic cluster.
* ``md_verlet`` -- velocity-Verlet molecular dynamics (NVE) whose every
  configuration is graded before its forces are used (Sec. II.F step 1):
  gamma(cfg) = max_i gamma_i below gamma_save: go on; between gamma_save and
  gamma_break: record the step and go on; above gamma_break: stop.

Units: Angstrom, eV, amu, fs.  The acceleration of a force of 1 eV/A on
1 amu, in A/fs^2, follows from the CODATA 2018 exact elementary charge and
the atomic mass constant: (1.602176634e-19 J / 1e-10 m) / 1.66053906660e-27
kg = 9.6485...e17 m/s^2 = 9.6485...e-3 A/fs^2.

* ``relax_fire`` -- structure relaxation (Sec. III.A, the relax command
  with extrapolation control) by FIRE (Bitzek, Koskinen, Gaehler, Moseler,
  Gumbsch, Phys. Rev. Lett. 97, 170201 (2006)); the paper names no
  minimizer, FIRE is our reading.  Each step: stop if max_i |F_i| < fmax;
  P = F.v; if P > 0: v <- (1 - alpha) v + alpha |v| F / |F| and, after more
  than N_min = 5 such steps in a row, dt <- min(1.1 dt, dt_max),
  alpha <- 0.99 alpha; else v <- 0, dt <- dt / 2, alpha <- 0.1 and the count
  restarts; then v <- v + dt F / m, x <- x + dt v (semi-implicit Euler); the
  new configuration is graded (as in ``md_verlet``) before its forces are
  used.  Norms |v|, |F| are over all 3N components.

Readings: the fragment takes distances strictly below the cutoff (as the
neighborhoods of Sec. II.A do) and lists its atoms ordered by (source atom,
image shift); the MD grades the configuration after each drift, before the
second half kick, and the initial configuration before the first step.
"""
from __future__ import annotations

import numpy as np

from . import mtp as om
from . import neighbors as onb

EV_PER_A_AMU_IN_A_PER_FS2 = (1.602176634e-19 / 1e-10) / 1.66053906660e-27 * 1e10 * 1e-30


def extrapolative_neighborhood(pos, types, cell, pbc, grades, cutoff):
    """Returns (center, src [k], shift [k, 3], pos [k, 3], types [k]) sorted by
    (src, shift); the center atom itself is the entry (center, 0, 0, 0)."""
    grades = np.asarray(grades)
    center = int(np.argmax(grades))          # lowest index among equal maxima
    pairs = onb.neighbors(pos, cell, pbc, cutoff, atoms=[center])
    items = [(center, (0, 0, 0))] + [(int(j), tuple(int(v) for v in s)) for j, s in zip(pairs.j, pairs.shift)]
    items.sort()
    src = np.array([j for j, _ in items], dtype=np.int64)
    shift = np.array([s for _, s in items], dtype=np.int64).reshape(-1, 3)
    p = np.asarray(pos, dtype=np.float64)[src] + shift @ np.asarray(cell, dtype=np.float64)
    return center, src, shift, p, np.asarray(types)[src]


def _grade_cfg(pot, theta, pos, types, cell, pbc, A, mode, keep):
    pairs = onb.neighbors(pos, cell, pbc, pot.r_cut)
    if mode == "full":
        rows = om.b_rows(pot, theta, pos, types, cell, pairs)[:, keep]
    else:
        rows = om.linear_rows(pot, theta, pos, types, cell, pairs)
    g = om.grades(rows, A)[0]
    return g, pairs


def md_verlet(pot, theta, pos, vel, types, cell, pbc, masses, dt, n_steps, A, mode, keep, gamma_save,
              gamma_break):
    """Velocity Verlet with extrapolation control (A None: without; gamma 0).
    Returns a dict with the
    final positions and velocities, gamma(cfg) of every graded configuration
    (step 0 = the initial one), the saved steps and the number of completed
    steps (fewer than n_steps when gamma_break was exceeded)."""
    x = np.array(pos, dtype=np.float64, copy=True)
    v = np.array(vel, dtype=np.float64, copy=True)
    inv_m = 1.0 / np.asarray(masses, dtype=np.float64)[np.asarray(types)]
    acc = EV_PER_A_AMU_IN_A_PER_FS2
    if A is None:   # no extrapolation control: plain NVE
        def _grade_cfg_or_none(x):
            return np.zeros(1), onb.neighbors(x, cell, pbc, pot.r_cut)
    else:
        def _grade_cfg_or_none(x):
            return _grade_cfg(pot, theta, x, types, cell, pbc, A, mode, keep)
    g, pairs = _grade_cfg_or_none(x)
    gam = [float(g.max())]
    saved = [0] if gamma_save < gam[0] <= gamma_break else []
    if gam[0] > gamma_break:
        return {"pos": x, "vel": v, "gamma": gam, "saved": saved, "steps": 0}
    F = om.energy_forces_stress(pot, theta, x, types, cell, pairs)[1]
    done = 0
    for step in range(1, n_steps + 1):
        v = v + (0.5 * dt * acc) * F * inv_m[:, None]
        x = x + dt * v
        g, pairs = _grade_cfg_or_none(x)
        gam.append(float(g.max()))
        if gam[-1] > gamma_break:
            break
        if gam[-1] > gamma_save:
            saved.append(step)
        F = om.energy_forces_stress(pot, theta, x, types, cell, pairs)[1]
        v = v + (0.5 * dt * acc) * F * inv_m[:, None]
        done = step
    return {"pos": x, "vel": v, "gamma": gam, "saved": saved, "steps": done}


def fire(x0, inv_m, forces, grade, dt0, dt_max, fmax, max_steps, gamma_save, gamma_break):
    """FIRE steps on any force field: forces(x) -> F [N, 3] (eV/A); grade(x)
    -> gamma(cfg) (called before forces(x) on every configuration);
    inv_m [N] 1/amu.  Returns a dict with the final positions, gamma(cfg)
    per graded configuration, the saved steps, the completed steps and
    whether max |F_i| < fmax was reached."""
    x = np.array(x0, dtype=np.float64, copy=True)
    v = np.zeros_like(x)
    acc = EV_PER_A_AMU_IN_A_PER_FS2
    gam = [float(grade(x))]
    saved = [0] if gamma_save < gam[0] <= gamma_break else []
    out = {"pos": x, "gamma": gam, "saved": saved, "steps": 0, "converged": False}
    if gam[0] > gamma_break:
        return out
    F = forces(x)
    dt, alpha, n_pos = dt0, 0.1, 0
    for step in range(1, max_steps + 1):
        if np.sqrt((F * F).sum(axis=1)).max() < fmax:
            out["converged"] = True
            break
        P = float((F * v).sum())
        if P > 0:
            v = (1.0 - alpha) * v + alpha * np.sqrt((v * v).sum()) * F / np.sqrt((F * F).sum())
            n_pos += 1
            if n_pos > 5:
                dt = min(1.1 * dt, dt_max)
                alpha *= 0.99
        else:
            v = np.zeros_like(v)
            dt *= 0.5
            alpha = 0.1
            n_pos = 0
        v = v + (dt * acc) * F * inv_m[:, None]
        x = x + dt * v
        gam.append(float(grade(x)))
        if gam[-1] > gamma_break:
            break
        if gam[-1] > gamma_save:
            saved.append(step)
        F = forces(x)
        out["steps"] = step
    else:
        out["converged"] = bool(np.sqrt((F * F).sum(axis=1)).max() < fmax)
    out["pos"] = x
    return out


def relax_fire(pot, theta, pos, types, cell, pbc, masses, dt0, dt_max, fmax, max_steps, A, mode, keep, gamma_save,
               gamma_break):
    """``fire`` with the potential's forces and grades (A None: gamma 0)."""
    inv_m = 1.0 / np.asarray(masses, dtype=np.float64)[np.asarray(types)]
    cache = {}

    def grade(x):
        if A is None:
            g, pairs = np.zeros(1), onb.neighbors(x, cell, pbc, pot.r_cut)
        else:
            g, pairs = _grade_cfg(pot, theta, x, types, cell, pbc, A, mode, keep)
        cache["pairs"] = pairs
        return g.max()

    def forces(x):
        return om.energy_forces_stress(pot, theta, x, types, cell, cache["pairs"])[1]

    return fire(pos, inv_m, forces, grade, dt0, dt_max, fmax, max_steps, gamma_save, gamma_break)
