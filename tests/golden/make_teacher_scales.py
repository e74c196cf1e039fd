"""Writes teacher_scales.json: the normalisation of the seeded teacher potentials.

Calls only the oracle.  For workload w, the raw draws (xi0, g, c) come from
paper_2304_13144_amd.synth.theta_raw; on a seeded reference snapshot the
oracle evaluates the basis values B_alpha, s_alpha = RMS over atoms of
B_alpha, then the forces of xi_alpha = g_alpha / s_alpha, and
force_factor = 1 / RMS|F| so that the teacher's RMS force is 1 eV/A.

Run:  python tests/golden/make_teacher_scales.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import mtp as om                      # noqa: E402
from oracle import neighbors as onb               # noqa: E402
from paper_2304_13144_amd import synth            # noqa: E402


def reference_snapshot(wid):
    if wid == 2:
        return synth.workload2_training(1)[0]
    if wid == 3:
        return synth._vacancy_config(synth.rng(3, synth.P_TRAIN), "fcc", 200, 0.06, 3, 0.15, 0.03)
    if wid == 4:
        return synth._vacancy_config(synth.rng(4, synth.P_TRAIN), "fcc", 256, 0.06, 2, 0.08, 0.0, 0.05)
    if wid == 5:
        return synth.workload5_training(1)[0]
    raise ValueError(wid)


SPEC = {2: (16, 2, 5.0), 3: (20, 3, 5.5), 4: (24, 2, 5.0), 5: (16, 1, 5.0)}


def main():
    out = {}
    for wid, (level, nt, rc) in SPEC.items():
        pot = om.Potential(level, nt, 2.0, rc)
        cfg = reference_snapshot(wid)
        xi0, g, c = synth.theta_raw(wid, nt, pot.n_lin, pot.n_rad)
        pairs = onb.neighbors(cfg.pos, cfg.cell, cfg.pbc, rc)
        theta = np.concatenate([xi0, np.zeros(pot.n_lin), c])
        lin = om.linear_rows(pot, theta, cfg.pos, cfg.types, cfg.cell, pairs)
        s = np.sqrt((lin[:, nt:] ** 2).mean(axis=0))
        theta = np.concatenate([xi0, g / s, c])
        F = om.energy_forces_stress(pot, theta, cfg.pos, cfg.types, cfg.cell, pairs)[1]
        lam = 1.0 / np.sqrt((F ** 2).sum(axis=1).mean())
        out[str(wid)] = {"level": level, "n_types": nt, "r_cut": rc, "n_ref_atoms": int(cfg.n),
                         "s_alpha": s.tolist(), "force_factor": float(lam)}
        print(wid, level, nt, cfg.n, "s range", s.min(), s.max(), "lam", lam, flush=True)
    with open(os.path.join(synth.DATA, "teacher_scales.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
