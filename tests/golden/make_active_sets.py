"""Writes active_w<k>_<mode>.npy: active sets of the seeded workloads, built by the oracle.

Calls only the oracle.  For each workload the pool is a set of seeded
training snapshots (paper_2304_13144_amd.synth.*_training); the rows are the
oracle's b_i (FULL: over the whole theta; LINEAR: (onehot, B_alpha)).  The
active set is the oracle's initial pick (column-pivoted QR of the pool)
followed by MaxVol (threshold 1.001) over the rest of the pool.  FULL sets
are stored with all theta columns so that any valid gauge can be applied.

Run:  python tests/golden/make_active_sets.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import mtp as om                      # noqa: E402
from oracle import neighbors as onb               # noqa: E402
from paper_2304_13144_amd import synth            # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def pool_rows(pot, theta, configs):
    full, lin = [], []
    for cfg in configs:
        pairs = onb.neighbors(cfg.pos, cfg.cell, cfg.pbc, pot.r_cut)
        full.append(om.b_rows(pot, theta, cfg.pos, cfg.types, cfg.cell, pairs))
        lin.append(om.linear_rows(pot, theta, cfg.pos, cfg.types, cfg.cell, pairs))
    return np.vstack(full), np.vstack(lin)


def select(rows):
    act = om.initial_active_set(rows)
    rest = np.setdiff1d(np.arange(len(rows)), act)
    A, _, swaps = om.maxvol(rows[act], rows[rest], threshold=1.001)
    return A, len(swaps)


def main():
    specs = {1: (synth.workload1(), synth.workload1_training(200)),
             2: (synth.workload2(reps=(4, 4, 4)), synth.workload2_training(8)),
             5: (synth.workload5(reps=(4, 4, 4)), synth.workload5_training(16))}
    for wid, (w, pool) in specs.items():
        t = time.time()
        pot = om.Potential(w.level, w.n_types, w.r_min, w.r_cut)
        if wid == 1:
            theta = synth.theta_normal(1, pot.n_types, pot.n_lin, pot.n_rad)
        else:
            theta = synth.theta_teacher(wid, pot.n_types, pot.n_lin, pot.n_rad)
        full, lin = pool_rows(pot, theta, pool)
        keep = om.kept_columns(pot, theta)
        Ak, nsw = select(full[:, keep])
        # recover the full-column rows of the selected neighborhoods
        idx = [int(np.argmin(np.abs(full[:, keep] - r).max(axis=1))) for r in Ak]
        A_full = full[idx]
        assert np.array_equal(A_full[:, keep], Ak)
        np.save(os.path.join(synth.DATA, f"active_w{wid}_full.npy"), A_full)
        Al, nsl = select(lin)
        np.save(os.path.join(synth.DATA, f"active_w{wid}_linear.npy"), Al)
        print(f"workload {wid}: pool {len(full)} rows, FULL m={Ak.shape[0]} ({nsw} swaps, "
              f"cond {np.linalg.cond(Ak):.3g}), LINEAR m={Al.shape[0]} ({nsl} swaps, cond {np.linalg.cond(Al):.3g}) "
              f"in {time.time() - t:.1f}s", flush=True)


if __name__ == "__main__":
    main()
