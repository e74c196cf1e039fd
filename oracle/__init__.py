"""FP64 CPU oracle for the Moment Tensor Potential hot path (MLIP-3 paper).

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, calls,
links or executes anything in this folder; only ``tests/``, the smoke check in
``__graft_entry__.py`` and the ``cpu_baseline`` leg of ``bench.py`` may.  The
oracle shares no code, header, table or generator with the HIP library.

It computes the plain definitions of the paper, slowly and in float64:

* ``basis``      -- the level rule (Sec. II.A, eqs. 5-6) and the basis set it
                    induces, enumerated by brute force over contraction graphs.
* ``mtp``        -- radial functions (eq. 4), dense moment tensors (eq. 3),
                    explicit index-sum contractions, site energies (eq. 2),
                    total energy (eq. 1), forces and stress as exact
                    derivatives (reverse-mode autograd of PyTorch CPU), the
                    rows b_i = dV_i/dtheta (Sec. II.D, eq. 10), the grade
                    gamma_i = max_p |(b_i A^-1)_p| by an LU solve (Sec. II.D),
                    MaxVol row swaps (Sec. II.C) and the gradient of the
                    fitting objective (eq. 7).
* ``neighbors``  -- the neighborhoods of Sec. II.A by brute force over all
                    atoms and all periodic images (a plain C triple loop with
                    a NumPy twin for tiny inputs).
* ``al``         -- extrapolation-controlled runs (Sec. II.F, Sec. III.A):
                    velocity-Verlet MD graded at every step and the
                    spherical fragment around the atom of largest grade.
* ``fit``        -- the BFGS minimization of eq. 7 (Sec. II.B).

``mtp.cfg_rows`` gives the configuration-mode rows of Sec. II.C (sums of the
neighborhood rows).

Every function cites the passage it follows.  Readings of passages where the
paper is silent are listed in the module docstrings.
"""
