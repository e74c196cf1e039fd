"""GPU parity of the extrapolation-controlled run pieces through the C ABI:
the spherical fragment around the atom of largest grade and velocity-Verlet
MD graded at every step, against oracle.al.

Bars: fragments bit-exact as sets of (source atom, shift) in the same order,
positions within 1e-12 A; MD positions within 1e-9 A and velocities within
1e-11 A/fs after the run, gamma(cfg) per step within 1e-9 relative, the
same saved steps (steps whose gamma lies within 1e-7 of a threshold are not
compared) and the same stopping step.
"""
import numpy as np
import pytest
import torch

from oracle import al as oal
from paper_2304_13144_amd import api, synth
from tests.helpers import active_rows, potential, theta_for

pytestmark = pytest.mark.gpu


def _cut_cases():
    slab = synth.fcc111_slab()
    thin = synth.cfg_pool(1, 3, stream=5)[2]          # a cell thinner than the cutoff: many images
    bulk = synth.workload1().configs[0]
    return [("slab_1620", slab, 8.0), ("thin_cell", thin, 8.0), ("bcc128", bulk, 6.5)]


@pytest.mark.parametrize("case", ["slab_1620", "thin_cell", "bcc128"])
def test_cut_neighborhood_matches_oracle(case):
    name, cfg, cutoff = [c for c in _cut_cases() if c[0] == case][0]
    grades = np.random.default_rng(61).random(cfg.n)
    center, src, shift, pos, types = oal.extrapolative_neighborhood(cfg.pos, cfg.types, cfg.cell, cfg.pbc, grades,
                                                                    cutoff)
    b = api.Batch([cfg])
    out = api.cut_neighborhood(b, torch.as_tensor(grades), cutoff)
    print(f"{name}: {len(src)} atoms around {center}")
    assert out["center"] == center
    got = list(zip(out["src"].cpu().numpy().tolist(), map(tuple, out["shift"].cpu().numpy().tolist())))
    want = list(zip(src.tolist(), map(tuple, shift.tolist())))
    assert got == want
    assert np.abs(out["pos"].cpu().numpy() - pos).max() <= 1e-12
    assert np.array_equal(out["types"].cpu().numpy(), types)


def test_cut_neighborhood_capacity():
    cfg = synth.workload1().configs[0]
    grades = np.zeros(cfg.n)
    grades[5] = 1.0
    b = api.Batch([cfg])
    out = api.cut_neighborhood(b, torch.as_tensor(grades), 6.5, capacity=10)
    _, src, shift, _, _ = oal.extrapolative_neighborhood(cfg.pos, cfg.types, cfg.cell, cfg.pbc, grades, 6.5)
    assert len(out["src"]) == 10
    assert out["src"].cpu().numpy().tolist() == src[:10].tolist()


def _md_setup():
    """Workload 1 with xi scaled by 1e-4 (forces of ~1 eV/A instead of ~1e4: E
    is linear in xi) and the LINEAR grade, whose rows (onehot, B_alpha) do
    not depend on xi, so that workload 1's LINEAR active set stays valid."""
    w = synth.workload1()
    pot = potential(w)
    theta = theta_for(1, pot).copy()
    theta[:pot.n_types + pot.n_lin] *= 1e-4
    m = api.Model.create(w.level, w.n_types, w.r_min, w.r_cut)
    m.set_params(theta)
    keep = m.kept_columns()
    A = active_rows(1, "linear")
    m.set_active_set("linear", A)
    cfg = w.configs[0]
    vel = np.random.default_rng(62).normal(0.0, 0.01, cfg.pos.shape)
    return w, pot, theta, m, keep, A, cfg, vel


def _gpu_md(m, cfg, vel, n_steps, save, brk):
    b = api.Batch([cfg])
    nb = api.Neighbors()
    v = torch.as_tensor(vel).cuda().contiguous()
    r = api.md_run(m, b, nb, v, [63.546], 1.0, n_steps, "fp64", "linear", save, brk)
    return r, b.pos.cpu().numpy(), v.cpu().numpy()


def _same_saved(got, want, gam, save, brk):
    near = {k for k, g in enumerate(gam) if min(abs(g - save), abs(g - brk)) <= 1e-7 * max(1.0, g)}
    return [k for k in got if k not in near] == [k for k in want if k not in near]


def test_md_run_matches_oracle():
    w, pot, theta, m, keep, A, cfg, vel = _md_setup()
    probe = oal.md_verlet(pot, theta, cfg.pos, vel, cfg.types, cfg.cell, cfg.pbc, [63.546], 1.0, 6, A, "linear",
                          keep, 1e300, 1e300)
    save = float(np.median(probe["gamma"]))     # about half of the steps are recorded
    want = oal.md_verlet(pot, theta, cfg.pos, vel, cfg.types, cfg.cell, cfg.pbc, [63.546], 1.0, 6, A, "linear", keep,
                         save, 1e300)
    r, pos, v = _gpu_md(m, cfg, vel, 6, save, 1e300)
    print(f"gamma(cfg) per step: {np.round(want['gamma'], 4).tolist()}, saved {want['saved']}")
    assert r["steps"] == want["steps"] == 6
    assert np.abs(pos - want["pos"]).max() <= 1e-9
    assert np.abs(v - want["vel"]).max() <= 1e-11
    assert np.allclose(r["gamma"], want["gamma"], rtol=1e-9, atol=0)
    assert _same_saved(r["saved"], want["saved"], want["gamma"], save, 1e300)


def test_md_run_stops_above_gamma_break():
    w, pot, theta, m, keep, A, cfg, vel = _md_setup()
    probe = oal.md_verlet(pot, theta, cfg.pos, vel, cfg.types, cfg.cell, cfg.pbc, [63.546], 1.0, 6, A, "linear",
                          keep, 1e300, 1e300)
    g = probe["gamma"]
    k = int(np.argmax(g[1:])) + 1                   # stop at the step of the largest grade
    brk = 0.5 * (g[k] + max(g[:k]))
    if not max(g[:k]) < brk < g[k]:
        pytest.skip("the grades do not rise above their earlier maximum")
    want = oal.md_verlet(pot, theta, cfg.pos, vel, cfg.types, cfg.cell, cfg.pbc, [63.546], 1.0, 6, A, "linear", keep,
                         1e300, brk)
    r, pos, v = _gpu_md(m, cfg, vel, 6, 1e300, brk)
    assert want["steps"] == k - 1 and r["steps"] == k - 1
    assert len(r["gamma"]) == k + 1
    assert np.abs(pos - want["pos"]).max() <= 1e-9


def test_md_run_without_steps_grades_the_start():
    w, pot, theta, m, keep, A, cfg, vel = _md_setup()
    r, pos, v = _gpu_md(m, cfg, vel, 0, 1e300, 1e300)
    want = oal.md_verlet(pot, theta, cfg.pos, vel, cfg.types, cfg.cell, cfg.pbc, [63.546], 1.0, 0, A, "linear",
                         keep, 1e300, 1e300)
    assert r["steps"] == 0 and len(r["gamma"]) == 1
    assert np.allclose(r["gamma"], want["gamma"], rtol=1e-9, atol=0)
    assert np.array_equal(pos, cfg.pos) and np.array_equal(v, vel)


def test_cut_neighborhood_zero_capacity():
    cfg = synth.workload1().configs[0]
    b = api.Batch([cfg])
    out = api.cut_neighborhood(b, torch.zeros(cfg.n, dtype=torch.float64), 6.5, capacity=0)
    assert len(out["src"]) == 0 and out["center"] == 0



def test_relax_fire_matches_oracle():
    """FIRE from a displaced workload-1 cell (xi scaled as in the MD tests):
    the same positions after 25 steps (no convergence in that time, so both
    sides take every step) and the same grades and saved steps."""
    w, pot, theta, m, keep, A, cfg, _ = _md_setup()
    start = cfg.pos + np.random.default_rng(63).normal(0.0, 0.03, cfg.pos.shape)
    probe = oal.relax_fire(pot, theta, start, cfg.types, cfg.cell, cfg.pbc, [63.546], 1.0, 10.0, 0.0, 25, A, "linear",
                           keep, 1e300, 1e300)
    save = float(np.median(probe["gamma"]))
    want = oal.relax_fire(pot, theta, start, cfg.types, cfg.cell, cfg.pbc, [63.546], 1.0, 10.0, 0.0, 25, A, "linear",
                          keep, save, 1e300)
    b = api.Batch([synth.Config(start, cfg.types, cfg.cell, cfg.pbc)])
    r = api.relax_fire(m, b, api.Neighbors(), [63.546], 1.0, 10.0, 0.0, 25, "fp64", "linear", save, 1e300)
    pos = b.pos.cpu().numpy()
    print(f"gamma(cfg): {np.round(want['gamma'][:6], 4).tolist()} ..., saved {len(want['saved'])}, "
          f"moved {np.abs(want['pos'] - start).max():.3g} A")
    assert r["steps"] == want["steps"] == 25 and not r["converged"]
    assert np.abs(pos - want["pos"]).max() <= 1e-9
    assert np.allclose(r["gamma"], want["gamma"], rtol=1e-9, atol=0)
    assert _same_saved(r["saved"], want["saved"], want["gamma"], save, 1e300)
