"""GPU parity of the BFGS fitting of eq. 7 (Sec. II.B) through the C ABI,
against oracle.fit (the same algorithm on the oracle's loss and gradient).

A teacher-student case at level 8: targets (E, F, S) of six small cells from
the oracle with the teacher's theta; both sides start from the same
perturbed theta.  Bars: the loss history of the first five iterations within
1e-7 relative (both follow the same steps in FP64), the loss after 15
iterations within 1e-3 relative of the oracle's and below 1 % of the start,
theta after the first iteration within 1e-8 relative.
"""
import numpy as np
import pytest

from oracle import fit as ofit
from oracle import mtp as om
from oracle import neighbors as onb
from paper_2304_13144_amd import api, synth
from tests.helpers import potential, theta_for

pytestmark = pytest.mark.gpu


def _case():
    w = synth.workload1()
    pot = potential(w)
    teacher = theta_for(1, pot).copy()
    teacher[:pot.n_types + pot.n_lin] *= 1e-3
    cfgs = synth.cfg_pool(1, 6, stream=6)
    confs, targets = [], []
    for c in cfgs:
        pairs = onb.neighbors(c.pos, c.cell, c.pbc, pot.r_cut)
        confs.append((c.pos, c.types, c.cell, pairs))
        E, F, S, _ = om.energy_forces_stress(pot, teacher, c.pos, c.types, c.cell, pairs)
        targets.append((E, F, S))
    start = teacher + np.random.default_rng(71).normal(0, 0.01, teacher.shape) * (np.abs(teacher) + 1e-3)
    return w, pot, cfgs, confs, targets, start


def test_fit_bfgs_matches_oracle():
    w, pot, cfgs, confs, targets, start = _case()
    th_or, hist_or = ofit.fit(pot, start, confs, targets, 1.0, 0.01, 0.001, 15)
    th1_or, _ = ofit.fit(pot, start, confs, targets, 1.0, 0.01, 0.001, 1)
    m = api.Model.create(w.level, w.n_types, w.r_min, w.r_cut)
    b = api.Batch(cfgs)
    nb = api.Neighbors().build(m, b, max_nbrs=64)
    E_t = np.array([t[0] for t in targets])
    F_t = np.concatenate([t[1] for t in targets])
    S_t = np.stack([t[2] for t in targets])
    m.set_params(start)
    th1, _ = api.fit_bfgs(m, b, nb, E_t, F_t, S_t, 1.0, 0.01, 0.001, max_iter=1)
    assert np.abs(th1 - th1_or).max() <= 1e-8 * np.abs(th1_or).max()
    m.set_params(start)
    th, hist = api.fit_bfgs(m, b, nb, E_t, F_t, S_t, 1.0, 0.01, 0.001, max_iter=15)
    print("loss gpu   ", np.array2string(hist[:6], precision=8))
    print("loss oracle", np.array2string(np.array(hist_or[:6]), precision=8), "... final", hist[-1], hist_or[-1])
    assert len(hist) == len(hist_or)
    assert np.allclose(hist[:6], hist_or[:6], rtol=1e-7, atol=0)
    assert abs(hist[-1] - hist_or[-1]) <= 1e-3 * hist_or[-1]
    assert hist[-1] < 0.01 * hist[0]
    assert np.array_equal(m.theta(), th)


def test_fit_bfgs_with_parameter_scale_matches_oracle():
    """The same case with a diagonal scale (the parameters' typical sizes)."""
    w, pot, cfgs, confs, targets, start = _case()
    scale = np.abs(start) + 1e-3
    th_or, hist_or = ofit.fit(pot, start, confs, targets, 1.0, 0.01, 0.001, 10, scale=scale)
    m = api.Model.create(w.level, w.n_types, w.r_min, w.r_cut)
    b = api.Batch(cfgs)
    nb = api.Neighbors().build(m, b, max_nbrs=64)
    m.set_params(start)
    th, hist = api.fit_bfgs(m, b, nb, np.array([t[0] for t in targets]), np.concatenate([t[1] for t in targets]),
                            np.stack([t[2] for t in targets]), 1.0, 0.01, 0.001, max_iter=10, scale=scale)
    print("loss gpu   ", np.array2string(hist, precision=8))
    print("loss oracle", np.array2string(np.array(hist_or), precision=8))
    assert len(hist) == len(hist_or)
    assert np.allclose(hist[:6], hist_or[:6], rtol=1e-7, atol=0)
    assert abs(hist[-1] - hist_or[-1]) <= 1e-3 * hist_or[-1]
