"""GPU parity of the training gradient (eq. 7) against the oracle.

The oracle differentiates the plain loss with reverse-mode autograd through
exact forces and stresses (itself pinned to central differences in
test_oracle_pins.py).  Bars: FP64 within 1e-9 relative (norm-wise); FP32
within 1e-3 relative."""
import numpy as np
import pytest
import torch

from oracle import mtp as om
from oracle import neighbors as onb
from paper_2304_13144_amd import api, synth
from tests.helpers import rel_err

pytestmark = pytest.mark.gpu

W_E, W_F, W_S = 1.0, 0.01, 0.001


def _case(level, n_types, n_cfg, seed, max_atoms=40):
    """Small strained multi-lattice configurations in the style of workload 3."""
    r = np.random.default_rng([seed, 1])
    cfgs = []
    kinds = ["bcc", "fcc", "hcp"]
    for k in range(n_cfg):
        n = int(r.integers(8, max_atoms + 1))
        cfgs.append(synth._vacancy_config(r, kinds[k % 3], n, 0.06, n_types, 0.15, 0.03))
    pot = om.Potential(level, n_types, 2.0, 5.5 if level >= 16 else 5.0)
    theta_t = np.random.default_rng([seed, 2]).normal(0, 0.1, pot.n_theta) * 0.3
    theta_s = np.random.default_rng([seed, 3]).normal(0, 0.1, pot.n_theta) * 0.3
    return pot, cfgs, theta_t, theta_s


def _oracle_targets(pot, cfgs, theta):
    out, geo = [], []
    for c in cfgs:
        pairs = onb.neighbors(c.pos, c.cell, c.pbc, pot.r_cut)
        E, F, S, _ = om.energy_forces_stress(pot, theta, c.pos, c.types, c.cell, pairs)
        out.append((E, F, S))
        geo.append((c.pos, c.types, c.cell, pairs))
    return out, geo


@pytest.mark.parametrize("level,n_types,precision", [(8, 2, "fp64"), (12, 3, "fp64"), (16, 2, "fp64"),
                                                     (16, 2, "mixed"), (20, 3, "fp64"), (20, 3, "mixed")])
def test_loss_gradient_matches_oracle(level, n_types, precision):
    if level not in api.compiled_levels():
        pytest.skip(f"level {level} not compiled into libmtp.so")
    pot, cfgs, theta_t, theta_s = _case(level, n_types, 4, seed=40 + level)
    targets, geo = _oracle_targets(pot, cfgs, theta_t)
    L_or, g_or = om.loss_and_grad(pot, theta_s, geo, targets, W_E, W_F, W_S)

    m = api.Model.create(level, n_types, pot.r_min, pot.r_cut)
    b = api.Batch(cfgs)
    m.set_params(theta_s)
    nb = api.Neighbors().build(m, b, max_nbrs=128)
    theta = torch.tensor(theta_s, dtype=torch.float64, device="cuda", requires_grad=True)
    E, F, S = api.MTPEnergy.apply(theta, m, b, nb, precision)
    Et = torch.tensor([t[0] for t in targets], dtype=torch.float64, device="cuda")
    Ft = torch.tensor(np.concatenate([t[1] for t in targets]), dtype=torch.float64, device="cuda")
    St = torch.tensor(np.stack([t[2] for t in targets]), dtype=torch.float64, device="cuda")
    loss = W_E * ((E - Et) ** 2).sum() + W_F * ((F - Ft) ** 2).sum() + W_S * ((S - St) ** 2).sum()
    loss.backward()
    g = theta.grad.cpu().numpy()
    print(f"level {level} {precision}: loss gpu {loss.item():.6g} oracle {L_or:.6g}, grad rel err {rel_err(g, g_or):.3g}")
    tol = 1e-9 if precision == "fp64" else 1e-3
    assert abs(loss.item() - L_or) <= (1e-10 if precision == "fp64" else 1e-4) * abs(L_or)
    assert rel_err(g, g_or) <= tol


def test_backward_parts_energy_only_equals_sum_of_rows():
    """With only dL/dE = 1 the gradient is sum_i dV_i/dtheta = the sum of the full b rows."""
    pot, cfgs, _, theta_s = _case(8, 2, 2, seed=77)
    m = api.Model.create(8, 2, pot.r_min, pot.r_cut)
    m.set_params(theta_s)
    b = api.Batch(cfgs)
    nb = api.Neighbors().build(m, b, max_nbrs=128)
    g = api.efs_backward(m, b, nb, gE=np.ones(len(cfgs))).cpu().numpy()
    rows = []
    for c in cfgs:
        pairs = onb.neighbors(c.pos, c.cell, c.pbc, pot.r_cut)
        rows.append(om.b_rows(pot, theta_s, c.pos, c.types, c.cell, pairs))
    want = np.concatenate(rows).sum(axis=0)
    assert rel_err(g, want) <= 1e-10
