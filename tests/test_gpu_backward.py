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


def test_backward_uses_the_theta_of_its_own_forward():
    """Two forwards at different theta, then the backward of the first: the
    gradient is the first theta's (the model is loaded with it again), equal
    to a single forward + backward at that theta."""
    pot, cfgs, theta_t, theta_s = _case(8, 2, 3, seed=81)
    m = api.Model.create(8, 2, pot.r_min, pot.r_cut)
    b = api.Batch(cfgs)
    m.set_params(theta_s)
    nb = api.Neighbors().build(m, b, max_nbrs=128)

    def loss_of(E, F, S):
        return (E ** 2).sum() + W_F * (F ** 2).sum() + W_S * (S ** 2).sum()

    t1 = torch.tensor(theta_s, dtype=torch.float64, device="cuda", requires_grad=True)
    ref = loss_of(*api.MTPEnergy.apply(t1, m, b, nb, "fp64"))
    ref.backward()
    want = t1.grad.clone()
    t1.grad = None
    l1 = loss_of(*api.MTPEnergy.apply(t1, m, b, nb, "fp64"))
    t2 = torch.tensor(theta_t, dtype=torch.float64, device="cuda", requires_grad=True)
    l2 = loss_of(*api.MTPEnergy.apply(t2, m, b, nb, "fp64"))
    l1.backward()
    assert torch.equal(t1.grad, want)
    l2.backward()
    assert not torch.equal(t2.grad, want)
    # a rebuild between forward and backward is refused
    l3 = loss_of(*api.MTPEnergy.apply(t1, m, b, nb, "fp64"))
    nb.build(m, b, max_nbrs=128)
    with pytest.raises(RuntimeError):
        l3.backward()


@pytest.mark.skipif(20 not in api.compiled_levels(), reason="level 20 not compiled into libmtp.so")
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_full_training_batch_gradient_on_sampled_configs(precision):
    """The level-20 training batch at full size (512 configurations of 8-256
    atoms, 3 species), in the launch configuration the benchmark times: the
    loss holds terms of six sampled configurations only (the upstream
    gradients of the others are zero), so the oracle computes it on those six."""
    w = synth.workload3()
    pot = om.Potential(w.level, w.n_types, w.r_min, w.r_cut)
    theta_t = synth.theta_teacher(3, w.n_types, pot.n_lin, pot.n_rad)
    theta_s = theta_t * (1.0 + 0.05 * np.random.default_rng(3).normal(size=theta_t.shape))
    pick = np.sort(np.random.default_rng(5).choice(len(w.configs), 6, replace=False))
    sub = [w.configs[k] for k in pick]
    targets, geo = _oracle_targets(pot, sub, theta_t)
    L_or, g_or = om.loss_and_grad(pot, theta_s, geo, targets, W_E, W_F, W_S)
    m = api.Model.create(w.level, w.n_types, w.r_min, w.r_cut)
    m.set_params(theta_s)
    b = api.Batch(w.configs)
    nb = api.Neighbors().build(m, b, max_nbrs=96)
    theta = torch.tensor(theta_s, dtype=torch.float64, device="cuda", requires_grad=True)
    E, F, S = api.MTPEnergy.apply(theta, m, b, nb, precision)
    off = b.cfg_off_host
    mask_c = torch.zeros(len(w.configs), dtype=torch.float64, device="cuda")
    mask_c[torch.as_tensor(pick)] = 1.0
    mask_a = torch.zeros(b.n_atoms, dtype=torch.float64, device="cuda")
    Et = torch.zeros(len(w.configs), dtype=torch.float64, device="cuda")
    Ft = torch.zeros((b.n_atoms, 3), dtype=torch.float64, device="cuda")
    St = torch.zeros((len(w.configs), 3, 3), dtype=torch.float64, device="cuda")
    for k, t in zip(pick, targets):
        mask_a[off[k]:off[k + 1]] = 1.0
        Et[k] = t[0]
        Ft[off[k]:off[k + 1]] = torch.as_tensor(t[1])
        St[k] = torch.as_tensor(t[2])
    loss = (W_E * (mask_c * (E - Et) ** 2).sum() + W_F * (mask_a[:, None] * (F - Ft) ** 2).sum()
            + W_S * (mask_c[:, None, None] * (S - St) ** 2).sum())
    loss.backward()
    g = theta.grad.cpu().numpy()
    err = rel_err(g, g_or)
    print(f"{precision}: configurations {list(pick)}, loss gpu {loss.item():.6g} oracle {L_or:.6g}, grad rel err {err:.3g}")
    assert abs(loss.item() - L_or) <= (1e-10 if precision == "fp64" else 1e-4) * abs(L_or)
    assert err <= (1e-9 if precision == "fp64" else 1e-3)
