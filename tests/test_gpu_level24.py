"""Level 24 against the FP64 oracle: the staged contraction program (graph
values, trie walk and reverse pass as separate launches that pass per-
neighborhood state through memory), on the batched uneven workload of that
level (2 species, FCC alloy with at least 5 % vacancies, atom counts
log-uniform in [16, 4096], seeded teacher potential).

Small configurations are compared whole; the full 1,024-configuration batch
(about 7.5e5 atoms) is compared on sampled atoms, in the launch
configuration the benchmark times.  Bars: FP64 within 1e-10 relative
(norm-wise); mixed form with forces within 1e-4 eV/A."""
import numpy as np
import pytest

from oracle import mtp as om
from oracle import neighbors as onb
from paper_2304_13144_amd import api, synth
from tests.helpers import oracle_local_forces, rel_err

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
MIXED_FORCE_TOL = 1e-4


@pytest.fixture(scope="module")
def w24():
    if 24 not in api.compiled_levels():
        pytest.skip("level 24 not compiled into libmtp.so")
    w = synth.workload4()
    pot = om.Potential(w.level, w.n_types, w.r_min, w.r_cut)
    theta = synth.theta_teacher(4, w.n_types, pot.n_lin, pot.n_rad)
    m = api.Model.create(w.level, w.n_types, w.r_min, w.r_cut)
    m.set_params(theta)
    return w, pot, theta, m


def _np(t):
    return t.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_small_configurations_match_oracle(w24, precision):
    w, pot, theta, m = w24
    cfgs = sorted(w.configs, key=lambda c: c.n)[:3] + [sorted(w.configs, key=lambda c: c.n)[40]]
    b = api.Batch(cfgs)
    nb = api.Neighbors().build(m, b, max_nbrs=64)
    got = api.energy_forces_stress(m, b, nb, precision)
    E, F, S, V = (_np(got[k]) for k in ("energy", "forces", "stress", "site_e"))
    for k, c in enumerate(cfgs):
        sl = slice(b.cfg_off_host[k], b.cfg_off_host[k + 1])
        pairs = onb.neighbors(c.pos, c.cell, c.pbc, pot.r_cut)
        E_or, F_or, S_or, V_or = om.energy_forces_stress(pot, theta, c.pos, c.types, c.cell, pairs)
        ef = np.abs(F[sl] - F_or).max()
        print(f"{precision} config of {c.n} atoms: E {E[k]:.6f} vs {E_or:.6f}, |dF| {ef:.3g}, "
              f"site_e rel {rel_err(V[sl], V_or):.3g}, stress rel {rel_err(S[k], S_or):.3g}")
        if precision == "fp64":
            assert rel_err(V[sl], V_or) <= FP64_TOL
            assert abs(E[k] - E_or) <= FP64_TOL * max(abs(E_or), np.abs(V_or).sum())
            assert rel_err(F[sl], F_or) <= FP64_TOL
            assert rel_err(S[k], S_or) <= FP64_TOL
        else:
            assert ef <= MIXED_FORCE_TOL


def test_rows_match_oracle(w24):
    """b rows of the staged program: LINEAR (onehot, B_alpha) and FULL (the
    gauge-fixed theta columns, m = 1114) on a few atoms."""
    w, pot, theta, m = w24
    c = sorted(w.configs, key=lambda c: c.n)[1]
    b = api.Batch([c])
    nb = api.Neighbors().build(m, b, max_nbrs=64)
    pairs = onb.neighbors(c.pos, c.cell, c.pbc, pot.r_cut)
    atoms = [0, 3, c.n - 1]
    lin = _np(api.b_rows(m, b, nb, atoms, mode="linear"))
    lin_or = om.linear_rows(pot, theta, c.pos, c.types, c.cell, pairs, atoms=atoms)
    assert lin.shape == lin_or.shape
    assert rel_err(lin, lin_or) <= FP64_TOL
    keep = m.kept_columns()
    assert len(keep) == m.m("full") == 1114
    full = _np(api.b_rows(m, b, nb, atoms, mode="full"))
    full_or = om.b_rows(pot, theta, c.pos, c.types, c.cell, pairs, atoms=atoms)[:, keep]
    print(f"rows: linear rel {rel_err(lin, lin_or):.3g}, full rel {rel_err(full, full_or):.3g}")
    assert rel_err(full, full_or) <= FP64_TOL


def test_full_batch_sampled_atoms_match_oracle(w24):
    """The whole 1,024-configuration batch in one evaluation per form; forces of
    sampled atoms (from small, middle and large configurations) against the
    oracle's exact local forces, site energies of the same atoms, and the
    energy of the smallest configurations."""
    w, pot, theta, m = w24
    b = api.Batch(w.configs)
    nb = api.Neighbors().build(m, b, max_nbrs=64)
    sizes = np.array([c.n for c in w.configs])
    order = np.argsort(sizes, kind="stable")
    picks = [int(order[0]), int(order[len(order) // 2]), int(order[-1])]
    rng = np.random.default_rng(24)
    res = {p: {k: _np(v) for k, v in api.energy_forces_stress(m, b, nb, p).items()} for p in ("fp64", "mixed")}
    for k in picks:
        c = w.configs[k]
        atoms = np.sort(rng.choice(c.n, size=2, replace=False))
        F_or, _ = oracle_local_forces(pot, theta, c, atoms)
        pairs = onb.neighbors(c.pos, c.cell, c.pbc, pot.r_cut, atoms=atoms)
        _, _, _, V_all = om.energy_forces_stress(pot, theta, c.pos, c.types, c.cell, pairs)
        gi = b.cfg_off_host[k] + atoms
        f64, mix = res["fp64"], res["mixed"]
        print(f"config {k} ({c.n} atoms), atoms {atoms.tolist()}: FP64 F rel {rel_err(f64['forces'][gi], F_or):.3g}, "
              f"mixed |dF| {np.abs(mix['forces'][gi] - F_or).max():.3g}")
        assert rel_err(f64["forces"][gi], F_or) <= FP64_TOL
        assert rel_err(f64["site_e"][gi], V_all[atoms]) <= FP64_TOL
        assert np.abs(mix["forces"][gi] - F_or).max() <= MIXED_FORCE_TOL
        if c.n <= 24:
            pairs = onb.neighbors(c.pos, c.cell, c.pbc, pot.r_cut)
            E_or, _, _, V_or = om.energy_forces_stress(pot, theta, c.pos, c.types, c.cell, pairs)
            assert abs(f64["energy"][k] - E_or) <= FP64_TOL * np.abs(V_or).sum()


def test_backward_is_refused(w24):
    w, pot, theta, m = w24
    c = sorted(w.configs, key=lambda c: c.n)[0]
    b = api.Batch([c])
    nb = api.Neighbors().build(m, b, max_nbrs=64)
    import torch
    th = torch.tensor(theta, dtype=torch.float64, device="cuda", requires_grad=True)
    E, F, S = api.MTPEnergy.apply(th, m, b, nb, "fp64")
    with pytest.raises(api.MtpError):
        E.sum().backward()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_grades_at_m_1114_match_oracle(w24, precision):
    """Grades of level-24 rows against a seeded well-conditioned active-set
    matrix of full size (m = 1114, beyond the register and int8 forms: the
    FP64 product with rows staged through LDS grades both forms), oracle rows
    solved by LU (Sec. II.D) for a few atoms; the preselection of the same
    call counts the atoms above 2 exactly as the oracle's grades do."""
    w, pot, theta, m = w24
    keep = m.kept_columns()
    mm = len(keep)
    assert mm == m.m("full") == 1114
    rng = np.random.default_rng(1114)
    A = np.eye(mm) * 4.0 + rng.normal(size=(mm, mm)) / np.sqrt(mm)   # kappa ~ 10
    A *= np.exp(rng.uniform(-3, 3, size=mm))[None, :]                 # columns of very different scale
    m.set_active_set("full", A)
    c = sorted(w.configs, key=lambda c: c.n)[2]
    b = api.Batch([c])
    nb = api.Neighbors().build(m, b, max_nbrs=64)
    out = api.evaluate(m, b, nb, precision, "full", gamma_save=2.0)
    atoms = [0, c.n // 2, c.n - 1]
    pairs = onb.neighbors(c.pos, c.cell, c.pbc, pot.r_cut)
    rows = om.b_rows(pot, theta, c.pos, c.types, c.cell, pairs, atoms=atoms)[:, keep]
    g_or, am_or, _ = om.grades(rows, A)
    g = _np(out["gamma"])[atoms]
    am = _np(out["argmax"])[atoms]
    print(f"{precision}: gamma {g} vs {g_or}")
    tol = 1e-10 if precision == "fp64" else 1e-5
    assert np.all(np.abs(g - g_or) <= tol * np.maximum(1.0, g_or))
    assert np.array_equal(am, am_or)


def test_grade_rows_at_m_1114_equals_the_evaluation(w24):
    """mtp_grade_rows at level 24 (m = 1114, rows staged through LDS): the
    evaluation's own rows, laid out column-major with zero padding to a
    multiple of 32 columns, grade bitwise as the evaluation does."""
    import torch
    w, pot, theta, m = w24
    mm = m.m("full")
    rng = np.random.default_rng(1115)
    A = np.eye(mm) * 4.0 + rng.normal(size=(mm, mm)) / np.sqrt(mm)
    m.set_active_set("full", A)
    c = sorted(w.configs, key=lambda c: c.n)[1]
    b = api.Batch([c])
    nb = api.Neighbors().build(m, b, max_nbrs=64)
    g = api.grade(m, b, nb, "fp64", "full", rows=True)
    rows = g["rows"]
    cm = torch.zeros(api.row_stride(mm, "fp64"), c.n, dtype=torch.float64, device=rows.device)
    cm[:mm] = rows.t()
    out = api.grade_rows(m, cm.contiguous(), "fp64", "full")
    torch.cuda.synchronize()
    assert np.array_equal(_np(out["gamma"]), _np(g["gamma"]))
    assert np.array_equal(_np(out["argmax"]), _np(g["argmax"]))
