"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bars (written per test): FP64 form within 1e-10 relative (norm-wise: max
|diff| / max |oracle|); mixed form with forces within 1e-4 eV/A and gamma
within 1e-5 max(1, gamma); neighbor lists bit-exact as sets.
"""
import os

import numpy as np
import pytest
import torch

from oracle import mtp as om
from oracle import neighbors as onb
from paper_2304_13144_amd import api, synth
from tests.helpers import active_rows, fp64_gamma_tol, kappa_eq, oracle_local_forces, potential, rel_err, theta_for

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
MIXED_GAMMA_TOL = 1e-5      # |dgamma| <= 1e-5 max(1, gamma)
MIXED_FORCE_TOL = 1e-4      # eV/A


def _model(w, theta, modes=("full", "linear")):
    m = api.Model.create(w.level, w.n_types, w.r_min, w.r_cut)
    m.set_params(theta)
    keep = m.kept_columns()
    if "full" in modes:
        m.set_active_set("full", active_rows(w.wid, "full")[:, keep])
    if "linear" in modes:
        m.set_active_set("linear", active_rows(w.wid, "linear"))
    return m, keep


def _nbr_sets(count, j, sh, atoms):
    out = {}
    for a in atoms:
        c = int(count[a])
        out[a] = sorted((int(j[a, q]),) + tuple(int(v) for v in sh[a, q]) for q in range(c))
    return out


def _oracle_sets(pairs, atoms):
    out = {a: [] for a in atoms}
    for i, j, s in zip(pairs.i, pairs.j, pairs.shift):
        if int(i) in out:
            out[int(i)].append((int(j),) + tuple(int(v) for v in s))
    return {a: sorted(v) for a, v in out.items()}


# ------------------------------------------------------------ neighbors ----
def _configs_for_neighbors():
    r = np.random.default_rng(5)
    out = []
    w1 = synth.workload1()
    out.append(("bcc128", w1.configs[0], 1))
    tri = synth.Config(np.array([[0.1, 0.2, 0.3], [1.7, 1.1, 0.9], [0.4, 2.5, 1.9]]),
                       np.array([0, 1, 1], np.int32),
                       np.array([[3.1, 0, 0], [0.9, 2.9, 0], [0.4, -0.7, 3.3]]))
    out.append(("triclinic_small", tri, 2))
    slab = synth.Config(r.random((40, 3)) @ np.diag([9.0, 9.5, 20.0]), r.integers(0, 2, 40).astype(np.int32),
                        np.diag([9.0, 9.5, 20.0]), (True, True, False))
    out.append(("slab_xy", slab, 2))
    return out


@pytest.mark.parametrize("case", ["bcc128", "triclinic_small", "slab_xy"])
def test_neighbors_match_oracle(case):
    name, cfg, nt = [c for c in _configs_for_neighbors() if c[0] == case][0]
    m = api.Model.create(8, nt, 2.0, 5.0)
    b = api.Batch([cfg])
    nb = api.Neighbors().build(m, b, max_nbrs=256)
    count, j, sh = (t.cpu().numpy() for t in nb.export(b))
    pairs = onb.neighbors(cfg.pos, cfg.cell, cfg.pbc, 5.0)
    atoms = list(range(cfg.n))
    assert _nbr_sets(count, j, sh, atoms) == _oracle_sets(pairs, atoms)


def test_neighbors_batched_configs_match_oracle():
    cfgs = [c for _, c, _ in _configs_for_neighbors()]
    m = api.Model.create(8, 2, 2.0, 5.0)
    b = api.Batch(cfgs)
    nb = api.Neighbors().build(m, b, max_nbrs=256)
    count, j, sh = (t.cpu().numpy() for t in nb.export(b))
    off = b.cfg_off_host
    for k, cfg in enumerate(cfgs):
        pairs = onb.neighbors(cfg.pos, cfg.cell, cfg.pbc, 5.0)
        atoms = list(range(cfg.n))
        got = _nbr_sets(count, j - off[k], sh, [a + off[k] for a in atoms])
        got = {a - off[k]: v for a, v in got.items()}
        assert got == _oracle_sets(pairs, atoms)


def test_neighbors_full_size_workload2_sampled():
    w = synth.workload2()
    cfg = w.configs[0]
    m = api.Model.create(16, 2, 2.0, 5.0)
    b = api.Batch([cfg])
    nb = api.Neighbors().build(m, b, max_nbrs=64)
    count, j, sh = (t.cpu().numpy() for t in nb.export(b))
    atoms = list(np.random.default_rng(6).choice(cfg.n, 48, replace=False)) + [0, cfg.n - 1]
    pairs = onb.neighbors(cfg.pos, cfg.cell, cfg.pbc, 5.0, atoms=atoms)
    assert _nbr_sets(count, j, sh, atoms) == _oracle_sets(pairs, atoms)


def test_neighbors_dense_cluster_mixed_bins():
    """A dense cluster in a sparse periodic box: bins next to the cluster have
    more candidates than one register window holds (the two-sweep path),
    the others take the one-window path; lists must match the oracle and be
    symmetric: (i, j, n) present iff (j, i, -n) is."""
    r = np.random.default_rng(11)
    dense = r.random((600, 3)) * 10.0
    sparse = r.random((100, 3)) * 20.0
    pos = np.vstack([dense, sparse])
    cfg = synth.Config(pos, r.integers(0, 2, len(pos)).astype(np.int32), np.diag([20.0, 20.0, 20.0]))
    m = api.Model.create(8, 2, 2.0, 5.0)
    b = api.Batch([cfg])
    nb = api.Neighbors().build(m, b, max_nbrs=512)
    count, j, sh = (t.cpu().numpy() for t in nb.export(b))
    atoms = list(range(cfg.n))
    got = _nbr_sets(count, j, sh, atoms)
    assert got == _oracle_sets(onb.neighbors(cfg.pos, cfg.cell, cfg.pbc, 5.0), atoms)
    directed = {(a,) + e for a, v in got.items() for e in v}
    assert all((e[1], e[0], -e[2], -e[3], -e[4]) in directed for e in directed)


def test_neighbor_capacity_and_overlap_are_reported():
    w = synth.workload1()
    m = api.Model.create(8, 1, 2.0, 5.0)
    b = api.Batch(w.configs)
    with pytest.raises(api.MtpError) as e:
        api.Neighbors().build(m, b, max_nbrs=8)
    assert e.value.status == "MTP_E_CAPACITY"
    cfg = w.configs[0]
    pos = cfg.pos.copy()
    pos[1] = pos[0]
    b2 = api.Batch([synth.Config(pos, cfg.types, cfg.cell)])
    with pytest.raises(api.MtpError) as e:
        api.Neighbors().build(m, b2, max_nbrs=64)
    assert e.value.status == "MTP_E_OVERLAP"


# ---------------------------------------------------------------- EFS ------
def _efs_case(w, cfg, theta, precision, lanes=None, monkeypatch=None):
    m = api.Model.create(w.level, w.n_types, w.r_min, w.r_cut)
    m.set_params(theta)
    b = api.Batch([cfg])
    nb = api.Neighbors().build(m, b, max_nbrs=64)
    out = api.energy_forces_stress(m, b, nb, precision)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def test_efs_fp64_workload1_matches_oracle():
    w = synth.workload1()
    pot = potential(w)
    theta = theta_for(1, pot)
    cfg = w.configs[0]
    pairs = onb.neighbors(cfg.pos, cfg.cell, cfg.pbc, w.r_cut)
    E, F, S, V = om.energy_forces_stress(pot, theta, cfg.pos, cfg.types, cfg.cell, pairs)
    g = _efs_case(w, cfg, theta, "fp64")
    assert rel_err(g["energy"][0], E) <= FP64_TOL
    assert rel_err(g["site_e"], V) <= FP64_TOL
    assert rel_err(g["forces"], F) <= FP64_TOL
    assert rel_err(g["stress"][0], S) <= FP64_TOL


@pytest.mark.parametrize("lanes", ["2", "4", "8"])
def test_efs_fp64_level16_two_species_small(lanes, monkeypatch):
    monkeypatch.setenv("MTP_LANES", lanes)
    w = synth.workload2(reps=(4, 4, 4))
    pot = potential(w)
    theta = theta_for(2, pot)
    cfg = w.configs[0]
    pairs = onb.neighbors(cfg.pos, cfg.cell, cfg.pbc, w.r_cut)
    E, F, S, V = om.energy_forces_stress(pot, theta, cfg.pos, cfg.types, cfg.cell, pairs)
    g = _efs_case(w, cfg, theta, "fp64")
    assert rel_err(g["energy"][0], E) <= FP64_TOL
    assert rel_err(g["site_e"], V) <= FP64_TOL
    assert rel_err(g["forces"], F) <= FP64_TOL
    assert rel_err(g["stress"][0], S) <= FP64_TOL


def test_efs_mixed_level16_two_species_small():
    w = synth.workload2(reps=(4, 4, 4))
    pot = potential(w)
    theta = theta_for(2, pot)
    cfg = w.configs[0]
    pairs = onb.neighbors(cfg.pos, cfg.cell, cfg.pbc, w.r_cut)
    E, F, S, V = om.energy_forces_stress(pot, theta, cfg.pos, cfg.types, cfg.cell, pairs)
    g = _efs_case(w, cfg, theta, "mixed")
    print("mixed errors: E %.3g  F %.3g eV/A  S %.3g" % (abs(g["energy"][0] - E), np.abs(g["forces"] - F).max(),
                                                         np.abs(g["stress"][0] - S).max()))
    assert np.abs(g["forces"] - F).max() <= 1e-4
    assert abs(g["energy"][0] - E) <= 1e-6 * max(1.0, abs(E)) * cfg.n
    assert np.abs(g["stress"][0] - S).max() <= 1e-5 * max(1.0, np.abs(S).max())


def test_efs_full_size_workload2_sampled():
    """Full 16,384-atom alloy in the benchmark's launch configuration; oracle on
    sampled atoms (site energies and forces), plus properties of the sums."""
    w = synth.workload2()
    pot = potential(w)
    theta = theta_for(2, pot)
    cfg = w.configs[0]
    atoms = np.sort(np.random.default_rng(7).choice(cfg.n, 24, replace=False))
    Fo, Vo = oracle_local_forces(pot, theta, cfg, atoms)
    for prec, ftol in (("fp64", None), ("mixed", 1e-4)):
        g = _efs_case(w, cfg, theta, prec)
        if ftol is None:
            assert rel_err(g["site_e"][atoms], Vo) <= FP64_TOL
            assert rel_err(g["forces"][atoms], Fo) <= FP64_TOL
            assert abs(g["energy"][0] - g["site_e"].sum()) <= 1e-12 * np.abs(g["site_e"]).sum()
        else:
            assert np.abs(g["forces"][atoms] - Fo).max() <= ftol
        assert np.abs(g["forces"].sum(axis=0)).max() <= 1e-6 * np.abs(g["forces"]).max() * cfg.n ** 0.5
        assert np.abs(g["stress"][0] - g["stress"][0].T).max() <= 1e-8 * np.abs(g["stress"][0]).max()


@pytest.mark.skipif(20 not in api.compiled_levels(), reason="level 20 not compiled into libmtp.so")
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_efs_level20_three_species_uneven_batch(precision):
    """Six configurations of the level-20, three-species training workload
    (uneven sizes, BCC/FCC/HCP, strained, vacancies) in one batch."""
    w = synth.workload3(n_cfg=6)
    pot = potential(w)
    theta = theta_for(3, pot)
    m = api.Model.create(w.level, w.n_types, w.r_min, w.r_cut)
    m.set_params(theta)
    b = api.Batch(w.configs)
    nb = api.Neighbors().build(m, b, max_nbrs=128)
    g = {k: v.cpu().numpy() for k, v in api.energy_forces_stress(m, b, nb, precision).items()}
    off = b.cfg_off_host
    for k, cfg in enumerate(w.configs):
        pairs = onb.neighbors(cfg.pos, cfg.cell, cfg.pbc, w.r_cut)
        E, F, S, V = om.energy_forces_stress(pot, theta, cfg.pos, cfg.types, cfg.cell, pairs)
        Fg = g["forces"][off[k]:off[k + 1]]
        if precision == "fp64":
            assert rel_err(g["energy"][k], E) <= FP64_TOL
            assert rel_err(g["site_e"][off[k]:off[k + 1]], V) <= FP64_TOL
            assert rel_err(Fg, F) <= FP64_TOL
            assert rel_err(g["stress"][k], S) <= FP64_TOL
        else:
            assert np.abs(Fg - F).max() <= 1e-4


def test_efs_fp64_bitwise_deterministic():
    w = synth.workload2(reps=(6, 6, 6))
    pot = potential(w)
    theta = theta_for(2, pot)
    a = _efs_case(w, w.configs[0], theta, "fp64")
    b = _efs_case(w, w.configs[0], theta, "fp64")
    for k in ("energy", "forces", "stress", "site_e"):
        assert np.array_equal(a[k], b[k]), k


def test_batched_equals_single_configs():
    w = synth.workload1()
    pot = potential(w)
    theta = theta_for(1, pot)
    cfgs = synth.workload1_training(3)
    m = api.Model.create(w.level, w.n_types, w.r_min, w.r_cut)
    m.set_params(theta)
    b = api.Batch(cfgs)
    nb = api.Neighbors().build(m, b, max_nbrs=64)
    together = {k: v.cpu().numpy() for k, v in api.energy_forces_stress(m, b, nb, "fp64").items()}
    for k, cfg in enumerate(cfgs):
        one = _efs_case(w, cfg, theta, "fp64")
        sl = slice(b.cfg_off_host[k], b.cfg_off_host[k + 1])
        assert np.array_equal(together["forces"][sl], one["forces"])
        assert np.array_equal(together["site_e"][sl], one["site_e"])
        assert together["energy"][k] == pytest.approx(one["energy"][0], rel=1e-14)


# --------------------------------------------------------------- grades ----
def _grade_case(wid, w, cfg, precision, mode, form=None):
    """form: a kernel form of the grade product (MTP_GRADE_FORM), else the
    library's choice"""
    pot = potential(w)
    theta = theta_for(wid, pot)
    m, keep = _model(w, theta)
    b = api.Batch([cfg])
    nb = api.Neighbors().build(m, b, max_nbrs=64)
    if form is not None:
        os.environ["MTP_GRADE_FORM"] = form
    try:
        out = api.grade(m, b, nb, precision, mode, rows=True)
    finally:
        os.environ.pop("MTP_GRADE_FORM", None)
    torch.cuda.synchronize()
    return pot, theta, keep, {k: v.cpu().numpy() for k, v in out.items()}


# the library's form for each precision, and the other FP64 forms (4: rows in
# registers in blocks of 32 rows, 5 and 6: k outermost)
@pytest.mark.parametrize("precision,form", [("fp64", None), ("mixed", None), ("fp64", "4"), ("fp64", "5"),
                                            ("fp64", "6")])
@pytest.mark.parametrize("mode", ["full", "linear"])
def test_grade_workload1(mode, precision, form):
    w = synth.workload1()
    cfg = w.configs[0]
    pot, theta, keep, g = _grade_case(1, w, cfg, precision, mode, form)
    pairs = onb.neighbors(cfg.pos, cfg.cell, cfg.pbc, w.r_cut)
    if mode == "full":
        assert list(keep) == om.kept_columns(pot, theta)
        rows = om.b_rows(pot, theta, cfg.pos, cfg.types, cfg.cell, pairs)[:, keep]
        A = active_rows(1, "full")[:, keep]
    else:
        rows = om.linear_rows(pot, theta, cfg.pos, cfg.types, cfg.cell, pairs)
        A = active_rows(1, "linear")
    assert rel_err(g["rows"], rows) <= FP64_TOL
    gam, am, _ = om.grades(rows, A)
    tol = fp64_gamma_tol(A)
    err = np.abs(g["gamma"] - gam) / np.maximum(1.0, gam)
    print(f"{precision}/{mode}: kappa {kappa_eq(A):.3g}, gamma rel err {rel_err(g['gamma'], gam):.3g}, "
          f"per-atom {err.max():.3g}")
    if precision == "fp64":
        assert rel_err(g["gamma"], gam) <= tol
    else:
        assert err.max() <= MIXED_GAMMA_TOL
    clear = np.sort(np.abs(_c(rows, A)), axis=1)
    unique = clear[:, -1] - clear[:, -2] > (1e-8 if precision == "fp64" else 1e-5) * clear[:, -1]
    assert np.array_equal(g["argmax"][unique], am[unique])


def _c(rows, A):
    return om.grades(rows, A)[2]


def _fp32_row_emulation(rows, A):
    """Oracle grade of the oracle's rows rounded to FP32 and solved in FP64:
    the error that FP32 rows alone force, whatever the product does."""
    g0 = om.grades(rows, A)[0]
    g1 = om.grades(rows.astype(np.float32).astype(np.float64), A)[0]
    return float((np.abs(g1 - g0) / np.maximum(1.0, g0)).max())


@pytest.mark.parametrize("precision,mode,form", [("fp64", "full", None), ("fp64", "linear", None),
                                                 ("mixed", "full", None), ("mixed", "linear", None),
                                                 ("fp64", "full", "5"), ("fp64", "linear", "5"),
                                                 ("fp64", "full", "6"), ("fp64", "linear", "6")])
def test_grade_level16_two_species_small(precision, mode, form):
    w = synth.workload2(reps=(4, 4, 4))
    cfg = w.configs[0]
    pot, theta, keep, g = _grade_case(2, w, cfg, precision, mode, form)
    pairs = onb.neighbors(cfg.pos, cfg.cell, cfg.pbc, w.r_cut)
    if mode == "full":
        rows = om.b_rows(pot, theta, cfg.pos, cfg.types, cfg.cell, pairs)[:, keep]
        A = active_rows(2, "full")[:, keep]
    else:
        rows = om.linear_rows(pot, theta, cfg.pos, cfg.types, cfg.cell, pairs)
        A = active_rows(2, "linear")
    gam, _, _ = om.grades(rows, A)
    err = np.abs(g["gamma"] - gam) / np.maximum(1.0, gam)
    emul = _fp32_row_emulation(rows, A)
    print(f"{precision}/{mode} gamma: max rel err {err.max():.3g} (FP32-row emulation {emul:.3g}), "
          f"gamma range {gam.min():.3g}..{gam.max():.3g}")
    if precision == "fp64":
        assert rel_err(g["rows"], rows) <= FP64_TOL
        tol = fp64_gamma_tol(A)
        print(f"kappa {kappa_eq(A):.3g}, norm-wise gamma rel err {rel_err(g['gamma'], gam):.3g}, tol {tol:.3g}")
        assert rel_err(g["gamma"], gam) <= tol
    else:
        # rows in FP64 (the grade's rows are FP64 in both forms), the product
        # from int8 digits with exact accumulation: gamma within 1e-5 max(1, gamma)
        assert rel_err(g["rows"], rows) <= FP64_TOL
        assert err.max() <= MIXED_GAMMA_TOL


def test_grade_full_size_workload2_sampled():
    """The benchmark's configuration (16,384-atom alloy, level 16, FULL, m = 212)
    in the benchmark's launch configuration (one fused evaluation with
    forces, stress and grades): rows, grades and forces of 96 sampled atoms
    against the oracle, in both forms."""
    w = synth.workload2()
    pot = potential(w)
    theta = theta_for(2, pot)
    cfg = w.configs[0]
    m, keep = _model(w, theta, modes=("full",))
    b = api.Batch([cfg])
    nb = api.Neighbors().build(m, b, max_nbrs=64)
    atoms = np.sort(np.random.default_rng(17).choice(cfg.n, 96, replace=False))
    pairs = onb.neighbors(cfg.pos, cfg.cell, cfg.pbc, w.r_cut, atoms=atoms)
    rows = om.b_rows(pot, theta, cfg.pos, cfg.types, cfg.cell, pairs, atoms=atoms)[:, keep]
    A = active_rows(2, "full")[:, keep]
    gam, am, C = om.grades(rows, A)
    Fo, _ = oracle_local_forces(pot, theta, cfg, atoms)
    for prec in ("fp64", "mixed"):
        out = {k: v.cpu().numpy() for k, v in api.evaluate(m, b, nb, prec, "full").items()}
        g = api.grade(m, b, nb, prec, "full", rows=True)
        assert np.array_equal(g["gamma"].cpu().numpy(), out["gamma"])
        assert rel_err(g["rows"].cpu().numpy()[atoms], rows) <= FP64_TOL
        err = np.abs(out["gamma"][atoms] - gam) / np.maximum(1.0, gam)
        ferr = np.abs(out["forces"][atoms] - Fo).max()
        print(f"{prec}: kappa {kappa_eq(A):.3g}, gamma {gam.min():.3g}..{gam.max():.3g}, max rel err "
              f"{err.max():.3g} (norm-wise {rel_err(out['gamma'][atoms], gam):.3g}), forces {ferr:.3g} eV/A")
        if prec == "fp64":
            assert rel_err(out["gamma"][atoms], gam) <= fp64_gamma_tol(A)
            assert rel_err(out["forces"][atoms], Fo) <= FP64_TOL
        else:
            assert err.max() <= MIXED_GAMMA_TOL
            assert ferr <= MIXED_FORCE_TOL
        srt = np.sort(np.abs(C), axis=1)
        clear = srt[:, -1] - srt[:, -2] > 1e-6 * srt[:, -1]
        assert np.array_equal(out["argmax"][atoms][clear], am[clear])


def test_gamma_is_one_on_active_rows():
    """Rows of the active set itself: gamma = 1 (the grade of an interpolation point)."""
    w = synth.workload1()
    pot = potential(w)
    theta = theta_for(1, pot)
    m, keep = _model(w, theta)
    A = torch.as_tensor(active_rows(1, "full")[:, keep]).cuda()
    # grade the active rows directly through the GEMM path: use MaxVol with no swap
    cand = A.clone().contiguous()
    sc, sj = api.maxvol_update(m, "full", cand, threshold=1.0 + 1e-9)
    assert len(sc) == 0


# -------------------------------------------------------------- MaxVol -----
def test_maxvol_matches_oracle_swap_sequence():
    w = synth.workload1()
    pot = potential(w)
    theta = theta_for(1, pot)
    m, keep = _model(w, theta)
    cfg = synth.workload1_training(1)[0]
    cfg = synth.Config(cfg.pos + np.random.default_rng(8).normal(0, 0.15, cfg.pos.shape), cfg.types, cfg.cell)
    pairs = onb.neighbors(cfg.pos, cfg.cell, cfg.pbc, w.r_cut)
    rows = om.b_rows(pot, theta, cfg.pos, cfg.types, cfg.cell, pairs)[:, keep]
    A0 = active_rows(1, "full")[:, keep]
    A_or, cand_or, swaps = om.maxvol(A0, rows, threshold=1.001)
    cand = torch.as_tensor(rows).cuda().contiguous()
    sc, sj = api.maxvol_update(m, "full", cand, threshold=1.001)
    assert [(int(a), int(b)) for a, b in zip(sc, sj)] == [(i, j) for i, j, _ in swaps]
    A_gpu, Ainv = m.get_active_set("full")
    assert np.array_equal(A_gpu.cpu().numpy(), A_or)
    assert np.array_equal(cand.cpu().numpy(), cand_or)
    assert rel_err(Ainv.cpu().numpy() @ A_or, np.eye(A_or.shape[0])) <= 1e-6


@pytest.mark.parametrize("case", ["workload2_full", "workload1_full", "pivoting", "singular"])
def test_active_set_inverse_matches_oracle_lu(case):
    """A^-1 by the multi-block Gauss-Jordan inverse against the oracle's LU
    solve of I = C A (Sec. II.C: A is the active set's matrix), row by row
    (row k of A^-1 carries 1 / (scale of column k of A)) within
    kappa_eq(A) m 1e-15, kappa_eq the condition number of A with unit
    max-abs columns; a singular A is refused."""
    w = synth.workload2() if case == "workload2_full" else synth.workload1()
    theta = theta_for(w.wid, potential(w))
    m, keep = _model(w, theta, modes=())
    if case in ("workload2_full", "workload1_full"):
        A = active_rows(w.wid, "full")[:, keep]
    else:
        k = len(keep)
        rng = np.random.default_rng(31)
        A = rng.normal(size=(k, k))
        A[np.arange(k), np.arange(k)] = 0.0          # every step has to pivot
        A[: k // 2] *= 1e-3                           # rows of very different scale
        if case == "singular":
            A[5] = 0.0                                # exactly singular: the last pivot is 0
    if case == "singular":
        with pytest.raises(api.MtpError):
            m.set_active_set("full", A)
        return
    m.set_active_set("full", A)
    _, Ainv = m.get_active_set("full")
    _, _, inv_or = om.grades(np.eye(A.shape[0]), A)
    tol = kappa_eq(A) * 1e-15 * A.shape[0]
    diff = np.abs(Ainv.cpu().numpy() - inv_or).max(axis=1) / np.abs(inv_or).max(axis=1)
    print(f"{case}: m = {A.shape[0]}, kappa_eq {kappa_eq(A):.3g}, worst row rel err {diff.max():.3g} (bar {tol:.3g})")
    assert diff.max() <= tol


@pytest.mark.parametrize("n,shift,cap", [(100000, 0.0, None), (1048577, 5.0, None), (300000, 5.0, 1000),
                                         (7, 0.0, None)])
def test_select_matches_numpy(n, shift, cap):
    """Indices with gamma > 2 in ascending order: few, all (past the block
    size, one more than 2^20), a capacity below the count, a tiny input."""
    g = torch.as_tensor(np.random.default_rng(9).exponential(1.0, n) + shift).cuda()
    idx, cnt = api.select(g, 2.0, capacity=cap)
    want = np.nonzero(g.cpu().numpy() > 2.0)[0]
    k = len(want) if cap is None else min(cap, len(want))
    assert int(cnt.item()) == k
    assert np.array_equal(idx[:k].cpu().numpy(), want[:k])


@pytest.mark.parametrize("precision,reps,q,cap", [("fp64", (16, 16, 16), 0.5, None), ("mixed", (16, 16, 16), 0.9, 100),
                                                  ("fp64", (5, 4, 3), 0.3, None), ("fp64", (5, 4, 3), 1.0, None)])
def test_evaluate_select_fused(precision, reps, q, cap):
    """Preselection fused into the evaluation (per-block counts written by the
    grade kernel): the grades equal mtp_grade's bit for bit and the indices
    are those with gamma above the threshold, ascending (a quantile of the
    grades as threshold; a capacity below the count; a ragged 240-atom cell;
    nothing selected)."""
    w = synth.workload2(reps=reps)
    cfg = w.configs[0]
    pot = potential(w)
    theta = theta_for(2, pot)
    m, _ = _model(w, theta, modes=("full",))
    b = api.Batch([cfg])
    nb = api.Neighbors().build(m, b, max_nbrs=64)
    g_ref = api.grade(m, b, nb, precision, "full")["gamma"].cpu().numpy()
    thr = float(np.quantile(g_ref, q))
    out = api.evaluate(m, b, nb, precision, "full", gamma_save=thr, capacity=cap)
    g = out["gamma"].cpu().numpy()
    assert np.array_equal(g, g_ref)
    want = np.nonzero(g > thr)[0]
    k = len(want) if cap is None else min(cap, len(want))
    assert int(out["sel_count"].item()) == k
    assert np.array_equal(out["sel_idx"][:k].cpu().numpy(), want[:k])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("lanes", [2, 4, 8])
def test_evaluate_select_sums_bitwise(precision, lanes, monkeypatch):
    """With a preselection the force gather runs as blocks of the
    preselection's launch and the per-32-atom sum partials come from the
    pair-gradient kernel (one, two or four chunks per block at eight, four or
    two lanes per neighborhood): energies, forces, stresses, site energies and
    grades equal the plain evaluation's bit for bit, on an uneven batch whose
    configurations straddle the chunks."""
    monkeypatch.setenv("MTP_LANES", str(lanes))
    w = synth.workload2(reps=(5, 4, 3))
    pot = potential(w)
    theta = theta_for(2, pot)
    m, _ = _model(w, theta, modes=("full",))
    b = api.Batch([w.configs[0]] + list(synth.cfg_pool(2, 40, stream=3)))
    assert b.n_atoms % 32 != 0
    nb = api.Neighbors().build(m, b, max_nbrs=64)
    plain = api.evaluate(m, b, nb, precision, "full")
    fused = api.evaluate(m, b, nb, precision, "full", gamma_save=1.0)
    for k in ("energy", "forces", "stress", "site_e", "gamma", "argmax"):
        assert torch.equal(plain[k], fused[k]), k
    assert int(fused["sel_count"].item()) == int((plain["gamma"] > 1.0).sum().item())


def test_singular_active_set_is_reported():
    w = synth.workload1()
    m = api.Model.create(w.level, w.n_types, w.r_min, w.r_cut)
    m.set_params(theta_for(1, potential(w)))
    A = torch.zeros((m.m("linear"), m.m("linear")), dtype=torch.float64).cuda()
    with pytest.raises(api.MtpError) as e:
        m.set_active_set("linear", A)
    assert e.value.status == "MTP_E_SINGULAR"


def test_model_file_round_trip(tmp_path):
    w = synth.workload1()
    pot = potential(w)
    theta = theta_for(1, pot)
    m, keep = _model(w, theta)
    path = tmp_path / "w1.mtp"
    m.save(path)
    m2 = api.Model.load(path)
    b = api.Batch(w.configs)
    nb = api.Neighbors().build(m, b)
    g1 = api.grade(m, b, nb, "fp64", "full")["gamma"].cpu().numpy()
    g2 = api.grade(m2, b, nb, "fp64", "full")["gamma"].cpu().numpy()
    assert np.array_equal(g1, g2)
