"""GPU parity of the neighborhood active-learning path (Sec. II.C-II.E) on
the BCC snapshot workload: grades of every neighborhood of a snapshot,
preselection gamma > gamma_save = 2, and FP64 MaxVol swaps of the selected
rows into A, with A carried from snapshot to snapshot -- against the FP64
oracle step by step; and the grades of the full 1,048,576-atom snapshot at
its largest displacement on sampled atoms."""
import numpy as np
import pytest
import torch

from oracle import mtp as om
from oracle import neighbors as onb
from paper_2304_13144_amd import api, synth
from tests.helpers import active_rows, potential, theta_for

pytestmark = pytest.mark.gpu

GAMMA_SAVE = 2.0


def _model(w, theta):
    """Library model with the workload's active sets; FULL columns are the
    library's own gauge choice (kept columns), applied to the oracle rows too."""
    m = api.Model.create(w.level, w.n_types, w.r_min, w.r_cut)
    m.set_params(theta)
    keep = m.kept_columns()
    m.set_active_set("full", active_rows(5, "full")[:, keep])
    m.set_active_set("linear", active_rows(5, "linear"))
    return m, keep


def _grade_bound(C, A, Ainv_gpu, g_or):
    """|gamma_gpu - gamma| allowed per row: 1e-10 relative plus the first-order
    effect of the library's rank-1-updated inverse, C (A Ainv_gpu - I)."""
    E = np.abs(A @ Ainv_gpu - np.eye(A.shape[0])).max()
    return 1e-10 * np.maximum(1.0, g_or) + np.abs(C).sum(axis=1) * E


def _oracle_rows(pot, theta, cfg, mode, keep, atoms=None):
    pairs = onb.neighbors(cfg.pos, cfg.cell, cfg.pbc, pot.r_cut, atoms=atoms)
    if mode == "full":
        return om.b_rows(pot, theta, cfg.pos, cfg.types, cfg.cell, pairs, atoms=atoms)[:, keep]
    return om.linear_rows(pot, theta, cfg.pos, cfg.types, cfg.cell, pairs, atoms=atoms)


@pytest.mark.parametrize("mode", ["full", "linear"])
def test_active_learning_snapshots_match_oracle(mode):
    """Four snapshots of a 4x4x8 BCC cell (256 atoms) at sigma 0.05 .. 0.40:
    gamma within 1e-10 relative (plus, after swaps, the first-order effect of
    the rank-1-updated inverse), the same preselected atoms (rows within that
    bound of 2 excepted), the same MaxVol swap sequence and the same A after
    every snapshot."""
    w = synth.workload5(reps=(4, 4, 8))
    pot = potential(w)
    theta = theta_for(5, pot)
    m, keep = _model(w, theta)
    A = (active_rows(5, "full")[:, keep] if mode == "full" else active_rows(5, "linear")).copy()
    total_swaps = 0
    for k in (0, 7, 13, 19):
        cfg = synth.workload5_snapshot(k, reps=(4, 4, 8))
        print(f"snapshot {k} mode {mode}", flush=True)
        b = api.Batch([cfg])
        nb = api.Neighbors().build(m, b, max_nbrs=64)
        g = api.grade(m, b, nb, "fp64", mode)["gamma"].cpu().numpy()
        rows = _oracle_rows(pot, theta, cfg, mode, keep)
        g_or, _, C = om.grades(rows, A)
        _, Ainv_gpu = m.get_active_set(mode)
        bound = _grade_bound(C, A, Ainv_gpu.cpu().numpy(), g_or)
        print(f"  max |dgamma| {np.abs(g - g_or).max():.3e}, bound {bound.min():.3e}..{bound.max():.3e}", flush=True)
        assert (np.abs(g - g_or) <= bound).all()
        idx, cnt = api.select(torch.as_tensor(g).cuda(), GAMMA_SAVE)
        sel = idx[: int(cnt.item())].cpu().numpy()
        sel_or = np.nonzero(g_or > GAMMA_SAVE)[0]
        clear = np.abs(g_or - GAMMA_SAVE) > bound
        assert set(sel[clear[sel]]) == set(sel_or[clear[sel_or]])
        if len(sel_or) == 0:
            continue
        # candidates: the oracle's rows of the selected atoms on both sides (the
        # swap sequence then depends only on the two MaxVol implementations)
        A, _, swaps = om.maxvol(A, rows[sel_or], threshold=1.001)
        cand = torch.as_tensor(rows[sel_or]).cuda().contiguous()
        sc, sj = api.maxvol_update(m, mode, cand, threshold=1.001)
        assert [(int(a), int(c)) for a, c in zip(sc, sj)] == [(i, j) for i, j, _ in swaps]
        A_gpu, _ = m.get_active_set(mode)
        assert np.array_equal(A_gpu.cpu().numpy(), A)
        total_swaps += len(swaps)
    assert total_swaps > 0   # the loop exercised MaxVol


def test_active_learning_gpu_rows_feed_maxvol():
    """The whole GPU loop on one snapshot: rows of the selected atoms from the
    library (not the oracle) swapped into A; every swap multiplies |det A| by
    more than the threshold, and after the loop no selected row has a grade
    above it."""
    w = synth.workload5(reps=(4, 4, 8))
    pot = potential(w)
    theta = theta_for(5, pot)
    m, keep = _model(w, theta)
    cfg = synth.workload5_snapshot(19, reps=(4, 4, 8))
    b = api.Batch([cfg])
    nb = api.Neighbors().build(m, b, max_nbrs=64)
    g = api.grade(m, b, nb, "fp64", "full")["gamma"]
    idx, cnt = api.select(g, GAMMA_SAVE)
    sel = idx[: int(cnt.item())]
    assert len(sel) > 0
    rows = api.b_rows(m, b, nb, sel, "full")
    A0, _ = m.get_active_set("full")
    d0 = np.linalg.slogdet(A0.cpu().numpy())[1]
    cand = rows.clone().contiguous()
    sc, sj = api.maxvol_update(m, "full", cand, threshold=1.001)
    A1, _ = m.get_active_set("full")
    d1 = np.linalg.slogdet(A1.cpu().numpy())[1]
    assert len(sc) > 0 and d1 > d0 + len(sc) * np.log(1.001) - 1e-9
    g_after = om.grades(rows.cpu().numpy(), A1.cpu().numpy())[0]
    assert g_after.max() <= 1.001 + 1e-9


def test_full_size_snapshot_grades_sampled():
    """The 1,048,576-atom BCC snapshot at sigma = 0.40: neighbor lists and
    grades (FULL and LINEAR, FP64) of 24 sampled atoms against the oracle."""
    w = synth.workload5()
    pot = potential(w)
    theta = theta_for(5, pot)
    m, keep = _model(w, theta)
    cfg = synth.workload5_snapshot(19)
    print(f"full-size snapshot: {cfg.n} atoms", flush=True)
    b = api.Batch([cfg])
    nb = api.Neighbors().build(m, b, max_nbrs=64)
    atoms = np.sort(np.random.default_rng(19).choice(cfg.n, 24, replace=False))
    count, j, sh = (t.cpu().numpy() for t in nb.export(b))
    pairs = onb.neighbors(cfg.pos, cfg.cell, cfg.pbc, w.r_cut, atoms=atoms)
    for a in atoms:
        got = sorted((int(j[a, q]),) + tuple(int(v) for v in sh[a, q]) for q in range(int(count[a])))
        want = sorted((int(jj),) + tuple(int(v) for v in s) for ii, jj, s in zip(pairs.i, pairs.j, pairs.shift)
                      if int(ii) == a)
        assert got == want
    for mode in ("full", "linear"):
        g = api.grade(m, b, nb, "fp64", mode)["gamma"].cpu().numpy()
        A = active_rows(5, "full")[:, keep] if mode == "full" else active_rows(5, "linear")
        g_or = om.grades(_oracle_rows(pot, theta, cfg, mode, keep, atoms=atoms), A)[0]
        # this active set (16 near-identical sigma = 0.05 copies) is ill-conditioned: the
        # FP64 bar is relaxed to kappa(A) 1e-15 (column-equilibrated kappa) when that is larger
        kappa = np.linalg.cond(A / np.abs(A).max(axis=0))
        tol = max(1e-10, kappa * 1e-15)
        err = np.abs(g[atoms] - g_or).max() / max(1.0, np.abs(g_or).max())
        print(f"{mode}: kappa {kappa:.3e}, max gamma {np.abs(g_or).max():.3e}, rel err {err:.3e}, tol {tol:.3e}")
        assert err <= tol
        idx, cnt = api.select(torch.as_tensor(g).cuda(), GAMMA_SAVE)
        want = np.nonzero(g > GAMMA_SAVE)[0]
        assert int(cnt.item()) == len(want)
        assert np.array_equal(idx[:len(want)].cpu().numpy(), want)
        # the preselection fused into the grade (past 1024 blocks of rows: the
        # block counts are scanned first), with and without a capacity
        for cap in (None, 1000):
            out = api.evaluate(m, b, nb, "fp64", mode, gamma_save=GAMMA_SAVE, capacity=cap,
                               out={"gamma": torch.empty(cfg.n, dtype=torch.float64, device=b.device)})
            assert np.array_equal(out["gamma"].cpu().numpy(), g)
            k = len(want) if cap is None else min(cap, len(want))
            assert int(out["sel_count"].item()) == k
            assert np.array_equal(out["sel_idx"][:k].cpu().numpy(), want[:k])
