"""Batching, graph capture and the autotuner (GPU).

* a batch of uneven configurations in one launch equals per-configuration runs;
* a captured step replayed several times, with eager work in between, equals
  the eager step every time (bitwise in FP64);
* the autotuner's choice agrees with every other schedule to rounding (the
  lanes change the summation order of the moments);
* a checked replay raises when its neighbor build overflows."""
import numpy as np
import pytest
import torch

from paper_2304_13144_amd import api, synth
from tests.helpers import active_rows, potential, theta_for

pytestmark = pytest.mark.gpu


def _uneven_configs(n_cfg=12, seed=90):
    r = np.random.default_rng(seed)
    sizes = np.round(np.exp(r.uniform(np.log(16), np.log(600), n_cfg))).astype(int)
    return [synth._vacancy_config(r, "fcc", int(n), 0.06, 2, 0.08, 0.0, vac_min_frac=0.05) for n in sizes]


def _model16():
    w = synth.workload2(reps=(4, 4, 4))
    pot = potential(w)
    m = api.Model.create(16, 2, 2.0, 5.0)
    m.set_params(theta_for(2, pot))
    keep = m.kept_columns()
    m.set_active_set("full", active_rows(2, "full")[:, keep])
    m.set_active_set("linear", active_rows(2, "linear"))
    return m


def _np(out):
    return {k: v.detach().cpu().numpy().copy() for k, v in out.items() if v is not None}


def test_uneven_batch_equals_single_configs():
    m = _model16()
    cfgs = _uneven_configs()
    b = api.Batch(cfgs)
    nb = api.Neighbors().build(m, b, max_nbrs=96)
    together = _np(api.evaluate(m, b, nb, "fp64", "full"))
    for k, cfg in enumerate(cfgs):
        bk = api.Batch([cfg])
        nk = api.Neighbors().build(m, bk, max_nbrs=96)
        one = _np(api.evaluate(m, bk, nk, "fp64", "full"))
        sl = slice(b.cfg_off_host[k], b.cfg_off_host[k + 1])
        assert np.array_equal(together["forces"][sl], one["forces"])
        assert np.array_equal(together["gamma"][sl], one["gamma"])
        assert np.array_equal(together["site_e"][sl], one["site_e"])
        assert together["energy"][k] == pytest.approx(one["energy"][0], rel=1e-13, abs=1e-12)
        assert np.allclose(together["stress"][k], one["stress"][0], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("precision,passes", [("fp64", 1), ("mixed", 1), ("fp64", 3)])
def test_graph_replay_equals_eager(precision, passes):
    m = _model16()
    b = api.Batch(_uneven_configs(8, seed=91))
    nb = api.Neighbors().build(m, b, max_nbrs=96)
    eager = _np(api.evaluate(m, b, nb, precision, "full"))
    step = api.CapturedStep(m, b, nb, precision, "full", max_nbrs=96, passes=passes)
    for rep in range(3):
        # eager work and a synchronisation between replays
        other = _np(api.evaluate(m, b, nb, precision, "linear"))
        torch.cuda.synchronize()
        got = _np(step.replay())
        torch.cuda.synchronize()
        for k in ("energy", "forces", "stress", "site_e", "gamma", "argmax"):
            assert np.array_equal(got[k], eager[k]), (rep, k)
        assert np.isfinite(other["gamma"]).all()


def test_autotuner_choice_agrees_to_rounding():
    m = _model16()
    b = api.Batch([synth.workload2(reps=(8, 8, 8)).configs[0]])
    nb = api.Neighbors().build(m, b, max_nbrs=64)
    lanes = api.tune(m, b, nb, "fp64", "full")
    assert lanes[0] in (2, 4, 8) and lanes[1] in (2, 4, 8)
    tuned = _np(api.evaluate(m, b, nb, "fp64", "full"))
    import os
    for k in ("2", "4", "8"):
        os.environ["MTP_LANES"] = k
        try:
            other = _np(api.evaluate(m, b, nb, "fp64", "full"))
        finally:
            del os.environ["MTP_LANES"]
        # lanes change the summation tree of the moments: equal to rounding
        assert np.allclose(other["forces"], tuned["forces"], rtol=0, atol=1e-10 * np.abs(tuned["forces"]).max())
        assert np.allclose(other["gamma"], tuned["gamma"], rtol=1e-9)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_grade_forms_agree_and_tuner_picks_one(precision):
    """Every kernel form of the grade product gives the same grades to the
    precision's bound, and the tuner returns one of the forms."""
    import os
    m = _model16()
    b = api.Batch([synth.workload2(reps=(6, 6, 6)).configs[0]])
    nb = api.Neighbors().build(m, b, max_nbrs=64)
    forms = {"1": "fp64-registers", "2": "fp64-lds", "4": "fp64-registers-32-row-blocks", "5": "fp64-k-outer",
             "6": "fp64-k-outer-2-step-chunks"} | \
        ({"3": "int8-slices"} if precision == "mixed" else {})
    lanes = api.tune(m, b, nb, precision, "full", with_grade=True)   # first: the lanes stay fixed below
    assert lanes[2] in forms.values()
    got = {}
    for k in forms:
        os.environ["MTP_GRADE_FORM"] = k
        try:
            got[k] = _np(api.evaluate(m, b, nb, precision, "full"))["gamma"]
        finally:
            del os.environ["MTP_GRADE_FORM"]
    # the FP64 products differ only in summation order
    assert np.allclose(got["2"], got["1"], rtol=1e-12, atol=0)
    assert np.allclose(got["4"], got["1"], rtol=1e-12, atol=0)
    assert np.allclose(got["5"], got["1"], rtol=1e-12, atol=0)
    assert np.array_equal(got["6"], got["5"])   # the same products in the same order
    if precision == "mixed":
        assert np.all(np.abs(got["3"] - got["1"]) <= 1e-5 * np.maximum(1.0, got["1"]))
    assert np.array_equal(_np(api.evaluate(m, b, nb, precision, "full"))["gamma"],
                          got[{v: k for k, v in forms.items()}[lanes[2]]])


def test_graph_replay_reports_neighbor_overflow_after_atoms_move():
    """The captured step rebuilds the lists on every replay; when the atoms of
    the captured positions are squeezed so that a neighborhood exceeds
    max_nbrs, the replay raises MTP_E_CAPACITY (the build's status words are
    read after every checked replay)."""
    m = _model16()
    cfg = synth.workload2(reps=(4, 4, 4)).configs[0]
    b = api.Batch([cfg])
    nb = api.Neighbors().build(m, b, max_nbrs=48)
    step = api.CapturedStep(m, b, nb, "fp64", "full", max_nbrs=48)
    step.replay()                              # 28-38 neighbors: fine
    with torch.no_grad():
        b.pos.mul_(0.8)                        # positions move in place (same buffer as captured)
        b.cells.mul_(0.8)
    torch.cuda.synchronize()
    with pytest.raises(api.MtpError) as e:
        step.replay()
    assert e.value.status == "MTP_E_CAPACITY"


def test_sustained_mfma_rate_is_plausible():
    """The measurement helper behind the roofline's sustained-rate figure:
    positive, below the nominal dense peaks (FP64 78.6 TFLOP/s, int8 5.0
    POP/s) with a small margin, and bad arguments are refused."""
    f64 = api.mfma_rate("f64", 2000)
    i8 = api.mfma_rate("i8", 2000)
    print(f"sustained MFMA: FP64 {f64:.1f} TFLOP/s, int8 {i8:.0f} TOP/s")
    assert 1.0 < f64 < 78.6 * 1.05
    assert 50.0 < i8 < 5000.0 * 1.05
    with pytest.raises(api.MtpError):
        api.mfma_rate("f64", 0)


@pytest.mark.parametrize("lanes", ["2", "4", "8"])
@pytest.mark.parametrize("mode", ["full", "linear"])
def test_fp64_rows_in_the_pair_pass_equal_the_row_blocks(mode, lanes):
    """An FP64 evaluation with forces computes the rows' remaining parts in the
    pair-gradient pass itself; mtp_grade (no forces) computes them in row
    blocks of their own.  Same sums in the same order: the grades are bitwise
    equal, and the forces are bitwise those of the launch without rows."""
    import os
    m = _model16()
    if mode == "linear":
        m.set_active_set("linear", active_rows(2, "linear"))
    b = api.Batch([synth.workload2(reps=(6, 6, 6)).configs[0]])
    nb = api.Neighbors().build(m, b, max_nbrs=64)
    os.environ["MTP_LANES"] = lanes
    try:
        fused = _np(api.evaluate(m, b, nb, "fp64", mode))
        sep = _np(api.grade(m, b, nb, "fp64", mode, rows=True))
        plain = _np(api.energy_forces_stress(m, b, nb, "fp64"))
    finally:
        del os.environ["MTP_LANES"]
    assert np.array_equal(fused["gamma"], sep["gamma"])
    assert np.array_equal(fused["argmax"], sep["argmax"])
    for key in ("forces", "energy", "stress"):
        assert np.array_equal(fused[key], plain[key]), key


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("mode", ["full", "linear"])
def test_grade_rows_equals_the_evaluation(precision, mode):
    """mtp_grade_rows on the evaluation's own rows (laid out column-major and
    zero-padded as the evaluation does) runs the same kernel form: the grades
    and argmax are bitwise those of the fused evaluation.  A row stride short
    of the padded length is refused."""
    m = _model16()
    if mode == "linear":
        m.set_active_set("linear", active_rows(2, "linear"))
    b = api.Batch([synth.workload2(reps=(6, 6, 6)).configs[0]])
    nb = api.Neighbors().build(m, b, max_nbrs=64)
    g = api.grade(m, b, nb, precision, mode, rows=True)
    rows = g["rows"]
    n, mm = rows.shape
    ldb = api.row_stride(mm, precision)
    cm = torch.zeros(ldb, n, dtype=torch.float64, device=rows.device)
    cm[:mm] = rows.t()
    out = api.grade_rows(m, cm.contiguous(), precision, mode)
    torch.cuda.synchronize()
    assert np.array_equal(out["gamma"].cpu().numpy(), g["gamma"].cpu().numpy())
    assert np.array_equal(out["argmax"].cpu().numpy(), g["argmax"].cpu().numpy())
    with pytest.raises(api.MtpError):
        api.grade_rows(m, cm[: mm // 32 * 32].contiguous(), precision, mode)
