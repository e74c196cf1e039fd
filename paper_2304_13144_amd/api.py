"""Python binding of libmtp over PyTorch device tensors.

PyTorch provides device memory and the current stream; every step of the
evaluation runs in the library's HIP kernels.  Names follow include/mtp.h.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import (MTP_FP64, MTP_GRADE_FULL, MTP_GRADE_FULL_CFG, MTP_GRADE_LINEAR, MTP_GRADE_LINEAR_CFG, MTP_MIXED,
                   MtpError, check)

PRECISION = {"fp64": MTP_FP64, "mixed": MTP_MIXED}
MODE = {"full": MTP_GRADE_FULL, "linear": MTP_GRADE_LINEAR, "full_cfg": MTP_GRADE_FULL_CFG,
        "linear_cfg": MTP_GRADE_LINEAR_CFG}


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _prec(p):
    return PRECISION[p] if isinstance(p, str) else int(p)


def _mode(g):
    return MODE[g] if isinstance(g, str) else int(g)


def _dev(device):
    return torch.device("cuda", device if isinstance(device, int) else torch.device(device).index or 0)


class Model:
    """An MTP (theta, basis, active sets) resident on one GPU."""

    def __init__(self, handle, device):
        self._h = handle
        self.device = _dev(device)

    @classmethod
    def load(cls, path, device=0):
        h = ctypes.c_void_p()
        dev = _dev(device)
        check(_lib.lib().mtp_load(str(path).encode(), dev.index, ctypes.byref(h)))
        return cls(h, dev)

    @classmethod
    def create(cls, level, n_types, r_min, r_cut, device=0):
        h = ctypes.c_void_p()
        dev = _dev(device)
        check(_lib.lib().mtp_create(level, n_types, float(r_min), float(r_cut), dev.index, ctypes.byref(h)))
        return cls(h, dev)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            try:
                _lib.lib().mtp_free(h)
            except Exception:
                pass
            self._h = None

    def save(self, path):
        check(_lib.lib().mtp_save(self._h, str(path).encode()))

    @property
    def info(self):
        i = _lib.ModelInfo()
        check(_lib.lib().mtp_info(self._h, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in _lib.ModelInfo._fields_}

    def m(self, mode):
        i = self.info
        return i["m_full"] if _mode(mode) in (MTP_GRADE_FULL, MTP_GRADE_FULL_CFG) else i["m_linear"]

    def theta(self):
        out = np.zeros(self.info["n_theta"])
        check(_lib.lib().mtp_get_params(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def set_params(self, theta):
        t = torch.as_tensor(theta, dtype=torch.float64).to(self.device).contiguous()
        assert t.numel() == self.info["n_theta"]
        check(_lib.lib().mtp_set_params(self._h, _p(t), _stream()))

    def kept_columns(self):
        out = np.zeros(self.info["m_full"], dtype=np.int32)
        check(_lib.lib().mtp_kept_columns(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def set_active_set(self, mode, A):
        m = self.m(mode)
        A = torch.as_tensor(A, dtype=torch.float64).to(self.device).contiguous()
        assert A.shape == (m, m), (A.shape, m)
        check(_lib.lib().mtp_set_active_set(self._h, _mode(mode), _p(A), _stream()))

    def get_active_set(self, mode):
        m = self.m(mode)
        A = torch.empty((m, m), dtype=torch.float64, device=self.device)
        Ai = torch.empty_like(A)
        check(_lib.lib().mtp_get_active_set(self._h, _mode(mode), _p(A), _p(Ai), _stream()))
        return A, Ai


class Batch:
    """Configurations packed for the library: device tensors + an mtp_system view."""

    def __init__(self, configs, device=0):
        dev = _dev(device)
        pos = np.concatenate([np.asarray(c.pos, dtype=np.float64) for c in configs]).reshape(-1, 3)
        types = np.concatenate([np.asarray(c.types, dtype=np.int32) for c in configs])
        cells = np.stack([np.asarray(c.cell, dtype=np.float64) for c in configs])
        pbc = np.array([[1 if p else 0 for p in c.pbc] for c in configs], dtype=np.uint8)
        off = np.zeros(len(configs) + 1, dtype=np.int64)
        np.cumsum([len(c.pos) for c in configs], out=off[1:])
        self.device = dev
        self.pos = torch.from_numpy(np.ascontiguousarray(pos)).to(dev)
        self.types = torch.from_numpy(types).to(dev)
        self.cells = torch.from_numpy(cells).to(dev)
        self.pbc = torch.from_numpy(pbc).to(dev)
        self.cfg_off = torch.from_numpy(off).to(dev)
        self.n_cfg = len(configs)
        self.n_atoms = int(off[-1])
        self.cfg_off_host = off

    def system(self):
        s = _lib.System()
        s.n_cfg = self.n_cfg
        s.n_atoms = self.n_atoms
        s.cfg_off = self.cfg_off.data_ptr()
        s.pos = self.pos.data_ptr()
        s.type = self.types.data_ptr()
        s.cell = self.cells.data_ptr()
        s.pbc = self.pbc.data_ptr()
        return s


class Neighbors:
    def __init__(self):
        self._h = ctypes.c_void_p()
        self.generation = 0   # counts builds (a backward checks that its lists were not rebuilt)
        check(_lib.lib().mtp_nbrs_create(ctypes.byref(self._h)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            try:
                _lib.lib().mtp_nbrs_free(h)
            except Exception:
                pass
            self._h = None

    def build(self, model, batch, max_nbrs=64, check_status=True):
        s = batch.system()
        check(_lib.lib().mtp_build_neighbors(model._h, ctypes.byref(s), max_nbrs, self._h, _stream()))
        self.max_nbrs = max_nbrs
        self.generation += 1
        if check_status:
            self.status()
        return self

    def status(self):
        check(_lib.lib().mtp_nbrs_status(self._h, _stream()))

    def export(self, batch):
        n = batch.n_atoms
        count = torch.empty(n, dtype=torch.int32, device=batch.device)
        stride = ctypes.c_int32()
        check(_lib.lib().mtp_nbrs_export(self._h, _p(count), None, None, ctypes.byref(stride), _stream()))
        j = torch.empty(n * stride.value, dtype=torch.int32, device=batch.device)
        sh = torch.empty(n * stride.value * 3, dtype=torch.int32, device=batch.device)
        check(_lib.lib().mtp_nbrs_export(self._h, None, _p(j), _p(sh), ctypes.byref(stride), _stream()))
        return count, j.view(n, stride.value), sh.view(n, stride.value, 3)


def _out(n, dtype, device, shape=None):
    return torch.empty(shape if shape is not None else n, dtype=dtype, device=device)


def energy_forces_stress(model, batch, nbrs, precision="fp64", site_energies=True):
    d = batch.device
    E = _out(batch.n_cfg, torch.float64, d)
    F = _out(None, torch.float64, d, (batch.n_atoms, 3))
    S = _out(None, torch.float64, d, (batch.n_cfg, 3, 3))
    V = _out(batch.n_atoms, torch.float64, d) if site_energies else None
    s = batch.system()
    check(_lib.lib().mtp_energy_forces_stress(model._h, ctypes.byref(s), nbrs._h, _prec(precision), _p(E), _p(F),
                                              _p(S), _p(V), _stream()))
    return {"energy": E, "forces": F, "stress": S, "site_e": V}


def energy_forces_stress_noalloc(model, batch, nbrs, precision="fp64", out=None):
    """energy_forces_stress through the entry point that allocates nothing
    (its scratch is the library's fixed device array); `out` reuses tensors."""
    d = batch.device
    if out is None:
        out = {"energy": _out(batch.n_cfg, torch.float64, d),
               "forces": _out(None, torch.float64, d, (batch.n_atoms, 3)),
               "stress": _out(None, torch.float64, d, (batch.n_cfg, 3, 3)),
               "site_e": _out(batch.n_atoms, torch.float64, d)}
    s = batch.system()
    check(_lib.lib().mtp_energy_forces_stress_noalloc(model._h, ctypes.byref(s), nbrs._h, _prec(precision),
                                                      _p(out["energy"]), _p(out["forces"]), _p(out["stress"]),
                                                      _p(out.get("site_e")), _stream()))
    return out


def grade(model, batch, nbrs, precision="fp64", mode="full", rows=False):
    d = batch.device
    g = _out(batch.n_atoms, torch.float64, d)
    am = _out(batch.n_atoms, torch.int32, d)
    b = None
    if rows:   # FP64 in both forms
        b = _out(None, torch.float64, d, (batch.n_atoms, model.m(mode)))
    s = batch.system()
    check(_lib.lib().mtp_grade(model._h, ctypes.byref(s), nbrs._h, _prec(precision), _mode(mode), _p(g), _p(am),
                               _p(b), _stream()))
    return {"gamma": g, "argmax": am, "rows": b}


def row_stride(m, precision="fp64"):
    """Columns of the column-major row layout the grade kernels read: m
    padded with zeros to a multiple of 32 (FP64) or 64 (mixed)."""
    q = 32 if precision == "fp64" else 64
    return (m + q - 1) // q * q


def grade_rows(model, rows_cm, precision="fp64", mode="full", out=None):
    """Grades of rows the caller holds: rows_cm is a contiguous FP64 device
    tensor [ldb, n] (column k of every row at rows_cm[k]; ldb >=
    row_stride(m), zeros past m), as the evaluation lays them out; `out`
    reuses a previous call's gamma / argmax tensors."""
    ldb, n = rows_cm.shape
    g = out["gamma"] if out else _out(n, torch.float64, rows_cm.device)
    am = out["argmax"] if out else _out(n, torch.int32, rows_cm.device)
    check(_lib.lib().mtp_grade_rows(model._h, _prec(precision), _mode(mode), _p(rows_cm), n, n, ldb, _p(g), _p(am),
                                    _stream()))
    return {"gamma": g, "argmax": am}


def grade_cfg(model, batch, nbrs, precision="fp64", mode="full_cfg", rows=False):
    """Configuration grades (mode "full_cfg" / "linear_cfg"): gamma [n_cfg],
    argmax [n_cfg] and, with rows=True, b(cfg) [n_cfg, m] FP64."""
    d = batch.device
    g = _out(batch.n_cfg, torch.float64, d)
    am = _out(batch.n_cfg, torch.int32, d)
    b = _out(None, torch.float64, d, (batch.n_cfg, model.m(mode))) if rows else None
    s = batch.system()
    check(_lib.lib().mtp_grade_cfg(model._h, ctypes.byref(s), nbrs._h, _prec(precision), _mode(mode), _p(g), _p(am),
                                   _p(b), _stream()))
    return {"gamma": g, "argmax": am, "rows": b}


def cfg_rows(model, batch, nbrs, precision="fp64", mode="full_cfg"):
    """b(cfg) = sum of the configuration's neighborhood rows, [n_cfg, m] FP64 (no active set needed)."""
    b = _out(None, torch.float64, batch.device, (batch.n_cfg, model.m(mode)))
    s = batch.system()
    check(_lib.lib().mtp_grade_cfg(model._h, ctypes.byref(s), nbrs._h, _prec(precision), _mode(mode), None, None,
                                   _p(b), _stream()))
    return b


def evaluate(model, batch, nbrs, precision="fp64", mode="full", out=None, gamma_save=None, capacity=None):
    """Fused energy, forces, stress, site energies and grades; `out` reuses tensors.

    With `gamma_save`, the preselection (gamma > gamma_save) runs in the same
    call: out["sel_idx"] (capacity, default n_atoms) and out["sel_count"]."""
    d = batch.device
    if out is None:
        out = {"energy": _out(batch.n_cfg, torch.float64, d),
               "forces": _out(None, torch.float64, d, (batch.n_atoms, 3)),
               "stress": _out(None, torch.float64, d, (batch.n_cfg, 3, 3)),
               "site_e": _out(batch.n_atoms, torch.float64, d),
               "gamma": _out(batch.n_atoms, torch.float64, d),
               "argmax": _out(batch.n_atoms, torch.int32, d)}
    s = batch.system()
    common = (model._h, ctypes.byref(s), nbrs._h, _prec(precision), _mode(mode), _p(out.get("energy")),
              _p(out.get("forces")), _p(out.get("stress")), _p(out.get("site_e")), _p(out.get("gamma")),
              _p(out.get("argmax")))
    if gamma_save is None:
        check(_lib.lib().mtp_evaluate(*common, _stream()))
        return out
    cap = batch.n_atoms if capacity is None else capacity
    if "sel_idx" not in out or out["sel_idx"].numel() < max(cap, 1):
        out["sel_idx"] = _out(max(cap, 1), torch.int32, d)
        out["sel_count"] = _out(1, torch.int32, d)
    check(_lib.lib().mtp_evaluate_select(*common, float(gamma_save), _p(out["sel_idx"]), cap,
                                         _p(out["sel_count"]), _stream()))
    return out


def b_rows(model, batch, nbrs, idx, mode="full"):
    idx = torch.as_tensor(idx, dtype=torch.int32).to(batch.device).contiguous()
    out = torch.empty((idx.numel(), model.m(mode)), dtype=torch.float64, device=batch.device)
    s = batch.system()
    check(_lib.lib().mtp_b_rows(model._h, ctypes.byref(s), nbrs._h, _mode(mode), _p(idx), idx.numel(), _p(out),
                                _stream()))
    return out


def select(gamma, threshold, capacity=None):
    n = gamma.numel()
    cap = n if capacity is None else capacity
    idx = torch.empty(max(cap, 1), dtype=torch.int32, device=gamma.device)
    cnt = torch.empty(1, dtype=torch.int32, device=gamma.device)
    check(_lib.lib().mtp_select(_p(gamma), n, float(threshold), _p(idx), cap, _p(cnt), _stream()))
    return idx, cnt


def cut_neighborhood(batch, grades, cutoff=8.0, capacity=None):
    """The spherical fragment (cutoff, A) around the atom of largest grade of a
    one-configuration batch: dict of pos [k, 3], types, src, shift [k, 3],
    center."""
    d = batch.device
    g = torch.as_tensor(grades, dtype=torch.float64).to(d).contiguous()
    if capacity is None:   # three times the atoms of the sphere at the cell's mean density, doubled while full
        vol = abs(float(np.linalg.det(batch.cells[0].cpu().numpy())))
        cap, grow = int(3 * 4.18879 * cutoff ** 3 * batch.n_atoms / vol) + 64, True
    else:
        cap, grow = capacity, False
    while True:
        pos = torch.empty((cap, 3), dtype=torch.float64, device=d)
        typ = torch.empty(cap, dtype=torch.int32, device=d)
        src = torch.empty(cap, dtype=torch.int32, device=d)
        sh = torch.empty((cap, 3), dtype=torch.int32, device=d)
        cnt, ctr = ctypes.c_int32(), ctypes.c_int32()
        s = batch.system()
        check(_lib.lib().mtp_cut_neighborhood(ctypes.byref(s), _p(g), float(cutoff), cap, _p(pos), _p(typ), _p(src),
                                              _p(sh), ctypes.byref(cnt), ctypes.byref(ctr), _stream()))
        if not grow or cnt.value < cap:
            break
        cap *= 2
    k = cnt.value
    return {"pos": pos[:k], "types": typ[:k], "src": src[:k], "shift": sh[:k], "center": ctr.value}


def md_run(model, batch, nbrs, vel, masses, dt, n_steps, precision="fp64", mode="full", gamma_save=2.0,
           gamma_break=10.0, max_nbrs=64):
    """Velocity-Verlet MD with extrapolation control on a one-configuration
    batch; batch.pos and vel (device [n, 3], A/fs) are updated in place.
    Returns gamma(cfg) per graded step, the saved steps and the steps done."""
    assert vel.dtype == torch.float64 and vel.is_contiguous() and vel.device == batch.pos.device
    m = np.ascontiguousarray(masses, dtype=np.float64)
    hist = np.full(n_steps + 1, np.nan)   # entries past the last graded step stay NaN
    saved = np.zeros(n_steps + 1, dtype=np.int32)
    ns, done = ctypes.c_int32(), ctypes.c_int32()
    s = batch.system()
    check(_lib.lib().mtp_md_run(model._h, ctypes.byref(s), nbrs._h, max_nbrs, _p(batch.pos), _p(vel),
                                m.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(dt), n_steps,
                                _prec(precision), _mode(mode), float(gamma_save), float(gamma_break),
                                hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                saved.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(ns),
                                ctypes.byref(done), _stream()))
    graded = int(np.count_nonzero(~np.isnan(hist)))
    return {"gamma": hist[:graded], "saved": saved[:ns.value].tolist(), "steps": done.value}


def relax_fire(model, batch, nbrs, masses, dt0=1.0, dt_max=10.0, fmax=1e-3, max_steps=1000, precision="fp64",
               mode="full", gamma_save=2.0, gamma_break=10.0, max_nbrs=64):
    """FIRE relaxation with extrapolation control of a one-configuration
    batch (batch.pos updated in place).  Returns gamma(cfg) per graded step,
    the saved steps, the steps done and whether fmax was reached."""
    m = np.ascontiguousarray(masses, dtype=np.float64)
    hist = np.full(max_steps + 1, np.nan)
    saved = np.zeros(max_steps + 1, dtype=np.int32)
    ns, done, conv = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    s = batch.system()
    check(_lib.lib().mtp_relax_fire(model._h, ctypes.byref(s), nbrs._h, max_nbrs, _p(batch.pos),
                                    m.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(dt0), float(dt_max),
                                    float(fmax), max_steps, _prec(precision), _mode(mode), float(gamma_save),
                                    float(gamma_break), hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    saved.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(ns),
                                    ctypes.byref(done), ctypes.byref(conv), _stream()))
    graded = int(np.count_nonzero(~np.isnan(hist)))
    return {"gamma": hist[:graded], "saved": saved[:ns.value].tolist(), "steps": done.value,
            "converged": bool(conv.value)}


def fit_bfgs(model, batch, nbrs, E_t=None, F_t=None, S_t=None, w_e=1.0, w_f=0.01, w_s=0.001, max_iter=50,
             gtol=1e-10, precision="fp64", scale=None):
    """BFGS on the objective of eq. 7 from the model's theta (which holds the
    result on return); targets E_t [n_cfg], F_t [n_atoms, 3], S_t [n_cfg, 3, 3];
    scale: typical size of each parameter (diagonal preconditioner) or None.
    Returns (theta, loss history)."""
    sc = None if scale is None else np.ascontiguousarray(scale, dtype=np.float64)
    def prep(t, shape):
        if t is None:
            return None
        return torch.as_tensor(t, dtype=torch.float64).to(batch.device).reshape(shape).contiguous()
    E_, F_, S_ = prep(E_t, (batch.n_cfg,)), prep(F_t, (batch.n_atoms, 3)), prep(S_t, (batch.n_cfg, 3, 3))
    hist = np.zeros(max_iter + 1)
    it = ctypes.c_int32()
    s = batch.system()
    check(_lib.lib().mtp_fit_bfgs(model._h, ctypes.byref(s), nbrs._h, _prec(precision), _p(E_), _p(F_), _p(S_),
                                  float(w_e if E_ is not None else 0.0), float(w_f if F_ is not None else 0.0),
                                  float(w_s if S_ is not None else 0.0), max_iter, float(gtol),
                                  None if sc is None else sc.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(it), _stream()))
    return model.theta(), hist[:it.value + 1]


def maxvol_update(model, mode, cand, threshold=1.001, max_swaps=None):
    """Swaps candidate rows (FP64 device [n, m], modified in place) into the active set."""
    m = model.m(mode)
    assert cand.dtype == torch.float64 and cand.is_contiguous() and cand.shape[1] == m
    ms = 10 * m if max_swaps is None else max_swaps
    sc = torch.empty(max(ms, 1), dtype=torch.int32, device=cand.device)
    sj = torch.empty(max(ms, 1), dtype=torch.int32, device=cand.device)
    n = ctypes.c_int32()
    check(_lib.lib().mtp_maxvol_update(model._h, _mode(mode), _p(cand), cand.shape[0], float(threshold), ms,
                                       _p(sc), _p(sj), ctypes.byref(n), _stream()))
    return sc[:n.value].cpu().numpy(), sj[:n.value].cpu().numpy()


def efs_backward(model, batch, nbrs, gE=None, gF=None, gS=None, precision="fp64"):
    """dL/dtheta for upstream gradients dL/dE [n_cfg], dL/dF [n_atoms, 3], dL/dS [n_cfg, 3, 3]."""
    def prep(t, shape):
        if t is None:
            return None
        return torch.as_tensor(t, dtype=torch.float64).to(batch.device).reshape(shape).contiguous()
    gE_, gF_, gS_ = prep(gE, (batch.n_cfg,)), prep(gF, (batch.n_atoms, 3)), prep(gS, (batch.n_cfg, 3, 3))
    out = torch.empty(model.info["n_theta"], dtype=torch.float64, device=batch.device)
    s = batch.system()
    check(_lib.lib().mtp_efs_backward(model._h, ctypes.byref(s), nbrs._h, _prec(precision), _p(gE_), _p(gF_),
                                      _p(gS_), _p(out), _stream()))
    return out


class MTPEnergy(torch.autograd.Function):
    """(E, F, S) = MTPEnergy.apply(theta, model, batch, nbrs, precision).

    Forward evaluates energies [n_cfg], forces [n_atoms, 3] and stresses
    [n_cfg, 3, 3] with theta loaded into the model; backward returns
    dL/dtheta from the library's backward kernels (moments recomputed) at the
    theta of its own forward: the model is loaded with that theta again if
    another forward or set_params changed it in between.  A backward after
    the neighbor lists were rebuilt raises (its positions are gone)."""

    @staticmethod
    def forward(ctx, theta, model, batch, nbrs, precision="fp64"):
        model.set_params(theta.detach())
        out = energy_forces_stress(model, batch, nbrs, precision, site_energies=False)
        ctx.save_for_backward(theta.detach().clone())
        ctx.model, ctx.batch, ctx.nbrs, ctx.precision = model, batch, nbrs, precision
        ctx.generation = nbrs.generation
        return out["energy"], out["forces"], out["stress"]

    @staticmethod
    def backward(ctx, gE, gF, gS):
        (theta,) = ctx.saved_tensors
        if ctx.nbrs.generation != ctx.generation:
            raise RuntimeError("MTPEnergy.backward: the neighbor lists were rebuilt after this forward")
        th = theta.cpu().numpy()
        if not np.array_equal(ctx.model.theta, th):
            ctx.model.set_params(th)
        g = efs_backward(ctx.model, ctx.batch, ctx.nbrs, gE, gF, gS, ctx.precision)
        return g, None, None, None, None


GRADE_FORMS = {0: "none", 1: "fp64-registers", 2: "fp64-lds", 3: "int8-slices", 4: "fp64-registers-32-row-blocks",
               5: "fp64-k-outer", 6: "fp64-k-outer-2-step-chunks"}


def tune(model, batch, nbrs, precision="fp64", mode="full", with_grade=False):
    """Runs the library's autotuner for this system; returns the chosen lanes
    per neighborhood as (moments / contraction, pair gradients), and with
    `with_grade` also the chosen kernel form of the grade product (a name
    from GRADE_FORMS; "none" when the mode has no active set)."""
    lanes = ctypes.c_int32()
    grade = ctypes.c_int32()
    s = batch.system()
    check(_lib.lib().mtp_tune(model._h, ctypes.byref(s), nbrs._h, _prec(precision), _mode(mode), ctypes.byref(lanes),
                              ctypes.byref(grade), _stream()))
    if with_grade:
        return lanes.value >> 4, lanes.value & 15, GRADE_FORMS[grade.value]
    return lanes.value >> 4, lanes.value & 15


def mfma_rate(kind, iters=20000):
    """Sustained MFMA rate of this GPU in TFLOP/s (TOP/s for int8): kind
    "f64" (v_mfma_f64_16x16x4) or "i8" (v_mfma_i32_16x16x64_i8)."""
    out = ctypes.c_double()
    check(_lib.lib().mtp_mfma_rate({"f64": 0, "i8": 1}[kind], iters, ctypes.byref(out), _stream()))
    return out.value


def basis_describe(level):
    n = ctypes.c_int32()
    buf = ctypes.create_string_buffer(1 << 22)
    check(_lib.lib().mtp_basis_describe(level, buf, len(buf), ctypes.byref(n)))
    return buf.value.decode().splitlines()


def compiled_levels():
    arr = (ctypes.c_int32 * 64)()
    n = _lib.lib().mtp_compiled_levels(arr, 64)
    return list(arr[:n])


__all__ = ["Model", "Batch", "Neighbors", "energy_forces_stress", "energy_forces_stress_noalloc", "grade", "grade_cfg", "cfg_rows", "evaluate",
           "b_rows", "select", "cut_neighborhood", "md_run", "relax_fire", "fit_bfgs",
           "maxvol_update", "efs_backward", "MTPEnergy", "tune", "CapturedStep", "basis_describe", "compiled_levels", "mfma_rate", "MtpError",
           "grade_rows", "row_stride"]


class CapturedStep:
    """One hot-path step (neighbor build if `rebuild`, fused evaluation,
    preselection) captured once in a HIP graph and replayed.

    `passes` > 1 captures that many passes of the step, one after the other,
    in the same graph: every replay then runs the step `passes` times over
    the same inputs (each pass rebuilds and re-evaluates in full).  A graph
    replay has a fixed start-up cost of its own, which several passes per
    replay share.

    The step must have run eagerly at least once at the same sizes so that
    every library workspace exists (nothing is allocated during capture).
    Outputs live in `self.out` and are overwritten by every pass."""

    def __init__(self, model, batch, nbrs, precision="fp64", mode="full", max_nbrs=64, gamma_save=2.0,
                 rebuild=True, passes=1, grades=True):
        if passes < 1:
            raise ValueError("passes must be at least 1")
        self.model, self.batch, self.nbrs = model, batch, nbrs
        self.args = (precision, mode, max_nbrs, gamma_save if grades else None)
        self.rebuild = rebuild
        self.passes = passes
        out = None
        if not grades:   # energy, forces, stress and site energies only (no active set needed)
            d = batch.device
            out = {"energy": _out(batch.n_cfg, torch.float64, d),
                   "forces": _out(None, torch.float64, d, (batch.n_atoms, 3)),
                   "stress": _out(None, torch.float64, d, (batch.n_cfg, 3, 3)),
                   "site_e": _out(batch.n_atoms, torch.float64, d)}
        self.out = evaluate(model, batch, nbrs, precision, mode, out=out, gamma_save=self.args[3])
        self._step()                      # eager warm-up: workspaces at their final size
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            for _ in range(passes):
                self._step()
        torch.cuda.synchronize()

    def _step(self):
        precision, mode, max_nbrs, gamma_save = self.args
        if self.rebuild:
            self.nbrs.build(self.model, self.batch, max_nbrs=max_nbrs, check_status=False)
        evaluate(self.model, self.batch, self.nbrs, precision, mode, out=self.out, gamma_save=gamma_save)
        self.sel = (self.out["sel_idx"], self.out["sel_count"]) if gamma_save is not None else None

    def replay(self, check=True):
        """Replays the step.  With `check` (the default) it waits for the step
        and raises MtpError if the neighbor build of this replay flagged a
        capacity overflow, an overlap or a non-finite position (the status
        words are written on the device by every replayed build); without it
        the replay is only enqueued, and status() checks later."""
        self.graph.replay()
        if check and self.rebuild:
            self.status()
        return self.out

    def status(self):
        """Raises MtpError for what the last replayed neighbor build flagged (synchronises)."""
        self.nbrs.status()
