#!/usr/bin/env python
"""Throughput of the MTP hot path on one MI355X: atom-steps/s of
energy + forces + stress + grade with the level-16 two-species potential.

Workload: random 50/50 FCC alloy, a = 4.05 A, 16x16x16 cells (16,384 atoms),
Gaussian displacements sigma = 0.08 A, R_cut = 5.0 A, R_min = 2.0 A, the
seeded normalised teacher potential and its oracle-built active set (FULL
grade mode, m = 212).  One step = neighbor build + fused evaluation (site
energies, total energy, forces, stress, b rows, grades) + preselection of
gamma > 2.  Inputs are resident in HBM before the timed region starts.

Prints one JSON line.  `--gpus` above 1 is not supported (one GPU only).
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_VALU_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz, FP64 and non-packed FP32
PEAK_MFMA_F64_TFLOPS = 78.6
PEAK_MFMA_BF16_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0
KERNELS = ("neighbors", "efs", "efs_moments", "efs_contract", "efs_forces", "force_gather", "cfg_sums", "grade",
           "select")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def efs_flops_per_atom(n_pairs_per_atom, nc, nr, contraction_flops, with_rows):
    """Algorithmic flops per neighborhood of the evaluation kernels.

    efs_moments, per pair:  r (6) + T_0..T_7 (12) + f_mu (16 nr + 2) + monomials (16) + moments (2 nc)
    efs_contract:           the generated contraction program (graph values, trie walk, reverse)
    efs_forces (one launch, two block ranges), per pair:
      pair gradients:       r (6) + T, T' (30) + f, f' (32 nr + 4 nr + 3) + monomials (16)
                            + P and grad P (8 nc) + g assembly (8 nr + 7) + virial (18)
      b-row c part:         r (6) + T (12) + cutoff (3) + monomials (16) + P (2 nc) + 2 nr NPOLY + NPOLY
    """
    p1 = 6 + 12 + 16 * nr + 2 + 16 + 2 * nc
    p3 = 6 + 30 + 36 * nr + 3 + 16 + 8 * nc + 8 * nr + 7 + 18
    p4 = 6 + 12 + 3 + 16 + 2 * nc + 2 * nr * 8 + 8
    return {"efs_moments": n_pairs_per_atom * p1, "efs_contract": float(contraction_flops),
            "efs_forces": n_pairs_per_atom * (p3 + (p4 if with_rows else 0))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64",
                    help="form reported as `value`; the other form is timed too")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=2048)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (for scaling HBM counters)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {a.gpus}); multi-GPU runs are not part of this build",
              file=sys.stderr)
        return 2

    import torch
    from paper_2304_13144_amd import _lib, api, synth

    dev = torch.device("cuda", 0)
    w = synth.workload2()
    cfg = w.configs[0]
    n_types, level = w.n_types, w.level
    model = api.Model.create(level, n_types, w.r_min, w.r_cut)
    info = model.info
    theta = synth.theta_teacher(2, n_types, info["n_lin"], info["n_rad"])
    model.set_params(theta)
    keep = model.kept_columns()
    A_full = np.load(os.path.join(ROOT, "tests", "golden", "active_w2_full.npy"))[:, keep]
    model.set_active_set("full", A_full)
    batch = api.Batch([cfg])
    nbrs = api.Neighbors().build(model, batch, max_nbrs=64)
    count, _, _ = nbrs.export(batch)
    pairs_per_atom = float(count.double().mean().item())
    outs = {p: api.evaluate(model, batch, nbrs, p, "full") for p in ("fp64", "mixed")}
    tuned = {p: api.tune(model, batch, nbrs, p, "full") for p in ("fp64", "mixed")}
    torch.cuda.synchronize()
    log(f"[bench] autotuned lanes per neighborhood: {tuned}")
    if a.copy_calibration:
        src = torch.ones(256 * 1024 * 1024 // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def step(prec):
        nbrs.build(model, batch, max_nbrs=64, check_status=False)
        o = api.evaluate(model, batch, nbrs, prec, "full", out=outs[prec])
        api.select(o["gamma"], 2.0)

    L = _lib.lib()
    results = {}
    for prec in ("fp64", "mixed"):
        # eager launches, every kernel bracketed by the library's event profiler
        for _ in range(a.warmup):
            step(prec)
        torch.cuda.synchronize()
        L.mtp_profile_enable(1)
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(a.steps):
            step(prec)
        t1.record()
        torch.cuda.synchronize()
        L.mtp_profile_enable(0)
        eager_ms = t0.elapsed_time(t1) / a.steps
        kern = {}
        for k in KERNELS:
            tot = ctypes.c_double()
            n = ctypes.c_int64()
            _lib.check(L.mtp_profile_read(k.encode(), ctypes.byref(tot), ctypes.byref(n)))
            kern[k] = {"avg_us": 1e3 * tot.value / max(n.value, 1), "launches": n.value}
        # the same step captured once in a HIP graph and replayed
        cap = api.CapturedStep(model, batch, nbrs, prec, "full", max_nbrs=64)
        for _ in range(a.warmup):
            cap.replay()
        torch.cuda.synchronize()
        t0.record()
        for _ in range(a.steps):
            cap.replay()
        t1.record()
        torch.cuda.synchronize()
        graph_ms = t0.elapsed_time(t1) / a.steps
        outs[prec] = {k: v.clone() for k, v in cap.out.items()}
        ms = min(eager_ms, graph_ms)
        results[prec] = {"ms_per_step": ms, "atom_steps_per_s": cfg.n / (ms * 1e-3), "kernels": kern,
                         "eager_ms_per_step": eager_ms, "graph_ms_per_step": graph_ms}
        log(f"[bench] {prec}: eager {eager_ms:.4f} ms/step, graph {graph_ms:.4f} ms/step, "
            f"{cfg.n / (ms * 1e-3):.4g} atom-steps/s; kernels (us): "
            + ", ".join(f"{k} {v['avg_us']:.1f}" for k, v in kern.items()))

    # agreement of the two forms on this workload (GPU vs GPU)
    f64 = {k: v.cpu().numpy() for k, v in outs["fp64"].items()}
    mix = {k: v.cpu().numpy() for k, v in outs["mixed"].items()}
    mixed_vs_fp64 = {"forces_max_abs_eVA": float(np.abs(mix["forces"] - f64["forces"]).max()),
                     "gamma_max_rel": float((np.abs(mix["gamma"] - f64["gamma"]) / np.maximum(1, f64["gamma"])).max()),
                     "energy_abs_eV": float(abs(mix["energy"][0] - f64["energy"][0]))}

    # roofline of the dominant evaluation kernel (largest share of the step)
    prec = a.precision
    r = results[prec]
    fl = efs_flops_per_atom(pairs_per_atom, info["n_comp"], info["n_rad"], info["contraction_flops"], True)
    per_kernel = {}
    for k, f in fl.items():
        us = r["kernels"][k]["avg_us"]
        per_kernel[k] = {"avg_us": us, "flops_per_atom": f,
                         "tflops": f * cfg.n / max(us * 1e-6, 1e-12) / 1e12}
    dom = max(per_kernel, key=lambda k: per_kernel[k]["avg_us"])
    achieved = per_kernel[dom]["tflops"]
    grade_us = r["kernels"]["grade"]["avg_us"]
    m = info["m_full"]
    grade_flops = 2.0 * cfg.n * m * m * (1 if prec == "fp64" else 6)
    out = {
        "metric": "atom-steps/s (E+F+stress+grade), level-16 MTP",
        "value": r["atom_steps_per_s"],
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": r["ms_per_step"],
        "launch": "hip-graph replay" if r["graph_ms_per_step"] <= r["eager_ms_per_step"] else "eager",
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else "f32+bf16x3",
        "data": "synthetic (seeded FCC alloy, seeded teacher potential)",
        "config": {"workload": "fcc-alloy-16x16x16-level16-2species", "atoms": cfg.n, "level": level,
                   "n_types": n_types, "r_cut": w.r_cut, "grade_mode": "full", "m": m,
                   "pairs_per_atom": pairs_per_atom, "step": "neighbors+evaluate(E,F,S,gamma)+select",
                   "lanes_per_neighborhood": tuned[prec]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_VALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_VALU_TFLOPS, "traffic": None, "kernel": dom,
                     "flops_per_atom": per_kernel[dom]["flops_per_atom"], "avg_us": per_kernel[dom]["avg_us"]},
        "evaluation_kernels": per_kernel,
        "grade_gemm": {"bound": "mfma", "avg_us": grade_us,
                       "achieved_tflops": grade_flops / (grade_us * 1e-6) / 1e12,
                       "peak": PEAK_MFMA_F64_TFLOPS if prec == "fp64" else PEAK_MFMA_BF16_TFLOPS},
        "forms": {p: {"atom_steps_per_s": v["atom_steps_per_s"], "ms_per_step": v["ms_per_step"],
                      "eager_ms_per_step": v["eager_ms_per_step"], "graph_ms_per_step": v["graph_ms_per_step"],
                      "kernels_us": {k: round(x["avg_us"], 2) for k, x in v["kernels"].items()}}
                  for p, v in results.items()},
        "mixed_speedup_vs_fp64": results["mixed"]["atom_steps_per_s"] / results["fp64"]["atom_steps_per_s"],
        "mixed_vs_fp64": mixed_vs_fp64,
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"], out["errors_vs_oracle"] = cpu_baseline(cfg, w, theta, keep, A_full, f64, mix,
                                                                   a.cpu_sample)
    print(json.dumps(out), flush=True)
    return 0


def cpu_baseline(cfg, w, theta, keep, A_full, f64, mix, sample):
    """The FP64 oracle on `sample` neighborhoods of the same configuration:
    site energies, pair gradients (forces / stress contributions), rows b_i and
    grades; also the GPU-vs-oracle errors on those atoms."""
    import torch

    from oracle import mtp as om
    from oracle import neighbors as onb

    pot = om.Potential(w.level, w.n_types, w.r_min, w.r_cut)
    # centers plus all their neighbors: forces on the centers are then exact
    centers = np.arange(max(1, sample // 34))
    around = onb.neighbors(cfg.pos, cfg.cell, cfg.pbc, w.r_cut, atoms=centers)
    atoms = np.unique(np.concatenate([centers, around.j]))
    pairs = onb.neighbors(cfg.pos, cfg.cell, cfg.pbc, w.r_cut, atoms=atoms)
    t = time.perf_counter()
    _, F, _, V = om.energy_forces_stress(pot, theta, cfg.pos, cfg.types, cfg.cell, pairs)
    rows = om.b_rows(pot, theta, cfg.pos, cfg.types, cfg.cell, pairs, atoms=atoms)[:, keep]
    gam = om.grades(rows, A_full)[0]
    dt = time.perf_counter() - t
    inner = centers
    errs = {}
    for name, g in (("fp64", f64), ("mixed", mix)):
        e = {"site_e_max_abs": float(np.abs(g["site_e"][atoms] - V[atoms]).max()),
             "gamma_max_rel": float((np.abs(g["gamma"][atoms] - gam) / np.maximum(1, gam)).max())}
        if len(inner):
            e["forces_max_abs_eVA"] = float(np.abs(g["forces"][inner] - F[inner]).max())
        errs[name] = e
    sample = len(atoms)
    base = {"value": sample / dt, "unit": "atom-steps/s", "cores": torch.get_num_threads(), "kind": "oracle",
            "sample": f"{sample} neighborhoods (16 atoms and all their neighbors) of the same 16,384-atom "
                      f"configuration: site energies, pair "
                      f"gradients, rows b_i and grades (neighbor search excluded)", "seconds": dt}
    return base, errs


if __name__ == "__main__":
    sys.exit(main())
