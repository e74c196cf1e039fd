#!/usr/bin/env python
"""Throughput of the MTP hot path on one MI355X: atom-steps/s of
energy + forces + stress + grade with the level-16 two-species potential.

Workload: random 50/50 FCC alloy, a = 4.05 A, 16x16x16 cells (16,384 atoms),
Gaussian displacements sigma = 0.08 A, R_cut = 5.0 A, R_min = 2.0 A, the
seeded normalised teacher potential and its oracle-built active set (FULL
grade mode, m = 212).  One step = fused evaluation (site energies, total
energy, forces, stress, b rows, grades) + preselection of gamma > 2 on a
built neighbor list; the neighbor build is timed on its own and a
"with_rebuild" rate (build + evaluation + preselection) is reported next to
it.  Inputs are resident in HBM before the timed region starts.

Prints one JSON line.  `--gpus` above 1 is not supported (one GPU only).
`--profile-summary` turns rocprofv3 output into the summaries kept under
profiles/.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_VALU_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz, FP64 and non-packed FP32
PEAK_MFMA_F64_TFLOPS = 78.6
PEAK_MFMA_I8_TOPS = 5000.0
GRADE_I8_PRODUCTS = 19     # int8 digit products of the mixed grade (levels s + t <= 5 of 5 x 5 slices)
PEAK_HBM_GBS = 8000.0
KERNELS = ("neighbors", "efs", "efs_moments", "efs_contract", "efs_forces", "force_gather", "cfg_sums", "grade",
           "select")
# kernels whose HBM traffic the profile summary records (rocprof name substrings)
TRAFFIC_KERNELS = ("efs_moments_contract<double, 16, true>", "efs_moments_contract8<double, 16, true>",
                   "efs_moments<double, 16, 8>", "efs_contract<double, 16, true>",
                   "efs_forces_fused<double, 16, 4, 2>", "efs_forces_fused<double, 16, 8, 2>",
                   "efs_forces_rows<float, double, 16, 4>", "efs_forces_rows<float, double, 16, 8>",
                   "grade_f64<", "grade_f64_wide<", "grade_f64_pair<", "grade_f64_kouter<7, 8, 1>",
                   "grade_f64_kouter<7, 2, 2>", "grade_i8<4>", "pair_search<false, 2>",
                   "reverse_pairs")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def efs_flops_per_atom(n_pairs_per_atom, nc, nr, contraction_flops, with_rows, fused_rows=True):
    """Algorithmic flops per neighborhood of the evaluation kernels.

    efs_moments, per pair:  r (6) + T_0..T_7 (12) + f_mu (16 nr + 2) + monomials (16) + moments (2 nc)
    efs_contract:           the generated contraction program (graph values, trie walk, reverse)
    efs_forces, per pair:
      pair gradients:       r (6) + T, T' (30) + f, f' (32 nr + 4 nr + 3) + monomials (16)
                            + P and grad P (8 nc) + g assembly (8 nr + 7) + virial (18)
      b-row c part, in the same pass (FP64, fused_rows): T_beta cut (NPOLY) + 2 nr NPOLY --
                            P and the Chebyshev values are the gradient's;
      in row blocks of their own (the mixed form, whose rows are FP64 and its
      pair gradients FP32): r (6) + T (12) + cutoff (3) + monomials (16) + P (2 nc)
                            + 2 nr NPOLY + NPOLY
    """
    p1 = 6 + 12 + 16 * nr + 2 + 16 + 2 * nc
    p3 = 6 + 30 + 36 * nr + 3 + 16 + 8 * nc + 8 * nr + 7 + 18
    p4 = 8 + 2 * nr * 8 if fused_rows else 6 + 12 + 3 + 16 + 2 * nc + 2 * nr * 8 + 8
    return {"efs_moments": n_pairs_per_atom * p1, "efs_contract": float(contraction_flops),
            "efs_forces": n_pairs_per_atom * (p3 + (p4 if with_rows else 0))}


def source_digest():
    """Digest of the library sources: HBM traffic figures recorded under
    profiles/ apply only while it is unchanged."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2304_13144_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp", ".cpp", ".h")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(f.encode() + b"\0" + fh.read())
    with open(os.path.join(ROOT, "paper_2304_13144_amd", "build.py"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_fcc-alloy-16x16x16_level16.md")


def recorded_traffic(kernel_substr):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated) of the
    kernel whose name contains kernel_substr, from the committed summary, or
    None when absent or recorded for other sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    digest = source_digest()
    for line in open(TRAFFIC_FILE):
        f = line.strip().strip("`").split()
        if len(f) >= 5 and f[0] == "traffic":
            kv = dict(x.split("=", 1) for x in f[2:] if "=" in x)
            if f[1] == kernel_substr.replace(" ", "") and kv.get("source") == digest:
                return float(kv["fetch_bytes"]) + float(kv["write_bytes"])
    return None


def profile_summary(trace_dir, fetch_dir, write_dir, kernels):
    """Markdown summary of rocprofv3 output: per-kernel durations from the
    kernel-trace statistics; FETCH_SIZE / WRITE_SIZE per dispatch (KiB),
    scaled by what the same counters read for the 256 MiB copy kernel of
    --copy-calibration; plus one `traffic` line per named kernel for
    recorded_traffic()."""
    import csv
    import glob

    def one(pattern):
        files = glob.glob(pattern, recursive=True)
        if not files:
            raise SystemExit(f"no file matches {pattern}")
        return files[0]

    stats = list(csv.DictReader(open(one(os.path.join(trace_dir, "**", "*kernel_stats.csv")))))

    def counter(d, name):
        agg = {}
        for r in csv.DictReader(open(one(os.path.join(d, "**", "*counter_collection.csv")))):
            if r["Counter_Name"] == name:
                agg.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return {k: sum(v) / len(v) for k, v in agg.items()}, {k: max(v) for k, v in agg.items()}

    (fetch, fmax), (write, wmax) = counter(fetch_dir, "FETCH_SIZE"), counter(write_dir, "WRITE_SIZE")
    copy = [k for k in fetch if "copyBuffer" in k]
    big = 256 * 1024.0   # KiB moved each way by the calibration copy (its largest dispatch)
    cf = big / max(fmax[k] for k in copy) if copy else 1.0
    cw = big / max(wmax.get(k, 0.0) for k in copy) if copy else 1.0
    dur = {r["Name"]: float(r["AverageNs"]) for r in stats}
    out = ["| kernel | calls | avg us | FETCH KiB | WRITE KiB | HBM GB/s (calibrated) |", "|---|---|---|---|---|---|"]
    for r in stats[:24]:
        k = r["Name"]
        fb = fetch.get(k, 0.0) * cf * 1024
        wb = write.get(k, 0.0) * cw * 1024
        gbs = (fb + wb) / max(float(r["AverageNs"]), 1.0) if k in fetch else float("nan")
        out.append(f"| `{k[:90]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                   f"{fetch.get(k, float('nan')):.0f} | {write.get(k, float('nan')):.0f} | {gbs:.0f} |")
    out.append("")
    out.append(f"calibration: copy kernel FETCH x{cf:.4f}, WRITE x{cw:.4f} (256 MiB each way)")
    out.append("")
    digest = source_digest()
    for sub in kernels:
        names = [k for k in fetch if sub in k]
        if not names:
            continue
        k = names[0]
        out.append(f"`traffic {sub.replace(' ', '')} fetch_bytes={fetch[k] * cf * 1024:.0f} write_bytes={write.get(k, 0.0) * cw * 1024:.0f} "
                   f"source={digest} avg_ns={dur.get(k, float('nan')):.0f}`")
    return "\n".join(out)


COUNTER_KERNELS = ("efs_moments_contract", "efs_forces_rows", "efs_forces_fused", "grade_f64", "grade_i8", "select_write")


def counter_summary(trace_dir, counter_dirs):
    """Markdown table of rocprofv3 --pmc counters (mean per dispatch, summed
    over the device) for the evaluation kernels, with derived figures: VALU
    busy and s_waitcnt shares of the waves' cycles, LDS bank-conflict share,
    and FP64 / FP32 FLOP/s counted from the per-type VALU instruction
    counters (an FMA is 2 flops, x 64 lanes) over the average duration from
    the trace run."""
    import csv
    import glob

    vals = {}
    for d in counter_dirs:
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                vals.setdefault(r["Kernel_Name"], {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    stats = list(csv.DictReader(open(glob.glob(os.path.join(trace_dir, "**", "*kernel_stats.csv"), recursive=True)[0])))
    dur = {r["Name"]: float(r["AverageNs"]) for r in stats}
    names = sorted({c for v in vals.values() for c in v})
    out = ["| kernel | avg us | " + " | ".join(names) + " |", "|---|---|" + "---|" * len(names)]
    derived = ["| kernel | VALU busy share (SQ_ACTIVE_INST_VALU / SQ_WAVE_CYCLES) | "
               "s_waitcnt share (SQ_WAIT_ANY / SQ_WAVE_CYCLES) | "
               "LDS bank-conflict share (SQ_LDS_BANK_CONFLICT / SQ_ACTIVE_INST_LDS) | FP64 TFLOP/s | FP32 TFLOP/s |",
               "|---|---|---|---|---|---|"]
    for k, c in vals.items():
        if not any(s in k for s in COUNTER_KERNELS):
            continue
        m = {n: sum(v) / len(v) for n, v in c.items()}
        us = dur.get(k, float("nan")) / 1e3
        out.append(f"| `{k[:80]}` | {us:.2f} | " + " | ".join(f"{m.get(n, float('nan')):.0f}" for n in names) + " |")
        g = lambda n: m.get(n, float("nan"))
        f64 = 64 * (2 * g("SQ_INSTS_VALU_FMA_F64") + g("SQ_INSTS_VALU_MUL_F64") + g("SQ_INSTS_VALU_ADD_F64"))
        f32 = 64 * (2 * g("SQ_INSTS_VALU_FMA_F32") + g("SQ_INSTS_VALU_MUL_F32") + g("SQ_INSTS_VALU_ADD_F32"))
        derived.append(f"| `{k[:80]}` | "
                       f"{g('SQ_ACTIVE_INST_VALU') / g('SQ_WAVE_CYCLES'):.3f} | {g('SQ_WAIT_ANY') / g('SQ_WAVE_CYCLES'):.3f} | "
                       f"{g('SQ_LDS_BANK_CONFLICT') / g('SQ_ACTIVE_INST_LDS'):.3f} | {f64 / (us * 1e-6) / 1e12:.2f} | "
                       f"{f32 / (us * 1e-6) / 1e12:.2f} |")
    return "\n".join(out + [""] + derived)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64",
                    help="form reported as `value`; the other form is timed too")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-centers", type=int, default=2048,
                    help="oracle sample: this many atoms and all their neighbors (about 10-30 s of host time)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (for scaling HBM counters)")
    ap.add_argument("--counter-summary", nargs="+", metavar="DIR",
                    help="print a markdown table of rocprofv3 --pmc output (TRACE_DIR then counter dirs) and exit")
    ap.add_argument("--profile-summary", nargs=3, metavar=("TRACE_DIR", "FETCH_DIR", "WRITE_DIR"),
                    help="print a markdown summary of rocprofv3 output and exit")
    ap.add_argument("--extra-workloads", action="store_true",
                    help="also time the level-20 training step (512 configurations, forward + backward) and the "
                         "grades of the 1,048,576-atom active-learning snapshots (adds `extra_workloads`)")
    a = ap.parse_args()
    if a.profile_summary:
        print(profile_summary(*a.profile_summary, kernels=TRAFFIC_KERNELS))
        return 0
    if a.counter_summary:
        print(counter_summary(a.counter_summary[0], a.counter_summary[1:]))
        return 0
    if a.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {a.gpus}); this benchmark measures one GPU only",
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
    A_full = synth.active_set(2, "full")[:, keep]
    model.set_active_set("full", A_full)
    batch = api.Batch([cfg])
    nbrs = api.Neighbors().build(model, batch, max_nbrs=64)
    count, _, _ = nbrs.export(batch)
    pairs_per_atom = float(count.double().mean().item())
    outs = {p: api.evaluate(model, batch, nbrs, p, "full", gamma_save=2.0) for p in ("fp64", "mixed")}
    tuned = {p: api.tune(model, batch, nbrs, p, "full", with_grade=True) for p in ("fp64", "mixed")}
    torch.cuda.synchronize()
    log(f"[bench] autotuned (moments lanes, pair-gradient lanes, grade form): {tuned}")
    if a.copy_calibration:
        src = torch.ones(256 * 1024 * 1024 // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def eval_step(prec):
        api.evaluate(model, batch, nbrs, prec, "full", out=outs[prec], gamma_save=2.0)

    def full_step(prec):
        nbrs.build(model, batch, max_nbrs=64, check_status=False)
        eval_step(prec)

    L = _lib.lib()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)

    def timed(fn, per_call=1):
        """ms per step of fn, which runs per_call steps: a.steps steps timed."""
        for _ in range(max(1, a.warmup // per_call)):
            fn()
        torch.cuda.synchronize()
        t0.record()
        for _ in range(a.steps // per_call):
            fn()
        t1.record()
        torch.cuda.synchronize()
        return t0.elapsed_time(t1) / a.steps

    # passes per graph replay: the largest divisor of the step count up to 10
    passes = max(d for d in range(1, 11) if a.steps % d == 0)

    results = {}
    for prec in ("fp64", "mixed"):
        # eager, every kernel group bracketed by the library's event profiler (with the rebuild)
        for _ in range(a.warmup):
            full_step(prec)
        torch.cuda.synchronize()
        L.mtp_profile_enable(1)
        prof_ms = timed(lambda: full_step(prec))
        L.mtp_profile_enable(0)
        kern = {}
        for k in KERNELS:
            tot = ctypes.c_double()
            n = ctypes.c_int64()
            _lib.check(L.mtp_profile_read(k.encode(), ctypes.byref(tot), ctypes.byref(n)))
            kern[k] = {"avg_us": 1e3 * tot.value / max(n.value, 1), "launches": n.value}
        # plain eager and HIP-graph replays: evaluation alone and with the rebuild
        eager_eval = timed(lambda: eval_step(prec))
        eager_full = timed(lambda: full_step(prec))
        # one pass per replay, and `passes` passes per replay (the K timed steps
        # are K / passes replays); status words of the rebuilds checked after timing
        cap_eval = api.CapturedStep(model, batch, nbrs, prec, "full", max_nbrs=64, rebuild=False)
        graph_eval = timed(cap_eval.replay)
        capk_eval = api.CapturedStep(model, batch, nbrs, prec, "full", max_nbrs=64, rebuild=False,
                                     passes=passes)
        graphk_eval = timed(lambda: capk_eval.replay(check=False), passes)
        cap_full = api.CapturedStep(model, batch, nbrs, prec, "full", max_nbrs=64, rebuild=True)
        graph_full = timed(lambda: cap_full.replay(check=False))
        cap_full.status()
        capk_full = api.CapturedStep(model, batch, nbrs, prec, "full", max_nbrs=64, rebuild=True, passes=passes)
        graphk_full = timed(lambda: capk_full.replay(check=False), passes)
        capk_full.status()
        outs[prec] = {k: v.clone() for k, v in capk_full.out.items()}
        ms_eval = min(eager_eval, graph_eval, graphk_eval)
        ms_full = min(eager_full, graph_full, graphk_full)
        results[prec] = {"ms_per_step": ms_eval, "atom_steps_per_s": cfg.n / (ms_eval * 1e-3),
                         "with_rebuild_ms_per_step": ms_full,
                         "with_rebuild_atom_steps_per_s": cfg.n / (ms_full * 1e-3),
                         "eager_ms_per_step": eager_eval, "graph_ms_per_step": graph_eval,
                         "graph_passes": passes, "graph_multi_pass_ms_per_step": graphk_eval,
                         "eager_with_rebuild_ms": eager_full, "graph_with_rebuild_ms": graph_full,
                         "graph_multi_pass_with_rebuild_ms": graphk_full,
                         "profiled_with_rebuild_ms": prof_ms, "kernels": kern}
        log(f"[bench] {prec}: evaluation {ms_eval:.4f} ms/step ({cfg.n / (ms_eval * 1e-3):.4g} atom-steps/s; "
            f"eager {eager_eval:.4f}, graph {graph_eval:.4f}, graph x{passes} {graphk_eval:.4f}); "
            f"with neighbor rebuild {ms_full:.4f} ms/step "
            f"({cfg.n / (ms_full * 1e-3):.4g}); kernels (us): "
            + ", ".join(f"{k} {v['avg_us']:.1f}" for k, v in kern.items()))

    # agreement of the two forms on this workload (GPU vs GPU)
    f64 = {k: v.cpu().numpy() for k, v in outs["fp64"].items()}
    mix = {k: v.cpu().numpy() for k, v in outs["mixed"].items()}
    mixed_vs_fp64 = {"forces_max_abs_eVA": float(np.abs(mix["forces"] - f64["forces"]).max()),
                     "gamma_max_rel": float((np.abs(mix["gamma"] - f64["gamma"]) / np.maximum(1, f64["gamma"])).max()),
                     "energy_abs_eV": float(abs(mix["energy"][0] - f64["energy"][0])),
                     "stress_max_abs_eV": float(np.abs(mix["stress"] - f64["stress"]).max())}

    # roofline of the dominant kernel of the evaluation (largest average launch time)
    prec = a.precision
    r = results[prec]
    m = info["m_full"]
    fl = efs_flops_per_atom(pairs_per_atom, info["n_comp"], info["n_rad"], info["contraction_flops"], True,
                            fused_rows=prec == "fp64")
    if r["kernels"]["efs_contract"]["launches"] == 0:   # four lanes: moments and contraction in one launch
        fl = {"efs_moments_contract": fl["efs_moments"] + fl["efs_contract"], "efs_forces": fl["efs_forces"]}
    per_kernel = {}
    for k, f in fl.items():
        us = r["kernels"]["efs_moments" if k == "efs_moments_contract" else k]["avg_us"]
        per_kernel[k] = {"avg_us": us, "flops_per_atom": f, "bound": "alu", "peak_tflops": PEAK_VALU_TFLOPS,
                         "tflops": f * cfg.n / max(us * 1e-6, 1e-12) / 1e12}
    # grade: 2 m^2 FP64 flops per row, or 19 int8 digit products of 2 m^2 ops each
    gform = tuned[prec][2]
    i8 = gform == "int8-slices"
    gf = 2.0 * m * m * (GRADE_I8_PRODUCTS if i8 else 1)
    gus = r["kernels"]["grade"]["avg_us"]
    # the grade kernel alone: back-to-back launches on the evaluation's own
    # rows (mtp_grade_rows, the same kernel form), between two events -- the
    # per-launch events of the profiled pass add their own time to each launch
    g_rows = api.grade(model, batch, nbrs, prec, "full", rows=True)["rows"]
    g_cm = torch.zeros(api.row_stride(m, prec), cfg.n, dtype=torch.float64, device=g_rows.device)
    g_cm[:m] = g_rows.t()
    g_cm = g_cm.contiguous()
    g_out = api.grade_rows(model, g_cm, prec, "full")
    for _ in range(5):
        api.grade_rows(model, g_cm, prec, "full", out=g_out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(100):
        api.grade_rows(model, g_cm, prec, "full", out=g_out)
    e1.record()
    torch.cuda.synchronize()
    gus_alone = e0.elapsed_time(e1) * 1e3 / 100
    log(f"[bench] grade kernel alone ({gform}): {gus_alone:.1f} us per launch ({gus:.1f} us in the profiled step)")
    per_kernel["grade"] = {"avg_us": gus, "flops_per_atom": gf, "bound": "mfma", "form": gform,
                           "peak_tflops": PEAK_MFMA_I8_TOPS if i8 else PEAK_MFMA_F64_TFLOPS,
                           "unit": "TOP/s (int8)" if i8 else "TFLOP/s",
                           "tflops": gf * cfg.n / max(gus * 1e-6, 1e-12) / 1e12}
    dom = max(per_kernel, key=lambda k: per_kernel[k]["avg_us"])
    d = dict(per_kernel[dom])
    if dom == "grade":   # its rate from the launches without per-launch events
        d["avg_us_in_step"] = d["avg_us"]
        d["avg_us"] = gus_alone
        d["tflops"] = gf * cfg.n / max(gus_alone * 1e-6, 1e-12) / 1e12
    # with grades the moments and contraction run in FP64 in both forms (FP64 rows)
    mc8 = "8" if tuned[prec][0] == 8 else ""
    rocprof_name = {"efs_moments": f"efs_moments<double, {level}, {tuned[prec][0]}>",
                    "efs_moments_contract": f"efs_moments_contract{mc8}<double, {level}, true>",
                    "efs_contract": f"efs_contract<double, {level}, true>",
                    # FP64 with forces and FULL rows: the pair pass carries the rows (R = 2)
                    "efs_forces": (f"efs_forces_fused<double, {level}, {tuned[prec][1]}, 2>" if prec == "fp64" else
                                   f"efs_forces_rows<float, double, {level}, {tuned[prec][1]}>"),
                    "grade": {"int8-slices": f"grade_i8<{(m + 63) // 64}>", "fp64-registers": "grade_f64<",
                              "fp64-lds": "grade_f64_wide<", "fp64-registers-32-row-blocks": "grade_f64_pair<",
                              "fp64-k-outer": f"grade_f64_kouter<{(m + 31) // 32}, 8, 1>",
                              "fp64-k-outer-2-step-chunks": f"grade_f64_kouter<{(m + 31) // 32}, 2, 2>"}[gform]}[dom]
    traffic = recorded_traffic(rocprof_name)
    # the rate this part sustains on the grade's MFMA form (register operands, no memory)
    ceiling = {"f64_tflops": api.mfma_rate("f64"), "i8_tops": api.mfma_rate("i8")}
    log(f"[bench] sustained MFMA rate: FP64 {ceiling['f64_tflops']:.1f} TFLOP/s, int8 {ceiling['i8_tops']:.0f} TOP/s")
    out = {
        "metric": "atom-steps/s (E+F+stress+grade), level-16 MTP",
        "value": r["atom_steps_per_s"],
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": r["ms_per_step"],
        "launch": {r["eager_ms_per_step"]: "eager", r["graph_ms_per_step"]: "hip-graph replay, one pass",
                   r["graph_multi_pass_ms_per_step"]: f"hip-graph replay, {r['graph_passes']} passes per replay"}[
                       r["ms_per_step"]],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else "f64 rows + f32 pair gradients + i8 slice MFMA",
        "data": "synthetic (seeded FCC alloy, seeded teacher potential)",
        "config": {"workload": "fcc-alloy-16x16x16-level16-2species", "atoms": cfg.n, "level": level,
                   "n_types": n_types, "r_cut": w.r_cut, "grade_mode": "full", "m": m,
                   "pairs_per_atom": pairs_per_atom,
                   "step": "evaluate(E, F, S, site energies, b rows, gamma, argmax) + preselection gamma > 2 (fused) "
                           "on a built neighbor list",
                   "lanes_per_neighborhood": {"moments_contraction": tuned[prec][0], "pair_gradients": tuned[prec][1]},
                   "grade_form": tuned[prec][2]},
        "with_rebuild": {"atom_steps_per_s": r["with_rebuild_atom_steps_per_s"],
                         "ms_per_step": r["with_rebuild_ms_per_step"],
                         "neighbor_build_us": r["kernels"]["neighbors"]["avg_us"]},
        "roofline": {"bound": d["bound"], "achieved": d["tflops"], "peak": d["peak_tflops"],
                     "unit": d.get("unit", "TFLOP/s"),
                     "frac": d["tflops"] / d["peak_tflops"], "traffic": traffic, "kernel": rocprof_name,
                     "flops_per_atom": d["flops_per_atom"], "atoms_per_launch": cfg.n, "avg_us": d["avg_us"],
                     "avg_us_in_step": d.get("avg_us_in_step"),
                     "sustained_mfma": ceiling,
                     "frac_of_sustained": (d["tflops"] / (ceiling["i8_tops"] if i8 else ceiling["f64_tflops"])
                                           if d["bound"] == "mfma" else None)},
        "evaluation_kernels": per_kernel,
        "forms": {p: {k: (round(v, 5) if isinstance(v, float) else v) for k, v in res.items() if k != "kernels"}
                  | {"kernels_us": {k: round(x["avg_us"], 2) for k, x in res["kernels"].items()}}
                  for p, res in results.items()},
        "mixed_speedup_vs_fp64": results["mixed"]["atom_steps_per_s"] / results["fp64"]["atom_steps_per_s"],
        "mixed_vs_fp64": mixed_vs_fp64,
    }
    if a.extra_workloads:
        out["extra_workloads"] = extra_workloads(timed, passes)
    if not a.no_cpu_baseline:
        out["cpu_baseline"], out["errors_vs_oracle"] = cpu_baseline(cfg, w, theta, keep, A_full, f64, mix,
                                                                   a.cpu_centers)
    print(json.dumps(out), flush=True)
    return 0


def extra_workloads(timed, passes):
    """The training workload (level 20, 3 species, 512 uneven configurations:
    loss forward + backward through MTPEnergy), the batched uneven evaluation
    at level 24 (1,024 configurations of 16-4096 atoms: E, F, S, site
    energies, eager and HIP-graph replay, both forms), the active-learning
    snapshots (level 16, 1,048,576 atoms: grades + preselection gamma > 2, FULL
    and LINEAR) at their full sizes, and configuration-mode grades of 1,024
    small alloy cells."""
    import torch

    from paper_2304_13144_amd import api, synth

    res = {}
    if 24 in api.compiled_levels():
        w4 = synth.workload4()
        m4 = api.Model.create(w4.level, w4.n_types, w4.r_min, w4.r_cut)
        inf4 = m4.info
        m4.set_params(synth.theta_teacher(4, w4.n_types, inf4["n_lin"], inf4["n_rad"]))
        b4 = api.Batch(w4.configs)
        nb4 = api.Neighbors().build(m4, b4, max_nbrs=64)
        for prec in ("fp64", "mixed"):
            lanes = api.tune(m4, b4, nb4, prec, "full")
            o4 = {"energy": torch.empty(b4.n_cfg, dtype=torch.float64, device=b4.device),
                  "forces": torch.empty((b4.n_atoms, 3), dtype=torch.float64, device=b4.device),
                  "stress": torch.empty((b4.n_cfg, 3, 3), dtype=torch.float64, device=b4.device),
                  "site_e": torch.empty(b4.n_atoms, dtype=torch.float64, device=b4.device)}
            eager = timed(lambda: api.evaluate(m4, b4, nb4, prec, "full", out=o4))
            cap = api.CapturedStep(m4, b4, nb4, prec, "full", max_nbrs=64, rebuild=False, passes=passes,
                                   grades=False)
            graph = timed(lambda: cap.replay(check=False), passes)
            ms = min(eager, graph)
            res[f"batched_level24_{prec}"] = {
                "configs": len(w4.configs), "atoms": b4.n_atoms, "ms_per_step": ms,
                "atom_steps_per_s": b4.n_atoms / (ms * 1e-3), "eager_ms": eager,
                "graph_ms_per_pass": graph, "graph_passes": passes,
                "lanes_per_neighborhood": {"moments": lanes[0], "pair_gradients": lanes[1]},
                "step": "E, F, S, site energies (staged contraction program, no grades)"}
            log(f"[bench] level 24 batch {prec}: {ms:.3f} ms/step ({b4.n_atoms / (ms * 1e-3):.4g} atom-steps/s; "
                f"eager {eager:.3f}, graph x{passes} {graph:.3f})")
        res["batched_level24_mixed_speedup"] = (res["batched_level24_fp64"]["ms_per_step"]
                                                / res["batched_level24_mixed"]["ms_per_step"])
        del m4, b4, nb4
    w = synth.workload3()
    n_lin = {20: 293}[w.level]
    n_rad = {20: 5}[w.level]
    theta = synth.theta_teacher(3, w.n_types, n_lin, n_rad)
    m = api.Model.create(w.level, w.n_types, w.r_min, w.r_cut)
    m.set_params(theta)
    b = api.Batch(w.configs)
    nb = api.Neighbors().build(m, b, max_nbrs=96)
    for prec in ("fp64", "mixed"):
        th = torch.tensor(theta, dtype=torch.float64, device="cuda", requires_grad=True)

        def step():
            E, F, S = api.MTPEnergy.apply(th, m, b, nb, prec)
            ((E ** 2).sum() + 0.01 * (F ** 2).sum() + 0.001 * (S ** 2).sum()).backward()

        ms = timed(step)
        res[f"training_level20_{prec}"] = {"configs": len(w.configs), "atoms": b.n_atoms, "ms_per_step": ms,
                                           "atom_steps_per_s": b.n_atoms / (ms * 1e-3),
                                           "step": "E, F, S forward + loss backward to theta"}
    w5 = synth.workload5()
    m5 = api.Model.create(w5.level, w5.n_types, w5.r_min, w5.r_cut)
    m5.set_params(synth.theta_teacher(5, w5.n_types, 92, 4))
    keep = m5.kept_columns()
    m5.set_active_set("full", synth.active_set(5, "full")[:, keep])
    m5.set_active_set("linear", synth.active_set(5, "linear"))
    for k in (0, 19):
        cfg = synth.workload5_snapshot(k)
        b5 = api.Batch([cfg])
        nb5 = api.Neighbors().build(m5, b5, max_nbrs=64)
        nbuild = timed(lambda: nb5.build(m5, b5, max_nbrs=64, check_status=False))
        for mode in ("full", "linear"):
            o5 = {"gamma": torch.empty(cfg.n, dtype=torch.float64, device=b5.device)}

            def g():
                return api.evaluate(m5, b5, nb5, "fp64", mode, out=o5, gamma_save=2.0)
            ms = timed(g)
            cnt = g()["sel_count"]
            res[f"active_learning_snapshot{k}_{mode}_fp64"] = {
                "atoms": cfg.n, "ms_per_step": ms, "grades_per_s": cfg.n / (ms * 1e-3),
                "selected_gamma_gt_2": int(cnt.item()), "neighbor_build_ms": nbuild}
    # configuration query mode (Sec. II.C) with workload 2's level-16 potential:
    # 1,024 small alloy cells graded against 212 configuration rows (the
    # library's own rows of another pool: a timing input, not a parity one)
    w2 = synth.workload2(reps=(2, 2, 2))
    m2 = api.Model.create(w2.level, w2.n_types, w2.r_min, w2.r_cut)
    m2.set_params(synth.theta_teacher(2, w2.n_types, 92, 4))
    pool = synth.cfg_pool(2, 212, stream=3)
    bp = api.Batch(pool)
    nbp = api.Neighbors().build(m2, bp, max_nbrs=64)
    m2.set_active_set("full_cfg", api.cfg_rows(m2, bp, nbp, "fp64", "full_cfg"))
    cfgs = synth.cfg_pool(2, 1024, stream=4)
    bc = api.Batch(cfgs)
    nbc = api.Neighbors().build(m2, bc, max_nbrs=64)
    for prec in ("fp64", "mixed"):
        ms = timed(lambda: api.grade_cfg(m2, bc, nbc, prec, "full_cfg"))
        g = api.grade_cfg(m2, bc, nbc, prec, "full_cfg")["gamma"]
        res[f"cfg_mode_level16_{prec}"] = {
            "configs": len(cfgs), "atoms": bc.n_atoms, "m": m2.m("full_cfg"), "ms_per_step": ms,
            "configs_per_s": len(cfgs) / (ms * 1e-3), "atom_steps_per_s": bc.n_atoms / (ms * 1e-3),
            "gamma_max": float(g.max().item()),
            "step": "neighborhood rows, per-configuration sums, FP64 grade GEMM (neighbor lists built)"}
    # BFGS fitting of eq. 7 on workload 3 (level 20, 512 configurations):
    # targets of the teacher from the library (a timing input), student =
    # teacher perturbed by 1 %, five iterations; the teacher's own parameter
    # sizes (0.1 for xi_0 and c, 0.1 lambda / s_alpha for xi_alpha, which span
    # many decades) as the diagonal scale
    fit_th = theta * (1.0 + 0.01 * np.random.default_rng([230413144, 3, 2, 9]).normal(size=theta.shape))
    s_alpha, lam = synth.teacher_scales(3)
    fit_scale = np.concatenate([np.full(w.n_types, 0.1), 0.1 * lam / s_alpha, np.full(len(theta) - w.n_types - n_lin,
                                                                                        0.1)])
    m.set_params(theta)
    tgt = api.energy_forces_stress(m, b, nb, "fp64", site_energies=False)
    for prec in ("fp64", "mixed"):
        m.set_params(fit_th)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, hist = api.fit_bfgs(m, b, nb, tgt["energy"], tgt["forces"], tgt["stress"], 1.0, 0.01, 0.001, max_iter=5,
                               precision=prec, scale=fit_scale)
        torch.cuda.synchronize()
        it_ms = (time.perf_counter() - t0) * 1e3 / max(1, len(hist) - 1)
        res[f"fit_bfgs_level20_{prec}"] = {
            "configs": len(w.configs), "atoms": b.n_atoms, "n_theta": len(theta), "iterations": len(hist) - 1,
            "ms_per_iteration": it_ms, "loss_first_last": [float(hist[0]), float(hist[-1])],
            "step": "one BFGS iteration: line-search forward evaluations + one backward, FP64 inverse-Hessian update"}
    # extrapolation-controlled MD on the 1,620-atom FCC(111) slab with the
    # one-species level-16 potential of workload 5 (LINEAR grades against its
    # active set; gamma_break disabled so every step is timed)
    slab = synth.fcc111_slab()
    mp = api.Model.create(16, 1, 2.0, 5.0)
    th = synth.theta_teacher(5, 1, 92, 4)
    mp.set_params(th)
    bs = api.Batch([slab])
    nbs = api.Neighbors().build(mp, bs, max_nbrs=64)
    # this teacher was scaled on BCC snapshots: on the FCC slab, scale xi (E is
    # linear in xi; the LINEAR rows do not depend on it) to max |F| = 0.5 eV/A
    fmax = float(api.energy_forces_stress(mp, bs, nbs)["forces"].abs().max().item())
    th[:93] *= min(1.0, 0.5 / max(fmax, 1e-30))
    mp.set_params(th)
    mp.set_active_set("linear", synth.active_set(5, "linear"))
    vel = torch.as_tensor(np.random.default_rng([230413144, 6, 1, 7]).normal(0.0, 0.002, slab.pos.shape)).cuda()
    api.md_run(mp, bs, nbs, vel, [63.546], 1.0, 2, "fp64", "linear", 2.0, 1e300)   # warm-up
    n_md = 50
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = api.md_run(mp, bs, nbs, vel, [63.546], 1.0, n_md, "fp64", "linear", 2.0, 1e300)
    torch.cuda.synchronize()
    dt_ms = (time.perf_counter() - t0) * 1e3 / n_md
    res["md_fcc111_slab_level16_fp64"] = {
        "atoms": slab.n, "steps": r["steps"], "ms_per_step": dt_ms, "atom_steps_per_s": slab.n / (dt_ms * 1e-3),
        "teacher_xi_scale": min(1.0, 0.5 / max(fmax, 1e-30)),
        "gamma_cfg_first_last": [float(r["gamma"][0]), float(r["gamma"][-1])], "saved_steps_gamma_gt_2": len(r["saved"]),
        "step": "velocity Verlet (dt 1 fs): neighbor rebuild, E/F/S + LINEAR grades, gamma(cfg) to the host"}
    # FIRE relaxation of the same slab from its displaced start (50 steps)
    bs2 = api.Batch([slab])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = api.relax_fire(mp, bs2, api.Neighbors(), [63.546], 1.0, 10.0, 0.0, 50, "fp64", "linear", 2.0, 1e300)
    torch.cuda.synchronize()
    dt_ms = (time.perf_counter() - t0) * 1e3 / max(1, r["steps"])
    res["relax_fire_fcc111_slab_level16_fp64"] = {
        "atoms": slab.n, "steps": r["steps"], "ms_per_step": dt_ms, "atom_steps_per_s": slab.n / (dt_ms * 1e-3),
        "step": "FIRE step: mixing, Euler step, neighbor rebuild, E/F/S + LINEAR grades, norms and gamma(cfg) to "
                "the host"}
    return res


def cpu_baseline(cfg, w, theta, keep, A_full, f64, mix, n_centers):
    """The FP64 oracle on a bounded sample of the same configuration: the
    first n_centers atoms and all their neighbors get site energies, pair
    gradients (forces / stress contributions), rows b_i and grades, on all
    host threads; the same on an eighth of the centers on one thread.  Also
    the GPU-vs-oracle errors: grades and site energies on the sample, and
    energy, forces and stress of the whole configuration (oracle run outside
    the timed sample)."""
    import torch

    from oracle import mtp as om
    from oracle import neighbors as onb

    pot = om.Potential(w.level, w.n_types, w.r_min, w.r_cut)

    def sample(n_c):
        centers = np.arange(max(1, min(n_c, cfg.n)))
        around = onb.neighbors(cfg.pos, cfg.cell, cfg.pbc, w.r_cut, atoms=centers)
        atoms = np.unique(np.concatenate([centers, around.j]))
        pairs = onb.neighbors(cfg.pos, cfg.cell, cfg.pbc, w.r_cut, atoms=atoms)
        t = time.perf_counter()
        _, F, _, V = om.energy_forces_stress(pot, theta, cfg.pos, cfg.types, cfg.cell, pairs)
        rows = om.b_rows(pot, theta, cfg.pos, cfg.types, cfg.cell, pairs, atoms=atoms)[:, keep]
        gam = om.grades(rows, A_full)[0]
        return time.perf_counter() - t, centers, atoms, V, rows, gam

    threads = torch.get_num_threads()
    dt, centers, atoms, V, rows, gam = sample(n_centers)
    torch.set_num_threads(1)
    try:
        dt1, _, atoms1, _, _, _ = sample(max(1, n_centers // 8))
    finally:
        torch.set_num_threads(threads)
    log(f"[bench] oracle sample: {len(atoms)} neighborhoods in {dt:.1f} s on {threads} threads, "
        f"{len(atoms1)} in {dt1:.1f} s on one thread")
    # whole-configuration energy, forces and stress (not timed)
    pairs_all = onb.neighbors(cfg.pos, cfg.cell, cfg.pbc, w.r_cut)
    E, F, S, _ = om.energy_forces_stress(pot, theta, cfg.pos, cfg.types, cfg.cell, pairs_all)
    errs = {}
    for name, g in (("fp64", f64), ("mixed", mix)):
        errs[name] = {"site_e_max_abs": float(np.abs(g["site_e"][atoms] - V[atoms]).max()),
                      "gamma_max_rel": float((np.abs(g["gamma"][atoms] - gam) / np.maximum(1, gam)).max()),
                      "gamma_normwise_rel": float(np.abs(g["gamma"][atoms] - gam).max() / np.abs(gam).max()),
                      "gamma_sample_atoms": int(len(atoms)),
                      "energy_rel": float(abs(g["energy"][0] - E) / abs(E)),
                      "forces_max_abs_eVA": float(np.abs(g["forces"] - F).max()),
                      "forces_normwise_rel": float(np.abs(g["forces"] - F).max() / np.abs(F).max()),
                      "stress_max_abs_eV": float(np.abs(g["stress"][0] - S).max()),
                      "stress_normwise_rel": float(np.abs(g["stress"][0] - S).max() / np.abs(S).max())}
    # what FP32 rows alone would force on a grade: the oracle's rows rounded to
    # FP32, graded in FP64; and the conditioning of A that amplifies it
    g32 = om.grades(rows.astype(np.float32).astype(np.float64), A_full)[0]
    errs["gamma_from_fp32_rows_predicted"] = float((np.abs(g32 - gam) / np.maximum(1, gam)).max())
    errs["kappa_A_column_equilibrated"] = float(np.linalg.cond(A_full / np.abs(A_full).max(axis=0)))
    base = {"value": len(atoms) / dt, "unit": "atom-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(atoms)} neighborhoods ({len(centers)} atoms and all their neighbors) of the same "
                      f"16,384-atom configuration: site energies, pair gradients, rows b_i and grades "
                      f"(neighbor search excluded)", "seconds": dt,
            "single_core": {"value": len(atoms1) / dt1, "unit": "atom-steps/s", "cores": 1,
                            "sample": f"{len(atoms1)} neighborhoods ({max(1, n_centers // 8)} atoms and all their "
                                      f"neighbors), the same steps", "seconds": dt1}}
    return base, errs


if __name__ == "__main__":
    sys.exit(main())
