"""Builds libmtp.so in-tree for gfx950.

Steps: compile the basis generator (g++) -> write one contraction header per
level -> one HIP translation unit per level with the fused kernel
instantiated for it (forward and backward, FP64 and FP32: four units per
level) -> compile every unit with hipcc in parallel -> link.

    python -m paper_2304_13144_amd.build [--levels 8,16] [-j 8]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(os.path.dirname(HERE), "_build")
GEN = os.path.join(BUILD, "gen")
LIB = os.path.join(HERE, "libmtp.so")

DEFAULT_LEVELS = (2, 4, 6, 8, 12, 16, 20, 24)
ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_FLAGS = ["-O3", f"--offload-arch={ARCH}", "-std=c++17", "-fPIC", "-Wno-unused-result",
             # no packed FP32 instructions anywhere in the device code
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", CSRC, "-I", GEN]
# units compiled with the machine scheduler's ILP strategy: the level-16 FP64
# moments / contraction kernel runs one wavefront per SIMD and waits on LDS
# results; scheduled for ILP it measured 21.4 -> 20.6 us per launch on the
# 16,384-atom alloy, while the pair pass measured slower under it (29.3 -> 32.3
# us) and keeps the default scheduler in a unit of its own
ILP_UNITS = ("efs_level16_f64_mc.hip",)
ILP_FLAGS = ["-mllvm", "--amdgpu-sched-strategy=max-ilp"]
HOST_SOURCES = ["api.cpp", "basis.cpp", "prof.cpp"]
# what the generated per-level units include (besides their level's program)
KERNEL_HEADERS = ["efs_kernel.hpp", "backward_kernel.hpp", "kernel_args.hpp", "device_util.hpp"]
HIP_SOURCES = ["neighbors.hip", "ops.hip", "grade.hip"]


def _run(cmd):
    t = time.time()
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + p.stdout + p.stderr)
    return time.time() - t


STAGE_R_PER_UNIT = 4   # reverse parts per translation unit of a staged level


def generate(levels):
    os.makedirs(GEN, exist_ok=True)
    gen_exe = os.path.join(BUILD, "gen_contract")
    _run(["g++", "-O2", "-std=c++17", "-o", gen_exe, os.path.join(CSRC, "gen_contract.cpp"),
          os.path.join(CSRC, "basis.cpp")])
    tmp = os.path.join(BUILD, "gen_tmp")
    if os.path.isdir(tmp):
        for f in os.listdir(tmp):
            os.remove(os.path.join(tmp, f))
    os.makedirs(tmp, exist_ok=True)
    _run([gen_exe, tmp] + [str(L) for L in levels])
    for f in os.listdir(tmp):   # keep the mtime of unchanged programs (incremental builds)
        _write_if_changed(os.path.join(GEN, f), open(os.path.join(tmp, f)).read())
    flops, staged = {}, {}
    for L in levels:
        txt = open(os.path.join(GEN, f"mtp_level{L}.inc")).read()
        flops[L] = sum(int(txt.split(f"FLOPS_{k} = ")[1].split(";")[0]) for k in ("GRAPHS", "TRIE", "REVERSE"))
        if "STAGED = true" in txt:   # (graph parts, reverse parts, graphs)
            staged[L] = (int(txt.split("STAGE_G = ")[1].split(",")[0]), int(txt.split("STAGE_R = ")[1].split(";")[0]),
                         int(txt.split("NGRAPH = ")[1].split(";")[0]))
    units = []

    def unit(name, body):
        path = os.path.join(GEN, name)
        _write_if_changed(path, body)
        units.append(path)

    for L in levels:   # units per (level, arithmetic type, forward / backward): they compile in parallel
        for T, tag in (("double", "f64"), ("float", "f32")):
            if L not in staged:
                # moments / contraction and the pair pass in units of their own
                # (ILP_UNITS compiles some of them differently), then the backward
                for name, macro in ((f"efs_level{L}_{tag}_mc", "MTP_EFS_MC_LEVEL_T"),
                                    (f"efs_level{L}_{tag}_fr", "MTP_EFS_FR_LEVEL_T"),
                                    (f"bwd_level{L}_{tag}", "MTP_BWD_LEVEL_T")):
                    unit(f"{name}.hip",
                         f'#include "efs_kernel.hpp"\n#include "backward_kernel.hpp"\nnamespace mtp {{\n'
                         f'#include "mtp_level{L}.inc"\n{macro}({L}, {T})\n}}  // namespace mtp\n')
                continue
            ng, nr, _ = staged[L]
            # the staged program: moments + trie walk + pair gradients in one unit, the graph
            # parts in one, the reverse parts in units of STAGE_R_PER_UNIT
            decl = "".join(f"template <> void launch_graphs_stage<{L}, {T}, {q}>(const EfsArgs &a);\n" for q in range(ng))
            decl += "".join(f"template <> void launch_reverse_stage<{L}, {T}, {q}>(const EfsArgs &a);\n" for q in range(nr))
            unit(f"efs_level{L}_{tag}.hip",
                 f'#include "efs_staged.hpp"\nnamespace mtp {{\n#include "mtp_level{L}.inc"\n{decl}'
                 f'MTP_EFS_STAGED_LEVEL_T({L}, {T})\nMTP_EFS_FR_LEVEL_T({L}, {T})\n}}  // namespace mtp\n')
            unit(f"stg_level{L}_{tag}_g.hip",
                 f'#include "efs_staged.hpp"\nnamespace mtp {{\n#include "mtp_level{L}.inc"\n'
                 + "".join(f'#include "mtp_level{L}_g{q}.inc"\nMTP_STAGE_G_T({L}, {T}, {q})\n' for q in range(ng))
                 + "}  // namespace mtp\n")
            for u in range(0, nr, STAGE_R_PER_UNIT):
                unit(f"stg_level{L}_{tag}_r{u // STAGE_R_PER_UNIT}.hip",
                     f'#include "efs_staged.hpp"\nnamespace mtp {{\n#include "mtp_level{L}.inc"\n'
                     + "".join(f'#include "mtp_level{L}_r{q}.inc"\nMTP_STAGE_R_T({L}, {T}, {q})\n'
                               for q in range(u, min(nr, u + STAGE_R_PER_UNIT)))
                     + "}  // namespace mtp\n")
    plain = [L for L in levels if L not in staged]
    decl = "".join(f"template <> int launch_mc_level_t<{L}, {T}>(const EfsArgs &a);\n"
                   f"template <> int launch_fr_level_t<{L}, {T}, {T}>(const EfsArgs &a);\n"
                   for L in levels for T in ("double", "float"))
    decl += "".join(f"template <> int launch_backward_level_t<{L}, {T}>(const BwdArgs &b);\n"
                    for L in plain for T in ("double", "float"))
    decl += "".join(f"template <> int launch_fr_level_t<{L}, float, double>(const EfsArgs &a);\n" for L in levels)
    # moments / contraction in FP64 for the FP64 form and for the mixed form when
    # it writes rows (rows are FP64); pair gradients in the form's own type
    mc = "".join(f"        case {L}: e = mc64 ? launch_mc_level_t<{L}, double>(a) : launch_mc_level_t<{L}, float>(a); break;\n"
                 for L in levels)
    fr = "".join(f"        case {L}: return f64 ? launch_fr_level_t<{L}, double, double>(a)\n"
                 f"                     : (mc64 ? launch_fr_level_t<{L}, float, double>(a) : launch_fr_level_t<{L}, float, float>(a));\n"
                 for L in levels)
    bcases = "".join(f"        case {L}: return f64 ? launch_backward_level_t<{L}, double>(b) : "
                     f"launch_backward_level_t<{L}, float>(b);\n" for L in plain)
    scases = "".join(f"        case {L}: return {staged[L][2]};\n" for L in staged)
    disp = ('#include "internal.hpp"\nnamespace mtp {\n'
            + "template <int L, typename T> int launch_mc_level_t(const EfsArgs &a);\n"
            + "template <int L, typename TF, typename TD> int launch_fr_level_t(const EfsArgs &a);\n"
            + "template <int L, typename T> int launch_backward_level_t(const BwdArgs &b);\n"
            + decl + "int launch_efs(int level, const EfsArgs &a) {\n    const bool f64 = a.precision == MTP_FP64;\n"
            + "    const bool mc64 = f64 || a.brow != nullptr;\n    int e = 0;\n"
            + "    switch (level) {\n" + mc + "        default: return -1;\n    }\n    if (e) return e;\n"
            + "    switch (level) {\n" + fr
            + "        default: return -1;\n    }\n}\n"
            + "int launch_backward(int level, const BwdArgs &b) {\n    const bool f64 = b.e.precision == MTP_FP64;\n"
            + "    switch (level) {\n" + bcases
            + "        default: return -1;\n    }\n}\n"
            + "int staged_graphs(int level) {\n    switch (level) {\n" + scases
            + "        default: return 0;\n    }\n}\n"
            + "std::vector<int> compiled_levels() { return {"
            + ", ".join(str(L) for L in levels) + "}; }\nlong contraction_flops(int level) {\n    switch (level) {\n"
            + "".join(f"        case {L}: return {flops[L]};\n" for L in levels)
            + "        default: return 0;\n    }\n}\n}  // namespace mtp\n")
    dpath = os.path.join(GEN, "dispatch.cpp")
    _write_if_changed(dpath, disp)
    return units, dpath


def _write_if_changed(path, text):
    if os.path.exists(path) and open(path).read() == text:
        return
    with open(path, "w") as fh:
        fh.write(text)


def _stale(src, obj, deps_mtime):
    return not os.path.exists(obj) or os.path.getmtime(obj) < max(os.path.getmtime(src), deps_mtime)


def build(levels=DEFAULT_LEVELS, jobs=None, verbose=True, force=True):
    """force=False recompiles only units older than their source or any
    header / generated program (development loop); the default rebuilds all."""
    t0 = time.time()
    units, dispatch = generate(levels)
    mt = os.path.getmtime
    # the per-level units see only the kernel headers and their level's program
    kernel_mtime = max(mt(d) for d in [os.path.join(CSRC, f) for f in KERNEL_HEADERS] + [os.path.abspath(__file__)])
    staged_mtime = max(kernel_mtime, mt(os.path.join(CSRC, "efs_staged.hpp")))
    deps = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))]
    deps += [os.path.join(os.path.dirname(HERE), "include", "mtp.h"), os.path.abspath(__file__)]
    host_mtime = max(mt(d) for d in deps)
    objs = []
    jobs_list = []
    for src in [os.path.join(CSRC, s) for s in HOST_SOURCES + HIP_SOURCES] + [dispatch] + units:
        obj = os.path.join(BUILD, os.path.basename(src) + ".o")
        objs.append(obj)
        if src in units:
            level = "".join(ch for ch in os.path.basename(src).split("_")[1] if ch.isdigit())
            progs = [f for f in os.listdir(GEN) if f == f"mtp_level{level}.inc" or f.startswith(f"mtp_level{level}_")]
            staged_unit = any(f.startswith(f"mtp_level{level}_") for f in progs)
            dm = max([staged_mtime if staged_unit else kernel_mtime] + [mt(os.path.join(GEN, f)) for f in progs])
        else:
            dm = host_mtime
        if force or _stale(src, obj, dm):
            extra = ILP_FLAGS if os.path.basename(src) in ILP_UNITS else []
            jobs_list.append([HIPCC] + HIP_FLAGS + extra + ["-c", src, "-o", obj])
    n = jobs or min(8, os.cpu_count() or 4)
    # longest units first (the backward units of the highest levels)
    jobs_list.sort(key=lambda c: ("bwd_level" not in c[-3], -int(''.join(ch for ch in os.path.basename(c[-3]) if ch.isdigit()) or 0)))
    with cf.ThreadPoolExecutor(n) as ex:
        times = list(ex.map(_run, jobs_list)) or [0.0]
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    if verbose:
        slow = sorted(zip(times, jobs_list), key=lambda t: -t[0])[:1]
        what = f"slowest unit {slow[0][0]:.1f}s: {os.path.basename(slow[0][1][-3])}" if slow else "nothing to compile"
        print(f"[build] libmtp.so with levels {list(levels)} in {time.time() - t0:.1f}s "
              f"({len(jobs_list)} units compiled, {what})", flush=True)
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--levels", default=",".join(str(L) for L in DEFAULT_LEVELS))
    ap.add_argument("-j", type=int, default=None)
    ap.add_argument("--incremental", action="store_true", help="compile only out-of-date units")
    a = ap.parse_args(argv)
    build(tuple(int(x) for x in a.levels.split(",")), a.j, force=not a.incremental)


if __name__ == "__main__":
    sys.exit(main())
