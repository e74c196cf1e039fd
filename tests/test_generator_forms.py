"""The two forms the contraction generator writes -- one program per level
(graph values as sums of prefix products, trie walk in registers) and the
staged program of the large levels (graph values in Horner form over each
graph's factor-prefix tree, trie walk streaming its graph values and dV/dg
through memory, reverse pass in parts) -- compute the same V, B_alpha and
dV/dM: both compiled for the host and compared on random moments."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2304_13144_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
@pytest.mark.parametrize("level", [12, 16])
def test_staged_program_equals_single_program(level, tmp_path):
    gen = tmp_path / "gen_contract"
    subprocess.run(["g++", "-O1", "-std=c++17", "-o", str(gen), os.path.join(CSRC, "gen_contract.cpp"),
                    os.path.join(CSRC, "basis.cpp")], check=True)
    single, staged = tmp_path / "single", tmp_path / "staged"
    single.mkdir()
    staged.mkdir()
    subprocess.run([str(gen), str(single), "--single", str(level)], check=True, capture_output=True)
    out = subprocess.run([str(gen), str(staged), "--staged", str(level)], check=True, capture_output=True, text=True)
    txt = (staged / f"mtp_level{level}.inc").read_text()
    ng = int(txt.split("STAGE_G = ")[1].split(",")[0])
    nr = int(txt.split("STAGE_R = ")[1].split(";")[0])
    parts = "".join(f'#include "{staged}/mtp_level{level}_g{q}.inc"\n' for q in range(ng))
    parts += "".join(f'#include "{staged}/mtp_level{level}_r{q}.inc"\n' for q in range(nr))
    (tmp_path / "parts.inc").write_text(parts)
    exe = tmp_path / "check"
    subprocess.run(["g++", "-O1", "-std=c++17", f"-DLV={level}", f'-DLEVEL_A="{single}/mtp_level{level}.inc"',
                    f'-DLEVEL_B="{staged}/mtp_level{level}.inc"', "-I", str(tmp_path),
                    os.path.join(HERE, "staged_check.cpp"), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    print(out.stdout.strip(), "|", r.stdout.strip())
    assert r.returncode == 0, r.stdout
