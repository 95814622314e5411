"""The host planning code (Smith form, plan, twiddles, canonical orders) built
with AddressSanitizer and UndefinedBehaviorSanitizer for the CPU and run on
regular, degenerate and overflowing matrices (no GPU involved)."""
import os
import shutil
import subprocess

import pytest

from oracle.lattice import determinantal_divisors

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MATS = [
    [[8, 0], [0, 8]], [[8, -4], [2, 7]], [[4, 4], [-4, 4]], [[-6, 1], [2, 3]], [[105, 0], [0, 3]],
    [[4096, 8192], [0, 1]], [[65536, 0], [1, 1]], [[3, 1, 0], [0, 2, 1], [1, 0, 4]], [[12, 0, 0], [0, 6, 0], [3, 0, 4]],
    [[1, 0, 0], [0, 256, 0], [0, 0, 256]], [[-127, 62, 1], [-14, 122, 68], [-72, 3, 125]],
    [[2, 0], [0, 1]], [[1, 0], [0, 1]],
]
ERRS = [[[2, 4], [1, 2]], [[1 << 40, 0], [0, 1 << 40]], [[11, 0], [0, 1]]]   # singular, overflow, prime 11


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host compiler")
def test_plan_code_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "plan_driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", os.path.join(ROOT, "tests", "sanitize", "plan_driver.cpp"),
           os.path.join(ROOT, "paper_1605_05712_amd", "csrc", "ahom_plan.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True)
    lines = []
    for M in MATS + ERRS:
        lines.append(" ".join([str(len(M))] + [str(v) for row in M for v in row]))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    out = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True, env=env, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "runtime error" not in out.stderr and "AddressSanitizer" not in out.stderr, out.stderr
    res = out.stdout.strip().splitlines()
    assert len(res) == len(MATS) + len(ERRS)
    for M, r in zip(MATS, res):
        f = r.split()
        assert f[0] == "ok", (M, r)
        e = [int(v) for v in f[2:]]
        assert e == [int(v) for v in determinantal_divisors(M)], (M, e)
    assert [r.split()[0] for r in res[len(MATS):]] == ["err"] * len(ERRS)
