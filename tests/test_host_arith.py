"""CPU checks of host-compilable code, plain and under the address and
undefined-behaviour sanitizers:
  - the library's modular-arithmetic helpers (Barrett reductions and balanced
    digit splits of the 32-bit paths, the reciprocal 128/64 remainder and the
    per-modulus constants of the 64-bit paths) against 128-bit integers;
  - the C oracle, driven through its pins' small cases by a C program.
Nothing here touches a GPU: the library's helpers are compiled host-only."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2307_06554_amd", "csrc")
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all"]


def _hipcc_host(src, out, sanitize):
    cmd = ["hipcc", "-x", "hip", "--offload-host-only", "-std=c++17", "-O2", "-I", CSRC, src, "-o", out]
    if sanitize:
        for f in SAN:
            cmd[1:1] = ["-Xarch_host", f]  # host code only: never a sanitized device build
    subprocess.run(cmd, check=True, capture_output=True, text=True)


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not found")
@pytest.mark.parametrize("sanitize", [False, True], ids=["plain", "asan_ubsan"])
def test_library_modular_arithmetic(tmp_path, sanitize):
    exe = str(tmp_path / "check_modarith")
    _hipcc_host(os.path.join(HERE, "host", "check_modarith.cpp"), exe, sanitize)
    for seed in ("1", "2"):
        res = subprocess.run([exe, seed], capture_output=True, text=True, timeout=300)
        assert res.returncode == 0, res.stdout + res.stderr
        assert res.stdout.startswith("ok "), res.stdout
        assert int(res.stdout.split()[1]) > 1_000_000


@pytest.mark.parametrize("sanitize", [False, True], ids=["plain", "asan_ubsan"])
def test_oracle_under_sanitizers(tmp_path, sanitize):
    exe = str(tmp_path / "oracle_drive")
    cmd = ["gcc", "-O1", "-std=c11", "-fopenmp", os.path.join(ROOT, "oracle", "polymul_oracle.c"),
           os.path.join(HERE, "host", "oracle_drive.c"), "-o", exe]
    if sanitize:
        cmd[1:1] = SAN
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, OMP_NUM_THREADS="2")
    res = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert res.returncode == 0, res.stdout + res.stderr
    assert res.stdout.startswith("ok "), res.stdout
