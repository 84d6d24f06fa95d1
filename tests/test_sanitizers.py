"""Host code under the address and undefined-behaviour sanitizers (CPU).

The scene validation of the C ABI (`csrc/validate.cpp`, host only) is built
with g++ and the sanitizers into a driver that feeds it a hand-built
hierarchy, every malformed case it names and seeded random corruptions; the
oracle's C sources are built with gcc and the sanitizers and the oracle's
own CPU test files are run against that build.  Any invalid read or write,
signed overflow or other undefined behaviour aborts the run."""
import os
import subprocess
import sys

import pytest

from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
ENV_SAN = {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True,
                          check=True).stdout.strip()
    if not os.path.isabs(path):
        pytest.skip(f"{name} is not installed")
    return path


def test_scene_validation_under_sanitizers(tmp_path):
    exe = str(tmp_path / "validate_driver")
    csrc = os.path.join(ROOT, "paper_2603_15186_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", "-O1", *SAN, "-I", os.path.join(ROOT, "include"), "-I", csrc,
                    os.path.join(csrc, "validate.cpp"), os.path.join(ROOT, "tests", "sanitize", "validate_driver.cpp"),
                    "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, env={**os.environ, **ENV_SAN}, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "validate_driver: ok" in r.stdout


def test_oracle_under_sanitizers(tmp_path):
    lib = O.build(force=True, out=str(tmp_path / "liboracle_san.so"), extra=SAN)
    env = {**os.environ, **ENV_SAN, O.SAN_ENV: lib, "OMP_NUM_THREADS": "4",
           "LD_PRELOAD": _runtime("libasan.so") + ":" + _runtime("libubsan.so")}
    files = ["test_oracle_pins.py", "test_learned_cut_oracle.py", "test_blend_oracle.py", "test_slice_oracle.py",
             "test_nav_oracle.py"]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-p", "no:xdist",
                        *[os.path.join(ROOT, "tests", f) for f in files]],
                       capture_output=True, text=True, env=env, cwd=ROOT, timeout=1200)
    out = r.stdout + r.stderr
    reports = [l for l in out.splitlines() if "Sanitizer" in l or "runtime error" in l]
    tail = "\n".join(reports[:10]) + "\n" + out[-3000:]
    assert r.returncode == 0, tail
    assert "passed" in r.stdout and "failed" not in r.stdout, tail
