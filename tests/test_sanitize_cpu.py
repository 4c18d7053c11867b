"""The library's host code (vfp.cpp: argument checks, context set-up, the
host tables; shtab.cpp: the spherical-harmonic matrices and harmonics) built
with AddressSanitizer and UndefinedBehaviorSanitizer on the host side only
(the device code of the other translation units is linked unchanged), then
run through tests/sanitize/host_checks.c on the CPU: any invalid access,
leak-free misuse or undefined behaviour on those paths stops the run.  Needs
the objects of a normal build in _build/ (python -m paper_2501_05110_amd.build)."""

import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2501_05110_amd", "csrc")
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    return None


def test_host_code_under_sanitizers(tmp_path):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not found")
    dev_objs = [o for o in glob.glob(os.path.join(ROOT, "_build", "*.hip.o")) if "_DVFP" not in os.path.basename(o)]
    if not dev_objs:
        pytest.skip("no build objects in _build/ (run python -m paper_2501_05110_amd.build)")
    inc = ["-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
    common = ["-O1", "-g", "-fPIC", *HOST_SAN, *inc]
    objs = []
    for src in ("vfp.cpp", "shtab.cpp"):
        o = str(tmp_path / (src + ".o"))
        r = subprocess.run([hipcc, "-std=c++17", *common, "-c", os.path.join(CSRC, src), "-o", o],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        objs.append(o)
    drv = str(tmp_path / "host_checks.o")
    r = subprocess.run([hipcc, *common, "-x", "c", "-c", os.path.join(ROOT, "tests", "sanitize", "host_checks.c"),
                        "-o", drv], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    exe = str(tmp_path / "host_checks")
    r = subprocess.run([hipcc, *HOST_SAN, drv, *objs, *sorted(dev_objs), "-o", exe, "-lm"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["HIP_VISIBLE_DEVICES"] = ""      # host paths only, also where a GPU is present
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ok: 0 failure(s)" in out, out[-2000:]
