"""The library's host code (symbolic analysis, host factorization, plan
construction, tune tables, the C ABI's host entry points) under
AddressSanitizer and UndefinedBehaviorSanitizer: built from the sources with
the device launchers stubbed out (tests/host_san/driver.cpp), then run on
random and malformed patterns.  CPU only."""

import json
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1604_02528_amd", "csrc")


def _hipcc():
    for c in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    return None


@pytest.mark.slow
def test_host_code_under_asan_and_ubsan(tmp_path):
    cc = _hipcc()
    if cc is None:
        pytest.skip("hipcc not found")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = ["-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-x", "hip", "-I", os.path.join(ROOT, "include"),
             "-I", CSRC, "-pthread"]
    exe = str(tmp_path / "driver")
    srcs = [os.path.join(CSRC, f) for f in ("symbolic.cpp", "factor_host.cpp", "tune.cpp", "capi.cpp")]
    srcs.append(os.path.join(ROOT, "tests", "host_san", "driver.cpp"))
    cmd = [cc, *flags, *san, *srcs, "-o", exe, "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    # a tune table for some of the runs
    table = tmp_path / "tune.json"
    key = dict(kv.split("=") for kv in _tune_key().split())
    table.write_text(json.dumps({"format": "selinv-tune-1", "entries": [
        {"arch": key["arch"], "rocm": key["rocm"], "dtype": dt, "s_max": 256, "c_max": 1 << 30,
         "dense": 1, "ydense": 1, "split_min_k": 64} for dt in ("f64", "c128")]}))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, str(table)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-6000:])
    assert "0 failures" in r.stdout


def _tune_key():
    from paper_1604_02528_amd import capi

    return capi.selinv_tune_key()
