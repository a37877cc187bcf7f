"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two programs are built with the sanitizers and run: the CPU oracle
(oracle/oracle.c) driven on small inputs, and the library's host code
(cpmi_host.cpp: tile lists, two-set lists, pruned tile lists, tune-cache
parsing and saving, bounds, layouts) driven through its host-only debug entry
points, linked with the library's other objects as built. The sanitizers are
applied to host code only; the device code of the library is built as usual.
Any report (or a failed check in a driver) fails the test.
"""
import glob
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{cmd[0]} failed ({r.returncode}):\n{r.stdout[-3000:]}\n{r.stderr[-6000:]}"
    return r


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-O1", "-g", "-std=c11", "-march=x86-64-v3", "-ffp-contract=off", "-fopenmp", *SAN,
          os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(HERE, "sanitize", "oracle_driver.c"), "-o", exe,
          "-lm"])
    r = _run([exe], env=dict(ENV, OMP_NUM_THREADS="4"))
    assert r.stdout.strip().endswith("ok")
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr


def _hipcc():
    h = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    return h if os.path.exists(h) else shutil.which("hipcc")


@pytest.mark.skipif(_hipcc() is None, reason="hipcc not found")
def test_library_host_code_under_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_1407_5609_amd", "csrc")
    build = os.path.join(ROOT, "paper_1407_5609_amd", "_build")
    objs = [o for o in sorted(glob.glob(os.path.join(build, "*.o"))) if not o.endswith("cpmi_host.o")]
    if len(objs) < 7:
        import importlib.util
        spec = importlib.util.spec_from_file_location("_cpmi_build", os.path.join(ROOT, "paper_1407_5609_amd",
                                                                                  "build.py"))
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        mod.build()
        objs = [o for o in sorted(glob.glob(os.path.join(build, "*.o"))) if not o.endswith("cpmi_host.o")]
    host_san = [a for f in SAN for a in ("-Xarch_host", f)]
    inc = ["-I", os.path.join(ROOT, "include"), "-I", csrc]
    host_o = str(tmp_path / "cpmi_host_san.o")
    _run([_hipcc(), "-x", "hip", "-O1", "-g", "-std=c++17", "-fPIC", "-ffp-contract=off", "--offload-arch=gfx950",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *host_san, *inc, "-c",
          os.path.join(csrc, "cpmi_host.cpp"), "-o", host_o])
    exe = str(tmp_path / "host_driver")
    _run([_hipcc(), "--offload-arch=gfx950", *host_san, *inc, "-x", "c", os.path.join(HERE, "sanitize",
          "host_driver.c"), "-x", "none", host_o, *objs, "-o", exe])
    r = _run([exe, str(tmp_path)], env=ENV)
    assert r.stdout.strip().endswith("ok")
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
