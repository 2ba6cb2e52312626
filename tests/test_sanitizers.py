"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host code (CPU
only, no GPU involved).

* The FP64 oracles (D2Q9 and D3Q19), compiled with gcc and the sanitizers into
  the drivers under tests/sanitize/, run every switch, velocity kind, planted
  mistake and the padded-window mode on small ragged and degenerate grids.
* The HIP library, built with the sanitizers on its host code only (the device
  code is compiled without optimisation to keep the build short; no kernel
  runs here), is linked into a C driver that walks the parameter validation of
  every entry point, the status strings and the batched form's host-side
  schedule check (items, neighbour lists and slot tables built by the
  library's own host code).

A sanitizer report aborts the driver, so each test only needs the exit status.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2203_05230_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = {**os.environ, "ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0", "UBSAN_OPTIONS": "print_stacktrace=1",
       "OMP_NUM_THREADS": "2"}


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, (" ".join(cmd), r.stdout[-3000:], r.stderr[-6000:])
    return r


@pytest.mark.parametrize("driver", ["oracle_driver", "oracle3_driver"])
def test_oracle_under_sanitizers(tmp_path, driver):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / driver)
    _run(["gcc", "-g", "-O1", "-fopenmp", *SAN_FLAGS, "-ffp-contract=off", "-std=c11", "-Wall",
          "-I", os.path.join(ROOT, "oracle"), "-o", exe, os.path.join(SAN, driver + ".c"), "-lm"])
    r = _run([exe], env=ENV, timeout=600)
    assert "0 failures" in r.stdout


def test_host_runtime_under_sanitizers(tmp_path):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("hipcc not found")
    sources = ["lbac", "lbac_batch", "lbac_mlp", "lbac_closure", "lbac3"]
    # the sanitizers go on the host code only; the device code is not run here
    host_san = [a for f in SAN_FLAGS for a in ("-Xarch_host", f)]
    procs = []
    for s in sources:
        cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-Xarch_device", "-O0", "-g", "-std=c++17", "-fPIC",
               "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *host_san,
               "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c", "-o", str(tmp_path / (s + ".o")),
               os.path.join(CSRC, s + ".hip")]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
    for cmd, p in procs:
        out, err = p.communicate(timeout=900)
        assert p.returncode == 0, (" ".join(cmd), err[-6000:])
    lib = str(tmp_path / "liblbac_san.so")
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *host_san, "-o", lib,
          *[str(tmp_path / (s + ".o")) for s in sources]])
    exe = str(tmp_path / "abi_driver")
    _run([CLANG, "-g", "-O1", *SAN_FLAGS, "-I", os.path.join(ROOT, "include"), "-o", exe,
          os.path.join(SAN, "abi_driver.c"), "-L", str(tmp_path), "-llbac_san", "-Wl,-rpath," + str(tmp_path), "-lm"])
    r = _run([exe], env=ENV, timeout=600)
    assert "0 failures" in r.stdout
