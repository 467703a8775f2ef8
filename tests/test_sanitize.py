"""AddressSanitizer and UndefinedBehaviorSanitizer builds, on the CPU:

* the FP64 oracles (D2Q8 and D3Q14), driven through every boundary kind, the
  smallest and ragged lattices, initial heat flux and wall-flux changes
  (``tests/sanitize/oracle2d_checks.c``, ``oracle3d_checks.c``, gcc);
* the host runtime of the HIP library (``lbm_runtime.cpp``,
  ``d3q14_runtime.cpp``), host code only (``-Xarch_host`` sanitizer flags),
  through the C ABI's validation and sizing paths and a create call on a host
  without a usable GPU (``tests/sanitize/runtime_checks.cpp``).

Any sanitizer report aborts the driver (``-fno-sanitize-recover``, ASan's
default), so the test is its exit status.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2010_01847_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="3")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r.stdout


@pytest.mark.parametrize("driver", ["oracle2d", "oracle3d"])
def test_oracle_under_sanitizers(driver, tmp_path):
    exe = str(tmp_path / driver)
    _run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
          "-fno-omit-frame-pointer", "-Wall", "-Wextra", "-Werror", os.path.join(SAN, f"{driver}_checks.c"), "-o", exe,
          "-lm"])
    out = _run([exe], env=ENV, timeout=600)
    assert "ok" in out


@pytest.mark.skipif(shutil.which(HIPCC) is None and not os.path.exists(HIPCC), reason="hipcc not installed")
def test_runtime_under_sanitizers(tmp_path):
    common = ["-std=c++17", "-fPIC", "--offload-arch=gfx950", "-ffp-contract=off", "-Xclang", "-target-feature",
              "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    san = ["-O1", "-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    objs = []
    for src in (os.path.join(CSRC, "lbm_runtime.cpp"), os.path.join(CSRC, "d3q14_runtime.cpp"),
                os.path.join(SAN, "runtime_checks.cpp")):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        _run([HIPCC] + san + common + ["-x", "hip", "-c", src, "-o", obj])
        objs.append(obj)
    # the device code itself is built without sanitizers (it only has to link)
    for name in ("lbm_device", "d3q14_device"):
        built = os.path.join(ROOT, "paper_2010_01847_amd", "_build", name + ".o")
        if not os.path.exists(built):
            built = str(tmp_path / (name + ".o"))
            _run([HIPCC, "-O3"] + common + ["-x", "hip", "-c", os.path.join(CSRC, name + ".hip"), "-o", built])
        objs.append(built)
    exe = str(tmp_path / "runtime_checks")
    _run([HIPCC, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
         + objs + ["-o", exe])
    out = _run([exe], env=ENV, timeout=300)
    assert "runtime sanitizer checks: ok" in out
