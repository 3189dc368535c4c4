"""The C ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

tacaw_plan.hip (descriptor checks, the plan's host preparation: windows, the
window's DFT, transform split and tables, mean strategy, error state) is compiled
with both sanitizers on its host side only (its device side is built as usual),
linked with the library's other objects and driven by tests/host_sanitize/
abi_driver.cpp through every path that needs no GPU. Without a GPU each plan stops
at its first device call and must release what it built, which LeakSanitizer
checks. Runs on the CPU; needs the objects build() leaves in _build/."""

import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2607_02236_amd", "csrc")
BUILD = os.path.join(ROOT, "_build")
DRIVER = os.path.join(ROOT, "tests", "host_sanitize", "abi_driver.cpp")
CLANG = "/opt/rocm/llvm/bin/clang++"


def _run(cmd, cwd):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


def test_host_code_under_asan_and_ubsan(tmp_path):
    compiler = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    others = [o for o in glob.glob(os.path.join(BUILD, "*.o"))
              if not os.path.basename(o).startswith("tacaw_plan")]
    if not others or not os.path.exists(CLANG) or not os.path.exists(compiler):
        pytest.skip("needs the library objects from build() and the ROCm compilers")
    inc = "-I" + os.path.join(ROOT, "include")
    # host-side instrumentation only: every sanitizer flag goes through -Xarch_host
    host_san = ["-Xarch_host", "-fsanitize=address",
                "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=undefined",
                "-Xarch_host", "-fno-omit-frame-pointer"]
    plan_obj = str(tmp_path / "plan_san.o")
    _run([compiler, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", inc, *host_san,
          "-c", os.path.join(CSRC, "tacaw_plan.hip"), "-o", plan_obj], tmp_path)
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]
    drv_obj = str(tmp_path / "driver.o")
    _run([CLANG, "-O1", "-g", "-std=c++17", inc, *san, "-c", DRIVER, "-o", drv_obj], tmp_path)
    exe = str(tmp_path / "abi_san")
    _run([CLANG, *san, drv_obj, plan_obj, *others, "-L/opt/rocm/lib", "-lamdhip64",
          "-Wl,-rpath,/opt/rocm/lib", "-o", exe], tmp_path)
    supp = tmp_path / "lsan.supp"
    # allocations the HIP and HSA runtimes keep until exit are theirs, not the library's
    supp.write_text("leak:libamdhip64\nleak:libhsa-runtime64\nleak:libhsakmt\n")
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["LSAN_OPTIONS"] = f"suppressions={supp}"
    r = subprocess.run([exe], cwd=tmp_path, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    print(r.stdout[-2000:])
    assert "ERROR: AddressSanitizer" not in out, out[-4000:]
    assert "ERROR: LeakSanitizer" not in out, out[-4000:]
    assert "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0 and "OK: 0 failed expectations" in r.stdout, out[-4000:]
