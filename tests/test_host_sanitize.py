"""The host code of libmsgfem under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

api.hip (plans, band geometry and nested dissection layout, plan options,
deflated-round sizing, coarse-store geometry, errors) is compiled with the
sanitizers on its host side only (each -fsanitize= behind -Xarch_host; the
device code is unchanged), linked with the library's other objects and the
C driver tests/host_sanitize/plan_host.c, and run: it exercises valid and
rejected plans of three meshes, both factor layouts, every option, coarse
stores and destruction, without touching a GPU.  Any sanitizer report
(invalid access, leak, undefined behaviour) or failed expectation fails the
test.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2211_13893_amd")
ROCM = "/opt/rocm"


def _tool(*names):
    for n in names:
        if os.path.exists(n):
            return n
        w = shutil.which(n)
        if w:
            return w
    return None


def test_host_code_sanitized(tmp_path):
    hipcc = _tool(f"{ROCM}/bin/hipcc", "hipcc")
    clang = _tool(f"{ROCM}/llvm/bin/clang")
    clangxx = _tool(f"{ROCM}/llvm/bin/clang++")
    if not (hipcc and clang and clangxx):
        pytest.skip("ROCm toolchain not found")
    from paper_2211_13893_amd import build
    objs = [os.path.join(PKG, "_build", s.replace(".hip", ".o")) for s in build.SOURCES if s != "api.hip"]
    if not all(os.path.exists(o) for o in objs):
        build.build()
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc")]
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer"]
    api = str(tmp_path / "api_san.o")
    subprocess.run([hipcc, "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + san + inc +
                   ["-c", os.path.join(PKG, "csrc", "api.hip"), "-o", api], check=True)
    drv = str(tmp_path / "plan_host.o")
    subprocess.run([clang, "-g", "-O1", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                    "-I", os.path.join(ROOT, "include"), "-c",
                    os.path.join(ROOT, "tests", "host_sanitize", "plan_host.c"), "-o", drv], check=True)
    exe = str(tmp_path / "plan_host")
    subprocess.run([clangxx, "-fsanitize=address,undefined", "-o", exe, drv, api] + objs +
                   [f"-L{ROCM}/lib", "-lamdhip64", f"-Wl,-rpath,{ROCM}/lib"], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, timeout=300)
    out = r.stdout.decode(errors="replace")
    print(out)
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out
    assert "all host checks passed" in out
