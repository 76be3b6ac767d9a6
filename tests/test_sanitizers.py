"""Host sanitizer builds, CPU only: the oracle's C walk and the host side of
the C ABI (argument checks, workspace sizing, the medium and size-bin
derivations) built with AddressSanitizer and UndefinedBehaviorSanitizer and
run through drivers that exercise them (tests/sanitize/*.c).  GPU code is
compiled as usual; the sanitizers apply to host code only, and no driver
does device work."""
import hashlib
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
OUT = os.path.join(HERE, "_build")
CSRC = os.path.join(ROOT, "paper_2507_23189_amd", "csrc")
LIB_SOURCES = ["capi.cpp", "mie_table.hip", "walk.hip", "metrics.hip"]
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")

pytestmark = pytest.mark.slow


def _digest(paths):
    h = hashlib.sha256()
    for p in paths:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def _tool(name):
    path = shutil.which(name) or os.path.join("/opt/rocm/bin", name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not found")
    return path


def test_oracle_walk_under_sanitizers():
    src = os.path.join(HERE, "oracle_driver.c")
    deps = [src, os.path.join(ROOT, "oracle", "walk.c")]
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, f"oracle_san_{_digest(deps)}")
    if not os.path.exists(exe):
        subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-D_DEFAULT_SOURCE", "-ffp-contract=off",
                        "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                        src, "-o", exe, "-lm"], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, env=SAN_ENV, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("OK"), r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr


def test_capi_host_checks_under_sanitizers():
    hipcc = _tool("hipcc")
    clang = "/opt/rocm/llvm/bin/clang"
    clangxx = "/opt/rocm/llvm/bin/clang++"
    driver = os.path.join(HERE, "capi_driver.c")
    header = os.path.join(ROOT, "include", "mcmie.h")
    deps = [driver, header] + [os.path.join(CSRC, s) for s in LIB_SOURCES + ["common.hpp", "philox.hpp"]]
    os.makedirs(OUT, exist_ok=True)
    tag = _digest(deps)
    exe = os.path.join(OUT, f"capi_san_{tag}")
    if not os.path.exists(exe):
        objs = []
        for s in LIB_SOURCES:
            obj = os.path.join(OUT, f"{os.path.splitext(s)[0]}_{tag}.o")
            subprocess.run([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}", "-c", os.path.join(CSRC, s), "-o", obj], check=True, capture_output=True)
            objs.append(obj)
        dobj = os.path.join(OUT, f"capi_driver_{tag}.o")
        subprocess.run([clang, "-O1", "-g", "-fsanitize=address,undefined", f"-I{os.path.join(ROOT, 'include')}",
                        "-c", driver, "-o", dobj], check=True)
        subprocess.run([clangxx, "-fsanitize=address,undefined", *objs, dobj, "-o", exe, "-L/opt/rocm/lib",
                        "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, env=SAN_ENV, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("OK"), r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
