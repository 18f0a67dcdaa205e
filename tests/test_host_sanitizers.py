"""The library's host code (fss_api.cpp: spec validation, quantisation, key
layouts, argument checks) built with AddressSanitizer and
UndefinedBehaviorSanitizer for the host only and driven on the CPU at the
interface's limits (tests/host/api_sanitize.cpp).  Kernel launchers are
replaced by stand-ins that report they cannot run; no GPU call is made."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2606_09551_amd", "csrc")
INC = os.path.join(ROOT, "include")
CLANG = "/opt/rocm/llvm/bin/clang++"
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, **kw)
    noise = ("packed-fp32-ops", "is not a recognized feature")
    out = "\n".join(l for l in r.stdout.splitlines() if not any(n in l for n in noise))
    return r.returncode, out


def test_host_code_under_asan_and_ubsan(tmp_path):
    if shutil.which("hipcc") is None or not os.path.exists(CLANG):
        pytest.skip("no ROCm toolchain")
    host_only = ["hipcc", "-O1", "-g", "-std=c++17", "-fPIC", "--offload-host-only", "--offload-arch=gfx950",
                 "-I", INC, "-I", CSRC]
    objs = []
    for src, flags in ((os.path.join(CSRC, "fss_api.cpp"), ["-x", "hip", *HOST_SAN]),
                       (os.path.join(HERE, "host", "api_sanitize.cpp"), HOST_SAN),
                       (os.path.join(HERE, "host", "launch_stubs.cpp"), ["-x", "hip"])):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        rc, out = _run(host_only + flags + ["-c", src, "-o", obj])
        assert rc == 0, out[-3000:]
        objs.append(obj)
    exe = str(tmp_path / "api_san")
    link = [CLANG, "-fsanitize=address,undefined", "-o", exe, *objs,
            "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"]
    rc, out = _run(link)
    assert rc == 0, out[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    rc, out = _run([exe], env=env, timeout=300)
    assert rc == 0 and out.strip().endswith("ok"), out[-3000:]
