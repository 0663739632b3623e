"""The library's host code (the C ABI's validation, unit conversion, state layout and the
pair-once row check) built with AddressSanitizer and UndefinedBehaviorSanitizer on the host side
only (the device code is compiled as usual), and run through tests/host_sanitize_main.cpp,
which needs no GPU: an out-of-bounds access, a use of freed memory or undefined behaviour in
those paths aborts the run."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _clangxx():
    for c in ("amdclang++", "/opt/rocm/llvm/bin/clang++", "/opt/rocm/lib/llvm/bin/clang++"):
        p = shutil.which(c) or (c if os.path.exists(c) else None)
        if p:
            return p
    return None


@pytest.mark.skipif(shutil.which("hipcc") is None or _clangxx() is None, reason="needs hipcc and clang++")
def test_host_code_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    from paper_1307_3711_amd import build as B
    objs = [os.path.join(B.HERE, "_build", f) for f in ("force.o", "step.o", "mlp.o")]
    if not all(os.path.exists(o) for o in objs):
        pytest.skip("the library's objects are not built")
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    api_o = str(tmp_path / "api.o")
    lib = str(tmp_path / "liblcmd_san.so")
    flags = [f for f in B.FLAGS if f != "-shared"]
    subprocess.check_call(["hipcc"] + flags + host_san + ["-c", "-o", api_o, os.path.join(B.CSRC, "api.hip")],
                          stderr=subprocess.DEVNULL)
    subprocess.check_call(["hipcc"] + B.FLAGS + host_san + ["-o", lib, api_o] + objs, stderr=subprocess.DEVNULL)
    exe = str(tmp_path / "host_sanitize")
    subprocess.check_call([_clangxx(), "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-o", exe,
                           os.path.join(HERE, "host_sanitize_main.cpp"), lib, "-Wl,-rpath," + str(tmp_path)])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
    assert "bad 0" in r.stdout
