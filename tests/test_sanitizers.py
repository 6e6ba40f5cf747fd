"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, without a
GPU: the library's host runtime (argument checks, plan and recode checks, the
serving scheduler in dry-run mode) and the oracle, each rebuilt with the
sanitizers and driven by the CPU tests in a child process."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1909_02871_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def _run_child(args, env_extra):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", **env_extra)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", *args], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]


@pytest.mark.slow
def test_host_runtime_under_sanitizers(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    rt = glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not rt:
        pytest.skip("clang sanitizer runtime not found")
    from paper_1909_02871_amd import build as hip_build
    # device-code files as built; the host-code files rebuilt with the sanitizers
    kernels = [os.path.join(hip_build.BUILD_DIR, s + ".o") for s in hip_build.SOURCES if s.endswith(".hip")]
    if not all(os.path.exists(k) for k in kernels):
        hip_build.build()
    objs = []
    procs = []
    for src in [s for s in hip_build.SOURCES if s.endswith(".cpp")]:
        obj = str(tmp_path / (src + ".o"))
        objs.append(obj)
        procs.append(subprocess.Popen(
            [HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
             "-I", os.path.join(ROOT, "include"), *SAN_HOST, "-c", os.path.join(CSRC, src), "-o", obj],
            stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
    for p in procs:
        out, _ = p.communicate(timeout=600)
        assert p.returncode == 0, out.decode()[-3000:]
    lib = str(tmp_path / "libgfnc_san.so")
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *SAN_HOST, "-shared-libsan", "-o", lib,
                        *objs, *kernels], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    _run_child(["tests/test_serve_sched.py", "tests/test_abi.py"], {"GFNC_LIB": lib, "LD_PRELOAD": rt[0]})


@pytest.mark.slow
def test_oracle_under_sanitizers(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan):
        pytest.skip("gcc's AddressSanitizer runtime not found")
    lib = str(tmp_path / "libgforacle_san.so")
    r = subprocess.run(["gcc", "-O1", "-g", "-std=c99", "-shared", "-fPIC", "-fno-omit-frame-pointer",
                        "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-o", lib,
                        os.path.join(ROOT, "oracle", "gforacle.c")], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    _run_child(["tests/test_oracle_ops.py", "tests/test_oracle_field.py", "-k", "not slow"],
               {"GFO_LIB": lib, "LD_PRELOAD": asan})
