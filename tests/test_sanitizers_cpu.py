"""CPU: the host runtime and the oracle under AddressSanitizer and
UndefinedBehaviorSanitizer.

Builds libiqp.so with the sanitizers on its host code only (device code is
compiled as usual) and the oracle with both, loads them in a child Python
with the sanitizer runtime preloaded, and runs the C-ABI tests (argument
validation, plan and workspace arithmetic, error texts, injected faults)
and the oracle's pins there; any sanitizer report fails. A planted
out-of-bounds write in a throwaway C file checks that reports do surface."""
import os
import subprocess
import sys

import pytest

from paper_2501_04776_amd import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LLVM = "/opt/rocm/llvm"
RT_DIR = os.path.join(LLVM, "lib", "clang")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _asan_runtime():
    if not os.path.isdir(RT_DIR):
        return None
    for ver in sorted(os.listdir(RT_DIR), reverse=True):
        p = os.path.join(RT_DIR, ver, "lib", "linux", "libclang_rt.asan-x86_64.so")
        if os.path.exists(p):
            return p
    return None


ASAN_RT = _asan_runtime()
pytestmark = pytest.mark.skipif(ASAN_RT is None or not os.path.exists(HIPCC),
                                reason="no clang sanitizer runtime or hipcc")

HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer"]


def _run_all(cmds):
    procs = [subprocess.Popen(c, stdout=subprocess.PIPE, stderr=subprocess.STDOUT) for c in cmds]
    for c, p in zip(cmds, procs):
        out = p.communicate()[0]
        assert p.returncode == 0, (" ".join(c), out.decode(errors="replace")[-3000:])


@pytest.fixture(scope="module")
def sanitized(tmp_path_factory):
    d = tmp_path_factory.mktemp("san")
    sha = build.source_sha256()
    cmds, objs = [], []
    for src in build.SOURCES:
        obj = str(d / (os.path.splitext(src)[0] + ".o"))
        objs.append(obj)
        cmds.append([HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
                     "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + HOST_SAN +
                    ["-I", os.path.join(ROOT, "include"), "-I", build.CSRC] +
                    (["-DIQP_SOURCE_SHA256=\"%s\"" % sha] if src == "iqp_api.cpp" else []) +
                    ["-c", os.path.join(build.CSRC, src), "-o", obj])
    oracle_so = str(d / "liboracle_san.so")
    cmds.append([os.path.join(LLVM, "bin", "clang"), "-O1", "-g", "-fno-omit-frame-pointer",
                 "-fsanitize=address,undefined", "-shared-libsan", "-std=c11", "-fPIC", "-shared",
                 "-o", oracle_so, os.path.join(ROOT, "oracle", "iqp_oracle.c"), "-lm",
                 "-lpthread"])
    _run_all(cmds)
    lib_so = str(d / "libiqp_san.so")
    _run_all([[HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-Xarch_host",
               "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-shared-libsan",
               "-o", lib_so] + objs])
    return d, lib_so, oracle_so


def _env(**extra):
    env = dict(os.environ)
    env.update(LD_PRELOAD=ASAN_RT, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    env.update(extra)
    return env


def test_sanitizer_reports_surface(sanitized):
    d, _, _ = sanitized
    src = d / "oob.c"
    src.write_text("#include <stdlib.h>\n"
                   "int oob(int i) { int *a = malloc(4 * sizeof(int)); a[i] = 1;"
                   " int r = a[0]; free(a); return r; }\n")
    so = str(d / "liboob.so")
    _run_all([[os.path.join(LLVM, "bin", "clang"), "-O1", "-g", "-fsanitize=address",
               "-shared-libsan", "-fPIC", "-shared", "-o", so, str(src)]])
    code = "import ctypes; L = ctypes.CDLL(%r); L.oob(3); print('fine', flush=True); L.oob(4)" % so
    r = subprocess.run([sys.executable, "-c", code], env=_env(), capture_output=True, text=True,
                       timeout=120)
    assert "fine" in r.stdout
    assert r.returncode != 0 and "heap-buffer-overflow" in r.stderr


def test_host_runtime_and_oracle_clean_under_sanitizers(sanitized):
    _, lib_so, oracle_so = sanitized
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "-m", "not gpu", "tests/test_abi_cpu.py", "tests/test_oracle.py",
                        "tests/test_oracle_indep.py", "tests/test_oracle_train.py"],
                       cwd=ROOT, env=_env(IQP_LIBRARY_PATH=lib_so, IQP_ORACLE_LIBRARY=oracle_so),
                       capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
