"""Host-side AddressSanitizer / UndefinedBehaviorSanitizer runs (CPU only):
the C oracle on small cases of every exported function, and the C ABI's
argument validation against a libbte whose host code is instrumented (the
device code is built as usual and never runs).  A planted overflow first
shows that the instrumentation is live."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANGXX = "/opt/rocm/llvm/bin/clang++"
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1")
GCC_SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-g", "-O1"]
# host side only: the GPU code of the library is compiled without sanitizers
HIP_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer"]


def run(cmd, **kw):
    return subprocess.run(cmd, capture_output=True, text=True, env=ENV, timeout=600, **kw)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_instrumentation_catches_a_planted_overflow(tmp_path):
    src = tmp_path / "planted.c"
    src.write_text("#include <stdlib.h>\nint main(void){int*p=malloc(4*sizeof(int));"
                   "p[4]=1;int r=p[0];free(p);return r;}\n")
    exe = tmp_path / "planted"
    r = run(["gcc", *GCC_SAN, str(src), "-o", str(exe)])
    assert r.returncode == 0, r.stderr
    r = run([str(exe)])
    # whichever instrumentation sees it first (UBSan object size or ASan) stops it
    assert r.returncode != 0
    assert "heap-buffer-overflow" in r.stderr or "runtime error" in r.stderr


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_san"
    r = run(["gcc", *GCC_SAN, "-std=c99", "-fopenmp", "-ffp-contract=off",
             os.path.join(SAN, "oracle_check.c"), os.path.join(ROOT, "oracle", "bte_oracle.c"),
             os.path.join(ROOT, "oracle", "characteristics.c"), "-lm", "-o", str(exe)])
    assert r.returncode == 0, r.stderr
    r = run([str(exe)])
    assert r.returncode == 0, r.stdout + r.stderr
    assert "oracle sanitizer run ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr


@pytest.mark.skipif(not os.path.exists(HIPCC) or not os.path.exists(CLANGXX),
                    reason="needs the ROCm compilers")
def test_abi_validation_under_sanitizers(tmp_path):
    sys.path.insert(0, ROOT)
    from paper_1401_6047_amd import build as B
    procs, objs = [], []
    for src in B.SOURCES:
        name = os.path.basename(src)
        obj = str(tmp_path / (name + ".o"))
        # the library's own flags, at -O1 with debug information
        flags = [f for f in B.HIPCC_FLAGS if f != "-O3"]
        cmd = [HIPCC, *flags, "-O1", "-g", *HIP_SAN, *B.EXTRA_FLAGS.get(name, []), "-c", src,
               "-o", obj]
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                                      env=ENV))
        objs.append(obj)
    for p in procs:
        _, err = p.communicate(timeout=600)
        assert p.returncode == 0, err.decode()[-2000:]
    drv = str(tmp_path / "drv.o")
    r = run([CLANGXX, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
             "-I", os.path.join(ROOT, "include"), "-c", os.path.join(SAN, "abi_host_check.cpp"),
             "-o", drv])
    assert r.returncode == 0, r.stderr
    exe = str(tmp_path / "abi_san")
    r = run([HIPCC, f"--offload-arch={B.ARCH}", *HIP_SAN, drv, *objs, "-o", exe])
    assert r.returncode == 0, r.stderr[-2000:]
    r = run([exe])
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "abi host sanitizer run ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
