"""The FP64 oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
on the host (g++), every entry point run once on small uniform, stretched
and all-wall grids with buildings (oracle/sanitize_check.cpp): any
out-of-range access, use after free, leak or undefined arithmetic aborts
the run and fails the test."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE = os.path.join(os.path.dirname(HERE), "oracle")


def _have_sanitizers():
    if shutil.which("g++") is None:
        return False
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "t.cpp")
        open(src, "w").write("int main() { return 0; }\n")
        r = subprocess.run(["g++", "-fsanitize=address,undefined", src, "-o", os.path.join(d, "t")],
                           capture_output=True)
        return r.returncode == 0


@pytest.mark.skipif(not _have_sanitizers(), reason="g++ with ASan/UBSan runtimes not available")
def test_oracle_clean_under_asan_and_ubsan():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "sanitize_check")
        cmd = ["g++", "-std=c++17", "-O1", "-g", "-fopenmp", "-ffp-contract=off",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
               os.path.join(ORACLE, "sanitize_check.cpp"), "-o", exe]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
        assert "sanitize_check: ok" in r.stdout


def _asan_runtime():
    import glob
    c = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return c[-1] if c else None


@pytest.mark.skipif(_asan_runtime() is None or shutil.which("/opt/rocm/bin/hipcc") is None,
                    reason="hipcc or clang's ASan runtime not available")
def test_host_code_clean_under_asan_and_ubsan():
    """The library's host code (argument checks, parameter validation, the
    boundary-range bijection, handle life cycle without a GPU) built with
    AddressSanitizer and UndefinedBehaviorSanitizer on the host side only
    (device code unchanged), then the CPU ABI tests run against that build
    with the sanitizer runtime preloaded."""
    from concurrent.futures import ThreadPoolExecutor
    from paper_1504_02264_amd import build as B
    with tempfile.TemporaryDirectory() as d:
        objs = []
        cmds = []
        for s in B.SOURCES:
            o = os.path.join(d, os.path.splitext(s)[0] + ".o")
            objs.append(o)
            cmds.append(["/opt/rocm/bin/hipcc", "-O1", "-g", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
                         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                         "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                         "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
                         "-I", os.path.join(os.path.dirname(HERE), "include"), "-c",
                         os.path.join(B.CSRC, s), "-o", o])
        with ThreadPoolExecutor(max_workers=min(8, len(cmds))) as ex:
            res = list(ex.map(lambda c: subprocess.run(c, capture_output=True, text=True), cmds))
        for r in res:
            assert r.returncode == 0, r.stderr[-3000:]
        lib = os.path.join(d, "libles_hostsan.so")
        r = subprocess.run(["/opt/rocm/bin/hipcc", "-shared", "-fPIC", "--offload-arch=gfx950", "-shared-libsan",
                            "-fsanitize=address,undefined", *objs, "-o", lib], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        env = dict(os.environ, LD_PRELOAD=_asan_runtime(), ASAN_OPTIONS="detect_leaks=0",
                   PAPER_1504_02264_AMD_LIB=lib)
        r = subprocess.run(["python3", "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                            os.path.join(HERE, "test_abi_cpu.py")],
                           capture_output=True, text=True, env=env, timeout=600,
                           cwd=os.path.dirname(HERE))
        assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
        assert "passed" in r.stdout and "ERROR: AddressSanitizer" not in r.stderr
