"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
code, CPU only): a sanitized build of tgo_oracle.c runs every exported routine
(threads included) in a child process, checked against the Python oracle
there; any memory error or undefined behaviour aborts the child."""
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
def test_c_oracle_under_asan_and_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("no AddressSanitizer runtime")
    lib = tmp_path / "libtgo_oracle_san.so"
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-pthread",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                    os.path.join(ROOT, "oracle", "tgo_oracle.c"), "-o", str(lib)], check=True)
    env = dict(os.environ, TGO_ORACLE_LIB=str(lib), LD_PRELOAD=asan, PYTHONPATH=ROOT,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, os.path.join(HERE, "sanitize", "oracle_workout.py")],
                       env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "workout done" in r.stdout and str(lib) in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]


def _hip_asan_runtime():
    clang = "/opt/rocm/llvm/bin/clang"
    if not os.path.exists(clang):
        return None
    p = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                       text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="no hipcc")
def test_library_host_code_under_asan_and_ubsan(tmp_path):
    """libtgo.so rebuilt with AddressSanitizer and UBSan on its host code
    (device code unchanged); the host-side boundary tests (argument checks,
    rank/unrank, symbol table) run against it in a child process."""
    from concurrent.futures import ThreadPoolExecutor
    from paper_1806_10113_amd import build as B
    rt = _hip_asan_runtime()
    if rt is None:
        pytest.skip("no clang AddressSanitizer runtime")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = [f for f in B.FLAGS if f != "-O3"] + ["-O1", "-g"] + san

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        subprocess.run([B.HIPCC, *flags, "-c", src, "-o", obj], check=True, capture_output=True)
        return obj

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, B.sources()))
    lib = tmp_path / "libtgo_san.so"
    subprocess.run([B.HIPCC, f"--offload-arch={B.ARCH}", "-shared", "-fPIC", *san, "-shared-libsan", *objs,
                    "-o", str(lib)], check=True, capture_output=True)
    env = dict(os.environ, TGO_LIB=str(lib), LD_PRELOAD=rt, PYTHONPATH=ROOT,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(HERE, "test_boundary.py"), "-q", "-x",
                        "-p", "no:cacheprovider", "-k", "not calibration"],
                       env=env, capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "runtime error" not in r.stdout + r.stderr
