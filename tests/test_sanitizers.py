"""Host code under sanitizers (runs without a GPU).

* AddressSanitizer + UndefinedBehaviorSanitizer: the library built with both on its host code
  (paper_1409_4441_amd/build.py, sanitize=True) runs the C-ABI tests (argument validation of every
  entry point) and the split-model tests (the reduced least squares, errors, cost model, search and
  its worker threads) with the sanitizer runtime preloaded; any report fails the run.
* ThreadSanitizer: the split model's source with a driver of conv_split_search_many (worker threads
  sharing one context and its SVD cache).
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang++"

pytestmark = pytest.mark.slow


def _asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def test_asan_ubsan_c_abi_and_split_model(tmp_path):
    rt = _asan_runtime()
    if rt is None or not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("hipcc or the clang sanitizer runtime is not installed")
    import importlib.util
    spec = importlib.util.spec_from_file_location("_san_build", os.path.join(ROOT, "paper_1409_4441_amd", "build.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    lib = b.build(sanitize=True, out_dir=str(tmp_path))
    env = dict(os.environ, CONVREAL_LIB=lib, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        os.path.join(ROOT, "tests", "test_abi.py"), os.path.join(ROOT, "tests", "test_split_model.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert " passed" in out


def test_tsan_split_search_threads(tmp_path):
    if not os.path.exists(CLANG):
        pytest.skip("clang++ is not installed")
    exe = str(tmp_path / "search_many_tsan")
    cmd = [CLANG, "-O1", "-g", "-std=c++17", "-fsanitize=thread", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROOT, "paper_1409_4441_amd", "csrc"),
           os.path.join(ROOT, "tests", "sanitize", "search_many_driver.cpp"),
           os.path.join(ROOT, "paper_1409_4441_amd", "csrc", "split.cpp"), "-o", exe, "-lpthread"]
    subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=600)
    r = subprocess.run([exe], env=dict(os.environ, TSAN_OPTIONS="halt_on_error=1"), capture_output=True, text=True,
                       timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ThreadSanitizer" not in out, out[-4000:]
    assert len(out.strip().splitlines()) == 12
