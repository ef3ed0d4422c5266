"""The C-ABI's host paths under AddressSanitizer and UndefinedBehaviorSanitizer.

``paper_2402_09996_amd/build.py`` compiles the library a second time with
its host code sanitized (every report fatal; device code as usual).  A child
pytest process preloads clang's ASan runtime, loads that twin through
``CPFFT_LIBRARY`` and runs the host-side ABI tests: descriptor validation
and the host tables of ``cpf_problem_create``, option checks and workspace
sizing of ``cpf_solver_create``, the lifecycle errors before binding and
the argument checks of the allocation-free histogram.  CPU only (no device
call is made).
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan_runtime():
    c = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return c[-1] if c else None


def test_abi_host_paths_under_asan_and_ubsan():
    rt = _asan_runtime()
    if rt is None or not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("hipcc or clang's ASan runtime not installed")
    sys.path.insert(0, ROOT)
    from paper_2402_09996_amd import build as hb
    if hb.sources_newer_than(hb.SAN_LIB):
        hb.build_sanitized()
    env = dict(os.environ)
    env.update(CPFFT_LIBRARY=hb.SAN_LIB, LD_PRELOAD=rt, HIP_VISIBLE_DEVICES="",
               ASAN_OPTIONS="detect_leaks=0:exitcode=86",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=87")
    p = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                        os.path.join(ROOT, "tests", "test_abi.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    report = p.stdout[-4000:] + p.stderr[-6000:]
    assert p.returncode == 0, report
    assert "AddressSanitizer" not in p.stderr and "runtime error" not in p.stderr, report
    assert " passed" in p.stdout
