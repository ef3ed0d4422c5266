"""Build the gfx950 HIP library ``libcpfft.so`` in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcpfft.so")
SOURCES = ["cpfft_api.hip", "cpfft_micro.hip"]
HEADERS = ["cpfft_device.hpp", "cpfft_kernels.hpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions stay off (the compiler would otherwise form
    # v_pk_* from scalar float code)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]
# roctx ranges (load step, iteration chunk, pass; adjoint step) for profiler runs
LIBS = ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]


# Host code under AddressSanitizer and UndefinedBehaviorSanitizer (every
# report fatal); device code is built as usual.  For the CPU tests of the
# C-ABI's host paths only: loading it needs the clang ASan runtime preloaded.
SAN_LIB = os.path.join(os.path.dirname(HERE), "_build", "libcpfft_hostsan.so")
SAN_FLAGS = [
    "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fno-omit-frame-pointer",
    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
    "-Xarch_host", "-fno-sanitize-recover=all",
]


def _command(flags, extra, tmp):
    return [HIPCC, *flags, *extra, "-o", tmp] + [os.path.join(CSRC, s) for s in SOURCES] + LIBS


def _build_with(flags, extra, out, verbose):
    tmp = out + ".tmp%d" % os.getpid()
    cmd = _command(flags, extra, tmp)
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(verbose: bool = False, extra=(), out: str = LIB) -> str:
    return _build_with(FLAGS, extra, out, verbose)


def build_sanitized(verbose: bool = False) -> str:
    os.makedirs(os.path.dirname(SAN_LIB), exist_ok=True)
    return _build_with(SAN_FLAGS, (), SAN_LIB, verbose)


def build_all(verbose: bool = False) -> None:
    """The library and its host-sanitized twin, compiled concurrently."""
    os.makedirs(os.path.dirname(SAN_LIB), exist_ok=True)
    jobs = []
    for flags, out in ((FLAGS, LIB), (SAN_FLAGS, SAN_LIB)):
        tmp = out + ".tmp%d" % os.getpid()
        cmd = _command(flags, (), tmp)
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        jobs.append((subprocess.Popen(cmd), tmp, out))
    failed = [out for p, tmp, out in jobs if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, "hipcc", "failed: " + ", ".join(failed))
    for _, tmp, out in jobs:
        os.replace(tmp, out)


def sources_newer_than(path: str) -> bool:
    if not os.path.exists(path):
        return True
    t = os.path.getmtime(path)
    return any(os.path.getmtime(os.path.join(CSRC, f)) > t for f in os.listdir(CSRC))


if __name__ == "__main__":
    if sys.argv[1:] == ["--sanitized"]:
        print(build_sanitized(verbose=True))
    else:
        print(build(verbose=True, extra=sys.argv[1:]))
