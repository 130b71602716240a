"""Build libdpf.so (HIP, gfx950) in-tree with hipcc."""

from __future__ import annotations

import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC_DIR = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdpf.so")
SOURCES = [os.path.join(SRC_DIR, "dpf.hip")]
HEADERS = [os.path.join(SRC_DIR, f) for f in os.listdir(SRC_DIR) if f.endswith(".hpp")] + [
    os.path.join(os.path.dirname(HERE), "include", "dpf.h")]

ARCH = os.environ.get("DPF_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # packed FP32 instructions are disabled for every kernel of this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    return "hipcc"


def source_hash() -> str:
    """Hash of the library's sources (embedded in the build, checked at load)."""
    h = hashlib.sha256()
    for p in sorted(SOURCES + HEADERS):
        with open(p, "rb") as fh:
            h.update(os.path.basename(p).encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def build(verbose: bool = False) -> str:
    """Compile the library unconditionally and return its path."""
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, f'-DDPF_SOURCE_HASH="{source_hash()}"', *SOURCES, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libdpf.so")
    os.replace(tmp, LIB)
    return LIB


def stale() -> bool:
    """True when the library is missing or was built from other sources."""
    if not os.path.exists(LIB):
        return True
    import ctypes
    lib = ctypes.CDLL(LIB)
    lib.dpf_version.restype = ctypes.c_char_p
    return not lib.dpf_version().decode().endswith("src " + source_hash())


if __name__ == "__main__":
    print(build(verbose=True))
