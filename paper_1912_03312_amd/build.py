"""Build the HIP library ``librexi.so`` in-tree for gfx950.

Usage: ``python -m paper_1912_03312_amd.build`` (or ``build()`` from Python).
Every call recompiles. Flags: -O3, wave64 gfx950 code object, packed FP32
instructions disabled (``-Xclang -target-feature -Xclang -packed-fp32-ops``).
hipcc hands -Xclang options to both of its passes; the host (x86) pass
ignores that feature with a warning. The driver cannot scope them to the
device pass (-Xarch_device refuses options that take arguments, and
-Xclang=...), so the warning stays; it changes nothing on the host side.

The build records a hash of its sources next to the library (``SOURCES``);
the test suite rebuilds when it differs.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librexi.so")
STAMP = os.path.join(HERE, "librexi.sources")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, os.path.join(CSRC, "api.hip"), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building librexi.so")
    os.replace(tmp, LIB)
    with open(STAMP, "w") as f:
        f.write(sources_hash() + "\n")
    return LIB


def sources_hash() -> str:
    """sha256 of the library's sources (kernels, C ABI, headers)."""
    import hashlib
    h = hashlib.sha256()
    for p in (os.path.join(CSRC, "kernels.hip"), os.path.join(CSRC, "api.hip"), os.path.join(CSRC, "rexi_internal.h"),
              os.path.join(HERE, "..", "include", "rexi.h")):
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def is_current() -> bool:
    """The built library exists and was built from the current sources."""
    if not (os.path.exists(LIB) and os.path.exists(STAMP)):
        return False
    with open(STAMP) as f:
        return f.read().strip() == sources_hash()


if __name__ == "__main__":
    print(build(verbose=True))
