"""Build libcpppl.so (gfx950) in-tree with hipcc.

    python -m paper_2503_10380_amd.build          # or build() from Python
"""
from __future__ import annotations

import hashlib
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libcpppl.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", f"-I{INCLUDE}"]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def source_hash() -> str:
    """SHA-256 over every HIP source and header the library is built from
    (csrc/*.hip, csrc/*.h, include/*.h), names and contents in sorted order.
    The build embeds it; the binding refuses a library whose hash differs."""
    files = []
    for d, exts in ((CSRC, (".hip", ".h")), (INCLUDE, (".h",))):
        files += [os.path.join(d, f) for f in os.listdir(d) if f.endswith(exts)]
    h = hashlib.sha256()
    for path in sorted(files, key=lambda f: os.path.relpath(f, os.path.dirname(HERE))):
        h.update(os.path.relpath(path, os.path.dirname(HERE)).encode())
        h.update(b"\0")
        with open(path, "rb") as f:
            h.update(f.read())
        h.update(b"\0")
    return h.hexdigest()


def _compile(src: str, src_hash: str) -> str:
    obj = os.path.join(OBJ, os.path.basename(src)[:-4] + ".o")
    cmd = [HIPCC, *FLAGS, f'-DCPPPL_SRC_HASH="{src_hash}"', "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    srcs = sources()
    jobs = min(len(srcs), max(1, min(8, os.cpu_count() or 1)))
    src_hash = source_hash()
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda f: _compile(f, src_hash), srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
