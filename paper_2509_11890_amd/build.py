"""Build libttipm.so (the HIP/C++ library behind include/ttipm.h) for gfx950.

Every source is compiled with hipcc for gfx950 only, with packed FP32 vector
instructions disabled, and linked into one shared library next to this file.
Objects are cached under _build/ and rebuilt when a source or header changes.
"""
from __future__ import annotations

import hashlib
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libttipm.so")
ARCH = os.environ.get("TTIPM_ARCH", "gfx950")

SOURCES = ["common.cpp", "gemm.hip", "dense.hip", "blocked.hip", "krylov.hip", "mlp.hip", "ttops.hip", "tt.hip", "amen.hip", "ipm.hip", "noalloc.hip", "capi.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-fvisibility=hidden", "-Wno-unused-result"]


def _headers_digest():
    h = hashlib.sha256()
    for d in (SRC, os.path.join(ROOT, "include")):
        for f in sorted(os.listdir(d)):
            if f.endswith((".hpp", ".h")):
                with open(os.path.join(d, f), "rb") as fh:
                    h.update(fh.read())
    return h.hexdigest()[:16]


def _obj(src, hdig):
    with open(os.path.join(SRC, src), "rb") as fh:
        dig = hashlib.sha256(fh.read() + hdig.encode() + " ".join(FLAGS).encode()).hexdigest()[:16]
    return os.path.join(BUILD, f"{src}.{dig}.o")


def _compile(src, obj, verbose):
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(SRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{out}")
    return out


def build(force=False, verbose=False, jobs=8):
    os.makedirs(BUILD, exist_ok=True)
    hdig = _headers_digest()
    objs = [_obj(s, hdig) for s in SOURCES]
    todo = [(s, o) for s, o in zip(SOURCES, objs) if force or not os.path.exists(o)]
    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        list(ex.map(lambda so: _compile(so[0], so[1], verbose), todo))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--force" in sys.argv, verbose="-v" in sys.argv))
