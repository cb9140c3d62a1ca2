"""Builds libcum.so (HIP kernels + C-ABI) in-tree for gfx950 with hipcc.

Every source is compiled to its own object in parallel, then linked.
``build()`` recompiles everything; ``build(incremental=True)`` (or
``python build.py --incremental``) reuses an object whose source and the
csrc headers are unchanged since it was made.
"""
from __future__ import annotations

import hashlib
import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libcum.so")
SOURCES = ["api.cpp", "tables.cpp", "kernels.hip", "combine_split.hip", "adjoint.hip", "noalloc.hip"]
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # keep the compiler from emitting packed FP32 vector instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def _clean(text: str) -> str:
    return "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l and l.strip())


def _includes(path: str, seen: set) -> None:
    """The project headers `path` includes, directly or not (quoted includes)."""
    with open(path) as f:
        for line in f:
            m = re.match(r'\s*#\s*include\s+"([^"]+)"', line)
            if m:
                inc = os.path.normpath(os.path.join(os.path.dirname(path), m.group(1)))
                if os.path.exists(inc) and inc not in seen:
                    seen.add(inc)
                    _includes(inc, seen)


def _digest(src: str) -> str:
    h = hashlib.sha256(" ".join(FLAGS).encode())
    deps = set()
    _includes(src, deps)
    for p in [src] + sorted(deps):
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:20]


def _compile(src: str, incremental: bool):
    path = os.path.join(CSRC, src)
    obj = os.path.join(OBJ, src + ".o")
    stamp = obj + ".sha"
    dig = _digest(path)
    if incremental and os.path.exists(obj) and os.path.exists(stamp):
        with open(stamp) as f:
            if f.read().strip() == dig:
                return src, 0, ""
    tmp = obj + ".tmp%d" % os.getpid()
    res = subprocess.run(["hipcc", *FLAGS, "-c", path, "-o", tmp], capture_output=True, text=True)
    if res.returncode == 0:
        os.replace(tmp, obj)
        with open(stamp, "w") as f:
            f.write(dig)
    return src, res.returncode, _clean(res.stdout + res.stderr)


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compiles every source and links libcum.so."""
    os.makedirs(OBJ, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        results = list(ex.map(lambda s: _compile(s, incremental), SOURCES))
    failed = [(s, out) for s, rc, out in results if rc != 0]
    if failed:
        raise RuntimeError("hipcc failed:\n" + "\n".join("%s:\n%s" % f for f in failed))
    if verbose:
        for s, _, out in results:
            if out:
                print(out)
    tmp = LIB + ".tmp%d" % os.getpid()
    objs = [os.path.join(OBJ, s + ".o") for s in SOURCES]
    res = subprocess.run(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp],
                         capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + _clean(res.stdout + res.stderr))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, incremental="--incremental" in sys.argv[1:]))
