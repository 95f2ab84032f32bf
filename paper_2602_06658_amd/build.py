"""Build libgwmi.so for gfx950 in-tree with hipcc.

Every .hip and .cpp file under csrc/ is compiled to an object with
``--offload-arch=gfx950`` and packed-FP32 instructions disabled, then linked
into ``paper_2602_06658_amd/libgwmi.so``.  Objects go to ``_build/`` beside
this file; unchanged sources are not recompiled unless ``force``.

``build_peaks`` compiles the instruction-rate microbenchmark
(peaks/peaks.hip) into its own ``libgwpeaks.so``, which bench.py runs to
derive the pass's roofline.
"""
from __future__ import annotations

import concurrent.futures as cf
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libgwmi.so")
PEAKS_SRC = os.path.join(HERE, "peaks", "peaks.hip")
PEAKS_OUT = os.path.join(HERE, "libgwpeaks.so")
BUILD = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
    # MFMA accumulators in ordinary VGPRs: the exp/add epilogue reads them
    # without a v_accvgpr_read per element
    "-mllvm", "--amdgpu-mfma-vgpr-form",
]
LIBS = ["-L/opt/rocm/lib", "-lrocsolver", "-lrocblas", "-lamdhip64", "-lpthread"]


def _sources():
    out = []
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".cpp")):
            out.append(os.path.join(CSRC, name))
    return out


def _headers_digest():
    h = hashlib.sha1()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith(".h"):
            with open(os.path.join(CSRC, name), "rb") as fh:
                h.update(fh.read())
    with open(os.path.join(os.path.dirname(HERE), "include", "gw.h"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:12]


def _compile(src, obj, force):
    stamp = obj + ".stamp"
    with open(src, "rb") as fh:
        key = hashlib.sha1(fh.read()).hexdigest() + _headers_digest() + " ".join(COMMON)
    if not force and os.path.exists(obj) and os.path.exists(stamp):
        with open(stamp) as fh:
            if fh.read() == key:
                return obj, False
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [HIPCC] + COMMON + ["-I", CSRC, "-c"] + lang + [src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    with open(stamp, "w") as fh:
        fh.write(key)
    return obj, True


def build(force: bool = False, jobs: int | None = None, verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = _sources()
    objs = [os.path.join(BUILD, os.path.basename(s) + ".o") for s in srcs]
    jobs = jobs or min(8, os.cpu_count() or 4)
    rebuilt = False
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = [ex.submit(_compile, s, o, force) for s, o in zip(srcs, objs)]
        for f in futs:
            _, did = f.result()
            rebuilt = rebuilt or did
    if force or rebuilt or not os.path.exists(OUT):
        tmp = OUT + ".tmp"
        cmd = [HIPCC, "-shared", "--offload-arch=gfx950", "-o", tmp] + objs + LIBS
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"link failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
        os.replace(tmp, OUT)
        if verbose:
            print("built", OUT, file=sys.stderr)
    return OUT


def build_peaks(verbose: bool = True) -> str:
    tmp = PEAKS_OUT + ".tmp"
    cmd = [HIPCC] + COMMON + ["-shared", "-x", "hip", PEAKS_SRC, "-o", tmp, "-L/opt/rocm/lib", "-lamdhip64"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"peaks build failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, PEAKS_OUT)
    if verbose:
        print("built", PEAKS_OUT, file=sys.stderr)
    return PEAKS_OUT


if __name__ == "__main__":
    build(force="--force" in sys.argv)
    build_peaks()
