"""Build the HIP library librpca.so for gfx950 in-tree with hipcc.

The library is the whole DCF-PCA hot path: kernels (rpca_vpass*.hip,
rpca_spass*.hip, rpca_bf16.hip, rpca_tail.hip, rpca_mlp.hip, with their shared
device helpers in rpca_device.h) and the C ABI (rpca_api.cpp, declared in include/rpca.h). Each
source is compiled to an object of its own, in parallel, and the objects are
linked into one shared library. Packed-FP32 instruction selection is disabled
for all device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "_lib")
LIB = os.path.join(LIBDIR, "librpca.so")
SOURCES = ["rpca_vpass.hip", "rpca_vpass_q.hip", "rpca_vpass_s.hip", "rpca_vpass_w.hip",
           "rpca_spass.hip", "rpca_spass_q.hip", "rpca_spass_s.hip", "rpca_spass_w.hip",
           "rpca_bf16.hip", "rpca_tail.hip", "rpca_api.cpp", "rpca_mlp.hip"]
ARCH = "gfx950"
# hipcc's host pass warns that it does not know the packed-fp32 feature.
_NOISE = "packed-fp32-ops"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found; the DCF-PCA library needs ROCm's hipcc")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [ln for ln in (res.stdout + res.stderr).splitlines() if _NOISE not in ln and ln.strip()]
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(msgs))
    if verbose and msgs:
        print("\n".join(msgs))


def build(verbose: bool = False) -> str:
    """Compile every source into one shared library; returns its path."""
    os.makedirs(LIBDIR, exist_ok=True)
    cc = hipcc()
    flags = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-result", "-I", os.path.join(ROOT, "include")]
    objs = [os.path.join(LIBDIR, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    jobs = [[cc] + flags + ["-x", "hip", "-c", os.path.join(CSRC, s), "-o", o]
            for s, o in zip(SOURCES, objs)]
    with cf.ThreadPoolExecutor(len(jobs)) as ex:
        for f in [ex.submit(_run, j, verbose) for j in jobs]:
            f.result()
    tmp = LIB + ".tmp"
    _run([cc, f"--offload-arch={ARCH}", "-shared", "-fPIC"] + objs + ["-o", tmp], verbose)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
