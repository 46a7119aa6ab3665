"""Build librsc.so (HIP for gfx950) in-tree with hipcc.

Usage: python -m paper_1806_04374_amd.build_lib [--verbose] [--resource-usage]
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "librsc.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", "-I", os.path.join(ROOT, "include"), "-I", CSRC]
# packed FP32 instructions are switched off for all device code
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

SOURCES = [
    ("rsc_basis.cpp", "host"),
    ("rsc_api.cpp", "hip"),
    ("rsc_project.hip", "hip"),
    ("rsc_encode.hip", "hip"),
    ("rsc_encode_annular.hip", "hip"),
    ("rsc_encode_lp.hip", "hip"),
    ("rsc_synth.hip", "hip"),
    ("rsc_images.hip", "hip"),
    ("rsc_rksvd.hip", "hip"),
    ("rsc_classify.hip", "hip"),
    ("rsc_rotate.hip", "hip"),
]


def _compile(src: str, kind: str, extra: list[str], verbose: bool) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    path = os.path.join(CSRC, src)
    if kind == "host":
        cmd = ["g++", *COMMON, "-c", path, "-o", obj]
    else:
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [HIPCC, *COMMON, *DEVICE, *lang, "-c", path, "-o", obj, *extra]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = r.stdout + r.stderr
    # hipcc's host pass does not know the gfx feature flag; that warning is harmless
    out = "\n".join(l for l in out.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{out}")
    if out.strip() and (verbose or extra):
        print(out)
    return obj


def build(verbose: bool = False, resource_usage: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    extra = ["-Rpass-analysis=kernel-resource-usage"] if resource_usage else []
    with ThreadPoolExecutor(max_workers=6) as ex:
        objs = list(ex.map(lambda s: _compile(s[0], s[1], extra if s[0].endswith(".hip") else [], verbose),
                           SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed\n{r.stdout}{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="--verbose" in sys.argv, resource_usage="--resource-usage" in sys.argv))
