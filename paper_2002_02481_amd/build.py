"""Build liblvmc.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIBRARY = os.path.join(PKG, "liblvmc.so")

ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", f"-I{INCLUDE}", f"-I{CSRC}"]
# packed FP32 instructions are kept out of the generated code on purpose
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]
# one translation unit per kernel family (the fused kernel once per precision and
# checkpoint segment), compiled in parallel: (source, device code, extra flags, object)
SOURCES = ([("lv_k_fwd.hip", True, [], "lv_k_fwd"), ("lv_k_rev.hip", True, [], "lv_k_rev"),
            ("lv_k_misc.hip", True, [], "lv_k_misc"), ("lv_k_opt.hip", True, [], "lv_k_opt"),
            ("lv_api.cpp", False, [], "lv_api")]
           + [("lv_k_fused.hip", True, [f"-DLV_FUSED_PREC={p}", f"-DLV_FUSED_SEG={g}"], f"lv_k_fused_p{p}_s{g}")
              for p in (32, 64) for g in (8, 16, 32)])


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build step failed: " + " ".join(cmd))
    return r


def build(verbose: bool = False) -> str:
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(BUILD, exist_ok=True)
    cmds, objs = [], []
    for name, device, flags, stem in SOURCES:
        src = os.path.join(CSRC, name)
        obj = os.path.join(BUILD, stem + ".o")
        cmds.append(["hipcc"] + COMMON + flags + (DEVICE + ["-x", "hip"] if device else []) + ["-c", src, "-o", obj])
        objs.append(obj)
    if verbose:
        for cmd in cmds:
            print(" ".join(cmd), flush=True)
    with ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 1)) as ex:
        list(ex.map(_run, cmds))
    tmp = LIBRARY + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    _run(cmd)
    os.replace(tmp, LIBRARY)
    return LIBRARY


if __name__ == "__main__":
    print(build(verbose=True))
