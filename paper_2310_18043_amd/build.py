"""Build the rfeig shared library for gfx950 with hipcc (in-tree).

    python -m paper_2310_18043_amd.build

produces ``paper_2310_18043_amd/librfeig.so``.  The library links only the HIP
runtime; it has no PyTorch dependency.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "librfeig.so")
SOURCES = ["rf_api.cpp", "rf_qz.cpp", "rf_band.hip", "rf_dense.hip", "rf_cluster.hip"]
ARCH = os.environ.get("RFEIG_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["-O3", "-std=c++17", "-fPIC", f"-I{INCLUDE}", f"-I{CSRC}",
          "-Wno-unused-result"]
# device code: gfx950 only; packed FP32 instructions disabled
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops", "-munsafe-fp-atomics"]


# per-source flags: the host QZ uses plain complex multiply/divide (its operands
# are finite; no Annex-G infinity recovery calls in the inner loops)
EXTRA = {"rf_qz.cpp": ["-fcx-limited-range"]}
# sources with host code only are compiled as C++ (no device pass), so that host-only
# attributes such as run-time CPU dispatch are available to them
HOST_ONLY = {"rf_qz.cpp"}


def _obj(src: str) -> str:
    return os.path.join(CSRC, "_build", os.path.splitext(src)[0] + ".o")


def build(verbose: bool = False, jobs: int = 4) -> str:
    os.makedirs(os.path.join(CSRC, "_build"), exist_ok=True)
    procs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        # every source includes HIP headers: compile them as HIP for gfx950, host-only ones as C++
        if src in HOST_ONLY:
            cmd = [HIPCC] + COMMON + EXTRA.get(src, []) + ["-x", "c++", "-c", path, "-o", _obj(src)]
        else:
            cmd = [HIPCC] + COMMON + DEVICE + EXTRA.get(src, []) + ["-x", "hip", "-c", path,
                                                                    "-o", _obj(src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                            stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _wait(procs.pop(0))
    while procs:
        _wait(procs.pop(0))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-o", tmp] + [_obj(s) for s in SOURCES] + \
          [f"--offload-arch={ARCH}", "-fPIC"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def _wait(item):
    src, p = item
    out, _ = p.communicate()
    text = out.decode(errors="replace")
    if p.returncode != 0:
        sys.stderr.write(text)
        raise RuntimeError(f"hipcc failed on {src}")
    # keep real warnings visible, skip the host-pass note about the device feature
    lines = [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
    if lines:
        sys.stderr.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
