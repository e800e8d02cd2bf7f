"""Build librxphy.so for gfx950 with hipcc (in-tree, next to the package)."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
OUT = os.path.join(PKG, "librxphy.so")
BUILD = os.path.join(PKG, "_build")
SOURCES = ["api.hip", "fft.hip", "csi.hip", "detect.hip", "detect_group.hip", "demod.hip", "backward.hip", "batch.hip",
           "stream.hip", "sense.hip", "precode.hip", "ldpc.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
         # keep the compiler from forming packed FP32 instructions
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # fuse a*b+c only within one source expression, never across them:
         # the same tile body then rounds the same way in every kernel that
         # inlines it (the batched kernel reproduces the per-stage kernels)
         "-ffp-contract=on",
         "-Wall", "-Wno-unused-function", "-pthread"]


# Per-source extra flags.  The persistent batched kernel holds every stage body
# in one item loop; machine-level loop-invariant code motion would hoist the
# constants of all of them out of that loop and run out of SGPRs.
EXTRA = {"batch.hip": ["-mllvm", "-disable-machine-licm"]}


def _compile(src):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + FLAGS + EXTRA.get(src, []) + ["-c", os.path.join(HERE, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr))
    noisy = [ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
    return obj, "\n".join(noisy)


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        results = list(ex.map(_compile, SOURCES))
    for _, msg in results:
        if msg and verbose:
            print(msg, file=sys.stderr)
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "-pthread", "--offload-arch=" + ARCH, "-o", tmp] + [o for o, _ in results]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
