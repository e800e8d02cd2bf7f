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


# Host-side AddressSanitizer + UndefinedBehaviorSanitizer build for CPU-only
# tests of the host code (argument checks, plan creation, the streaming
# runtime, the sensing host helpers).  Each -fsanitize= applies to the host
# pass only (-Xarch_host); the device code is compiled but never run from it.
# Loading it needs the sanitizer runtime preloaded into the process.
SAN_BUILD = os.path.join(PKG, "_build_san")
SAN_OUT = os.path.join(SAN_BUILD, "librxphy_san.so")
SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-ffp-contract=on", "-pthread",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined"]


def _compile(src, sanitize=False):
    if sanitize:
        obj = os.path.join(SAN_BUILD, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC] + SAN_FLAGS + ["-c", os.path.join(HERE, src), "-o", obj]
    else:
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


def sanitized_is_current() -> bool:
    """True when the sanitized library exists and is newer than every source."""
    if not os.path.exists(SAN_OUT):
        return False
    t = os.path.getmtime(SAN_OUT)
    deps = [os.path.join(HERE, f) for f in os.listdir(HERE) if f.endswith((".hip", ".h"))]
    deps.append(os.path.join(os.path.dirname(PKG), "include", "rxphy.h"))
    return all(os.path.getmtime(d) <= t for d in deps)


def build_sanitized() -> str:
    """The host-sanitized librxphy (SAN_OUT); rebuilt only when a source is newer."""
    if sanitized_is_current():
        return SAN_OUT
    os.makedirs(SAN_BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        results = list(ex.map(lambda f: _compile(f, sanitize=True), SOURCES))
    tmp = SAN_OUT + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "-pthread", "--offload-arch=" + ARCH, "-shared-libasan",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-o", tmp] + \
        [o for o, _ in results]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, SAN_OUT)
    return SAN_OUT


if __name__ == "__main__":
    print(build(verbose=True))
