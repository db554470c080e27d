"""Build the HIP library liblbm_mi355x.so for gfx950 in-tree (paper_1705_10045_amd/_build/), and
the benchmark's bandwidth-ceiling probe libceiling.so beside it.

Every source is compiled by hipcc for gfx950 only, with packed FP32 instructions disabled;
objects are compiled in parallel and linked into one shared library exposing the C ABI of
include/lbm_mi355x.h.
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "liblbm_mi355x.so")
SOURCES = ["api.hip", "kernels.hip", "kernels_red.hip", "serve.hip", "noalloc.hip"]
# the bandwidth-ceiling probe of the benchmark, a library of its own (not part of the ABI)
PROBE_SOURCES = ["ceiling.hip"]
PROBE_LIB = os.path.join(OUT_DIR, "libceiling.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile(src, verbose):
    obj = os.path.join(OUT_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s%s" % (src, r.stdout, r.stderr))
    # the host pass does not know the packed-fp32 feature; that warning is expected
    noise = [l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip()
             and "warning generated" not in l]
    if noise and verbose:
        print("\n".join(noise))
    return obj


def _link(objs, out, verbose):
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)


def build(verbose=False):
    os.makedirs(OUT_DIR, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=len(SOURCES) + len(PROBE_SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES + PROBE_SOURCES))
    _link(objs[:len(SOURCES)], LIB, verbose)
    _link(objs[len(SOURCES):], PROBE_LIB, verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
