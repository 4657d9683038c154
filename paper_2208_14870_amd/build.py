"""Build of the HIP library (gfx950) in-tree: paper_2208_14870_amd/liblbm.so."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "liblbm.so")
SOURCES = [os.path.join(CSRC, f) for f in
           ("lbm_capi.hip", "lbm_batch.hip", "lbm_wave.hip", "lbm_wave_inplace.hip",
            "lbm_wave_batch.hip")]
HEADERS = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp")) + [
    os.path.join(ROOT, "include", "lbm.h")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Wall", "-Wno-unused-function",
    # packed FP32 instructions are disabled for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
]


def build(verbose: bool = True) -> str:
    """Compile every HIP source into liblbm.so (always recompiles): one hipcc
    process per source, in parallel, then one link."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    srcs = [s for s in SOURCES if os.path.exists(s)]
    tag = "%d" % os.getpid()
    objs = [os.path.join(CSRC, os.path.basename(s)[:-4] + ".o.tmp" + tag) for s in srcs]
    procs = []
    try:
        for src, obj in zip(srcs, objs):
            cmd = [hipcc] + HIPCC_FLAGS + ["-c", "-o", obj, src]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append(subprocess.Popen(cmd))
        failed = [src for src, p in zip(srcs, procs) if p.wait() != 0]
        if failed:
            raise subprocess.CalledProcessError(1, "hipcc " + " ".join(failed))
        tmp = LIB + ".tmp" + tag
        cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    finally:
        for p in procs:
            if p.poll() is None:
                p.kill()
                p.wait()
        for obj in objs:
            if os.path.exists(obj):
                os.remove(obj)
    return LIB


CONSUMER_SRC = os.path.join(ROOT, "tests", "capi_consumer.c")
CONSUMER = os.path.join(ROOT, "tests", "capi_consumer")


def build_c_consumer(verbose: bool = True) -> str:
    """Compile the plain C consumer of the ABI used by the tests (gcc, linked
    against liblbm.so and the HIP runtime, found through rpath)."""
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    tmp = CONSUMER + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-D__HIP_PLATFORM_AMD__",
           "-I" + os.path.join(rocm, "include"), "-I" + os.path.join(ROOT, "include"),
           CONSUMER_SRC, "-o", tmp, "-L" + PKG, "-llbm", "-L" + os.path.join(rocm, "lib"),
           "-lamdhip64", "-Wl,-rpath,$ORIGIN/../paper_2208_14870_amd",
           "-Wl,-rpath," + os.path.join(rocm, "lib")]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, CONSUMER)
    return CONSUMER


if __name__ == "__main__":
    build()
    build_c_consumer()
    sys.exit(0)
