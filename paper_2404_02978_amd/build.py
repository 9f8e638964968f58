"""Build libqrfs.so (the HIP path) and libqrfs_peaks.so (throughput probes
for the roofline denominators) for gfx950 with hipcc, in-tree."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libqrfs.so")
PEAKS_LIB = os.path.join(HERE, "libqrfs_peaks.so")
PEAKS_SOURCES = ["qrfs_peaks.hip"]
SOURCES = ["qrfs_frequencies.hip", "qrfs_kernels.hip", "qrfs_wide.hip", "qrfs_temporal.hip", "qrfs_measures.hip",
           "qrfs_pairs.hip", "qrfs_proposal.hip", "qrfs_api.cpp", "qrfs_batch.cpp", "qrfs_proposal_api.cpp",
           "qrfs_plan.cpp"]
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-Wall", "-Werror",
         "-Wno-unused-function",
         # no packed-FP32 instructions anywhere in device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-fvisibility=hidden", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
# The point-set measures run on finite coordinates only; without IEEE-mode
# NaN quieting, minima of values loaded from LDS need no canonicalising
# instruction before each v_min_f64 (15 % of the pair loop).
FILE_FLAGS = {"qrfs_pairs.hip": ["-fno-honor-nans", "-mno-amdgpu-ieee"]}


def build(verbose=False, jobs=4):
    objs = []
    procs = []
    for src in SOURCES + PEAKS_SOURCES:
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        cmd = (["hipcc"] + FLAGS + FILE_FLAGS.get(src, []) + lang +
               ["-c", os.path.join(CSRC, src), "-o", obj])
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd, stderr=subprocess.PIPE, text=True))
        objs.append(obj)
    errs = []
    for p, src in zip(procs, SOURCES + PEAKS_SOURCES):
        _, err = p.communicate()
        err = "\n".join(l for l in err.splitlines()
                        if "packed-fp32-ops" not in l)
        if p.returncode != 0:
            errs.append(f"{src}:\n{err}")
    if errs:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errs))
    n = len(SOURCES)
    for lib, lib_objs in ((LIB, objs[:n]), (PEAKS_LIB, objs[n:])):
        cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", lib + ".tmp"] + lib_objs
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        os.replace(lib + ".tmp", lib)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
