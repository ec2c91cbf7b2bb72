"""Compile librewl.so (HIP kernels + C-ABI host runtime) for gfx950, in-tree."""
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librewl.so")
SOURCES = [os.path.join(CSRC, "rewl_kernels.hip"), os.path.join(CSRC, "rewl_runtime.hip"),
           os.path.join(CSRC, "rewl_batch.hip"), os.path.join(CSRC, "rewl_trimer.hip"),
           os.path.join(CSRC, "rewl_lipid.hip"), os.path.join(CSRC, "rewl_structure.hip")]
HEADERS = [os.path.join(CSRC, "rewl_device.h"), os.path.join(CSRC, "rewl_host.h"),
           os.path.join(os.path.dirname(HERE), "include", "rewl.h")]

# -ffp-contract=off: the acceptance test must round every binary64/binary32
# operation separately, in source order, exactly like a plain IEEE evaluation.
# -packed-fp32-ops off: no packed FP32 instructions are generated.
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall",
         "-Wno-unused-function", "-Wno-unknown-pragmas"]


# The LDS bandwidth microbenchmark the benchmark measures its LDS roofline
# against (not part of the REWL library).
LDS_PEAK_SRC = os.path.join(CSRC, "lds_peak.hip")
LDS_PEAK_LIB = os.path.join(HERE, "liblds_peak.so")


def hipcc():
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def build_lds_peak(force=True):
    if not force and os.path.exists(LDS_PEAK_LIB) and os.path.getmtime(LDS_PEAK_LIB) >= os.path.getmtime(LDS_PEAK_SRC):
        return LDS_PEAK_LIB
    tmp = LDS_PEAK_LIB + ".tmp"
    res = subprocess.run([hipcc()] + FLAGS + [LDS_PEAK_SRC, "-o", tmp], capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("liblds_peak build failed:\n" + res.stderr[-8000:])
    os.replace(tmp, LDS_PEAK_LIB)
    return LDS_PEAK_LIB


def build(force=True, verbose=False):
    if not force and os.path.exists(LIB):
        newest = max(os.path.getmtime(p) for p in SOURCES + HEADERS)
        if os.path.getmtime(LIB) >= newest:
            return LIB
    tmp = LIB + ".tmp"
    cmd = [hipcc()] + FLAGS + SOURCES + ["-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("librewl build failed:\n" + res.stderr[-8000:])
    if verbose and res.stderr:
        print(res.stderr[-4000:])
    os.replace(tmp, LIB)
    build_lds_peak(force=force)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
