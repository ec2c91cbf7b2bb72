"""Compile librewl.so (HIP kernels + C-ABI host runtime) for gfx950, in-tree."""
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librewl.so")
CLOCKS_LIB = os.path.join(HERE, "librewl_clocks.so")
SOURCES = [os.path.join(CSRC, "rewl_kernels.hip"), os.path.join(CSRC, "rewl_runtime.hip"),
           os.path.join(CSRC, "rewl_batch.hip"), os.path.join(CSRC, "rewl_trimer.hip"),
           os.path.join(CSRC, "rewl_lipid.hip"), os.path.join(CSRC, "rewl_structure.hip")]
HEADERS = [os.path.join(CSRC, "rewl_device.h"), os.path.join(CSRC, "rewl_host.h"),
           os.path.join(os.path.dirname(HERE), "include", "rewl.h"),
           os.path.join(os.path.dirname(HERE), "include", "rewl_phase_clocks.h")]

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
    """Compile librewl.so and its profiling build librewl_clocks.so (the same
    sources with REWL_PHASE_CLOCKS: per-walker cycle counters of the attempt
    loop, include/rewl_phase_clocks.h) side by side, then liblds_peak.so."""
    if not force and os.path.exists(LIB) and os.path.exists(CLOCKS_LIB):
        newest = max(os.path.getmtime(p) for p in SOURCES + HEADERS)
        if min(os.path.getmtime(LIB), os.path.getmtime(CLOCKS_LIB)) >= newest:
            return LIB
    jobs = []
    for out, extra in ((LIB, []), (CLOCKS_LIB, ["-DREWL_PHASE_CLOCKS"])):
        cmd = [hipcc()] + FLAGS + extra + SOURCES + ["-o", out + ".tmp"]
        jobs.append((out, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
    errors = []
    for out, proc in jobs:
        _, err = proc.communicate()
        if proc.returncode != 0:
            errors.append(f"{os.path.basename(out)} build failed:\n" + err[-8000:])
        elif verbose and err:
            print(err[-4000:])
    if errors:
        raise RuntimeError("\n".join(errors))
    for out, _ in jobs:
        os.replace(out + ".tmp", out)
    build_lds_peak(force=force)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
