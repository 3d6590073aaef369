"""Build the HIP library libstgv.so for gfx950 in-tree (hipcc, no JIT cache).

    python -m paper_2605_14505_amd.build

compiles every csrc/*.hip translation unit in parallel into _build/, links
paper_2605_14505_amd/lib/libstgv.so and the command-line driver
paper_2605_14505_amd/bin/stgv_run (csrc/stgv_run.cpp, C ABI only).  It always
recompiles.
"""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIBDIR = os.path.join(PKG, "lib")
LIB = os.path.join(LIBDIR, "libstgv.so")
BINDIR = os.path.join(PKG, "bin")
RUNNER = os.path.join(BINDIR, "stgv_run")
ARCH = "gfx950"

CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
    # keep the compiler from emitting packed FP32 VALU ops
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # fuse a * b + c only within one source expression: the rounding of every
    # kernel then follows its source, so two kernels that share the collision
    # code (the plain and the learned step) round it identically
    "-ffp-contract=on",
    # MFMA results in ordinary VGPRs rather than accumulation registers: the fused
    # learned step reads every product back into VALU code, which AGPRs would turn
    # into one v_accvgpr_read per result register
    "-mllvm", "-amdgpu-mfma-vgpr-form=1",
]


def hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found: the ROCm toolchain is required to build libstgv.so")
    return exe


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [hipcc(), *CFLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lrocfft"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    os.makedirs(BINDIR, exist_ok=True)
    cmd = [hipcc(), "-O2", "-std=c++17", "-Wall", os.path.join(CSRC, "stgv_run.cpp"), "-o", RUNNER + ".tmp",
           f"-L{LIBDIR}", "-lstgv", "-Wl,-rpath,$ORIGIN/../lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"driver build failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(RUNNER + ".tmp", RUNNER)
    if verbose:
        print(f"built {LIB} and {RUNNER}", flush=True)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
