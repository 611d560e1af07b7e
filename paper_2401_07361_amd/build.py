"""Builds libstc.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2401_07361_amd.build

Every source is recompiled on each call.  Flags:
* --offload-arch=gfx950, -O3, C++17;
* packed FP32 instructions are disabled for all device code;
* the tree kernels, the adaptive-mesh kernels and the host geometry are
  compiled without floating-point contraction, so point location, the
  acceptance criterion and the refinement tests use exactly the IEEE
  operations written in the source.
"""

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(HERE, "libstc.so")
BUILD = os.path.join(HERE, "_build")

ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
CLANG = os.path.join(ROCM, "llvm", "bin", "clang++")

COMMON = ["-O3", "-std=c++17", "-fPIC", "-I", INCLUDE, "-I", CSRC]
DEVICE = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]

SOURCES = [
    # (file, extra flags, is_device)
    ("geometry.cpp", ["-ffp-contract=off"], False),
    ("k_sort.hip", [], True),
    ("k_tree.hip", ["-ffp-contract=off"], True),
    # matrix-core operands and results in ordinary VGPRs (no copies through
    # the accumulation registers in the target-proxy kernel's inner loop)
    ("k_eval.hip", ["-mllvm", "-amdgpu-mfma-vgpr-form"], True),
    ("k_mlp.hip", [], True),
    ("k_learned.hip", [], True),
    ("amr.hip", ["-ffp-contract=off"], True),
    ("stc_api.hip", [], True),
]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + "\n")
        raise RuntimeError("compilation failed: " + os.path.basename(cmd[-1]))
    return r.stdout


def build(verbose=False, jobs=None, out=None):
    """Compiles every source and links libstc.so (or `out`).  Environment
    STC_FAR_MFMA=1 builds the matrix-core form of the FP32 target-proxy
    kernel instead of the VALU one (kept for measurement; slower)."""
    lib = out or OUT
    os.makedirs(BUILD, exist_ok=True)
    far_mfma = os.environ.get("STC_FAR_MFMA", "0") == "1"
    objs = []
    procs = []
    for name, extra, dev in SOURCES:
        src = os.path.join(CSRC, name)
        obj = os.path.join(BUILD, name + ".o")
        if dev:
            cmd = [HIPCC] + COMMON + DEVICE + extra + ["-c", "-o", obj, src]
            if far_mfma and name == "k_eval.hip":
                cmd.insert(-4, "-DSTC_FAR_MFMA=1")
        else:
            cmd = [CLANG] + COMMON + extra + ["-x", "c++", "-c", "-o", obj, src]
        if verbose:
            print(" ".join(cmd))
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        objs.append(obj)
    failed = []
    for cmd, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            failed.append((cmd, out))
        elif verbose and out.strip():
            print(out)
    if failed:
        for cmd, out in failed:
            sys.stderr.write(" ".join(cmd) + "\n" + out + "\n")
        raise RuntimeError("compilation failed")
    tmp = lib + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    shutil.move(tmp, lib)
    return lib


if __name__ == "__main__":
    dst = None
    if "-o" in sys.argv:
        dst = os.path.abspath(sys.argv[sys.argv.index("-o") + 1])
    print(build(verbose="-v" in sys.argv, out=dst))
