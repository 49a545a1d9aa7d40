"""Build the gfx950 HIP library (librbgs.so) in-tree with hipcc.

Usage: python -m paper_2111_14641_amd.build   (or build() from Python)
"""
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "librbgs.so")
ARCH = "gfx950"

SOURCES = ["rbgs_api.hip", "sketch_kernels.hip", "update_kernels.hip", "small_kernels.hip",
           "krylov_kernels.hip", "post_kernels.hip", "batch_kernels.hip"]

# Packed FP32 instructions are disabled: the compiler would otherwise form
# v_pk_* FP32 operations from scalar code.
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument", "-fvisibility=hidden",
    "-I", INCLUDE, "-I", CSRC,
]


# Per-source additions.  The dense sketch keeps its matrix-core accumulators in
# ordinary vector registers (the VGPR form of the MFMA instructions): with the
# accumulation-register form the 16-column kernel copied all of them to and
# from those registers around every 4-row step.
SOURCE_FLAGS = {
    "sketch_kernels.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
}


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose=False, jobs=4):
    """Compile every source to an object file (in parallel) and link librbgs.so."""
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    cc = hipcc()
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        cmd = [cc, *FLAGS, *SOURCE_FLAGS.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _wait(procs.pop(0))
    for p in procs:
        _wait(p)
    tmp = LIB + ".tmp"
    cmd = [cc, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    out = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if out.returncode != 0:
        raise RuntimeError("link failed:\n" + out.stdout.decode())
    os.replace(tmp, LIB)
    return LIB


def _wait(item):
    src, p = item
    out, _ = p.communicate()
    text = out.decode()
    if p.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{text}")
    # the host pass does not know the packed-fp32 feature; that warning is expected
    lines = [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
    if lines:
        sys.stderr.write(f"[{src}]\n" + "\n".join(lines) + "\n")


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
