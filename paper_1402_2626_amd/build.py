"""Build the HIP library in-tree: ``paper_1402_2626_amd/libpolyeval.so``.

    python -m paper_1402_2626_amd.build [-v] [-j JOBS]

Compiles for gfx950 with hipcc.  The kernel launchers are compiled once per
(level, kind) from ``csrc/instances.hip`` so that the objects build in
parallel; ``csrc/polyeval.hip`` (the C ABI) and ``csrc/packer.cpp`` (the host
packer) are compiled on their own, and everything is linked into one shared
library.  Floating-point contraction is off (the error-free transformations
rely on it) and packed FP32 instructions are disabled for all HIP code.
"""
import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpolyeval.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("PE_OFFLOAD_ARCH", "gfx950")

LEVELS = (1, 2, 4)
KINDS = (0, 1, 2, 3, 4)  # rows, adjoint, batch, Gauss-Newton, least squares
# real-arithmetic level codes (8 | limbs) and the kinds compiled for them
REAL_LEVELS = (9, 10, 12)
REAL_KINDS = (0, 3, 4)

FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-ffp-contract=off", "-fno-fast-math",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def compile_commands(objdir):
    """(object file, hipcc command) for every translation unit."""
    cmds = []
    for src in ("polyeval.hip", "packer.cpp"):
        obj = os.path.join(objdir, src + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmds.append((obj, [HIPCC, *FLAGS, "-c", *lang, os.path.join(CSRC, src), "-o", obj]))
    pairs = [(L, K) for L in LEVELS for K in KINDS] + [(L, K) for L in REAL_LEVELS for K in REAL_KINDS]
    for L, K in pairs:
        obj = os.path.join(objdir, f"instances_L{L}_K{K}.o")
        cmds.append((obj, [HIPCC, *FLAGS, f"-DPE_LEVEL={L}", f"-DPE_KIND={K}", "-c",
                           os.path.join(CSRC, "instances.hip"), "-o", obj]))
    return cmds


def build(verbose: bool = False, jobs: int | None = None) -> str:
    jobs = jobs or min(len(LEVELS) * len(KINDS) + len(REAL_LEVELS) * len(REAL_KINDS) + 2,
                       max(1, os.cpu_count() or 1), 16)
    objdir = tempfile.mkdtemp(prefix="pe_build_")
    try:
        cmds = compile_commands(objdir)

        def run(cmd):
            return subprocess.run(cmd, capture_output=True, text=True)

        with ThreadPoolExecutor(jobs) as pool:
            results = list(pool.map(run, [c for _, c in cmds]))
        for (obj, cmd), res in zip(cmds, results):
            if res.returncode != 0:
                sys.stderr.write(" ".join(cmd) + "\n" + res.stdout + res.stderr)
                raise RuntimeError(f"hipcc failed on {os.path.basename(obj)}")
            if verbose and res.stderr:
                sys.stderr.write(res.stderr)
        tmp = LIB + ".tmp"
        link = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *[o for o, _ in cmds], "-o", tmp]
        res = subprocess.run(link, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("linking libpolyeval.so failed")
        os.replace(tmp, LIB)
    finally:
        shutil.rmtree(objdir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    j = None
    if "-j" in sys.argv:
        j = int(sys.argv[sys.argv.index("-j") + 1])
    print(build(verbose="-v" in sys.argv, jobs=j))
