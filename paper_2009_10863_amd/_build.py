"""Build the libguess shared library for gfx950 with hipcc (in-tree).

Every HIP source under ``csrc/`` is compiled to an object file under
``_build/`` at the repository root, then linked into
``paper_2009_10863_amd/_lib/libguess.so``.  Called by ``__graft_entry__.build()``;
it always recompiles.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "_lib", "libguess.so")
# (source, object name, extra flags).  PCG's stencil kernel issues ~30 loads
# per chunk and the projection kernels up to 2M + 2 streams per chunk; the
# max-ILP scheduler groups those loads (measured in the step loop at 256^3:
# the fused apply 8 % and the second Gram-Schmidt pass 3 % faster; the
# extrapolation kernels gained nothing, so they keep the default).  The
# projection kernels are compiled once per storage format and variant (bit 1:
# rolling QR, bit 2: l2 inner product), the raw-solution projection once per
# storage format.  The FP16 / BF16 projection units are built for at least three
# waves per SIMD: their 2-byte columns keep fewer bytes in flight per wave (at
# 256^3, M = 8: fused apply 90 -> 81 us, write pass 104 -> 94 us, rolling write
# pass 132-140 -> 95 us; FP32 ran 1 % slower that way, so FP32 and FP64 keep the
# default).
_DTYPES = ["GUESS_F64", "GUESS_F32", "GUESS_F16", "GUESS_BF16"]
_MAX_ILP = ["-mllvm", "-amdgpu-sched-strategy=max-ilp"]
UNITS = [("proj_inst.hip", f"proj_{dt[6:].lower()}_v{vf}",
          [f"-DLG_PROJ_DT={dt}", f"-DLG_PROJ_VF={vf}", *_MAX_ILP,
           *(["-DLG_WAVES_MIN=3"] if dt in ("GUESS_F16", "GUESS_BF16") else [])])
         for dt in _DTYPES for vf in range(4)]
UNITS += [("rawproj_inst.hip", f"rawproj_{dt[6:].lower()}", [f"-DLG_RAW_DT={dt}", *_MAX_ILP]) for dt in _DTYPES]
UNITS += [("pcg.hip", "pcg", [*_MAX_ILP, "-DLG_WAVES_MIN=2"])]
UNITS += [(src, src[:-4], []) for src in ("extrap.hip", "proj.hip", "rawproj.hip", "op.hip", "vec.hip", "host.hip")]
SOURCES = sorted({u[0] for u in UNITS})
ARCH = "gfx950"

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-function",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # no mixed-precision FMA: FP16 history is widened with v_cvt_f32_f16,
    # which keeps FP16 subnormals exact (the mixed FMA's FP16 operands did not)
    "-Xclang", "-target-feature", "-Xclang", "-fma-mix-insts",
    f"-I{INCLUDE}",
    f"-I{CSRC}",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(unit) -> str:
    src, name, extra = unit
    obj = os.path.join(OBJDIR, name + ".o")
    cmd = [hipcc(), *HIPCC_FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs: int = None) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    jobs = jobs or min(len(UNITS), os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, UNITS))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
