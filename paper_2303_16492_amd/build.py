"""Builds the gfx950 HIP library ``libtrsgd.so`` in-tree with hipcc.

Every ``csrc/*.hip`` file is compiled for gfx950 only, with packed FP32
instructions disabled, then linked into one shared library.  The library is
linked against the HIP runtime that ships inside the installed PyTorch so
that a process which imports torch maps a single HIP runtime (streams and
device pointers from torch are then valid in the library).

Run ``python -m paper_2303_16492_amd.build`` or call ``build()``.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(ROOT, "_build", "obj")
LIB = os.path.join(HERE, "libtrsgd.so")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = [
    "-std=c++17", "-O3", "-fPIC", f"--offload-arch={ARCH}",
    "-mcode-object-version=5",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def _torch_lib_dir() -> str | None:
    try:
        import importlib.util
        spec = importlib.util.find_spec("torch")
        if spec is None or not spec.origin:
            return None
        d = os.path.join(os.path.dirname(spec.origin), "lib")
        return d if os.path.exists(os.path.join(d, "libamdhip64.so")) else None
    except Exception:
        return None


# Per-source code-generation options.  sweep.hip: the FP64 matrix-core
# accumulators of the one-workgroup inverse are selected in ordinary vector
# registers (the VGPR form of the MFMA instructions), which removes the
# copies between accumulation and vector registers from every block step.
PER_SOURCE = {
    "sweep.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"],
}


def _compile(src: str) -> str:
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    cmd = [HIPCC, *COMMON, *PER_SOURCE.get(os.path.basename(src), []), "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    jobs = min(len(srcs), max(1, min(8, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tlib = _torch_lib_dir()
    link = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", LIB + ".tmp", *objs]
    if tlib:
        # Resolve libamdhip64 to torch's copy first (DT_RUNPATH), so one
        # process never maps two HIP runtimes.
        link = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-no-hip-rt",
                "-o", LIB + ".tmp", *objs, f"-L{tlib}", "-lamdhip64",
                f"-Wl,-rpath,{tlib}", "-Wl,--enable-new-dtags"]
    r = subprocess.run(link, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    shutil.move(LIB + ".tmp", LIB)
    if verbose:
        print(f"built {LIB} from {len(srcs)} sources", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
