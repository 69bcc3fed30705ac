"""Build libsar_rda.so (HIP, gfx950) in-tree with hipcc.

    python paper_2604_03585_amd/build.py

Every source under csrc/ is compiled to an object in _build/ (in parallel)
and the objects are linked into paper_2604_03585_amd/libsar_rda.so.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libsar_rda.so")
ARCH = "gfx950"

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang++"


def hip_runtime_dir() -> str:
    """Directory of the HIP runtime the process will use.

    PyTorch wheels for ROCm carry their own libamdhip64.so (and HSA runtime);
    a second HIP runtime loaded into the same process cannot open the GPU.
    The library therefore links against torch's copy when torch is installed,
    and against /opt/rocm otherwise."""
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec and spec.origin:
        d = os.path.join(os.path.dirname(spec.origin), "lib")
        if os.path.exists(os.path.join(d, "libamdhip64.so")):
            return d
    return "/opt/rocm/lib"

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wall", "-Wno-unused-function", "-mcode-object-version=5",
]
# Packed FP32 (v_pk_*_f32) is kept out of every kernel.
DEVICE_ONLY = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def sources(csrc: str = CSRC):
    return sorted(os.path.join(csrc, f) for f in os.listdir(csrc)
                  if f.endswith((".hip", ".cpp")))


def _compile(src: str, build_dir: str = BUILD) -> str:
    obj = os.path.join(build_dir, os.path.basename(src) + ".o")
    inc = ["-I", os.path.dirname(src)]
    cmd = [HIPCC, *COMMON, *inc, *DEVICE_ONLY, "-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass does not know the packed-fp32 feature and says so
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in r.stderr.splitlines() if noise not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{err}")
    if err.strip():
        sys.stderr.write(err + "\n")
    return obj


def build(verbose: bool = False, csrc: str = CSRC, lib: str = LIB,
          build_dir: str = BUILD) -> str:
    """Compile every source of `csrc` and link `lib` (defaults: this package)."""
    os.makedirs(build_dir, exist_ok=True)
    srcs = sources(csrc)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda f: _compile(f, build_dir), srcs))
    tmp = lib + ".tmp"
    rt = hip_runtime_dir()
    cmd = [CLANG, "-shared", "-fPIC", *objs, "-o", tmp,
           f"-L{rt}", "-l:libamdhip64.so", f"-Wl,-rpath,{rt}", "-Wl,--no-undefined",
           "-Wl,--as-needed"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print(f"built {lib}")
    return lib


if __name__ == "__main__":
    build(verbose=True)
