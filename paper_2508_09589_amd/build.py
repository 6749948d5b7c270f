"""Build libst.so (the HIP library behind include/st_api.h) for gfx950, in-tree.

    python -m paper_2508_09589_amd.build [--jobs N]

Every source under csrc/ is compiled by hipcc for gfx950 only, with packed-FP32
instruction selection disabled, and linked into paper_2508_09589_amd/libst.so.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libst.so")

SOURCES = ["kernels_fine.hip", "kernels_level.hip", "kernels_krylov.hip", "kernels_coarse.hip",
           "kernels_smooth.hip", "kernels_sstep.hip", "kernels_design.hip", "noalloc.hip",
           "solver.cpp"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
         "-Wno-unused-variable", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    return "hipcc"


def _compile(src):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc(), "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj] + FLAGS
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj, r.stderr


def build(jobs=4, verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        results = list(ex.map(_compile, SOURCES))
    if verbose:
        for _, err in results:
            if err.strip():
                sys.stderr.write(err)
    objs = [o for o, _ in results]
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


def build_host_check(out_dir=None):
    """Build tests/host_check.cpp against the library's host code compiled
    with AddressSanitizer and UndefinedBehaviorSanitizer (host side only: the
    kernels stay as built) and return the executable's path.  Needs the
    kernel objects of build()."""
    out_dir = out_dir or os.path.join(BUILD, "san")
    os.makedirs(out_dir, exist_ok=True)
    san_obj = os.path.join(out_dir, "solver_san.o")
    cmd = [_hipcc(), "-x", "hip", "-c", os.path.join(CSRC, "solver.cpp"), "-o", san_obj] + FLAGS + [
        "-O1", "-g", "-fno-omit-frame-pointer",
        "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for the sanitized host code:\n{r.stderr}")
    drv_obj = os.path.join(out_dir, "host_check.o")
    gxx = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-I", os.path.join(ROOT, "include")]
    r = subprocess.run(gxx + ["-c", os.path.join(ROOT, "tests", "host_check.cpp"), "-o", drv_obj],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"g++ failed for host_check.cpp:\n{r.stderr}")
    kern = [os.path.join(BUILD, os.path.splitext(x)[0] + ".o") for x in SOURCES if x != "solver.cpp"]
    exe = os.path.join(out_dir, "host_check")
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    r = subprocess.run(gxx + ["-o", exe, drv_obj, san_obj] + kern +
                       ["-L", os.path.join(rocm, "lib"), "-Wl,-rpath," + os.path.join(rocm, "lib"),
                        "-lamdhip64"], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link of host_check failed:\n{r.stderr}")
    return exe


if __name__ == "__main__":
    jobs = 4
    if "--jobs" in sys.argv:
        jobs = int(sys.argv[sys.argv.index("--jobs") + 1])
    print(build(jobs, verbose=True))
