"""Build libclmap.so (HIP for gfx950) in-tree with hipcc.

The library is the product's compute path; the Python binding loads it from
this directory and fails loudly when it is missing.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libclmap.so")
BUILD = os.path.join(HERE, "_build")

SOURCES = ["build_kernels.hip", "sweep_kernels.hip", "sweep_half.hip", "md_kernels.hip", "kclosest_kernels.hip",
           "calib_kernels.hip", "static_map.hip", "nl_sort.hip",
           "clmap_api.cpp", "md_api.cpp", "kclosest_api.cpp", "calib_api.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# -ffp-contract=off: the canonical FP64 arithmetic (wrap, image shift,
# squared distance) must not be fused; FP32 code requests FMA explicitly.
# -packed-fp32-ops: packed FP32 VALU instructions are kept out of the code.
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-ffp-contract=off",
    "-fno-fast-math", "-Wall", "-Wno-unused-function",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = (r.stdout or "") + (r.stderr or "")
    # the host pass does not know the GPU-only target feature: harmless
    lines = [l for l in out.splitlines() if "packed-fp32-ops" not in l and l.strip()]
    if r.returncode != 0:
        sys.stderr.write(out)
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}")
    if verbose and lines:
        print("\n".join(lines))


def build(verbose=False, jobs=None):
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [HIPCC] + FLAGS + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
        objs.append(obj)
        procs.append(cmd)
    # compile in parallel
    import concurrent.futures as cf
    with cf.ThreadPoolExecutor(max_workers=jobs or min(4, len(procs))) as ex:
        list(ex.map(lambda c: _run(c, verbose), procs))
    tmp = LIB + ".tmp"
    # export only the C-ABI (clm_*), see csrc/libclmap.map
    exports = "-Wl,--version-script=" + os.path.join(CSRC, "libclmap.map")
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", exports] + objs + ["-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
