"""Build libscmc.so (HIP for gfx950) in-tree with hipcc.

Every translation unit is compiled to an object in parallel, then linked into
``paper_2112_02574_amd/libscmc.so``.  All HIP code is compiled with packed
FP32 instructions disabled.
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libscmc.so")
# (source, object name, extra defines): the fused kernels are instantiated
# once per storage format and stencil order so that they compile in parallel
SOURCES = [("step_kernels.hip", "step_kernels", []),
           ("fused_kernels.hip", "fused_kernels", []),
           ("obs_kernels.hip", "obs_kernels", []),
           ("ceiling_kernels.hip", "ceiling_kernels", []),
           ("scmc_api.cpp", "scmc_api", [])]
for _st in ("StoreF32", "StoreF16", "StoreBF16"):
    for _order in (4, 6):
        SOURCES.append(("fused_inst.hip", f"fused_{_st}_{_order}",
                        [f"-DSCMC_INST_STORE=scmc::{_st}", f"-DSCMC_INST_ORDER={_order}"]))
ARCH = os.environ.get("SCMC_OFFLOAD_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function"]


def _compile(item):
    src, name, defines = item
    obj = os.path.join(BUILD, name + ".o")
    lang = ["-x", "hip"] if src.endswith(".cpp") else []
    cmd = ["hipcc"] + FLAGS + defines + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{err}")
    return obj, err


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    workers = min(len(SOURCES), os.cpu_count() or 1)
    with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
        results = list(ex.map(_compile, SOURCES))
    for _, err in results:
        if verbose and err.strip():
            print(err, file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + [o for o, _ in results]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
