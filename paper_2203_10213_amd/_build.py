"""Build libvkt.so (HIP for gfx950) in-tree with hipcc.

Each csrc/*.hip translation unit is compiled to an object in parallel, then
linked into paper_2203_10213_amd/libvkt.so.  Packed-FP32 instruction
selection is disabled for all device code.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libvkt.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-pass-failed",
         "-I", os.path.join(PKG, "..", "include")]


# Translation units compiled more than once, with their per-object flags.
# The matrix-core kernels are built per tile shape, all with MFMA accumulators
# in VGPRs: the 16x16 build so that the per-plane lane shift needs no copies;
# the 32x32 build because it then needs no accumulator copies either (1024^3
# 9^3 float32 13.45 -> 13.07 ms, 2048x2048x1024 11^3 uint16 75.5 -> 71.7 ms,
# and fewer registers: the 11^3 uint16 kernel 435 -> 321).
VARIANTS = {
    "vkt_filter_mfma.hip": [
        ("vkt_filter_mfma16", ["-DVKT_MFMA_SHAPE=16", "-mllvm", "--amdgpu-mfma-vgpr-form"]),
        ("vkt_filter_mfma32", ["-DVKT_MFMA_SHAPE=32", "-mllvm", "--amdgpu-mfma-vgpr-form"]),
    ],
    "vkt_filter_mfma_rp.hip": [("vkt_filter_mfma_rp", ["-mllvm", "--amdgpu-mfma-vgpr-form"])],
}


def sources():
    """(source, object stem, extra flags) for every object of the library."""
    out = []
    for f in sorted(os.listdir(CSRC)):
        if not f.endswith(".hip"):
            continue
        for stem, extra in VARIANTS.get(f, [(f[:-4], [])]):
            out.append((os.path.join(CSRC, f), stem, extra))
    return out


def _compile(unit, verbose):
    src, stem, extra = unit
    obj = os.path.join(OUT, stem + ".o")
    cmd = [HIPCC, *FLAGS, *extra, "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                    if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{msg}")
    if msg.strip() and verbose:
        print(msg, file=sys.stderr)
    return obj


def build_lib(verbose: bool = False, jobs: int = 0) -> str:
    """Always recompile every translation unit and relink."""
    os.makedirs(OUT, exist_ok=True)
    units = sources()
    jobs = jobs or min(len(units), os.cpu_count() or 1, 8)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda u: _compile(u, verbose), units))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_lib(verbose=True))
