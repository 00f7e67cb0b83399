"""Builds liblpgpu_emu.so: the library's own HIP sources compiled for the host CPU against
emu_hip.h, a CPU emulation of the part of HIP they use.  Test infrastructure only: the
package never loads it; tests/test_emu_cpu.py points the binding at it in its own process.

Every GPU thread runs as a fiber, one workgroup at a time; barriers and wave operations
(shuffles, ballots, readlane, DPP moves, the FP64 MFMA tile) are resolved by a scheduler
once every live lane of the wave (or workgroup) has reached them; device and pinned host
allocations, and each launch's dynamic LDS, sit against guard pages, so an out-of-bounds
access stops the run with the kernel, workgroup and thread named.  The whole-wave
reductions of lp_wave.h (DPP trees) are replaced by single wave operations with the same
results; wave_sum keeps its xor-butterfly order, so every dot product rounds as on the
device.  The rocBLAS calls of the large-block reinversion run as plain loops.

    python tests/emu/build.py [OUT.so]
"""
import os
import re
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(ROOT, "paper_1803_04378_amd", "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(BUILD, "liblpgpu_emu.so")
SOURCES = ["lp_kernels.hip", "lp_mixed.hip", "lp_reinv.hip", "lp_phase.hip", "lp_api.hip", "lp_batch.hip",
           "lp_batch_api.hip"]
CXX = os.environ.get("EMU_CXX", "/opt/rocm/llvm/bin/clang++")

# The whole-wave reductions as single wave operations (emu_hip.h); the DPP versions stay,
# renamed, unused.
WAVE_OPS = """
__device__ __forceinline__ void wave_lexmin(double& d, int& j) { emu_wave_lexmin(d, j); }
__device__ __forceinline__ void wave_lexmin_payload(double& d, int& j, int& p) { emu_wave_lexmin_payload(d, j, p); }
__device__ __forceinline__ void wave_two_smallest(double& a, double& b) { emu_wave_two_smallest(a, b); }
__device__ __forceinline__ int wave_min_int(int v) { return emu_wave_min_int(v); }
__device__ __forceinline__ int wave_sum_int(int v) { return emu_wave_sum_int(v); }
__device__ __forceinline__ double wave_min(double v) { return emu_wave_min(v); }
__device__ __forceinline__ double wave_sum(double v) { return emu_wave_sum(v); }
"""


def prepare(dst):
    """Copies the sources, turning dynamic LDS declarations into the launch's buffer."""
    for f in os.listdir(SRC):
        s = open(os.path.join(SRC, f)).read()
        s = re.sub(r"extern __shared__ (?:__align__\(\d+\) )?((?:unsigned )?\w+) (\w+)\[\];",
                   r"\1* \2 = (\1*)emu::dyn_lds();", s)
        s = re.sub(r"__attribute__\(\(amdgpu_\w+\([^)]*\)\)\)", "", s)  # register budgets: device only
        if f == "lp_wave.h":
            for fn in ("wave_lexmin_payload", "wave_lexmin", "wave_two_smallest", "wave_min_int", "wave_sum_int",
                       "wave_min", "wave_sum"):
                s = re.sub(r"(__device__ __forceinline__ \w+ )" + fn + r"\(", r"\1" + fn + "_dpp(", s)
            s = s.replace("namespace detail {", "namespace detail {\n" + WAVE_OPS, 1)
        with open(os.path.join(dst, f), "w") as fh:
            fh.write(s)


def build(out=LIB, opt="-O1"):
    src_dir = os.path.join(BUILD, "src")
    shutil.rmtree(src_dir, ignore_errors=True)
    os.makedirs(src_dir)
    prepare(src_dir)
    flags = ["-std=c++17", opt, "-g", "-fPIC", "-ffp-contract=off", "-I", os.path.join(HERE, "fakeinc"), "-I",
             src_dir, "-I", os.path.join(ROOT, "include"), "-include", os.path.join(HERE, "emu_hip.h"),
             "-Wno-everything"]

    def compile_one(name):
        src = os.path.join(src_dir, name) if name.endswith(".hip") else os.path.join(HERE, name)
        obj = os.path.join(src_dir, name + ".o")
        res = subprocess.run([CXX, *flags, "-x", "c++", "-c", src, "-o", obj], capture_output=True, text=True)
        return name, obj, res

    with ThreadPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
        results = list(ex.map(compile_one, SOURCES + ["emu_rt.cpp", "glue.cpp"]))
    for name, _, res in results:
        if res.returncode:
            raise RuntimeError(f"emulation build of {name} failed:\n{res.stderr[-4000:]}")
    tmp = out + ".tmp"
    res = subprocess.run([CXX, "-shared", "-o", tmp] + [o for _, o, _ in results] + ["-lpthread"],
                         capture_output=True, text=True)
    if res.returncode:
        raise RuntimeError("linking the emulation library failed:\n" + res.stderr[-4000:])
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(sys.argv[1] if len(sys.argv) > 1 else LIB))
