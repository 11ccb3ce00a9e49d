"""Build libifa.so for gfx950 with hipcc (cross-compiles without a GPU)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libifa.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
          f"-I{os.path.join(ROOT, 'include')}"]
# Packed FP32 instructions stay off in every device compile.
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

SOURCES = ["ifa_scan.hip", "ifa_runtime.cpp", "ifa_sam.cpp", "ifa_seed.cpp"]


def build(force=True, verbose=False):
    if not force and os.path.exists(LIB):
        return LIB
    objs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(CSRC, src + ".o")
        cmd = [HIPCC, *COMMON, "-c", path, "-o", obj]
        if src.endswith(".hip"):
            # matrix-core results stay in VGPRs: the filter reads every one
            cmd[1:1] = DEVICE + ["-x", "hip", "-mllvm", "-amdgpu-mfma-vgpr-form"]
        else:
            cmd[1:1] = ["-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"]
        if verbose:
            print(" ".join(cmd))
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *DEVICE, "-shared", "-fPIC", *objs, "-o", tmp, "-lpthread"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    build_calib(verbose)
    return LIB


CALIB_LIB = os.path.join(HERE, "libifa_calib.so")


def build_calib(verbose=False):
    """The copy kernel that calibrates HBM byte counters (measurement only)."""
    tmp = CALIB_LIB + ".tmp"
    cmd = [HIPCC, *DEVICE, "-x", "hip", *COMMON, "-shared",
           os.path.join(CSRC, "ifa_calib.hip"), "-o", tmp]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, CALIB_LIB)
    return CALIB_LIB


if __name__ == "__main__":
    print(build(verbose=True))
