"""Build step: compile the HIP library (and its CPU emulation test tool).

    python -m paper_1805_06018_amd.build

libpc.so      hipcc, gfx950, the product library (C ABI in include/pc.h)
libpc_emu.so  host-only build of the same kernel phases, for CPU tests
libpc_emu_asan.so  the same with AddressSanitizer on the host code
workloads/libblur.so  exact spatially varying blur (the black-box operator)
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("PC_OFFLOAD_ARCH", "gfx950")

LIB = os.path.join(HERE, "libpc.so")
EMU = os.path.join(HERE, "libpc_emu.so")
EMU_ASAN = os.path.join(HERE, "libpc_emu_asan.so")
BLUR_SRC = os.path.join(ROOT, "workloads", "csrc")
BLUR = os.path.join(ROOT, "workloads", "libblur.so")

COMMON = ["-std=c++17", "-fPIC", "-shared", "-I" + os.path.join(ROOT, "include")]
# packed FP32 instructions are kept out of every device build
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd, out):
    tmp = out + ".tmp%d" % os.getpid()
    full = cmd + ["-o", tmp]
    r = subprocess.run(full, cwd=CSRC, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build failed: " + " ".join(full))
    os.replace(tmp, out)
    return out


def build_lib():
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-O3", "-fopenmp"] + COMMON + DEVICE_FLAGS + [
        "pc_kernels.hip", "pc_host.cpp", "pc_plan.cpp", "pc_plan3.cpp"]
    return _run(cmd, LIB)


def build_emu(asan=False):
    cmd = [HIPCC, "-x", "hip", "--offload-host-only", "-O1", "-g", "-fopenmp"] + COMMON
    if asan:
        cmd += ["-Xarch_host", "-fsanitize=address", "-fno-omit-frame-pointer"]
    cmd += ["pc_emu.cpp", "pc_plan.cpp", "pc_plan3.cpp"]
    return _run(cmd, EMU_ASAN if asan else EMU)


def build_blur():
    """The exact blur operator used as the estimator's black-box adjoint."""
    tmp = BLUR + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared"] + DEVICE_FLAGS + [
        "blur_direct.hip", "-o", tmp]
    r = subprocess.run(cmd, cwd=BLUR_SRC, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build failed: " + " ".join(cmd))
    os.replace(tmp, BLUR)
    return BLUR


def build_all():
    build_lib()
    build_blur()
    build_emu(False)
    build_emu(True)


if __name__ == "__main__":
    build_all()
    print("built", LIB)
