"""Build libtdse_emu.so: the library's kernels and C ABI compiled for the CPU
against tests/emu/hip_emu.h (test harness only; "device" pointers are host
pointers)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2001_06113_amd", "csrc")
OUT = os.path.join(HERE, "libtdse_emu.so")
SOURCES = [os.path.join(CSRC, "periodic_kernels.hip"), os.path.join(CSRC, "freespace_kernels.hip"),
           os.path.join(CSRC, "batch_fp64.hip"), os.path.join(CSRC, "batch_split.hip"),
           os.path.join(CSRC, "adjoint_kernels.hip"), os.path.join(CSRC, "far_kernels.hip"),
           os.path.join(CSRC, "run1d_kernels.hip"), os.path.join(CSRC, "persist2d_kernels.hip"),
           os.path.join(CSRC, "diag_kernels.hip"),
           os.path.join(CSRC, "tdse_api.cpp"),
           os.path.join(HERE, "emu_globals.cpp")]


TSAN_DRIVER = os.path.join(HERE, "tsan_batch_adjoint.cpp")
TSAN_OUT = os.path.join(HERE, "tsan_batch_adjoint")


def build(sanitize: bool = False) -> str:
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", "-shared", "-pthread", "-include", os.path.join(HERE, "hip_emu.h"),
             f"-I{os.path.join(HERE, 'stub')}", f"-I{CSRC}", f"-I{os.path.join(ROOT, 'include')}", "-x", "c++"]
    if sanitize:
        flags = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer"] + flags
    cmd = ["g++", *flags, *SOURCES, "-o", OUT]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(" ".join(cmd) + "\n" + r.stderr[-4000:])
    return OUT


def build_tsan_driver() -> str:
    """The library's host code and kernels with the batch-adjoint driver in one
    ThreadSanitizer executable (host CPU build; no GPU code is involved)."""
    flags = ["-O1", "-g", "-std=c++17", "-pthread", "-fsanitize=thread", "-fno-omit-frame-pointer",
             "-include", os.path.join(HERE, "hip_emu.h"), f"-I{os.path.join(HERE, 'stub')}", f"-I{CSRC}",
             f"-I{os.path.join(ROOT, 'include')}", "-x", "c++"]
    cmd = ["g++", *flags, *SOURCES, TSAN_DRIVER, "-o", TSAN_OUT]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(" ".join(cmd) + "\n" + r.stderr[-4000:])
    return TSAN_OUT


if __name__ == "__main__":
    print(build())
