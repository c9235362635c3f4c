"""Builds the CPU emulation of libcgl (host code + HIP kernels compiled as
host C++ against the emulated runtime in this directory) with
AddressSanitizer and UndefinedBehaviorSanitizer, plus the driver."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2403_02816_amd", "csrc")
OUT = os.path.join(ROOT, "_build", "emu")
CXX = "/opt/rocm/llvm/bin/clang++"
FLAGS = ["-std=c++20", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
         "-fno-sanitize-recover=undefined", "-I", HERE, "-Wno-unknown-attributes", "-Wno-psabi"]


def build() -> str:
    os.makedirs(OUT, exist_ok=True)
    srcs = [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC)) if f.endswith((".cpp", ".hip"))]
    srcs.append(os.path.join(HERE, "emu_driver.cpp"))

    def comp(src):
        obj = os.path.join(OUT, os.path.basename(src) + ".o")
        lang = ["-x", "c++"] if src.endswith(".hip") else []
        r = subprocess.run([CXX, *FLAGS, *lang, "-c", src, "-o", obj], capture_output=True, text=True)
        if r.returncode:
            raise RuntimeError(r.stderr)
        return obj

    with cf.ThreadPoolExecutor(8) as ex:
        objs = list(ex.map(comp, srcs))
    exe = os.path.join(OUT, "emu_driver")
    r = subprocess.run([CXX, *FLAGS, *objs, "-o", exe, "-lpthread"], capture_output=True, text=True)
    if r.returncode:
        raise RuntimeError(r.stderr)
    return exe


if __name__ == "__main__":
    print(build())
