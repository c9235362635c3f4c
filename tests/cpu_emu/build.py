"""Builds the CPU emulation of libcgl (host code + HIP kernels compiled as
host C++ against the emulated runtime in this directory) with
AddressSanitizer and UndefinedBehaviorSanitizer, plus the driver."""
from __future__ import annotations

import concurrent.futures as cf
import hashlib
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2403_02816_amd", "csrc")
OUT = os.path.join(ROOT, "_build", "emu")
CXX = "/opt/rocm/llvm/bin/clang++"
FLAGS = ["-std=c++20", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
         "-fno-sanitize-recover=undefined", "-I", HERE, "-Wno-unknown-attributes", "-Wno-psabi"]


def _digest(srcs) -> str:
    """Hash of every source and header the emulation build reads, and the flags."""
    h = hashlib.sha256(" ".join(FLAGS).encode())
    files = list(srcs)
    for d in (CSRC, os.path.join(ROOT, "include"), os.path.join(HERE, "hip")):
        files += [os.path.join(d, f) for f in sorted(os.listdir(d)) if f.endswith((".h", ".hpp"))]
    for f in files:
        with open(f, "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()


def build() -> str:
    """Builds the driver, or returns it when nothing it is built from changed."""
    os.makedirs(OUT, exist_ok=True)
    srcs = [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC)) if f.endswith((".cpp", ".hip"))]
    srcs.append(os.path.join(HERE, "emu_driver.cpp"))
    exe = os.path.join(OUT, "emu_driver")
    stamp = os.path.join(OUT, "stamp")
    digest = _digest(srcs)
    if os.path.exists(exe) and os.path.exists(stamp) and open(stamp).read() == digest:
        return exe

    def comp(src):
        obj = os.path.join(OUT, os.path.basename(src) + ".o")
        lang = ["-x", "c++"] if src.endswith(".hip") else []
        r = subprocess.run([CXX, *FLAGS, *lang, "-c", src, "-o", obj], capture_output=True, text=True)
        if r.returncode:
            raise RuntimeError(r.stderr)
        return obj

    with cf.ThreadPoolExecutor(8) as ex:
        objs = list(ex.map(comp, srcs))
    r = subprocess.run([CXX, *FLAGS, *objs, "-o", exe, "-lpthread"], capture_output=True, text=True)
    if r.returncode:
        raise RuntimeError(r.stderr)
    with open(stamp, "w") as fh:
        fh.write(digest)
    return exe


if __name__ == "__main__":
    print(build())
