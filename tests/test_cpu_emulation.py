"""Runs the library's host code and HIP kernels on the CPU (emulated HIP
runtime, one host thread per lane, emulated MFMA) under AddressSanitizer and
UndefinedBehaviorSanitizer: every entry point, both precisions, every kernel
variant (mu = 1 contiguous, mu > 1 strided, ragged tiles), d = 1..3, graph
replay.  Fails on any out-of-bounds access, UB, or a mode product / Tucker
result off the naive reference."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


FULL = os.environ.get("CGL_EMU_FULL") == "1"


@pytest.mark.skipif(not os.path.exists("/opt/rocm/llvm/bin/clang++"), reason="needs ROCm clang++")
def test_library_under_cpu_emulation_with_sanitizers():
    """By default one case of every kernel family (about 3 minutes); with
    CGL_EMU_FULL=1 the full sweep: every tile shape, ragged tiles, every
    stepper and method on several grids (about 15 minutes on 8 cores)."""
    from tests.cpu_emu import build as emu_build
    exe = emu_build.build()
    # the full sweep covers every split tile shape (the autotuner's timing is
    # not emulated); its runs are independent processes, started together
    procs = []
    modes = (("0", "quick"), ("1", "split"), ("0", "fft")) if FULL else (("0", "smoke"),)
    for tile, mode in modes:
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
                   UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", CGL_SPLIT_TILE=tile)
        procs.append((tile, mode, subprocess.Popen([exe, mode], stdout=subprocess.PIPE,
                                                   stderr=subprocess.PIPE, text=True, env=env)))
    for tile, mode, pr in procs:
        out, err = pr.communicate(timeout=900)
        print(out[-4000:])
        print(err[-4000:])
        assert pr.returncode == 0, (tile, mode)
        assert "PASSED (0 failures)" in out
