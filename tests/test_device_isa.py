"""The device code, compiled with the library's own flags, assembles cleanly.

The backend hands its instructions straight to the encoder when it builds
the library; an operand the instruction cannot encode (a 64-bit literal in a
scalar move, for one) is then silently cut down instead of rejected.  Running
the same compile to assembly text and through the assembler, which does check
operands, keeps such instructions out of the shipped code object.
"""
import os
import subprocess
import tempfile

import pytest

from paper_2604_13144_amd import build

LLVM_MC = "/opt/rocm/llvm/bin/llvm-mc"


@pytest.mark.slow
@pytest.mark.skipif(not os.path.exists(LLVM_MC), reason="llvm-mc not installed")
@pytest.mark.parametrize("source", ["kernels.hip", "queue.hip"])
def test_device_assembly_is_encodable(source):
    flags = [f for f in build.HIPCC_FLAGS if f not in ("-shared", "-fPIC")]
    with tempfile.TemporaryDirectory() as d:
        asm = os.path.join(d, "kernels.s")
        cmd = [build.hipcc(), *flags, "--cuda-device-only", "-S",
               "-I", build.INCLUDE, "-I", build.CSRC,
               os.path.join(build.CSRC, source), "-o", asm]
        res = subprocess.run(cmd, capture_output=True, text=True)
        assert res.returncode == 0, res.stderr[-2000:]
        res = subprocess.run([LLVM_MC, "-triple=amdgcn-amd-amdhsa", "-mcpu=gfx950",
                              "-filetype=obj", asm, "-o", os.path.join(d, "k.o")],
                             capture_output=True, text=True)
        errors = [l for l in res.stderr.splitlines() if "error:" in l]
        context = []
        if errors:
            lines = open(asm).read().splitlines()
            for e in errors[:5]:
                n = int(e.split(":")[1])
                context.append(lines[n - 1].strip())
        assert res.returncode == 0 and not errors, (len(errors), errors[:5], context)
