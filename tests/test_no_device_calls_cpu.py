"""The built library's gfx950 code makes no device-function calls: every
kernel's device functions are inlined, so that kernels keep the LDS vectors
in LDS address space (no generic pointers) and use no call stack.  The
compiler outlines a large device function on its own when it is called from
several kernels; a forced outline changes the code the launch forms were
measured and tested with, so this check fails if one appears.  Reads the
AMD assembly of the library built here (llvm-objdump from ROCm)."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2304_04876_amd", "libgdsw.so")
OBJDUMP = "/opt/rocm/llvm/bin/llvm-objdump"


@pytest.mark.skipif(not os.path.exists(LIB) or not os.path.exists(OBJDUMP),
                    reason="needs the built library and ROCm's llvm-objdump")
def test_library_makes_no_device_calls():
    with tempfile.TemporaryDirectory() as tmp:
        so = os.path.join(tmp, "libgdsw.so")
        shutil.copy(LIB, so)
        # (extracts the offload bundles next to the copy)
        subprocess.run([OBJDUMP, "--offloading", so], cwd=tmp, check=True, capture_output=True, timeout=300)
        objs = [f for f in os.listdir(tmp) if "amdgcn" in f and "gfx950" in f]
        assert objs, os.listdir(tmp)
        for f in objs:
            asm = subprocess.run([OBJDUMP, "-d", "--mcpu=gfx950", os.path.join(tmp, f)], check=True,
                                 capture_output=True, text=True, timeout=600).stdout
            assert "s_endpgm" in asm   # (the kernels were disassembled)
            calls = [ln for ln in asm.splitlines() if "s_swappc" in ln or "s_call_b64" in ln]
            assert not calls, calls[:5]
