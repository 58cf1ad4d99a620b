"""Checks on the compiled gfx950 code objects of the library (CPU only).

Every kernel keeps its values in registers: a kernel that spills VGPRs to
scratch memory is slow and, past the per-wave scratch the hardware can
address, computes with overwritten spill slots.  The code-object metadata
that the compiler writes for each kernel states its VGPR spill count.
"""
import glob
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OBJ = os.path.join(ROOT, "paper_2602_09020_amd", "_build")
LLVM = "/opt/rocm/llvm/bin"


def kernel_metadata(obj, tmp):
    """(kernel name, vgpr count, vgpr spill count) of every kernel in one object's gfx950 code."""
    fat = os.path.join(tmp, os.path.basename(obj) + ".fatbin")
    dev = os.path.join(tmp, os.path.basename(obj) + ".gfx950.o")
    subprocess.run([f"{LLVM}/llvm-objcopy", "--dump-section", f".hip_fatbin={fat}", obj,
                    os.path.join(tmp, "host.o")], check=True, capture_output=True)
    subprocess.run([f"{LLVM}/clang-offload-bundler", "--unbundle", "--type=o", f"--input={fat}",
                    "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", f"--output={dev}"], check=True,
                   capture_output=True)
    notes = subprocess.run([f"{LLVM}/llvm-readelf", "--notes", dev], check=True, capture_output=True,
                           text=True).stdout
    out = []
    for block in notes.split("  - .agpr_count")[1:]:
        name = re.search(r"\.name:\s+(\S+)", block).group(1)
        vgpr = int(re.search(r"\.vgpr_count:\s+(\d+)", block).group(1))
        spill = int(re.search(r"\.vgpr_spill_count:\s+(\d+)", block).group(1))
        out.append((name, vgpr, spill))
    return out


def device_objects():
    objs = []
    for o in sorted(glob.glob(os.path.join(OBJ, "*.o"))):
        sections = subprocess.run([f"{LLVM}/llvm-objdump", "-h", o], capture_output=True, text=True).stdout
        if ".hip_fatbin" in sections:
            objs.append(o)
    return objs


@pytest.mark.skipif(not os.path.isdir(OBJ) or not os.path.exists(f"{LLVM}/llvm-readelf"),
                    reason="library objects or ROCm LLVM tools not present")
def test_no_kernel_spills_vgprs(tmp_path):
    objs = device_objects()
    assert objs, "no device code objects under _build"
    kernels = [k for o in objs for k in kernel_metadata(o, str(tmp_path))]
    assert len(kernels) > 50
    spilling = [(n, v, s) for n, v, s in kernels if s]
    assert not spilling, spilling[:10]
