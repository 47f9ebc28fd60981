"""The step kernel's register and LDS budgets, read from the code object of the built library
(CPU only: the AMDGPU metadata that the compiler records for each kernel).

* No instantiation of the step kernel spills vector registers to memory (a spill reload
  waits on the vector memory counter, which would drain the gathers in flight).
* The shapes the benchmark runs keep their occupancy: with the populations in registers,
  FP32 fits three waves per SIMD (at most 168 VGPRs) with three workgroups of 256 lanes per
  CU in 160 KB of LDS, and FP64 fits two (at most 256 VGPRs) with two workgroups per CU.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1512_01977_amd", "liblbm_axi.so")
LLVM = "/opt/rocm/llvm/bin"
LDS_PER_CU = 160 * 1024


def tool(name):
    path = os.path.join(LLVM, name)
    return path if os.path.exists(path) else shutil.which(name)


@pytest.fixture(scope="module")
def kernels(tmp_path_factory):
    tools = [tool(t) for t in ("llvm-objcopy", "clang-offload-bundler", "llvm-readelf")]
    if not os.path.exists(LIB) or not all(tools):
        pytest.skip("built library or LLVM tools not available")
    objcopy, bundler, readelf = tools
    d = tmp_path_factory.mktemp("codeobj")
    fat, co = str(d / "fat.bin"), str(d / "co.o")
    subprocess.run([objcopy, "--dump-section", f".hip_fatbin={fat}", LIB], check=True, capture_output=True)
    subprocess.run([bundler, "--unbundle", "--type=o", "--targets=hipv4-amdgcn-amd-amdhsa--gfx950",
                    f"--input={fat}", f"--output={co}"], check=True, capture_output=True)
    notes = subprocess.run([readelf, "--notes", co], check=True, capture_output=True, text=True).stdout
    out = {}
    for block in re.split(r"\n\s+- (?=\.)", notes):
        m = re.search(r"\.name:\s+(_ZN3lbm7k_sweepI\S+)", block)
        if not m:
            continue
        fl = re.search(r"k_sweepI([fd])Li(\d+)E((?:Lb[01]E)+)", m.group(1))
        moments, persist, regf, guo, mid = (int(b) for b in re.findall(r"Lb([01])E", fl.group(3)))

        def num(key):
            v = re.search(r"\." + key + r":\s+(\d+)", block)
            return int(v.group(1)) if v else 0

        out[m.group(1)] = dict(fp=fl.group(1), width=int(fl.group(2)), moments=moments, persist=persist,
                               regf=regf, guo=guo, mid=mid, vgpr=num("vgpr_count"), agpr=num("agpr_count"),
                               vspill=num("vgpr_spill_count"), scratch=num("private_segment_fixed_size"),
                               lds=num("group_segment_fixed_size"))
    assert len(out) >= 60, "step kernel instantiations not found in the code object"
    return out


def test_no_vector_spills(kernels):
    bad = [n for n, k in kernels.items() if k["vspill"] or k["scratch"]]
    assert not bad, bad


@pytest.mark.parametrize("fp,waves,wgs", [("f", 3, 3), ("d", 2, 2)])
def test_register_carry_shapes_keep_their_occupancy(kernels, fp, waves, wgs):
    shapes = [k for k in kernels.values()
              if k["fp"] == fp and k["regf"] and not (k["persist"] or k["mid"] or k["moments"])]
    assert shapes
    for k in shapes:
        assert k["vgpr"] + k["agpr"] <= 512 // waves // 8 * 8, k
        assert not k["vspill"] and not k["scratch"], k
        if k["width"] == 256:
            assert wgs * k["lds"] <= LDS_PER_CU, k
