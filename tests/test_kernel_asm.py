"""Invariants of the machine code of the kernels that copy global memory
straight into LDS: the MFMA grid matchers and the two top-k passes (CPU: hipcc
cross-compiles).

Their stage copies are issued from inline assembly that writes m0, a register
the compiler reserves and does not restore after inline assembly; the kernels
are correct only while no other instruction of theirs reads or writes m0."""
import os
import re
import shutil
import subprocess

import pytest

from paper_1501_04140_amd import build

KERNELS = [f"fic::kt_match_mfma8<{f16}, {tab}>" for f16 in ("true", "false") for tab in ("true", "false")]
TOPK = ["fic::k_tk_max", "fic::k_tk_collect"]


def _device_asm(tmp_path) -> str:
    src = tmp_path / "m8.hip"
    src.write_text("#include <hip/hip_runtime.h>\n#include \"fic_kernels.hip\"\n#include \"fic_mlp_kernels.hip\"\n" +
                   "".join(f"template __global__ void {k}(fic::Lvl, const fic::Lvl*);\n" for k in KERNELS) +
                   "")
    out = tmp_path / "m8.s"
    cmd = [build.hipcc(), f"--offload-arch={build.ARCH}", "-O3", "-std=c++17", "--cuda-device-only", "-S",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-mllvm", "-amdgpu-mfma-vgpr-form",
           "-I", os.path.join(build.ROOT, "include"), "-I", build.CSRC, "-o", str(out), str(src)]
    subprocess.run(cmd, check=True, capture_output=True)
    return out.read_text()


def _bodies(asm: str):
    for m in re.finditer(r"^(_ZN3fic(?:14kt_match_mfma8\w*|8k_tk_max\w*|12k_tk_collect\w*)):", asm, re.M):
        end = asm.index("s_endpgm", m.end())
        yield m.group(1), asm[m.end():end]


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not available")
def test_m0_only_in_the_stage_copies(tmp_path):
    asm = _device_asm(tmp_path)
    bodies = list(_bodies(asm))
    assert len(bodies) == len(KERNELS) + len(TOPK)
    for name, body in bodies:
        # the inline-assembly blocks with instructions (the others are empty
        # register pins): m0 set, then the copy that reads it
        blocks = [b for b in re.findall(r";;#ASMSTART\n(.*?);;#ASMEND", body, re.S) if b.strip()]
        assert blocks, name
        for b in blocks:
            lines = [ln.strip() for ln in b.strip().splitlines()]
            assert re.fullmatch(r"s_mov_b32 m0, s\d+", lines[0]), (name, lines)
            assert lines[-1].startswith("global_load_lds_dwordx4"), (name, lines)
        outside = re.sub(r";;#ASMSTART\n.*?;;#ASMEND", "", body, flags=re.S)
        uses = [ln for ln in outside.splitlines() if re.search(r"\bm0\b", ln) and not ln.strip().startswith(";")]
        assert not uses, (name, uses[:5])
