"""The built library's gfx950 code carries no packed FP32 arithmetic.

The build passes `-Xclang -target-feature -Xclang -packed-fp32-ops` to hipcc.
The host pass prints that it does not know the feature (it is an AMDGPU
feature); the device pass honours it.  This test reads the library's own
offload bundles (code built here from this repository's sources), disassembles
every gfx950 code object and checks that none of the packed FP32 add, multiply
or fused multiply-add instructions appears.  No GPU needed."""

import os
import re
import shutil
import subprocess
import tempfile

import pytest

from paper_2601_02540_amd import binding

LLVM = "/opt/rocm/llvm/bin"
MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"
PACKED_F32 = re.compile(rb"\bv_pk_(add|mul|fma)_f32\b")


def _tools():
    tools = {t: os.path.join(LLVM, t) for t in ("llvm-objcopy", "clang-offload-bundler", "llvm-objdump")}
    if not all(os.path.exists(p) for p in tools.values()):
        pytest.skip("ROCm LLVM tools not found")
    return tools


def gfx950_code_objects(lib_path, workdir):
    """Paths of the gfx950 code objects of every offload bundle in lib_path."""
    t = _tools()
    fatbin = os.path.join(workdir, "fatbin")
    subprocess.check_call([t["llvm-objcopy"], f"--dump-section=.hip_fatbin={fatbin}", lib_path,
                           os.path.join(workdir, "lib.copy")])
    data = open(fatbin, "rb").read()
    starts = [m.start() for m in re.finditer(re.escape(MAGIC), data)]
    assert starts, "no offload bundle in the library"
    out = []
    for k, a in enumerate(starts):
        b = starts[k + 1] if k + 1 < len(starts) else len(data)
        part = os.path.join(workdir, f"bundle{k}")
        with open(part, "wb") as f:
            f.write(data[a:b])
        co = os.path.join(workdir, f"gfx950_{k}.co")
        subprocess.check_call([t["clang-offload-bundler"], "--unbundle", "--type=o", f"--input={part}",
                               "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", f"--output={co}"])
        out.append(co)
    return out


def test_no_packed_fp32_instructions():
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("library not built")
    t = _tools()
    work = tempfile.mkdtemp(prefix="sgn_isa_")
    try:
        cos = gfx950_code_objects(binding.LIB_PATH, work)
        # one code object per translation unit of the library
        assert len(cos) >= 5
        for co in cos:
            p = subprocess.Popen([t["llvm-objdump"], "-d", co], stdout=subprocess.PIPE)
            hits, kernels = [], 0
            for line in p.stdout:
                if line.endswith(b">:\n"):
                    kernels += 1
                if PACKED_F32.search(line):
                    hits.append(line.strip())
            assert p.wait() == 0
            assert kernels > 0, co
            assert not hits, (co, hits[:5])
    finally:
        shutil.rmtree(work, ignore_errors=True)
