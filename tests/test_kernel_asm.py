"""Checks on the gfx950 assembly of this library's own MMA kernels (CPU,
compiled here): every gather stays an LDS access (no flat loads, which
would also break the explicit vmcnt accounting of the LDS-DMA pipelines)
and no kernel spills to scratch."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2506_22969_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-ffp-contract=fast", "--cuda-device-only", "-S"]


def kernels(asm: str):
    """(name, body) of every pipelined sweep kernel in an assembly listing."""
    out = []
    for m in re.finditer(r"^(_ZN2ss\S*k_(?:mma|lds)\S*):", asm, flags=re.M):
        name = m.group(1)
        end = asm.find(".Lfunc_end", m.end())
        out.append((name, asm[m.end():end]))
    return out


SOURCES = ["mma2d_f32_r1.hip", "mma2d_f32_r2.hip", "mma2d_f32_r3.hip", "mma2d_f16.hip", "mma2d_planes.hip", "mma2d_planes3.hip", "mma3d.hip", "mma2d_f64.hip", "mma1d.hip", "direct2d.hip"]


@pytest.fixture(scope="module")
def listings(tmp_path_factory):
    """Device assembly of every kernel source, compiled in parallel."""
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("asm")
    procs = {src: subprocess.Popen([HIPCC] + FLAGS + [os.path.join(CSRC, src), "-o", str(d / (src + ".s"))],
                                   stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
             for src in SOURCES}
    for src, p in procs.items():
        assert p.wait() == 0, src
    return {src: (d / (src + ".s")).read_text() for src in SOURCES}


@pytest.mark.parametrize("src", SOURCES)
def test_kernels_use_lds_and_do_not_spill(src, listings):
    asm = listings[src]
    ks = kernels(asm)
    assert ks, "no kernels found"
    for name, body in ks:
        assert "flat_load" not in body and "flat_store" not in body, name
    for m in re.finditer(r"^\s*\.set\s+(\S*k_(?:mma|lds)\S*)\.private_seg_size,\s*(\d+)", asm, flags=re.M):
        assert int(m.group(2)) == 0, m.group(1)
    scratch = re.findall(r"; ScratchSize: (\d+)", asm)
    assert scratch and all(int(x) == 0 for x in scratch)
