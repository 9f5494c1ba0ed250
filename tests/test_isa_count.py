"""Instruction count of the steady-state loops in the gfx950 assembly.

Compares the kernels' per-block work with the paper's count of SIMD
instructions per 512-bit register (Sections "Encoding" and "Decoding") and
guards the loop structure the design relies on: two rounds of U wave-wide
vector loads (and stores) per iteration, and exactly one LDS lookup per
character.
"""
import shutil

import pytest

from paper_1910_05109_amd import isa_count
from paper_1910_05109_amd.build import hipcc

pytestmark = pytest.mark.skipif(shutil.which(hipcc()) is None, reason="hipcc not found")


@pytest.fixture(scope="module")
def rows():
    return {r["kernel"]: r for r in isa_count.report()}


def test_loop_memory_structure(rows):
    for name, (_, u, _) in isa_count.KERNELS.items():
        r = rows[name]
        assert r["vmem load"] == 2 * u, r
        assert r["vmem store"] == (0 if "validate" in name else 2 * u), r
        # one LDS byte lookup per character: 16 per lane chunk
        assert r["lds"] == 2 * u * 16, r


def test_compute_per_block_within_bound(rows):
    # wave instructions (VALU + LDS + SALU) per 64 input bytes; the paper's
    # AVX-512 loops spend 4 (3 per 48 B) to encode and 5 to decode.  The
    # bounds leave headroom for compiler drift but catch a loop that stopped
    # being straight-line (guarded loads, spilled state).
    assert rows["k_encode<4, nt>"]["compute_instr_per_64B"] < 6.0
    assert rows["k_decode<8, nt>"]["compute_instr_per_64B"] < 5.0
    assert rows["k_validate<8, nt>"]["compute_instr_per_64B"] < 3.5


def test_no_kernel_uses_scratch_memory():
    # A kernel's scratch is per-lane memory the compiler falls back to (an
    # indexed local array, state it cannot keep in registers); each access is
    # a memory round trip and its writes are HBM traffic.  One slipped into
    # the whitespace decode's prediction once and tripled its writes.
    sizes = isa_count.scratch_sizes()
    assert len(sizes) > 50, len(sizes)             # the descriptors were found
    assert any("k_ws_predict" in k for k in sizes) and any("k_encode" in k for k in sizes)
    used = {k: v for k, v in sizes.items() if v}
    assert not used, used
