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
