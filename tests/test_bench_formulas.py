"""The bench's algorithmic bytes and flops per subcarrier-vector against
per-configuration figures worked out by hand (complex64 in and out, one uint8
hard decision per user; Hermitian Gram at half cost, U^3/6 complex MACs for
the factorisation, one U^2 solve per estimate)."""
import pytest

import bench


@pytest.mark.parametrize("algo,B,U,C,T,bytes_vec,mflop", [
    ("admm", 256, 32, 8, 5, 67872, 1.824),    # headline, C = 8
    ("admm", 256, 32, 4, 5, 67872, 1.485),    # headline, C = 4
    ("admm", 128, 16, 8, 5, 17552, 0.281),    # configuration 2, ADMM
    ("cg", 128, 16, 8, 5, 17552, 0.180),      # configuration 2, CG
    ("dl", 256, 32, 16, 5, 67840, 1.398),     # configuration 3
    ("admm", 512, 64, 8, 5, 266816, 12.889),  # configuration 4
])
def test_one_shot_formulas(algo, B, U, C, T, bytes_vec, mflop):
    assert bench.algorithmic_bytes(algo, B, U, C) == bytes_vec
    assert abs(bench.algorithmic_flops(algo, B, U, C, T) / 1e6 - mflop) < 0.0015


def test_resident_forms():
    B, U, C, T = 256, 32, 8, 5
    # the factors add 8 C U^2 bytes; the FP16 channel halves H and adds one float scale per cluster
    assert bench.algorithmic_bytes("admm", B, U, C, "resident") == 67872 + 8 * C * U * (U + 1) // 2
    assert bench.algorithmic_bytes("admm", B, U, C, "resident_h16") == 67872 + 8 * C * U * (U + 1) // 2 - 4 * B * U + 4 * C
    # no Gram and no factorisation: H^H y, then T estimates with one U^2 product each
    assert bench.algorithmic_flops("admm", B, U, C, T, "resident") == 8.0 * (B * U + T * C * U * U)
