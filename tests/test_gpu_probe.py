"""The binary16 three-way maximum that the local-mode int16 search uses in
place of two integer maxima: over every operand pattern that search can
produce (positive and negative normal binary16, against the offset floor),
it must return the operand of greatest sign-magnitude order."""
import pytest

from paper_1701_01575_amd import binding as B

pytestmark = pytest.mark.gpu


def test_max3_order_exhaustive():
    import torch
    torch.cuda.init()
    assert B.dsa_probe(7, 1) == 0.0


def test_spread_and_cell_rates():
    """The byte sign spread of the 8-bit probe is exact on the device, and
    both cell-rate probes run (their rates are recorded with the profiles)."""
    import torch
    torch.cuda.init()
    assert B.dsa_probe(10, 1) == 0.0
    r16, r8 = B.dsa_probe(8, 4096), B.dsa_probe(9, 4096)
    assert r16 > 0 and r8 > 0
    rw = [B.dsa_probe(10 + w, 1024) for w in (1, 2, 3, 4)]  # 1..4 waves per SIMD
    assert all(r > 0 for r in rw)
