"""Measured ceilings on the current GPU (dsa_probe): VALU issue rate of the
instructions the alignment kernels use, an HBM copy of known size (also
the reference kernel for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE), and the
local-mode cell rate of a bare 16-row column in packed int16 against 8-bit
lanes of 32-bit words.

    python paper_1701_01575_amd/probe.py            # all probes
    python paper_1701_01575_amd/probe.py copy BYTES # one copy of BYTES
    python paper_1701_01575_amd/probe.py cells      # the two cell rates only
"""
import os
import sys

if __package__ in (None, ""):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from paper_1701_01575_amd import binding as B  # noqa: E402

# which -> (name, 16-bit results per instruction)
NAMES = {0: ("v_pk_add_i16 (clamp)", 2), 1: ("v_pk_max_i16", 2), 2: ("v_pk_sub_u16 (clamp)", 2),
         6: ("v_pk_maximum3_f16", 2), 3: ("v_add_u32", 1), 4: ("v_max_i32", 1)}


def main(argv):
    import torch
    torch.cuda.init()
    if len(argv) >= 2 and argv[0] == "copy":
        r = B.dsa_probe(5, int(argv[1]))
        print(f"copy of {int(argv[1])} bytes x 6 launches: {r / 1e9:.0f} GB/s (read + write)")
        return
    if len(argv) >= 1 and argv[0] == "cells":
        cells()
        return
    for w, (n, per) in NAMES.items():
        r = B.dsa_probe(w, 20000)
        print(f"{n:22s} {r / 1e12:7.2f} T lane-instructions/s  ({r * per / 1e12:.2f} T 16-bit ops/s)")
    r = B.dsa_probe(5, 4 << 30)
    print(f"HBM copy of 4 GiB: {r / 1e9:.0f} GB/s (read + write)")
    bad = B.dsa_probe(7, 1)
    print(f"v_pk_maximum3_f16 order check (offset local-mode operands): {int(bad)} wrong results")
    cells()


def cells():
    bad = B.dsa_probe(10, 1)
    print(f"byte sign spread check (8-bit probe): {int(bad)} wrong results")
    r16, r8 = B.dsa_probe(8, 65536), B.dsa_probe(9, 65536)
    print(f"local cells, packed int16 (2 targets per lane):  {r16 / 1e12:6.2f} T cells/s")
    print(f"local cells, 8-bit lanes (4 targets per lane):   {r8 / 1e12:6.2f} T cells/s")
    print(f"int16 / 8-bit: {r16 / r8:.2f}")
    for w in (1, 2, 3, 4):
        r = B.dsa_probe(10 + w, 16384)
        print(f"local cells, packed int16, {w} wave(s) per SIMD: {r / 1e12:6.2f} T cells/s")


if __name__ == "__main__":
    main(sys.argv[1:])
