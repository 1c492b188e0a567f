"""Alphabets, substitution matrices and background frequencies.

These are inputs of the alignment method: the paper takes a score matrix as one
of its three input datasets (Section II.B.1, "Map").  Nothing here computes an
alignment.

Protein codes follow the 24-letter order in which BLOSUM62 is distributed
(A R N D C Q E G H I L K M F P S T W Y V B Z X *); the 20 standard residues
are codes 0..19.  DNA codes are A C G T N (0..4).
"""
from __future__ import annotations

import os

import numpy as np

PROTEIN_ALPHABET = "ARNDCQEGHILKMFPSTWYVBZX*"
PROTEIN_STANDARD = PROTEIN_ALPHABET[:20]
DNA_ALPHABET = "ACGTN"

_HERE = os.path.dirname(os.path.abspath(__file__))

# Amino-acid background frequencies of Robinson & Robinson, "Distribution of
# glutamine and asparagine residues and their near neighbors in peptides and
# proteins", PNAS 88:8880-8884 (1991), in the order A R N D C Q E G H I L K M F
# P S T W Y V.  The published values sum to 1.00000; they are renormalised
# anyway so the vector is an exact probability distribution.
_ROBINSON_1991 = np.array([
    0.07805, 0.05129, 0.04487, 0.05364, 0.01925, 0.04264, 0.06295,
    0.07377, 0.02199, 0.05142, 0.09019, 0.05744, 0.02243, 0.03856,
    0.05203, 0.07120, 0.05841, 0.01330, 0.03216, 0.06441,
], dtype=np.float64)
BACKGROUND_FREQ = _ROBINSON_1991 / _ROBINSON_1991.sum()


def blosum62() -> np.ndarray:
    """BLOSUM62 as a (24, 24) int8 array, row = query code, column = target code."""
    path = os.path.join(_HERE, "blosum62.txt")
    rows = []
    header = None
    with open(path, "r", encoding="ascii") as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            if header is None:
                header = parts
                continue
            rows.append([int(x) for x in parts[1:]])
            if parts[0] != header[len(rows) - 1]:
                raise ValueError("BLOSUM62 row order does not match its header")
    if "".join(header) != PROTEIN_ALPHABET:
        raise ValueError("BLOSUM62 header is not in the expected letter order")
    mat = np.array(rows, dtype=np.int8)
    if mat.shape != (24, 24):
        raise ValueError("BLOSUM62 must be 24 x 24")
    return mat


def dna_matrix(match: int = 2, mismatch: int = -3) -> np.ndarray:
    """(5, 5) int8 DNA matrix over A C G T N.

    A base scores `match` against itself; every other pair, N against anything
    (N included), scores `mismatch`.
    """
    mat = np.full((5, 5), mismatch, dtype=np.int8)
    for c in range(4):
        mat[c, c] = match
    return mat


def encode(seq: str, alphabet: str = PROTEIN_ALPHABET, unknown: str | None = None) -> np.ndarray:
    """ASCII letters to uint8 codes.  Letters outside the alphabet map to
    `unknown` (X for protein, N for DNA) when given, else raise."""
    lut = np.full(256, 255, dtype=np.uint8)
    for k, ch in enumerate(alphabet):
        lut[ord(ch)] = k
        lut[ord(ch.lower())] = k
    raw = np.frombuffer(seq.encode("ascii"), dtype=np.uint8)
    codes = lut[raw]
    bad = codes == 255
    if bad.any():
        if unknown is None:
            raise ValueError(f"letters outside the alphabet: {set(seq[i] for i in np.nonzero(bad)[0])}")
        codes[bad] = alphabet.index(unknown)
    return codes


def decode(codes, alphabet: str = PROTEIN_ALPHABET) -> str:
    return "".join(alphabet[int(c)] for c in codes)
