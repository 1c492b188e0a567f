"""Seeded synthetic workloads and scoring inputs.

This package feeds both the HIP path and the CPU oracle.  It holds no
alignment arithmetic: only alphabets, matrices, background frequencies and
random sequence generators.
"""
from .matrices import (  # noqa: F401
    BACKGROUND_FREQ, DNA_ALPHABET, PROTEIN_ALPHABET, PROTEIN_STANDARD,
    blosum62, decode, dna_matrix, encode,
)
from .gen import SeqSet  # noqa: F401
