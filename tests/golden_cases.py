"""Reader for tests/golden/handworked.txt (hand-derived alignments)."""
import os

import numpy as np

from workloads import blosum62, dna_matrix, encode, PROTEIN_ALPHABET

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "handworked.txt")


def matrix(name):
    if name == "dna23":
        return dna_matrix(2, -3), "ACGTN"
    if name == "dna33":
        return dna_matrix(3, -3), "ACGTN"
    if name == "blosum62":
        return blosum62(), PROTEIN_ALPHABET
    raise KeyError(name)


def load():
    cases = []
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            f = [x.strip() for x in line.split("|")]
            S, alpha = matrix(f[1])
            cases.append(dict(
                name=f[0], S=S, o=int(f[2]), e=int(f[3]), mode=f[4], ends=int(f[5]),
                query=encode(f[6], alpha) if f[6] else np.zeros(0, np.uint8),
                target=encode(f[7], alpha) if f[7] else np.zeros(0, np.uint8),
                score=int(f[8]), q_begin=int(f[9]), q_end=int(f[10]),
                t_begin=int(f[11]), t_end=int(f[12]), cigar=f[13]))
    return cases
