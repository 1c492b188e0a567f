"""Scoring inputs and the seeded workload generators."""
import math

import numpy as np

from workloads import BACKGROUND_FREQ, PROTEIN_ALPHABET, blosum62, decode, dna_matrix, encode
from workloads import gen


def test_blosum62_shape_symmetry_range():
    S = blosum62()
    assert S.shape == (24, 24) and S.dtype == np.int8
    assert (S == S.T).all()
    assert S.min() == -4 and S.max() == 11
    assert int(S[PROTEIN_ALPHABET.index("W"), PROTEIN_ALPHABET.index("W")]) == 11
    assert all(S[k, k] > 0 for k in range(20))
    # sum of the 20 standard diagonal entries of the published table
    assert int(np.trace(S[:20, :20])) == 116


def test_background_frequencies():
    assert BACKGROUND_FREQ.shape == (20,)
    assert abs(BACKGROUND_FREQ.sum() - 1.0) < 1e-12
    assert (BACKGROUND_FREQ > 0).all()
    # leucine is the most frequent residue and tryptophan the rarest
    assert PROTEIN_ALPHABET[int(np.argmax(BACKGROUND_FREQ))] == "L"
    assert PROTEIN_ALPHABET[int(np.argmin(BACKGROUND_FREQ))] == "W"


def test_dna_matrix_n_always_mismatches():
    D = dna_matrix(2, -3)
    assert D.shape == (5, 5)
    assert [int(D[k, k]) for k in range(5)] == [2, 2, 2, 2, -3]
    assert (D[4] == -3).all() and (D[:, 4] == -3).all()


def test_encode_roundtrip():
    s = "MKVLAAGIW*BZX"
    assert decode(encode(s)) == s
    assert decode(encode("mkv")) == "MKV"
    assert decode(encode("MKJ", unknown="X")) == "MKX"


def test_cfg1_shape_and_determinism():
    a = gen.cfg1()
    b = gen.cfg1()
    assert (a["targets"].codes == b["targets"].codes).all()
    L = a["targets"].lengths
    assert len(L) == 1000 and L.min() >= 50 and L.max() <= 400
    assert len(a["queries"]) == 1 and a["queries"].lengths[0] == 64
    assert a["targets"].codes.max() < 20


def test_cfg2_lengths_lognormal():
    c = gen.cfg2(n_targets=20000)
    L = c["targets"].lengths
    assert L.min() >= 20 and L.max() <= 35000
    assert abs(np.median(L) - 300) < 10
    # mean of a log-normal with sigma 0.58 is median * exp(sigma^2 / 2) ~ 355
    assert abs(L.mean() - 300 * math.exp(0.58 ** 2 / 2)) < 8
    assert list(c["queries"].lengths) == [144, 464, 1000, 2000, 5000]
    freq = np.bincount(c["targets"].codes, minlength=20) / len(c["targets"].codes)
    assert np.abs(freq - BACKGROUND_FREQ).max() < 0.002


def test_cfg3_reads_and_windows():
    c = gen.cfg3(n_pairs=300)
    W = c["targets"].lengths
    R = c["queries"].lengths
    assert W.min() >= 500 and W.max() <= 1000
    assert R.min() >= 90 and R.max() <= 270
    assert c["targets"].codes.max() < 4 and c["queries"].codes.max() < 4


def test_cfg4_lengths_and_identity():
    c = gen.cfg4(n_pairs=200)
    L = c["targets"].lengths
    assert L.min() >= 100 and L.max() <= 3000
    ql = c["queries"].lengths
    assert np.corrcoef(L, ql)[0, 1] > 0.95


def test_cfg5_requests():
    reqs = gen.cfg5_requests(50)
    arr = np.array([t for t, _ in reqs])
    assert (np.diff(arr) >= 0).all()
    nq = [len(q) for _, q in reqs]
    assert min(nq) >= 1 and max(nq) <= 64
    lens = np.concatenate([q.lengths for _, q in reqs])
    assert lens.min() >= 30 and lens.max() <= 5000
