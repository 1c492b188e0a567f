"""Seeded synthetic workloads.

The paper's own datasets (UniProt-derived reference sets and queries, Table I)
are not available, so every workload here is synthetic, drawn from numpy
`SeedSequence([170101575, k])` streams.  Shapes follow the paper's two uses of
the method: protein database search against a large reference set
(Section III.A) and read-mapping style pairwise alignment (Section I).

Five workloads are defined:

* ``cfg1``  1 protein query (length 64) vs 1,000 targets, lengths uniform in
  [50, 400]; BLOSUM62, gap open 11 / extend 1; local.
* ``cfg2``  protein queries of lengths 144, 464, 1000, 2000, 5000 vs 200,000
  targets with log-normal lengths (median 300, sigma 0.58, clipped to
  [20, 35000]); local, score + end.
* ``cfg3``  100,000 DNA pairs: a read of length U[100, 250] cut from a random
  ACGT window of length U[500, 1000], with 1% substitutions and 0.1% indel
  events (geometric length, mean 2); match +2 / mismatch -3, open 5 / extend 2;
  local with traceback.
* ``cfg4``  50,000 protein pairs, target length log-uniform in [100, 3000],
  query derived at identity U(0.3, 0.9) (90% substitutions, 10% indels of
  geometric length); BLOSUM62, open 10 / extend 1; global and semi-global
  (target ends free) with traceback.
* ``cfg5``  serving: 500,000 log-normal targets resident on the device;
  Poisson request stream (rate 200/s), each request 1..64 queries with lengths
  log-uniform in [30, 5000]; local, top-10 hits with traceback.

Every generator accepts a size argument so tests can draw the same recipe at
reduced scale.  Residues are i.i.d. from the Robinson & Robinson background
(protein) or uniform ACGT (DNA).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .matrices import BACKGROUND_FREQ, blosum62, dna_matrix

ROOT_SEED = 170101575


@dataclasses.dataclass
class SeqSet:
    """A set of sequences: concatenated uint8 codes plus int64 offsets (n+1)."""
    codes: np.ndarray
    offsets: np.ndarray

    def __post_init__(self):
        self.codes = np.ascontiguousarray(self.codes, dtype=np.uint8)
        self.offsets = np.ascontiguousarray(self.offsets, dtype=np.int64)

    def __len__(self) -> int:
        return len(self.offsets) - 1

    def __getitem__(self, k: int) -> np.ndarray:
        return self.codes[self.offsets[k]:self.offsets[k + 1]]

    @property
    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets)

    @classmethod
    def from_list(cls, seqs) -> "SeqSet":
        seqs = [np.asarray(s, dtype=np.uint8) for s in seqs]
        offs = np.zeros(len(seqs) + 1, dtype=np.int64)
        if seqs:
            offs[1:] = np.cumsum([len(s) for s in seqs])
            codes = np.concatenate(seqs) if offs[-1] > 0 else np.zeros(0, np.uint8)
        else:
            codes = np.zeros(0, np.uint8)
        return cls(codes, offs)

    def subset(self, idx) -> "SeqSet":
        return SeqSet.from_list([self[int(k)] for k in idx])


def streams(k: int, n: int):
    """n independent child generators of workload k."""
    ss = np.random.SeedSequence([ROOT_SEED, k])
    return [np.random.default_rng(c) for c in ss.spawn(n)]


def background_residues(rng, count: int) -> np.ndarray:
    """i.i.d. residue codes 0..19 from the background frequency vector."""
    cdf = np.cumsum(BACKGROUND_FREQ)
    cdf[-1] = 1.0
    u = rng.random(count)
    return np.searchsorted(cdf, u, side="right").astype(np.uint8)


def lognormal_lengths(rng, n: int, median: float = 300.0, sigma: float = 0.58,
                      lo: int = 20, hi: int = 35000) -> np.ndarray:
    x = np.exp(rng.normal(math.log(median), sigma, size=n))
    return np.clip(np.rint(x), lo, hi).astype(np.int64)


def loguniform_lengths(rng, n: int, lo: float, hi: float) -> np.ndarray:
    x = np.exp(rng.uniform(math.log(lo), math.log(hi), size=n))
    return np.rint(x).astype(np.int64)


def random_protein_set(rng_len_or_lengths, rng_res) -> SeqSet:
    lengths = np.asarray(rng_len_or_lengths, dtype=np.int64)
    offs = np.zeros(len(lengths) + 1, dtype=np.int64)
    offs[1:] = np.cumsum(lengths)
    return SeqSet(background_residues(rng_res, int(offs[-1])), offs)


def geometric_half(rng, size=None):
    """Geometric length on {1, 2, ...} with success probability 1/2 (mean 2)."""
    return rng.geometric(0.5, size=size)


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------

def cfg1(n_targets: int = 1000, query_len: int = 64) -> dict:
    r_len, r_q, r_t = streams(1, 3)
    q = random_protein_set([query_len], r_q)
    lengths = r_len.integers(50, 401, size=n_targets)
    t = random_protein_set(lengths, r_t)
    return dict(name="cfg1", queries=q, targets=t, matrix=blosum62(),
                gap_open=11, gap_extend=1, mode="local", traceback=False)


CFG2_QUERY_LENGTHS = (144, 464, 1000, 2000, 5000)


def cfg2(n_targets: int = 200_000, query_lengths=CFG2_QUERY_LENGTHS) -> dict:
    r_len, r_q, r_t = streams(2, 3)
    q = random_protein_set(list(query_lengths), r_q)
    lengths = lognormal_lengths(r_len, n_targets)
    t = random_protein_set(lengths, r_t)
    return dict(name="cfg2", queries=q, targets=t, matrix=blosum62(),
                gap_open=11, gap_extend=1, mode="local", traceback=False)


def _mutate_read(rng, window: np.ndarray, start: int, length: int,
                 p_sub: float = 0.01, p_indel: float = 0.001) -> np.ndarray:
    """Cut window[start:start+length] and inject substitutions and indels.

    Each base independently: with p_sub it becomes one of the other 3 bases;
    with p_indel an indel event starts there (insertion or deletion with
    probability 1/2 each, length geometric with mean 2; inserted bases are
    uniform ACGT, a deletion removes this base and the following ones)."""
    read = window[start:start + length].copy()
    sub = rng.random(length) < p_sub
    if sub.any():
        shift = rng.integers(1, 4, size=int(sub.sum())).astype(np.uint8)
        read[sub] = (read[sub] + shift) % 4
    ev = np.nonzero(rng.random(length) < p_indel)[0]
    if len(ev) == 0:
        return read
    out = []
    pos = 0
    for k in ev:
        if k < pos:
            continue  # already removed by an earlier deletion
        out.append(read[pos:k])
        L = int(geometric_half(rng))
        if rng.random() < 0.5:  # insertion before base k
            out.append(rng.integers(0, 4, size=L).astype(np.uint8))
            pos = k
        else:  # deletion of bases k .. k+L-1
            pos = min(length, k + L)
    out.append(read[pos:])
    return np.concatenate(out).astype(np.uint8)


def cfg3(n_pairs: int = 100_000) -> dict:
    r_w, r_r, r_res, r_mut = streams(3, 4)
    wlen = r_w.integers(500, 1001, size=n_pairs)
    rlen = r_r.integers(100, 251, size=n_pairs)
    starts = (r_r.random(n_pairs) * (wlen - rlen + 1)).astype(np.int64)
    woffs = np.zeros(n_pairs + 1, dtype=np.int64)
    woffs[1:] = np.cumsum(wlen)
    wcodes = r_res.integers(0, 4, size=int(woffs[-1])).astype(np.uint8)
    windows = SeqSet(wcodes, woffs)
    reads = [_mutate_read(r_mut, windows[k], int(starts[k]), int(rlen[k]))
             for k in range(n_pairs)]
    return dict(name="cfg3", queries=SeqSet.from_list(reads), targets=windows,
                matrix=dna_matrix(2, -3), gap_open=5, gap_extend=2,
                mode="local", traceback=True, pairwise=True)


def _derive_protein(rng, target: np.ndarray, identity: float,
                    p_sub_share: float = 0.9) -> np.ndarray:
    """Query derived from a target: each position kept with probability
    `identity`; otherwise a mutation event, a substitution (to a different
    background residue) with probability 0.9, else an indel (insertion or
    deletion with probability 1/2 each, geometric length, mean 2)."""
    n = len(target)
    u = rng.random(n)
    keep = u < identity
    v = rng.random(n)
    is_sub = (~keep) & (v < p_sub_share)
    is_indel = (~keep) & (~is_sub)
    out_pos = target.copy()
    ns = int(is_sub.sum())
    if ns:
        repl = background_residues(rng, ns)
        same = repl == out_pos[is_sub]
        while same.any():
            repl[same] = background_residues(rng, int(same.sum()))
            same = repl == out_pos[is_sub]
        out_pos[is_sub] = repl
    ev = np.nonzero(is_indel)[0]
    if len(ev) == 0:
        return out_pos
    pieces = []
    pos = 0
    for k in ev:
        if k < pos:
            continue
        pieces.append(out_pos[pos:k])
        L = int(geometric_half(rng))
        if rng.random() < 0.5:  # insertion, then the original residue k
            pieces.append(background_residues(rng, L))
            pieces.append(target[k:k + 1])
            pos = k + 1
        else:  # deletion of target residues k .. k+L-1
            pos = min(n, k + L)
    pieces.append(out_pos[pos:])
    return np.concatenate(pieces).astype(np.uint8)


def cfg4(n_pairs: int = 50_000) -> dict:
    r_len, r_res, r_id, r_mut = streams(4, 4)
    lengths = loguniform_lengths(r_len, n_pairs, 100, 3000)
    targets = random_protein_set(lengths, r_res)
    ident = r_id.uniform(0.3, 0.9, size=n_pairs)
    queries = [_derive_protein(r_mut, targets[k], float(ident[k])) for k in range(n_pairs)]
    return dict(name="cfg4", queries=SeqSet.from_list(queries), targets=targets,
                matrix=blosum62(), gap_open=10, gap_extend=1,
                modes=("global", "semiglobal"), traceback=True, pairwise=True)


def cfg5_db(n_targets: int = 500_000) -> dict:
    r_len, r_t = streams(5, 2)
    lengths = lognormal_lengths(r_len, n_targets)
    return dict(name="cfg5", targets=random_protein_set(lengths, r_t),
                matrix=blosum62(), gap_open=11, gap_extend=1, mode="local", top_k=10)


def cfg5_requests(n_requests: int, rate: float = 200.0, seed_offset: int = 0):
    """Poisson request stream: list of (arrival_seconds, SeqSet of queries)."""
    ss = np.random.SeedSequence([ROOT_SEED, 5, 1000 + seed_offset])
    r_arr, r_n, r_len, r_res = [np.random.default_rng(c) for c in ss.spawn(4)]
    gaps = r_arr.exponential(1.0 / rate, size=n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    reqs = []
    for k in range(n_requests):
        nq = int(r_n.integers(1, 65))
        lens = loguniform_lengths(r_len, nq, 30, 5000)
        reqs.append((float(arrivals[k]), random_protein_set(lens, r_res)))
    return reqs


def random_pairs(seed: int, n: int, max_len: int, alphabet_size: int,
                 min_len: int = 0) -> tuple[SeqSet, SeqSet]:
    """Uniform random small pairs for tests (codes uniform over the alphabet)."""
    rng = np.random.default_rng([ROOT_SEED, 99, seed])
    ql = rng.integers(min_len, max_len + 1, size=n)
    tl = rng.integers(min_len, max_len + 1, size=n)
    q = SeqSet.from_list([rng.integers(0, alphabet_size, size=int(L)).astype(np.uint8) for L in ql])
    t = SeqSet.from_list([rng.integers(0, alphabet_size, size=int(L)).astype(np.uint8) for L in tl])
    return q, t


def related_pairs(seed: int, n: int, min_len: int, max_len: int,
                  identity=(0.3, 0.95)) -> tuple[SeqSet, SeqSet]:
    """Protein pairs where the query is derived from the target (cfg4 recipe,
    other lengths) so that alignments have long gapped paths."""
    rng = np.random.default_rng([ROOT_SEED, 98, seed])
    lengths = rng.integers(min_len, max_len + 1, size=n)
    targets = random_protein_set(lengths, rng)
    ident = rng.uniform(identity[0], identity[1], size=n)
    queries = [_derive_protein(rng, targets[k], float(ident[k])) for k in range(n)]
    return SeqSet.from_list(queries), targets
