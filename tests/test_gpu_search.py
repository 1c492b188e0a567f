"""GPU parity of database search (every query vs every target) against the
CPU oracle: score, query end and target end must be bit-identical.

Inputs span several strips and a ragged last strip (query lengths around
multiples of 16 and 32), empty targets and queries, several groups with a
ragged last group, every mode, the plain and persistent forms and the int32
kernel; a scaled matrix forces int16 saturation and the int32 rerun.
"""
import numpy as np
import pytest

import oracle
from gpu_util import compare_search, gpu_search, log
from workloads import gen
from workloads.gen import SeqSet

pytestmark = pytest.mark.gpu

QLENS = [0, 1, 2, 15, 16, 17, 31, 32, 33, 63, 64, 65, 100, 257]


def _targets(seed, n, max_len, alphabet=20, extra=()):
    rng = np.random.default_rng([170101575, 50, seed])
    lens = list(rng.integers(0, max_len + 1, size=n)) + list(extra)
    lens[0] = 0
    return SeqSet.from_list([gen.background_residues(rng, int(L)) % alphabet for L in lens])


def _queries(seed, lens):
    rng = np.random.default_rng([170101575, 51, seed])
    return SeqSet.from_list([gen.background_residues(rng, int(L)) for L in lens])


CASES = [
    ("local", None), ("global", None), ("semiglobal", None),
    ("semiglobal", 1 | 4), ("semiglobal", 4), ("semiglobal", 8), ("semiglobal", 1 | 8),
]


@pytest.mark.parametrize("mode,ends", CASES)
@pytest.mark.parametrize("plain", [False, True], ids=["persistent", "plain"])
@pytest.mark.parametrize("strip", ["16", "32"])
def test_search_modes(mode, ends, plain, strip, blosum, monkeypatch):
    monkeypatch.setenv("DSA_INTRA_BUDGET", "1000000000")  # inter-sequence kernel only
    monkeypatch.setenv("DSA_STRIP", strip)
    T = _targets(1, 300, 180, extra=[1, 2, 3, 4, 5, 399, 400])
    Q = _queries(2, QLENS)
    log(f"search mode={mode} ends={ends} plain={plain} strip={strip} nq={len(Q)} nt={len(T)}")
    got, _ = gpu_search(Q, T, blosum, 11, 1, mode, ends, plain=plain)
    exp = oracle.search(Q, T, blosum, 11, 1, mode=mode, ends=ends)
    compare_search(got, exp, len(Q), len(T), label=f"{mode}/{ends}/{plain}")


QE_ENDS = [2, 2 | 8, 1 | 2, 2 | 4, 15]


@pytest.mark.parametrize("ends", QE_ENDS)
@pytest.mark.parametrize("plain", [False, True], ids=["persistent", "plain"])
def test_search_free_query_end(ends, plain, blosum):
    """Semi-global with a free query end (the last column is a candidate
    too, row 0 included): the search runs the exact int32 kernel."""
    T = _targets(12, 300, 400, extra=[1, 2, 1200])
    Q = _queries(13, [0, 1, 15, 16, 17, 33, 100, 700])
    log(f"search QE ends={ends} plain={plain}")
    got, _ = gpu_search(Q, T, blosum, 11, 1, "semiglobal", ends, plain=plain)
    exp = oracle.search(Q, T, blosum, 11, 1, mode="semiglobal", ends=ends)
    compare_search(got, exp, len(Q), len(T), label=f"QE {ends}/{plain}")
    # some results end before the last query residue
    assert (exp["q_end"] < np.repeat(Q.lengths - 1, len(T))).any()


@pytest.mark.parametrize("mode,ends", CASES[:3])
def test_search_force_int32(mode, ends, blosum):
    T = _targets(3, 200, 150)
    Q = _queries(4, [1, 16, 17, 40, 130])
    log(f"force_int32 mode={mode}")
    got, _ = gpu_search(Q, T, blosum, 10, 1, mode, ends, force_int32=True)
    exp = oracle.search(Q, T, blosum, 10, 1, mode=mode, ends=ends)
    compare_search(got, exp, len(Q), len(T), label=f"int32 {mode}")
    assert (got["status"] & 1).all()


@pytest.mark.parametrize("mode", ["local", "global", "semiglobal"])
def test_search_int16_overflow_rerun(mode, blosum):
    # x5 matrix: self-similar pairs exceed 32767 and must come from the int32 pass
    S = (blosum.astype(np.int32) * 5).clip(-128, 127).astype(np.int8)
    rng = np.random.default_rng([170101575, 52])
    base = gen.background_residues(rng, 1400)
    seqs = [base[:k] for k in (300, 700, 1400)] + [gen.background_residues(rng, 500) for _ in range(40)]
    T = SeqSet.from_list(seqs)
    Q = SeqSet.from_list([base, base[:200]])
    log(f"overflow mode={mode}")
    got, _ = gpu_search(Q, T, S, 40, 4, mode)
    exp = oracle.search(Q, T, S, 40, 4, mode=mode)
    compare_search(got, exp, len(Q), len(T), label=f"ovf {mode}")
    if mode == "local":
        assert exp["score"].max() > 32767
        big = exp["score"] > 32767
        assert (got["status"][big] & 1).all()


def test_search_dna_alphabet(dna):
    rng = np.random.default_rng([170101575, 53])
    T = SeqSet.from_list([rng.integers(0, 5, size=int(L)).astype(np.uint8)
                          for L in rng.integers(0, 300, size=150)])
    Q = SeqSet.from_list([rng.integers(0, 4, size=L).astype(np.uint8) for L in (20, 150)])
    got, _ = gpu_search(Q, T, dna, 5, 2, "local")
    exp = oracle.search(Q, T, dna, 5, 2, mode="local")
    compare_search(got, exp, len(Q), len(T), label="dna")


def test_cfg1_full_parity():
    c = gen.cfg1()
    log("cfg1 full")
    for plain in (True, False):
        got, _ = gpu_search(c["queries"], c["targets"], c["matrix"], 11, 1, "local", plain=plain)
        exp = oracle.search(c["queries"], c["targets"], c["matrix"], 11, 1)
        compare_search(got, exp, 1, 1000, label=f"cfg1 plain={plain}")


def test_cfg2_reduced_full_parity():
    c = gen.cfg2(n_targets=3000, query_lengths=(144, 464, 1000))
    log("cfg2 reduced: 3 queries x 3000 targets")
    got, _ = gpu_search(c["queries"], c["targets"], c["matrix"], 11, 1, "local")
    exp = oracle.search(c["queries"], c["targets"], c["matrix"], 11, 1)
    compare_search(got, exp, 3, 3000, label="cfg2 reduced")


INTRA_QLENS = [1, 15, 16, 17, 100, 700, 1023, 1024, 1025, 2100]
ROUTES = [None, "wavefront", "pipelined"]


def _route(monkeypatch, route):
    """Send every group at least 128 columns wide (the long groups) to the
    wavefront units, or to the strip-pipelined units (local mode, 16-row
    strips, persistent form; elsewhere the wavefront units take them)."""
    if route is not None:
        monkeypatch.setenv("DSA_INTRA_BUDGET", "1")
        monkeypatch.setenv("DSA_KS_BUDGET", "0" if route == "wavefront" else str(1 << 40))


@pytest.mark.parametrize("mode,ends", CASES)
@pytest.mark.parametrize("route", ROUTES, ids=["default-routing", "wavefront", "pipelined"])
def test_search_wavefront_long_targets(mode, ends, route, blosum, monkeypatch):
    """Long targets of long queries go through the wavefront kernel (lanes =
    16-row strips, up to three 1024-row passes) or the strip-pipelined units
    (a block's waves share a query's strips); the routing budget 1 sends
    every group wider than 128 columns there."""
    _route(monkeypatch, route)
    T = _targets(5, 260, 1500, extra=[1, 2, 1501, 1777, 2001])
    Q = _queries(6, INTRA_QLENS)
    log(f"wavefront mode={mode} ends={ends} route={route}")
    for plain in (False, True):
        got, _ = gpu_search(Q, T, blosum, 11, 1, mode, ends, plain=plain)
        exp = oracle.search(Q, T, blosum, 11, 1, mode=mode, ends=ends)
        compare_search(got, exp, len(Q), len(T), label=f"wavefront {mode}/{ends}/{plain}")


@pytest.mark.parametrize("strip,waves", [("32", "8"), ("16", "2"), ("32", "1")])
def test_search_wavefront_launch_shapes(strip, waves, blosum, monkeypatch):
    """Wavefront units inside the persistent kernel at other strip heights and
    block sizes (a unit takes as many long pairs as the block has waves)."""
    monkeypatch.setenv("DSA_STRIP", strip)
    monkeypatch.setenv("DSA_WAVES", waves)
    monkeypatch.setenv("DSA_INTRA_BUDGET", "20000")
    T = _targets(9, 260, 1500, extra=[1, 2, 1501, 1777, 2001])
    Q = _queries(10, INTRA_QLENS)
    for mode, ends in (("local", None), ("semiglobal", None)):
        log(f"wavefront shapes strip={strip} waves={waves} mode={mode}")
        got, _ = gpu_search(Q, T, blosum, 11, 1, mode, ends)
        exp = oracle.search(Q, T, blosum, 11, 1, mode=mode, ends=ends)
        compare_search(got, exp, len(Q), len(T), label=f"shapes {strip}/{waves}/{mode}")


@pytest.mark.parametrize("waves", ["8", "4", "3", "2"])
def test_search_strip_pipelined_block_sizes(waves, blosum, monkeypatch):
    """Strip-pipelined units with 8, 4, 3 and 2 waves per block: queries of
    fewer strips than waves (idle waves), of a ragged last round, and of many
    rounds (the last wave hands its strip to the first wave's next one
    through the boundary row), against groups from 128 columns up."""
    monkeypatch.setenv("DSA_STRIP", "16")
    monkeypatch.setenv("DSA_WAVES", waves)
    _route(monkeypatch, "pipelined")
    T = _targets(13, 300, 1500, extra=[1, 2, 128, 1501, 1777, 2001])
    Q = _queries(14, INTRA_QLENS + [33, 48, 49, 129, 4000])
    log(f"strip-pipelined waves={waves}")
    got, _ = gpu_search(Q, T, blosum, 11, 1, "local")
    exp = oracle.search(Q, T, blosum, 11, 1, mode="local")
    compare_search(got, exp, len(Q), len(T), label=f"pipelined {waves}")


@pytest.mark.parametrize("mode,ends", CASES[:3])
def test_search_small_databases_full_alphabet(mode, ends, blosum):
    """A one-target database, a database of length-1 targets only, and
    residues drawn from all 24 BLOSUM62 letters (B, Z, X and * included)."""
    rng = np.random.default_rng([170101575, 57])
    Q = SeqSet.from_list([rng.integers(0, 24, size=L).astype(np.uint8) for L in (1, 7, 40, 300)])
    dbs = [SeqSet.from_list([rng.integers(0, 24, size=120).astype(np.uint8)]),
           SeqSet.from_list([rng.integers(0, 24, size=1).astype(np.uint8) for _ in range(200)]),
           SeqSet.from_list([rng.integers(0, 24, size=int(L)).astype(np.uint8)
                             for L in rng.integers(0, 400, size=300)])]
    for k, T in enumerate(dbs):
        log(f"small db {k} mode={mode}")
        got, _ = gpu_search(Q, T, blosum, 11, 1, mode, ends)
        exp = oracle.search(Q, T, blosum, 11, 1, mode=mode, ends=ends)
        compare_search(got, exp, len(Q), len(T), label=f"small db {k} {mode}")


@pytest.mark.parametrize("mode,ends", CASES[:3])
def test_search_longest_targets(mode, ends, blosum):
    """Targets at 35,000 residues (where the length law is clipped) and at the
    65,532-residue maximum, next to ordinary ones; a short and a two-pass
    query.  Global scores against the longest target leave the int16 range,
    so that query also runs through the int32 path."""
    rng = np.random.default_rng([170101575, 56])
    lens = [35000, 65532, 20, 300, 1, 5000]
    T = SeqSet.from_list([gen.background_residues(rng, L) for L in lens])
    Q = _queries(11, [50, 1100])
    log(f"longest targets mode={mode}")
    got, _ = gpu_search(Q, T, blosum, 11, 1, mode, ends)
    exp = oracle.search(Q, T, blosum, 11, 1, mode=mode, ends=ends)
    compare_search(got, exp, len(Q), len(T), label=f"longest {mode}")


@pytest.mark.parametrize("route", ROUTES[1:])
def test_search_wavefront_overflow_rerun(route, blosum, monkeypatch):
    _route(monkeypatch, route)
    S = (blosum.astype(np.int32) * 5).clip(-128, 127).astype(np.int8)
    rng = np.random.default_rng([170101575, 55])
    base = gen.background_residues(rng, 1600)
    seqs = [base[:k] for k in (600, 1600)] + [gen.background_residues(rng, 900) for _ in range(130)]
    T = SeqSet.from_list(seqs)
    Q = SeqSet.from_list([base, base[:300]])
    got, _ = gpu_search(Q, T, S, 40, 4, "local")
    exp = oracle.search(Q, T, S, 40, 4, mode="local")
    compare_search(got, exp, len(Q), len(T), label="wavefront ovf")
    assert exp["score"].max() > 32767


@pytest.mark.parametrize("mode,ends", CASES[:3])
def test_search_rounds_of_one_query(mode, ends, blosum, monkeypatch):
    """A tiny boundary-memory budget makes the persistent form run one query
    per round (one query slot)."""
    monkeypatch.setenv("DSA_BND_BUDGET", "1")
    T = _targets(7, 300, 1200, extra=[1, 1300])
    Q = _queries(8, [5, 40, 700, 1500])
    got, _ = gpu_search(Q, T, blosum, 11, 1, mode, ends)
    exp = oracle.search(Q, T, blosum, 11, 1, mode=mode, ends=ends)
    compare_search(got, exp, len(Q), len(T), label=f"rounds {mode}")


def _slot_bytes(T):
    """Boundary bytes of one query slot for database T: per group of 128
    length-sorted targets, (H, F) int32-sized per column and lane; per pair
    of a group at least 128 columns wide, one word per column."""
    lens = np.sort(np.asarray(T.lengths, dtype=np.int64), kind="stable")
    total = 0
    long_words = 0
    for g0 in range(0, len(lens), 128):
        grp = lens[g0:g0 + 128]
        ncols = (int(grp.max()) + 3) // 4 * 4
        total += 2 * ncols * 64 * 8
        if ncols >= 128:
            grp = np.concatenate([grp, np.zeros(128 - len(grp), dtype=np.int64)])
            long_words += int(np.maximum(grp[0::2], grp[1::2]).sum())
    return total + max(long_words, 1) * 8


@pytest.mark.parametrize("per_round", [2, 3])
def test_search_rounds_of_several_queries(per_round, blosum, monkeypatch):
    """A boundary budget of a few query slots splits the queries into rounds
    of 2 or 3; they are dealt longest first in snake order (an empty query
    among them)."""
    T = _targets(15, 300, 1200, extra=[1, 1300])
    Q = _queries(16, [5, 40, 700, 1500, 0, 300, 2000, 64])
    monkeypatch.setenv("DSA_BND_BUDGET", str(per_round * _slot_bytes(T) + 7))
    log(f"rounds of {per_round}")
    got, _ = gpu_search(Q, T, blosum, 11, 1, "local")
    exp = oracle.search(Q, T, blosum, 11, 1, mode="local")
    compare_search(got, exp, len(Q), len(T), label=f"rounds of {per_round}")


LOCAL16_MAX = 28544  # highest local score the offset int16 pass computes exactly


@pytest.mark.parametrize("route", ROUTES, ids=["inter", "wavefront", "pipelined"])
def test_search_local_exact_range_edge(route, blosum, monkeypatch):
    """Scores on both sides of the offset int16 range's top: those at or
    below it come from the int16 pass, those above (still below 32767, where
    the packed values would not saturate) must come from the int32 rerun.
    Self-similar prefixes under a x5 matrix place scores around the edge."""
    _route(monkeypatch, route)
    S = (blosum.astype(np.int32) * 5).clip(-128, 127).astype(np.int8)
    rng = np.random.default_rng([170101575, 57])
    base = gen.background_residues(rng, 1400)
    diag = np.cumsum(S[base, base].astype(np.int64))
    picks = [int(np.searchsorted(diag, v)) + 1 for v in
             (28000, 28400, 28500, 28520, 28540, 28548, 28560, 28700, 29600, 31500, 32600)]
    seqs = [base[:k] for k in picks] + [gen.background_residues(rng, 400) for _ in range(30)]
    T = SeqSet.from_list(seqs)
    Q = SeqSet.from_list([base, base[:1000]])
    log(f"local exact-range edge route={route}")
    got, _ = gpu_search(Q, T, S, 40, 4, "local")
    exp = oracle.search(Q, T, S, 40, 4, mode="local")
    compare_search(got, exp, len(Q), len(T), label="local edge")
    sc = np.asarray(exp["score"])
    above = (sc > LOCAL16_MAX) & (sc < 32767)
    near = (sc <= LOCAL16_MAX) & (sc > LOCAL16_MAX - 600)
    assert above.any() and near.any(), sorted(sc[sc > 20000])
    assert (got["status"][above] & 1).all()


@pytest.mark.parametrize("route", ROUTES, ids=["inter", "wavefront", "pipelined"])
@pytest.mark.parametrize("o,e,int32", [(1500, 1100, True), (1000, 300, True), (1024, 256, False),
                                       (900, 0, False), (60, 60, False), (7, 3, False), (11, 1, False),
                                       (6, 4, False), (9, 5, False)])
def test_search_local_gap_penalties(o, e, int32, route, blosum, monkeypatch):
    """Gap penalties at and beyond the offset int16 range (gap_open <= 1024,
    gap_extend <= 256): beyond it a local search runs the exact int32 kernel;
    at its edge, with no extension cost and with open = extend, the int16
    pass must still be exact.  Its column frame is taken back every
    4 * max(1, 256 // e) columns in the inter-sequence kernel, and in
    wavefront units (which use the frame up to gap_extend 4) every R
    columns, R the largest power of two with R * e <= 1024; targets reach
    1,500 residues so that this happens several times."""
    _route(monkeypatch, route)
    rng = np.random.default_rng([170101575, 58])
    lens = list(rng.integers(0, 400, size=90)) + [1100, 1500]
    T = SeqSet.from_list([gen.background_residues(rng, int(L)) for L in lens])
    Q = _queries(12, [40, 300])
    got, _ = gpu_search(Q, T, blosum, o, e, "local")
    exp = oracle.search(Q, T, blosum, o, e, mode="local")
    compare_search(got, exp, len(Q), len(T), label=f"gaps {o}/{e}")
    assert bool((got["status"] & 1).all()) == int32


@pytest.mark.parametrize("seed", range(7))
@pytest.mark.parametrize("route", ROUTES, ids=["inter", "wavefront", "pipelined"])
def test_search_local_random_scoring(seed, route, monkeypatch):
    """Random alphabets (4 to 24 letters), random matrices that reach the
    int8 extremes (-128, +127) and random gap penalties within the offset
    int16 range, so that profile entries s + e span their whole range; both
    unit kinds and routes, bit-exact against the oracle."""
    _route(monkeypatch, route)
    rng = np.random.default_rng([170101575, 59, seed])
    A = int(rng.integers(4, 25))
    S = rng.integers(-12, 9, size=(A, A)).astype(np.int8)
    S[rng.integers(0, A), rng.integers(0, A)] = 127
    S[rng.integers(0, A), rng.integers(0, A)] = -128
    e = [0, 1, 2, 4, 5, 17, 256][seed]
    o = int(rng.integers(e, min(1024, e + 60) + 1))
    T = SeqSet.from_list([rng.integers(0, A, size=int(L)).astype(np.uint8)
                          for L in list(rng.integers(0, 500, size=150)) + [1200]])
    Q = SeqSet.from_list([rng.integers(0, A, size=int(L)).astype(np.uint8) for L in (1, 37, 260, 1100)])
    log(f"random scoring seed={seed} A={A} o={o} e={e} route={route}")
    got, _ = gpu_search(Q, T, S, o, e, "local")
    exp = oracle.search(Q, T, S, o, e, mode="local")
    compare_search(got, exp, len(Q), len(T), label=f"random {seed}")
