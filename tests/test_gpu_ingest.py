"""A database and queries read from files by the library's ingest, then
searched on the GPU: a FASTA database of log-normal targets plus long tails
(35,000, 41,234 and 65,532 residues, which the wavefront units take) and
FASTQ queries; the codes read back equal the generator's, and every search
result (and the top-10 hits with traceback of one query) equals the oracle's."""
import numpy as np
import pytest

import oracle
from gpu_util import compare_search, log
from workloads import PROTEIN_ALPHABET, gen
from workloads.gen import SeqSet

pytestmark = pytest.mark.gpu


def _write_fasta(path, seqs, width=70):
    with open(path, "w") as fh:
        for k in range(len(seqs)):
            s = "".join(PROTEIN_ALPHABET[c] for c in seqs[k])
            if k % 3 == 1:
                s = s.lower()
            fh.write(f">target_{k} synthetic\n")
            for i in range(0, len(s), width):
                fh.write(s[i:i + width] + "\n")


def _write_fastq(path, seqs):
    with open(path, "w") as fh:
        for k in range(len(seqs)):
            s = "".join(PROTEIN_ALPHABET[c] for c in seqs[k])
            fh.write(f"@query_{k}\n{s[:len(s) // 2]}\n{s[len(s) // 2:]}\n+\n{'@' * len(s)}\n")


def test_search_database_read_from_fasta(blosum, tmp_path):
    import torch
    import paper_1701_01575_amd as dsa
    rng = np.random.default_rng([170101575, 97])
    lens = np.concatenate([gen.lognormal_lengths(rng, 3000), [35000, 41234, 65532]])
    rng.shuffle(lens)
    T = gen.random_protein_set(lens, rng)
    Q = gen.random_protein_set(np.array([300, 1200]), rng)
    _write_fasta(tmp_path / "db.fasta", T)
    _write_fastq(tmp_path / "q.fastq", Q)
    log("ingest: 3003 targets (tails to 65,532) from FASTA, 2 queries from FASTQ")
    qs = dsa.Sequences.from_file(tmp_path / "q.fastq", "protein")
    assert qs.format == "fastq" and qs.names == ["query_0", "query_1"]
    assert (qs.codes == Q.codes).all() and (qs.offsets == Q.offsets).all()
    db = dsa.Database.from_file(tmp_path / "db.fasta", "protein")
    assert db.names[5] == "target_5 synthetic"
    assert (db._codes == T.codes).all() and (db._offsets == T.offsets).all()
    r = dsa.align(qs, db=db, matrix=blosum, gap_open=11, gap_extend=1)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in r.items() if hasattr(v, "cpu")}
    exp = oracle.search(Q, T, blosum, 11, 1)
    compare_search(got, exp, len(Q), len(T), label="ingest")
    log("ingest: top-10 with traceback of the 300-residue query")
    Q0 = SeqSet.from_list([Q[0]])
    r = dsa.align(Q0, db=db, matrix=blosum, gap_open=11, gap_extend=1, top_k=10, traceback=True)
    torch.cuda.synchronize()
    hits = r["t_index"].cpu().numpy()
    sc = exp["score"][:len(T)]
    assert (hits == oracle.top_k(sc, 10)).all()
    tr = oracle.align_index(np.zeros(10, np.int64), hits, Q0, T, blosum, 11, 1, mode="local",
                            traceback=True)
    cig = dsa.cigars(r)
    for f in ("score", "q_begin", "q_end", "t_begin", "t_end"):
        assert (r[f].cpu().numpy() == tr[f]).all(), f
    for k in range(10):
        assert (cig[k] == tr["cigars"][k]).all(), k
    db.close()
