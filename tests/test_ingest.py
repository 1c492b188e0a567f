"""FASTA / FASTQ ingest of the library (dsa_seqset_*, host code, no GPU)
against a plain Python reader written here from the format definitions:
multi-line records, case, unknown letters, CRLF line ends, blank lines,
empty records, skipped bytes, FASTQ qualities that start with '@' or '+',
every split of the text into two pieces, random piece sizes, a file read in
4 MiB pieces, and the errors (text before the first header, FASTQ quality of
the wrong length, a FASTQ record cut before its '+' line)."""
import os

import numpy as np
import pytest

PROTEIN_ORDER = "ARNDCQEGHILKMFPSTWYVBZX*"


def ref_code(ch, alphabet):
    """Code of one byte on a sequence line, or None when it is skipped."""
    if alphabet == "protein":
        if ch == "*":
            return 23
        if ch.isascii() and ch.isalpha():
            up = ch.upper()
            return PROTEIN_ORDER.index(up) if up in PROTEIN_ORDER else 22
        return None
    if ch.isascii() and ch.isalpha():
        up = ch.upper()
        return {"A": 0, "C": 1, "G": 2, "T": 3, "U": 3}.get(up, 4)
    return None


def ref_parse(text, alphabet):
    """(list of code lists, list of names, format) by the format definitions."""
    lines = text.split("\n")
    seqs, names = [], []
    k = 0
    while k < len(lines) and lines[k].strip(" \t\r") == "":
        k += 1
    if k == len(lines):
        return [], [], 0
    fmt = {">": 1, "@": 2}.get(lines[k].lstrip(" \t\r")[:1], None)
    if fmt is None:
        raise ValueError("no header")
    if fmt == 1:
        cur = None
        for line in lines[k:]:
            if line.startswith(">") or (cur is None and line.lstrip(" \t\r").startswith(">")):
                if cur is not None:
                    seqs.append(cur)
                name = line.lstrip(" \t\r")[1:]
                names.append(name[:-1] if name.endswith("\r") else name)
                cur = []
            elif cur is None:
                if line.strip(" \t\r"):
                    raise ValueError("text before header")
            else:
                cur.extend(c for c in (ref_code(ch, alphabet) for ch in line) if c is not None)
        if cur is not None:
            seqs.append(cur)
        return seqs, names, fmt
    # FASTQ: header, sequence lines up to '+', quality lines up to the length
    while k < len(lines):
        line = lines[k]
        if line.strip(" \t\r") == "":
            k += 1
            continue
        head = line.lstrip(" \t\r")
        if not head.startswith("@"):
            raise ValueError("expected @")
        name = head[1:]
        names.append(name[:-1] if name.endswith("\r") else name)
        k += 1
        cur = []
        while k < len(lines) and not lines[k].startswith("+"):
            cur.extend(c for c in (ref_code(ch, alphabet) for ch in lines[k]) if c is not None)
            k += 1
        if k == len(lines):
            raise ValueError("no + line")
        k += 1
        need = len(cur)
        while need > 0:
            if k == len(lines):
                raise ValueError("quality short")
            q = lines[k].replace("\r", "")
            if len(q) > need:
                raise ValueError("quality long")
            need -= len(q)
            k += 1
        seqs.append(cur)
    return seqs, names, fmt


@pytest.fixture(scope="module")
def dsa():
    import paper_1701_01575_amd as m
    return m


def check(dsa, text, alphabet, pieces=None):
    seqs, names, fmt = ref_parse(text, alphabet)
    got = dsa.Sequences.from_text(pieces if pieces is not None else [text], alphabet)
    assert len(got) == len(seqs)
    assert got.names == names
    for k, s in enumerate(seqs):
        assert list(got[k]) == s, k
    assert got.codes.dtype == np.uint8 and got.offsets[0] == 0
    if seqs:
        assert got.format == ("fasta" if fmt == 1 else "fastq")
    return got


FASTA = (">sp|P1|first protein\nMKTAYIAKQR\nqisfvksHFS\n\n>second desc\r\nACDEFGHIK*\r\nJOUBZX-..12 L\n"
         ">empty\n>last no newline\nWWWYV")
FASTQ = ("@read1 x\nACGTNRYU\n+\nIIIIIIII\n@read2\nacg\ntt\n+read2\n@@+\nII\n@empty\n\n+\n\n"
         "@r4\r\nGGA\r\n+\r\n+@I\r\n")


def test_fasta_protein(dsa):
    got = check(dsa, FASTA, "protein")
    assert got.names[0] == "sp|P1|first protein" and len(got[2]) == 0
    # J O U -> X; B Z X; '-', '.', digits and the space skipped; L
    assert list(got[1][-7:]) == [22, 22, 22, 20, 21, 22, 10]
    assert list(got[1][:10]) == [0, 4, 3, 6, 13, 7, 8, 9, 11, 23]


def test_fasta_dna(dsa):
    check(dsa, ">a\nACGTU\nnryk\n>b\n\n>c\nGATTACA", "dna")


def test_fastq(dsa):
    got = check(dsa, FASTQ, "dna")
    assert got.format == "fastq" and got.names == ["read1 x", "read2", "empty", "r4"]
    assert list(got[0]) == [0, 1, 2, 3, 4, 4, 4, 3]


def test_every_two_piece_split(dsa):
    for text, alpha in ((FASTA, "protein"), (FASTQ, "dna")):
        for cut in range(len(text) + 1):
            check(dsa, text, alpha, pieces=[text[:cut], text[cut:]])


def test_random_pieces(dsa):
    rng = np.random.default_rng([170101575, 95])
    text = FASTA * 7 + "\n"
    for _ in range(20):
        cuts = np.sort(rng.integers(0, len(text), size=int(rng.integers(1, 30))))
        pieces = [text[a:b] for a, b in zip(np.concatenate([[0], cuts]), np.concatenate([cuts, [len(text)]]))]
        check(dsa, text, "protein", pieces=pieces)


def test_blank_and_empty_inputs(dsa):
    assert len(dsa.Sequences.from_text("", "protein")) == 0
    assert len(dsa.Sequences.from_text("\n \r\n", "protein")) == 0
    check(dsa, "\n\n>x\nAC\n", "protein")


@pytest.mark.parametrize("text,alpha,words", [
    ("ACGT\n>x\nAC\n", "protein", "header"),
    ("@r\nACG\n+\nIIII\n", "dna", "longer"),
    ("@r\nACG\n+\nII", "dna", "shorter"),
    ("@r\nACG\n", "dna", "'+'"),
    (">x\nAC\n@r\n", "dna", None),   # '@' inside FASTA is a skipped byte, not an error
])
def test_errors(dsa, text, alpha, words):
    from paper_1701_01575_amd import binding as B
    if words is None:
        check(dsa, text, alpha)
        return
    with pytest.raises(B.DsaError) as ei:
        dsa.Sequences.from_text(text, alpha)
    assert ei.value.status == B.DSA_E_INVAL and words in str(ei.value)


def test_file_in_pieces(dsa, tmp_path):
    """About 9 MB of FASTA with 60-column lines: more than two 4 MiB pieces."""
    rng = np.random.default_rng([170101575, 96])
    lens = rng.integers(1, 4000, size=4500)
    letters = np.frombuffer(b"ARNDCQEGHILKMFPSTWYVarndx", dtype=np.uint8)
    parts = []
    for k, L in enumerate(lens):
        s = letters[rng.integers(0, len(letters), size=int(L))].tobytes().decode()
        body = "\n".join(s[i:i + 60] for i in range(0, len(s), 60))
        parts.append(f">seq{k} len={L}\n{body}\n")
    text = "".join(parts)
    path = tmp_path / "db.fasta"
    path.write_text(text)
    assert os.path.getsize(path) > 8 << 20
    got = dsa.Sequences.from_file(path, "protein")
    seqs, names, _ = ref_parse(text, "protein")
    assert got.names == names and len(got) == 4500
    assert (got.lengths == np.array([len(s) for s in seqs])).all()
    assert (got.codes == np.concatenate([np.array(s, np.uint8) for s in seqs])).all()
