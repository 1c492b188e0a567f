// Sequence ingest: FASTA and FASTQ text, streamed in pieces of any size,
// mapped to residue codes and collected into concatenated codes + offsets
// (+ record names), ready for dsa_db_create or as a query set.
//
// The paper's converter (Section II.B.1, "Map") turns the input files into
// the alignment workers' layout, and its data API takes FASTA, FASTQ and
// ADAM files (Section II.C.1; ADAM, a columnar store, is not read here).
// The residue mapping follows the standard alphabets of the score matrices:
//   protein  A R N D C Q E G H I L K M F P S T W Y V B Z X * -> codes 0..23
//            (BLOSUM62's distribution order); any other letter (J, O, U, ...)
//            is X (22)
//   DNA      A C G T -> 0..3, U -> T, any other letter (N and the IUPAC
//            ambiguity codes) -> N (4)
// Letters are case-insensitive.  On sequence lines every byte that is not a
// letter (or '*' for protein) is skipped: spaces, tabs, '\r', digits,
// alignment gaps '-' and '.'.
//
// FASTA: a record is a '>' header line (the name is the rest of the line,
// without a trailing '\r') followed by any number of sequence lines; text
// before the first '>' other than blank lines is an error.
// FASTQ: a record is an '@' header line, sequence lines up to a line starting
// with '+', then quality lines until as many quality bytes as residues have
// been read (so a quality line may start with '@' or '+'); the quality
// values are not kept.  A file is FASTA or FASTQ by its first non-blank byte.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "dsa.h"

namespace dsa {
void set_last_error(const std::string &msg);  // runtime: the text dsa_last_error returns
}

namespace {

int ingest_fail(int code, const std::string &msg) {
    dsa::set_last_error(msg);
    return code;
}

enum Format { FMT_NONE = 0, FMT_FASTA = 1, FMT_FASTQ = 2 };
// where the parser is inside the text
enum State {
    ST_START,      // between records (FASTQ) or before the first one: blank lines only
    ST_HEADER,     // in a header line (after '>' or '@')
    ST_SEQ_BOL,    // at the beginning of a sequence line
    ST_SEQ,        // inside a sequence line
    ST_PLUS,       // FASTQ: inside the '+' separator line
    ST_QUAL,       // FASTQ: inside the quality lines
};

}  // namespace

struct dsa_seqset {
    int32_t alphabet = 0;
    uint8_t map[256];
    std::vector<uint8_t> codes;
    std::vector<int64_t> offsets{0};
    std::vector<std::pair<int64_t, int64_t>> name_span;  // [begin, end) of each record's name in `names`
    std::string names;
    int format = FMT_NONE;
    State st = ST_START;
    int64_t qual_need = 0;     // FASTQ: quality bytes still expected for this record
    int64_t line = 1;          // input line (for error messages)
    bool finished = false;
};

namespace {

void build_map(dsa_seqset *s) {
    // 255 = skip this byte
    memset(s->map, 255, sizeof(s->map));
    if (s->alphabet == DSA_ALPHA_PROTEIN) {
        static const char order[] = "ARNDCQEGHILKMFPSTWYVBZX*";
        for (int c = 'A'; c <= 'Z'; c++) s->map[c] = s->map[c + 32] = 22;  // X
        for (int k = 0; k < 24; k++) {
            const unsigned char c = (unsigned char)order[k];
            s->map[c] = (uint8_t)k;
            if (c >= 'A' && c <= 'Z') s->map[c + 32] = (uint8_t)k;
        }
    } else {
        for (int c = 'A'; c <= 'Z'; c++) s->map[c] = s->map[c + 32] = 4;  // N
        const char *acgt = "ACGT";
        for (int k = 0; k < 4; k++) {
            s->map[(unsigned char)acgt[k]] = (uint8_t)k;
            s->map[(unsigned char)acgt[k] + 32] = (uint8_t)k;
        }
        s->map['U'] = s->map['u'] = 3;
    }
}

void open_record(dsa_seqset *s) {
    const int64_t at = (int64_t)s->names.size();
    s->name_span.push_back({at, at});
    s->st = ST_HEADER;
}

void end_header(dsa_seqset *s) {
    auto &sp = s->name_span.back();
    if ((int64_t)s->names.size() > sp.first && s->names.back() == '\r') s->names.pop_back();
    sp.second = (int64_t)s->names.size();
}

void close_record(dsa_seqset *s) { s->offsets.push_back((int64_t)s->codes.size()); }

int64_t cur_len(const dsa_seqset *s) { return (int64_t)s->codes.size() - s->offsets.back(); }

std::string where(const dsa_seqset *s) { return "line " + std::to_string(s->line) + ": "; }

// Feed bytes; every state change happens at a byte, so pieces may split the
// text anywhere.
int feed(dsa_seqset *s, const char *p, size_t n) {
    for (size_t k = 0; k < n; k++) {
        const unsigned char c = (unsigned char)p[k];
        if (s->st == ST_START) {
            if (c == '\n') { s->line++; continue; }
            if (c == ' ' || c == '\t' || c == '\r') continue;
            if (s->format == FMT_NONE) s->format = (c == '>') ? FMT_FASTA : (c == '@') ? FMT_FASTQ : FMT_NONE;
            if ((s->format == FMT_FASTA && c == '>') || (s->format == FMT_FASTQ && c == '@')) {
                open_record(s);
                continue;
            }
            return ingest_fail(DSA_E_INVAL, where(s) + "expected a FASTA ('>') or FASTQ ('@') header");
        }
        if (s->st == ST_HEADER) {
            if (c == '\n') {
                end_header(s);
                s->line++;
                s->st = ST_SEQ_BOL;
            } else {
                s->names.push_back((char)c);
            }
            continue;
        }
        if (s->st == ST_SEQ_BOL) {
            if (s->format == FMT_FASTA && c == '>') {
                close_record(s);
                open_record(s);
                continue;
            }
            if (s->format == FMT_FASTQ && c == '+') {
                s->qual_need = cur_len(s);
                s->st = ST_PLUS;
                continue;
            }
            s->st = ST_SEQ;  // and read c as a sequence byte
        }
        if (s->st == ST_SEQ) {
            if (c == '\n') {
                s->line++;
                s->st = ST_SEQ_BOL;
            } else if (s->map[c] != 255) {
                s->codes.push_back(s->map[c]);
            }
            continue;
        }
        if (s->st == ST_PLUS) {
            if (c == '\n') {
                s->line++;
                if (s->qual_need == 0) {
                    close_record(s);
                    s->st = ST_START;
                } else {
                    s->st = ST_QUAL;
                }
            }
            continue;
        }
        // ST_QUAL: count quality bytes up to the sequence length
        if (c == '\n') {
            s->line++;
            if (s->qual_need == 0) {
                close_record(s);
                s->st = ST_START;
            }
            continue;
        }
        if (c == '\r') continue;
        if (s->qual_need == 0)
            return ingest_fail(DSA_E_INVAL, where(s) + "FASTQ quality longer than its sequence (record " +
                                                std::to_string(s->offsets.size()) + ")");
        s->qual_need--;
    }
    return DSA_OK;
}

}  // namespace

extern "C" int dsa_seqset_create(int32_t alphabet, dsa_seqset **out) {
    if (!out) return ingest_fail(DSA_E_INVAL, "out is NULL");
    *out = nullptr;
    if (alphabet != DSA_ALPHA_PROTEIN && alphabet != DSA_ALPHA_DNA)
        return ingest_fail(DSA_E_INVAL, "alphabet must be DSA_ALPHA_PROTEIN or DSA_ALPHA_DNA");
    dsa_seqset *s = new dsa_seqset();
    s->alphabet = alphabet;
    build_map(s);
    *out = s;
    return DSA_OK;
}

extern "C" int dsa_seqset_feed(dsa_seqset *s, const char *bytes, size_t len) {
    if (!s) return ingest_fail(DSA_E_INVAL, "seqset is NULL");
    if (s->finished) return ingest_fail(DSA_E_INVAL, "seqset already finished");
    if (len && !bytes) return ingest_fail(DSA_E_INVAL, "bytes is NULL");
    return feed(s, bytes, len);
}

extern "C" int dsa_seqset_finish(dsa_seqset *s) {
    if (!s) return ingest_fail(DSA_E_INVAL, "seqset is NULL");
    if (s->finished) return DSA_OK;
    switch (s->st) {
        case ST_START:
            break;
        case ST_HEADER:
        case ST_SEQ_BOL:
        case ST_SEQ:
            if (s->format == FMT_FASTQ)
                return ingest_fail(DSA_E_INVAL, "FASTQ record " + std::to_string(s->offsets.size()) +
                                                    " ends before its '+' line");
            if (s->st == ST_HEADER) end_header(s);
            close_record(s);
            break;
        case ST_PLUS:
        case ST_QUAL:
            if (s->qual_need != 0)
                return ingest_fail(DSA_E_INVAL, "FASTQ record " + std::to_string(s->offsets.size()) +
                                                    ": quality shorter than its sequence");
            close_record(s);
            break;
    }
    s->finished = true;
    return DSA_OK;
}

extern "C" int dsa_seqset_read_file(dsa_seqset *s, const char *path) {
    if (!s || !path) return ingest_fail(DSA_E_INVAL, "seqset or path is NULL");
    FILE *f = fopen(path, "rb");
    if (!f) return ingest_fail(DSA_E_INVAL, std::string("cannot open ") + path);
    std::vector<char> buf((size_t)4 << 20);
    int rc = DSA_OK;
    size_t r;
    while (rc == DSA_OK && (r = fread(buf.data(), 1, buf.size(), f)) > 0) rc = dsa_seqset_feed(s, buf.data(), r);
    const bool err = ferror(f) != 0;
    fclose(f);
    if (rc) return rc;
    if (err) return ingest_fail(DSA_E_INVAL, std::string("read error on ") + path);
    return dsa_seqset_finish(s);
}

extern "C" int dsa_seqset_info(const dsa_seqset *s, int64_t *n_seqs, int64_t *n_residues, int32_t *format) {
    if (!s) return ingest_fail(DSA_E_INVAL, "seqset is NULL");
    if (n_seqs) *n_seqs = (int64_t)s->offsets.size() - 1;
    if (n_residues) *n_residues = s->offsets.back();
    if (format) *format = s->format;
    return DSA_OK;
}

extern "C" int dsa_seqset_codes(const dsa_seqset *s, const uint8_t **codes, const int64_t **offsets) {
    if (!s || !codes || !offsets) return ingest_fail(DSA_E_INVAL, "NULL argument");
    if (!s->finished) return ingest_fail(DSA_E_INVAL, "call dsa_seqset_finish first");
    *codes = s->codes.data();
    *offsets = s->offsets.data();
    return DSA_OK;
}

extern "C" int dsa_seqset_name(const dsa_seqset *s, int64_t k, const char **name, int64_t *len) {
    if (!s || !name || !len) return ingest_fail(DSA_E_INVAL, "NULL argument");
    if (!s->finished) return ingest_fail(DSA_E_INVAL, "call dsa_seqset_finish first");
    const int64_t n = (int64_t)s->offsets.size() - 1;
    if (k < 0 || k >= n) return ingest_fail(DSA_E_INVAL, "record index out of range");
    const auto &sp = s->name_span[(size_t)k];
    *name = s->names.data() + sp.first;
    *len = sp.second - sp.first;
    return DSA_OK;
}

extern "C" int dsa_seqset_destroy(dsa_seqset *s) {
    delete s;
    return DSA_OK;
}
