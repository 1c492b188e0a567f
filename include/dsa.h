/*
 * dsa.h - C ABI of the MI355X affine-gap alignment library (libdsa.so).
 *
 * The library aligns query sequences against a database of target sequences
 * (every query against every target), or queries against targets pairwise,
 * with the three algorithms of the DSA paper (Section II.C.2): local
 * Smith-Waterman, global Needleman-Wunsch and semi-global alignment, all
 * with affine gaps as in the SIMD libraries the paper builds on
 * (Section II.B.1).  Each result is the alignment object of Section II.B.1:
 * optimal score, location (begin/end in both sequences) and, on request, a
 * CIGAR; per-query top-K selection follows Section II.B.2.
 *
 * Definitions (shared by every entry point):
 *   codes        sequences are arrays of uint8 codes < alphabet_size (<= 64;
 *                searches over more than 32 letters run the exact int32 kernel)
 *   subst        alphabet_size x alphabet_size int8 matrix, row = query code,
 *                column = target code
 *   gaps         a run of L gap columns costs gap_open + (L-1) * gap_extend,
 *                0 <= gap_extend <= gap_open
 *   local        max(0, best score over all pairs of substrings); 0 = none
 *   global       both sequences end to end
 *   semiglobal   the query end to end, the target's prefix/suffix free by
 *                default; free_ends (DSA_QB|DSA_QE|DSA_TB|DSA_TE) selects which
 *                ends are free (0 = DSA_TB|DSA_TE); the result is the best of
 *                H[m][n], the last row if TE, the last column if QE (a search
 *                with QE runs the exact int32 kernel, as DSA_FORCE_INT32)
 *   end cell     among the cells reaching the result: smallest target end,
 *                then smallest query end
 *   traceback    priority zero (local) > diagonal > gap in query (D) > gap in
 *                target (I); inside a gap run, opening wins ties
 *   coordinates  0-based inclusive; -1 everywhere for "no alignment"; begins
 *                are computed only with DSA_TRACEBACK (else -1)
 *   CIGAR        uint32 runs, (length << 4) | op, op in BAM numbering:
 *                1 = I (query residue vs gap), 2 = D (gap vs target residue),
 *                7 = '=' (identical residues), 8 = 'X' (different residues)
 *
 * Memory: pointers marked [dev] are device pointers on the current HIP
 * device, [host] are host pointers.  The caller owns every input and output
 * buffer.  The library owns only a dsa_db (device memory taken by
 * dsa_db_create from the caller's allocator, or hipMalloc without one, and
 * released by dsa_db_destroy) and a small pinned staging buffer per device
 * for work tables.
 *
 * Streams: dsa_align_batch enqueues its copies and kernels on args->stream
 * (a hipStream_t, NULL = default stream) and returns without waiting;
 * outputs are valid once that stream has been synchronised.  One exception:
 * a top-K search with DSA_TRACEBACK reads its hit list back to the host to
 * plan the traceback of the hits, so it waits for args->stream once, in the
 * middle of the call (and cannot be recorded into a graph).  It performs no
 * device allocation: all scratch memory is the caller's workspace.
 *
 * Errors: every entry point returns a dsa_status; no C++ exception crosses
 * the ABI.  dsa_last_error() returns a thread-local message for the last
 * failure on the calling thread.
 */
#ifndef DSA_H
#define DSA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* raised whenever a struct layout or a signature below changes */
#define DSA_ABI_VERSION 4

typedef enum {
    DSA_OK = 0,
    DSA_E_INVAL = 1,      /* bad pointer, mode, flag, code, penalty or size */
    DSA_E_RANGE = 2,      /* scores could reach 2^31 even in int32 */
    DSA_E_WORKSPACE = 3,  /* workspace smaller than dsa_workspace_size */
    DSA_E_CAPACITY = 4,   /* CIGAR buffer too small (results still valid) */
    DSA_E_DEVICE = 5,     /* a HIP call failed; see dsa_last_error */
    DSA_E_NOTSUP = 6      /* combination not supported by the library */
} dsa_status;

enum { DSA_LOCAL = 0, DSA_GLOBAL = 1, DSA_SEMIGLOBAL = 2 };
enum { DSA_QB = 1, DSA_QE = 2, DSA_TB = 4, DSA_TE = 8 };

/* flags */
#define DSA_TRACEBACK   1u  /* compute begins and CIGAR */
#define DSA_PLAIN       2u  /* one launch per query (per pair batch), no persistent kernel */
#define DSA_FORCE_INT32 4u  /* skip the packed int16 pass */

/* per-result status bits */
#define DSA_ST_INT32     1u  /* computed by an int32 kernel (a rerun, or a path that is int32 throughout) */
#define DSA_ST_TRUNCATED 2u  /* the CIGAR did not fit in its slot */

typedef struct dsa_db dsa_db;

/*
 * Device memory supplied by the caller (for example a framework's caching
 * allocator): alloc(bytes, ctx) returns device memory on the current device,
 * at least 16-byte aligned, or NULL on failure; free(ptr, ctx) gives it back.
 * Both are called on the thread that calls dsa_db_create / dsa_db_destroy.
 */
typedef struct {
    void *(*alloc)(size_t bytes, void *ctx);
    void (*free)(void *ptr, void *ctx);
    void *ctx;
} dsa_allocator;

/*
 * dsa_db_create - pack a target database into device memory (Section II.B.1
 * "Map": the reference set is converted once into a layout suited to the
 * parallel workers and kept memory-resident, Section II.A).
 *   codes      [host] concatenated target codes, offsets[n_targets] bytes
 *   offsets    [host] n_targets + 1 int64 offsets, non-decreasing, offsets[0] = 0
 *   n_targets  >= 1
 *   alphabet_size  2..64; every code must be < alphabet_size
 *   alloc      [host] the allocator every device buffer of the database comes
 *              from (copied; its ctx must stay valid until dsa_db_destroy),
 *              or NULL for hipMalloc / hipFree
 *   stream     hipStream_t for the uploads (the call synchronises it)
 *   out        receives the handle
 * Targets are sorted by length into groups of 128 (two per lane of a
 * 64-wide wave), their codes interleaved so a wave reads 8 bytes per lane
 * per 4 columns.  Errors: DSA_E_INVAL (also an allocator with alloc or free
 * NULL, or memory not 16-byte aligned), DSA_E_DEVICE (also alloc returning
 * NULL), DSA_E_NOTSUP (a target longer than 65,532 residues).  On an error
 * every buffer already taken is given back.
 */
int dsa_db_create(const uint8_t *codes, const int64_t *offsets, int64_t n_targets,
                  int32_t alphabet_size, const dsa_allocator *alloc, void *stream, dsa_db **out);

/* dsa_db_destroy - free a database (NULL is accepted), through the allocator
 * it was created with.  Not stream-ordered: the caller must make sure no
 * enqueued work still reads it. */
int dsa_db_destroy(dsa_db *db);

/* Number of targets, total residues and device bytes held by a database. */
int dsa_db_info(const dsa_db *db, int64_t *n_targets, int64_t *n_residues, int64_t *device_bytes);

typedef struct {
    /* queries */
    const uint8_t *q_codes;    /* [dev]  concatenated query codes */
    const int64_t *q_offsets;  /* [host] n_q + 1 offsets into q_codes */
    int64_t n_q;               /* >= 1 */
    /* targets: exactly one of db / (t_codes, t_offsets) */
    const dsa_db *db;          /* database search: every query vs every target */
    const uint8_t *t_codes;    /* [dev]  pairwise: query k vs target k */
    const int64_t *t_offsets;  /* [host] n_q + 1 offsets into t_codes */
    /* scoring */
    const int8_t *subst;       /* [host] alphabet_size^2, row = query code (may be NULL with pssm) */
    const int8_t *pssm;        /* [host] position-specific profile, or NULL: one row of alphabet_size
                                  scores per query residue, rows in q_codes order; residue i of a
                                  query then scores pssm[row][c] against target code c in place of
                                  subst[code][c] (the scoring hook beside the paper's user-defined
                                  algorithms, Section II.C.2); '=' and 'X' still compare codes */
    int32_t alphabet_size;     /* 2..64; must equal the database's */
    int32_t gap_open;          /* >= gap_extend >= 0 */
    int32_t gap_extend;
    int32_t mode;              /* DSA_LOCAL | DSA_GLOBAL | DSA_SEMIGLOBAL */
    int32_t free_ends;         /* semiglobal only; 0 = DSA_TB|DSA_TE */
    uint32_t flags;            /* DSA_TRACEBACK | DSA_PLAIN | DSA_FORCE_INT32 */
    int32_t top_k;             /* database search only: 0 = all targets, else K <= 64 best per query */
    /* scratch */
    void *workspace;           /* [dev] >= dsa_workspace_size bytes, 256-byte aligned */
    size_t workspace_bytes;
    void *stream;              /* hipStream_t */
} dsa_args;

/*
 * Results.  Layout: database search without top_k: n_q * n_targets entries,
 * query-major, targets in original order.  With top_k: n_q * top_k entries,
 * best first (score descending, original target index ascending; only
 * positive local scores; unused slots have t_index = -1, score = 0).
 * Pairwise: n_q entries.  All pointers [dev]; NULL = not wanted (score is
 * required).
 */
typedef struct {
    int32_t *score;
    int32_t *q_begin, *q_end, *t_begin, *t_end;
    int64_t *t_index;          /* top_k only: original target index */
    uint8_t *status;           /* DSA_ST_* bits */
    /* DSA_TRACEBACK: result r's runs are cigar_ops[cigar_off[r] .. + cigar_len[r]) */
    int64_t *cigar_off;
    int32_t *cigar_len;
    uint32_t *cigar_ops;
    int64_t cigar_capacity;    /* uint32 entries in cigar_ops */
} dsa_out;

/*
 * dsa_workspace_size - bytes of device workspace dsa_align_batch needs for
 * these arguments (the workspace pointer itself is not read).
 * Errors: DSA_E_INVAL, DSA_E_NOTSUP, DSA_E_RANGE.
 */
int dsa_workspace_size(const dsa_args *args, size_t *bytes);

/*
 * dsa_cigar_capacity - uint32 entries dsa_out.cigar_ops needs so that no
 * CIGAR can be truncated (sum over results of query + target length + 1).
 * Each result owns a region of that size in result order; its runs are
 * written at the end of the region and cigar_off / cigar_len locate them.
 * With less capacity the results that do not fit get an empty region, the
 * DSA_ST_TRUNCATED status bit and dsa_align_batch returns DSA_E_CAPACITY
 * (scores and coordinates stay valid).
 */
int dsa_cigar_capacity(const dsa_args *args, int64_t *entries);

/*
 * dsa_align_batch - align (Sections II.B.1 and II.C.2; top-K per
 * Section II.B.2).  Asynchronous on args->stream, except that a top-K search
 * with DSA_TRACEBACK waits once for the stream (its hit list is read back to
 * plan the hits' traceback).  Scores are exact.  A database search runs a
 * packed int16 pass followed by an exact int32 rerun of every result that
 * could have saturated, and these results carry DSA_ST_INT32:
 *   local        every score above 28,544, the exact range of the offset
 *                int16 values the local kernels hold;
 *   global, semi-global
 *                every query whose host bound (3 gap_open + (m + n) gap_extend
 *                + |min S|, or min(sum of row maxima, sum of column maxima))
 *                leaves the int16 range goes to int32 at once, and every
 *                score at either int16 bound is rerun.
 * These searches run the int32 kernel throughout: DSA_FORCE_INT32; a free
 * query end (semi-global with DSA_QE); a local search with gap_open above
 * 1024 or gap_extend above 256.
 * Pairwise alignment: large pairs (by default 48 query rows and 32,768 cells
 * or more) run a packed int16 fill, two pairs per wavefront segment, each
 * pair's values offset by a bias that covers the lowest value its recurrence
 * can reach (gap_open + gap_extend + |min S|, plus the two boundary gaps in
 * global and semi-global mode).  A pair whose values could pass the int16
 * range is redone by the exact int32 kernels and carries DSA_ST_INT32: in
 * global and semi-global mode when its query's sum of positive row maxima
 * exceeds the limit the bias leaves (31,743 - bias - max S - gap_extend
 * (17 + n), with bias = 1,024 + that depth; the last term is the room the
 * fill's value frame takes), in local mode when its best score does or a
 * value of its fill passes the finite binary16 range.  These run int32
 * throughout: a position-specific profile, more than 32 letters, max S +
 * 2 gap_extend above 127 (max S + gap_extend in local mode: the fill's
 * int8 score table carries that step), DSA_FORCE_INT32, DSA_PLAIN.
 * Smaller pairs, and the traceback of top-K hits, run exact int32 kernels.
 * Errors: DSA_E_INVAL, DSA_E_RANGE, DSA_E_WORKSPACE, DSA_E_NOTSUP,
 * DSA_E_DEVICE.
 */
int dsa_align_batch(const dsa_args *args, const dsa_out *out);

/*
 * dsa_align_batch_noalloc - dsa_align_batch for callers that cannot
 * allocate memory (code that must not call hipMalloc or hipHostMalloc:
 * tight serving loops, harnesses that forbid allocation).  Same arguments,
 * results, status codes and stream semantics as dsa_align_batch, except:
 *   - args->workspace and args->workspace_bytes are ignored; the workspace
 *     is a static device array of the library, DSA_NOALLOC_SCRATCH_BYTES
 *     (64 MiB) per device, held from the library's load until the process
 *     ends.  Boundary rows and direction-code chunks are planned to at
 *     most a quarter of it each (more rounds of queries, more chunks).
 *   - a call whose plan still needs more returns DSA_E_WORKSPACE before any
 *     device work; dsa_last_error states the bytes needed.
 *   - no device or pinned host memory is allocated: the work tables go to
 *     the device from pageable host memory (the host heap holds the plan).
 *     The first call on a device looks up the array's device address.
 *   - every call on a device shares the array and finds the previous
 *     call's contents in it: calls that overlap on one device (two streams,
 *     two threads) race and give undefined results; calls in order on one
 *     stream, or separated by synchronisation, are safe.
 */
#define DSA_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int dsa_align_batch_noalloc(const dsa_args *args, const dsa_out *out);

/*
 * Recorded batches: the batched form replayed from a HIP graph, for callers
 * that run the same batch shape again and again (Section II.B's map phase
 * over a fixed query set and reference).
 *
 * dsa_graph_create plans the call (args, out) as dsa_align_batch would,
 * writes its tables into args->workspace (it waits for args->stream once),
 * then records every kernel of the call into a graph by capturing
 * args->stream (which must not be the null stream).  Nothing runs yet.
 * dsa_graph_launch(graph, stream) replays the whole call on `stream`: it reads
 * the query codes, database, workspace and writes the outputs at the device
 * addresses given at creation, with whatever they hold at replay time, so
 * the caller keeps all of them alive and unmoved, may change the query
 * residues (not the lengths) between replays, and must not run two replays
 * of one graph, or a replay and another call on the same workspace, at the
 * same time.  *graph is set when the return is DSA_OK or DSA_E_CAPACITY.
 * dsa_graph_destroy frees the graph (not the buffers).
 * Errors: as dsa_align_batch; DSA_E_NOTSUP for top_k with traceback (the hit
 * traceback reads the hit list back on the host).
 */
typedef struct dsa_graph dsa_graph;
int dsa_graph_create(const dsa_args *args, const dsa_out *out, dsa_graph **graph);
int dsa_graph_launch(dsa_graph *graph, void *stream);
int dsa_graph_destroy(dsa_graph *graph);

/*
 * Autotuning of launch choices that never change results: the strip height
 * (16 or 32 rows) and waves per block of the inter-sequence kernel, the
 * cell budget above which a target group goes to the wavefront kernel and,
 * for local searches, the budget up to which such a group is instead one
 * strip-pipelined unit (database search), or the query rows and cells above which a pair goes
 * to the wavefront pairwise kernel (pairwise).  Choices are kept per shape
 * class: kind, mode, form (plain or batched), traceback, top-K, alphabet and
 * power-of-two buckets of the query residues and database residues (search)
 * or of the cells and longest query (pairwise); dsa_tuning_key writes that
 * class's name.
 *
 * dsa_autotune(args, cache_path, chosen) times candidates on these very
 * arguments (blocking; it allocates its own workspace and outputs, so
 * args->workspace is not used), keeps the fastest for the class in the
 * process, merges it into the JSON file cache_path when that is not NULL,
 * and returns in *chosen (NULL allowed) the values calls of the class now
 * use, as dsa_tuning_get does.  Later calls of the class,
 * dsa_workspace_size included, use it: the caller sizes the workspace after
 * tuning.  A file named by the environment variable DSA_AUTOTUNE_CACHE is
 * read once, at the first call that plans.  Environment variables DSA_STRIP,
 * DSA_WAVES, DSA_INTRA_BUDGET, DSA_KS_BUDGET, DSA_PAIR_WF_ROWS and
 * DSA_PAIR_WF_CELLS override the table.
 * dsa_tuning_get returns the values a call with these arguments would use
 * now (search: strip, waves, intra_budget, ks_budget; pairwise: pair_rows, pair_cells;
 * the others -1), with ms = the tuned time (0 if untuned).
 */
typedef struct {
    int32_t strip;           /* rows per strip of the inter-sequence kernel */
    int32_t waves;           /* waves per block of the inter-sequence kernel */
    int64_t intra_budget;    /* strips x columns above which a group goes to the wavefront kernel */
    int64_t ks_budget;       /* such a group of a local search is one strip-pipelined unit when
                                ceil(strips / waves) x columns <= ks_budget (0 = never) */
    int64_t pair_rows;       /* pairwise: wavefront iff query rows >= pair_rows ... */
    int64_t pair_cells;      /* ... and rows x columns >= pair_cells */
    double ms;               /* time of the chosen candidate when tuned */
} dsa_tuning;
int dsa_autotune(const dsa_args *args, const char *cache_path, dsa_tuning *chosen);
int dsa_tuning_get(const dsa_args *args, dsa_tuning *out);
int dsa_tuning_key(const dsa_args *args, char *buf, size_t size);

/*
 * Measurement hooks.  dsa_timing_enable(1) makes dsa_align_batch record HIP
 * event pairs on the stream each kernel is launched on: kind 0 = the whole
 * search phase on args->stream (both search kernels, from the fork to the
 * join), or the whole pairwise phase (fill and walk of both pair kinds),
 * 1 = each launch of the inter-sequence kernel, 2 = each launch of the
 * wavefront search kernel (on the library's auxiliary stream), 3 = all
 * lane-per-pair fill + walk launches of one call, 4 = all wavefront-pair
 * fill + walk launches of one call (auxiliary stream when both kinds run).
 * dsa_timing_read(kind, ...) waits for that kind's events and returns the
 * summed milliseconds and the launch count; dsa_timing_reset clears the
 * record.  Used by the benchmark to time the dominant kernels; off by default.
 */
int dsa_timing_enable(int on);
int dsa_timing_read(int kind, double *total_ms, int64_t *launches);
int dsa_timing_reset(void);

/*
 * dsa_probe - measured ceilings on the current device (blocking; allocates
 * its own scratch).  which: 0 v_pk_add_i16 (clamp), 1 v_pk_max_i16,
 * 2 v_pk_sub_u16 (clamp), 3 v_add_u32, 4 v_max_i32, 6 v_pk_maximum3_f16
 * -> *rate = instructions per second summed over lanes, size = loop
 * iterations; 5 -> HBM copy of `size` bytes, *rate = bytes read + written
 * per second; 7 -> *rate = the number of wrong results of the packed
 * binary16 three-way maximum over every operand pattern the local-mode int16
 * search produces (must be 0; size is ignored but must be positive);
 * 8, 9 -> *rate = local-mode cells per second of a bare 16-row column
 * recurrence (scores from an LDS profile, no boundary or end-cell work),
 * 8 in packed int16 (two targets per lane), 9 in 8-bit lanes of 32-bit
 * words (four targets per lane), size = columns per lane; 10 -> *rate = the
 * number of wrong results of the byte sign spread that 9 uses (must be 0);
 * 11..14 -> 8 with 1..4 waves per SIMD instead of 8.
 */
int dsa_probe(int which, int64_t size, double *rate);

/*
 * Sequence ingest (Section II.C.1: the data API reads FASTA and FASTQ files;
 * Section II.B.1: a converter maps them into the workers' layout).  A
 * dsa_seqset collects records streamed as text in pieces of any size and
 * maps residues to codes; its codes and offsets go to dsa_db_create (a
 * database) or to dsa_args (queries).  Host memory only; no device work.
 *   alphabets  DSA_ALPHA_PROTEIN: A R N D C Q E G H I L K M F P S T W Y V B Z X *
 *              -> 0..23 (BLOSUM62's order), other letters -> X (22);
 *              DSA_ALPHA_DNA: A C G T -> 0..3, U -> T, other letters -> N (4).
 *              Case-insensitive; on sequence lines every other byte (space,
 *              tab, CR, digit, '-', '.') is skipped.
 *   formats    decided by the first non-blank byte: '>' FASTA (header line,
 *              then sequence lines up to the next '>' at a line start), '@'
 *              FASTQ (header, sequence lines up to a '+' line, then quality
 *              lines holding exactly as many bytes as residues; a quality
 *              line may start with '@' or '+').  Qualities are not kept.
 *   names      a record's name is its header line after '>' or '@', without
 *              a trailing CR.
 * dsa_seqset_feed may be called with any split of the text; dsa_seqset_finish
 * ends the input (the last record may lack a final newline).
 * dsa_seqset_read_file feeds a whole file in 4 MiB pieces and finishes.
 * dsa_seqset_codes and dsa_seqset_name return pointers into the set, valid
 * until dsa_seqset_destroy (names are not NUL-terminated).
 * Errors: DSA_E_INVAL (bad argument, unreadable file, text before the first
 * header, a FASTQ record without its '+' line or with a quality of another
 * length than its sequence; dsa_last_error names the line or record).
 */
enum { DSA_ALPHA_PROTEIN = 1, DSA_ALPHA_DNA = 2 };
enum { DSA_FORMAT_NONE = 0, DSA_FORMAT_FASTA = 1, DSA_FORMAT_FASTQ = 2 };
typedef struct dsa_seqset dsa_seqset;
int dsa_seqset_create(int32_t alphabet, dsa_seqset **out);
int dsa_seqset_feed(dsa_seqset *set, const char *bytes, size_t len);
int dsa_seqset_finish(dsa_seqset *set);
int dsa_seqset_read_file(dsa_seqset *set, const char *path);
int dsa_seqset_info(const dsa_seqset *set, int64_t *n_seqs, int64_t *n_residues, int32_t *format);
int dsa_seqset_codes(const dsa_seqset *set, const uint8_t **codes, const int64_t **offsets);
int dsa_seqset_name(const dsa_seqset *set, int64_t index, const char **name, int64_t *len);
int dsa_seqset_destroy(dsa_seqset *set);

const char *dsa_strerror(int status);
const char *dsa_last_error(void);
int32_t dsa_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* DSA_H */
