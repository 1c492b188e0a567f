/*
 * CPU oracle for affine-gap (Gotoh) pairwise sequence alignment.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code, header,
 * table or helper with the GPU library and must never be called by it.
 *
 * What it computes (the paper's three algorithms, Section II.C.2: local
 * Smith-Waterman "DSW", global Needleman-Wunsch "DNW" and semi-global "DSG";
 * Section II.B.1 names affine-gap libraries for them, and Section II.B.1's
 * alignment object carries score, location and CIGAR):
 *
 *   A gap run of length L costs  open + (L-1)*extend  (0 <= extend <= open).
 *   E[i][j] = max(E[i][j-1] - e, H[i][j-1] - o)      gap in the query (D, consumes b_j)
 *   F[i][j] = max(F[i-1][j] - e, H[i-1][j] - o)      gap in the target (I, consumes a_i)
 *   H[i][j] = max([0 if local], H[i-1][j-1] + S[a_i][b_j], E[i][j], F[i][j])
 *   With a position-specific score profile P (one row of A scores per query
 *   position; the extension point for user-defined scoring next to the
 *   paper's algorithm template, Section II.C.2), S[a_i][b_j] is P[i][b_j].
 *
 *   Boundaries: H[0][0] = 0; E[i][0] = F[0][j] = -inf;
 *     local:      H[0][j] = H[i][0] = 0
 *     global:     H[0][j] = -(o+(j-1)e),  H[i][0] = -(o+(i-1)e)
 *     semiglobal: as global, except H[0][j] = 0 if the target begin is free
 *                 (TB) and H[i][0] = 0 if the query begin is free (QB).
 *   Result:
 *     local:      max(0, max H); 0 means "no alignment"
 *     global:     H[m][n]
 *     semiglobal: max over H[m][n], the last row if TE, the last column if QE
 *   End-cell rule (where several cells attain the result): smallest target
 *   end j, then smallest query end i.
 *   Traceback from the end cell in state H, ties broken
 *     zero (local) > diagonal > E (D) > F (I);   in E or F: open wins ties.
 *
 * Plain O(m*n) dynamic programming in int64 with full matrices when a
 * traceback is asked for, two rolling rows otherwise; no SIMD, no blocking.
 *
 * Pins (tests that do not run this code's formulas again):
 *   scores and end cells: brute force over every alignment of short
 *   sequences, closed forms, textbook reductions (linear gaps, LCS,
 *   Levenshtein, Kadane) and invariants; paths: membership of every CIGAR
 *   in the brute-forced optimal set, rescoring, and hand-worked cases.
 *   Parity unpinned by the paper: which optimal path is reported among
 *   equal-score paths.  The tie rule above fixes it; an independently written
 *   Python traceback (pyref.py) and the hand-worked cases agree with it.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_LOCAL 0
#define OR_GLOBAL 1
#define OR_SEMIGLOBAL 2

#define OR_QB 1
#define OR_QE 2
#define OR_TB 4
#define OR_TE 8

/* CIGAR operation codes: the BAM numbering. */
#define OP_I 1
#define OP_D 2
#define OP_EQ 7
#define OP_X 8

#define NEG (INT64_MIN / 4)

static int64_t max2(int64_t x, int64_t y) { return x > y ? x : y; }

static int64_t gap_cost(int64_t o, int64_t e, int64_t len) {
    return len <= 0 ? 0 : o + (len - 1) * e;
}

/* Is candidate end cell (i, j) with score h better than the current one
 * (score *bs at (*bi, *bj))?  Order: score descending, then j ascending,
 * then i ascending. */
static int better(int64_t h, int64_t i, int64_t j, int64_t bs, int64_t bi, int64_t bj) {
    if (h != bs) return h > bs;
    if (j != bj) return j < bj;
    return i < bi;
}

typedef struct {
    int64_t score;
    int32_t q_begin, q_end, t_begin, t_end;
    int32_t n_ops;   /* CIGAR runs of the alignment (may exceed capacity) */
    int32_t status;  /* 0 ok, 1 CIGAR truncated, -1 bad arguments, -2 out of memory */
} or_result;

/* The score of query position i (1-based) against target code c. */
static int64_t score_at(const uint8_t *a, const int8_t *S, const int8_t *P, int32_t A, int64_t i, uint8_t c) {
    return P ? (int64_t)P[(i - 1) * A + c] : (int64_t)S[(int64_t)a[i - 1] * A + c];
}

/*
 * Align query a[0..m) with target b[0..n).
 * S is an A x A int8 matrix, row = query code, column = target code; when P
 * is not NULL it holds m rows of A scores, row i - 1 scoring query position i.
 * cigar (capacity cap, may be NULL when want_tb == 0) receives the run-length
 * encoded path, len << 4 | op, in forward order.
 */
int or_align(const uint8_t *a, int64_t m, const uint8_t *b, int64_t n,
             const int8_t *S, const int8_t *P, int32_t A, int64_t o, int64_t e,
             int32_t mode, int32_t ends, int32_t want_tb,
             uint32_t *cigar, int64_t cap, or_result *res)
{
    memset(res, 0, sizeof(*res));
    res->q_begin = res->q_end = res->t_begin = res->t_end = -1;
    if (m < 0 || n < 0 || A <= 0 || o < 0 || e < 0 || e > o) { res->status = -1; return -1; }
    if (mode == OR_GLOBAL) ends = 0;
    if (mode == OR_LOCAL) ends = 0;

    const int64_t W = n + 1;
    const int64_t rows = want_tb ? (m + 1) : 2;
    int64_t *H = (int64_t *)malloc(sizeof(int64_t) * rows * W);
    int64_t *E = (int64_t *)malloc(sizeof(int64_t) * rows * W);
    int64_t *F = (int64_t *)malloc(sizeof(int64_t) * rows * W);
    if (!H || !E || !F) { free(H); free(E); free(F); res->status = -2; return -2; }
#define AT(M, i, j) (M)[((want_tb ? (i) : ((i) & 1)) * W) + (j)]

    int64_t best = (mode == OR_LOCAL) ? 0 : NEG;
    int64_t bi = 0, bj = 0;

    for (int64_t i = 0; i <= m; i++) {
        for (int64_t j = 0; j <= n; j++) {
            int64_t h, ev, fv;
            if (i == 0 && j == 0) {
                h = 0; ev = NEG; fv = NEG;
            } else if (i == 0) {
                ev = NEG; fv = NEG;
                if (mode == OR_LOCAL || (ends & OR_TB)) h = 0;
                else h = -gap_cost(o, e, j);
            } else if (j == 0) {
                ev = NEG; fv = NEG;
                if (mode == OR_LOCAL || (ends & OR_QB)) h = 0;
                else h = -gap_cost(o, e, i);
            } else {
                ev = max2(AT(E, i, j - 1) - e, AT(H, i, j - 1) - o);
                fv = max2(AT(F, i - 1, j) - e, AT(H, i - 1, j) - o);
                int64_t diag = AT(H, i - 1, j - 1) + score_at(a, S, P, A, i, b[j - 1]);
                h = max2(diag, max2(ev, fv));
                if (mode == OR_LOCAL) h = max2(h, 0);
            }
            AT(H, i, j) = h; AT(E, i, j) = ev; AT(F, i, j) = fv;

            /* end-cell candidates */
            if (mode == OR_LOCAL) {
                if (i >= 1 && j >= 1 && h > 0 && better(h, i, j, best, bi, bj)) { best = h; bi = i; bj = j; }
            } else {
                int cand = (i == m && j == n);
                if (mode == OR_SEMIGLOBAL) {
                    if ((ends & OR_TE) && i == m) cand = 1;
                    if ((ends & OR_QE) && j == n) cand = 1;
                }
                if (cand && (best == NEG || better(h, i, j, best, bi, bj))) { best = h; bi = i; bj = j; }
            }
        }
    }

    res->score = best;
    if (mode == OR_LOCAL && best == 0) {
        free(H); free(E); free(F);
        return 0;  /* no alignment */
    }
    res->q_end = (int32_t)(bi - 1);
    res->t_end = (int32_t)(bj - 1);

    if (want_tb) {
        /* Walk back from (bi, bj); ops are collected in reverse order. */
        int64_t maxops = m + n + 1;
        uint8_t *rev = (uint8_t *)malloc((size_t)maxops);
        if (!rev) { free(H); free(E); free(F); res->status = -2; return -2; }
        int64_t nrev = 0;
        int64_t i = bi, j = bj;
        int state = 0; /* 0 = H, 1 = E, 2 = F */
        for (;;) {
            if (state == 0) {
                if (i == 0 && j == 0) break;
                if (mode == OR_LOCAL && AT(H, i, j) == 0) break;
                if (i == 0) {
                    if (ends & OR_TB) break;
                    while (j > 0) { rev[nrev++] = OP_D; j--; }
                    break;
                }
                if (j == 0) {
                    if (ends & OR_QB) break;
                    while (i > 0) { rev[nrev++] = OP_I; i--; }
                    break;
                }
                int64_t s = score_at(a, S, P, A, i, b[j - 1]);
                if (AT(H, i, j) == AT(H, i - 1, j - 1) + s) {
                    rev[nrev++] = (a[i - 1] == b[j - 1]) ? OP_EQ : OP_X;
                    i--; j--;
                } else if (AT(H, i, j) == AT(E, i, j)) {
                    state = 1;
                } else {
                    state = 2;
                }
            } else if (state == 1) {
                rev[nrev++] = OP_D;
                if (AT(E, i, j) == AT(H, i, j - 1) - o) state = 0;
                j--;
            } else {
                rev[nrev++] = OP_I;
                if (AT(F, i, j) == AT(H, i - 1, j) - o) state = 0;
                i--;
            }
        }
        res->q_begin = (int32_t)i;
        res->t_begin = (int32_t)j;
        /* run-length encode in forward order */
        int64_t runs = 0;
        for (int64_t k = nrev - 1; k >= 0;) {
            uint8_t op = rev[k];
            int64_t len = 0;
            while (k >= 0 && rev[k] == op) { len++; k--; }
            if (runs < cap && cigar) cigar[runs] = (uint32_t)((len << 4) | op);
            runs++;
        }
        res->n_ops = (int32_t)runs;
        if (runs > cap) res->status = 1;
        free(rev);
    }
    free(H); free(E); free(F);
#undef AT
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Batches of (query index, target index) pairs over a thread pool.        */

typedef struct {
    int64_t n;
    const int64_t *qi, *ti;
    const uint8_t *q_codes; const int64_t *q_off;
    const uint8_t *t_codes; const int64_t *t_off;
    const int8_t *S; const int8_t *P; int32_t A; int64_t o, e; int32_t mode, ends, want_tb;
    int64_t *score; int32_t *coords; int32_t *n_ops; int32_t *status;
    uint32_t *cigar; const int64_t *cig_off; const int64_t *cig_cap;
    int64_t next;
    int32_t err;
} or_batch;

static void *batch_worker(void *p) {
    or_batch *B = (or_batch *)p;
    for (;;) {
        int64_t k = __atomic_fetch_add(&B->next, 1, __ATOMIC_RELAXED);
        if (k >= B->n) break;
        int64_t q = B->qi[k], t = B->ti[k];
        or_result r;
        uint32_t *cg = (B->want_tb && B->cigar) ? B->cigar + B->cig_off[k] : NULL;
        int64_t cap = (B->want_tb && B->cigar) ? B->cig_cap[k] : 0;
        int rc = or_align(B->q_codes + B->q_off[q], B->q_off[q + 1] - B->q_off[q],
                          B->t_codes + B->t_off[t], B->t_off[t + 1] - B->t_off[t],
                          B->S, B->P ? B->P + B->q_off[q] * B->A : NULL,
                          B->A, B->o, B->e, B->mode, B->ends, B->want_tb, cg, cap, &r);
        if (rc != 0) __atomic_store_n(&B->err, rc, __ATOMIC_RELAXED);
        B->score[k] = r.score;
        B->coords[4 * k + 0] = r.q_begin;
        B->coords[4 * k + 1] = r.q_end;
        B->coords[4 * k + 2] = r.t_begin;
        B->coords[4 * k + 3] = r.t_end;
        if (B->n_ops) B->n_ops[k] = r.n_ops;
        if (B->status) B->status[k] = r.status;
    }
    return NULL;
}

/*
 * Align n pairs (q_codes[q_off[qi[k]]..], t_codes[t_off[ti[k]]..]) for
 * k in [0, n) on n_threads threads.  Outputs per pair: score, coords (4 per
 * pair: q_begin, q_end, t_begin, t_end), and with want_tb the CIGAR runs at
 * cigar + cig_off[k] (capacity cig_cap[k]), run count n_ops[k], status[k].
 * pssm (NULL = score with S) holds a row of A scores per query residue, in
 * the order of q_codes.  Returns 0, or the first nonzero or_align code.
 */
int or_align_batch(int64_t n, const int64_t *qi, const int64_t *ti,
                   const uint8_t *q_codes, const int64_t *q_off,
                   const uint8_t *t_codes, const int64_t *t_off,
                   const int8_t *S, const int8_t *pssm, int32_t A, int64_t o, int64_t e,
                   int32_t mode, int32_t ends, int32_t want_tb, int32_t n_threads,
                   int64_t *score, int32_t *coords, int32_t *n_ops, int32_t *status,
                   uint32_t *cigar, const int64_t *cig_off, const int64_t *cig_cap)
{
    or_batch B;
    memset(&B, 0, sizeof(B));
    B.n = n; B.qi = qi; B.ti = ti;
    B.q_codes = q_codes; B.q_off = q_off; B.t_codes = t_codes; B.t_off = t_off;
    B.S = S; B.P = pssm; B.A = A; B.o = o; B.e = e; B.mode = mode; B.ends = ends; B.want_tb = want_tb;
    B.score = score; B.coords = coords; B.n_ops = n_ops; B.status = status;
    B.cigar = cigar; B.cig_off = cig_off; B.cig_cap = cig_cap;
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 256) n_threads = 256;
    pthread_t th[256];
    int started = 0;
    for (int t = 1; t < n_threads; t++) {
        if (pthread_create(&th[t], NULL, batch_worker, &B) == 0) started++;
        else break;
    }
    batch_worker(&B);
    for (int t = 1; t <= started; t++) pthread_join(th[t], NULL);
    return B.err;
}
