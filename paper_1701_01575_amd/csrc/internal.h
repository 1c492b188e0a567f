// Internal types shared by the host runtime and the kernels of libdsa.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dsa {

constexpr int kWave = 64;
constexpr int kGroup = 128;          // targets per group: 64 lanes x 2 int16 halves
constexpr int kPadLen = 4;           // group column count is a multiple of this
constexpr int kMaxAlphabet = 64;     // the int32 kernels' (A + 1)^2 LDS tables stay small
constexpr int kMaxAlphabet16 = 32;   // the int16 search's pair profiles in LDS: larger alphabets run int32
constexpr int kMaxLen16 = 65532;     // int16 kernels index rows/columns with uint16
constexpr int kT32 = 16;             // strip height of the int32 kernels
constexpr int32_t kKsBase = 1 << 29;  // work-list code of strip-pipelined units
// Local-mode int16 search holds H, E and F as value + an offset of at least
// kBias16: every value is then a positive normal binary16 bit pattern, whose
// binary16 order is its integer order, so one packed binary16 three-way
// maximum does the work of two integer maxima.  The inter-sequence kernel
// adds up to kShift16 more (a per-column offset that grows by gap_extend per
// column and is taken back every few columns).  Exact while every H <=
// kLocal16Max (H + offset + s stays at most 0x7bff, the largest finite
// binary16, for s <= 127), and while H - gap_open stays normal
// (gap_open <= kLocal16GapMax) and the column offset stays within kShift16
// (gap_extend <= kLocal16ExtMax).
constexpr int kBias16 = 2048;
constexpr int kShift16 = 1024;
constexpr int kLocal16Max = 0x7b80 - kBias16 - kShift16;
constexpr int kLocal16GapMax = kBias16 - 1024;
constexpr int kLocal16ExtMax = kShift16 / 4;

enum Mode { LOCAL = 0, GLOBAL = 1, SEMIGLOBAL = 2 };

// The value of lane - 1 of the wave (0 for lane 0): one VALU op with a
// wave-wide DPP shift, where a shuffle would take an LDS round trip.  The
// wavefront kernels call it at the top of each step with every lane of a
// segment active, and a segment's first lane replaces what it receives.
__device__ __forceinline__ int lane_above(int v) {
    return __builtin_amdgcn_update_dpp(0, v, 0x138 /* wave_shr:1 */, 0xf, 0xf, false);
}
enum Ends { QB = 1, QE = 2, TB = 4, TE = 8 };

// Score of query residue gi (an index into the query code buffer) of query
// q against target code t: its residue's matrix row, or, when a
// position-specific profile is given, its own profile row.  The device
// profile holds rows of A + 1 int8 (the last column is padding), each query's
// rows followed by one padding row, so query q's row i is row
// q_off + q + i and its padding row is row q_off + q + m.
__device__ __forceinline__ int qscore(const int8_t *pssm, const int8_t *subst, const uint8_t *q_codes, int A,
                                      int64_t gi, int q, int t) {
    return pssm ? (int)pssm[(gi + q) * (A + 1) + t] : (int)subst[min((int)q_codes[gi], A - 1) * A + t];
}
constexpr int kPssmPad = -128;   // score of the profile's padding row and column

// One group of 128 length-sorted targets.
struct GroupInfo {
    int64_t off;      // first uint2 of the group's column blocks in `packed`
    int64_t bnd;      // first uint2 of the group's boundary words inside one query slot
    int32_t ncols;    // columns, multiple of 4 (max target length, rounded up)
    int32_t slot0;    // first slot: slots slot0 .. slot0+127
};

struct QueryInfo {
    int64_t off;      // into the query code buffer
    int64_t prof;     // first dword of the query's pair profile (int16 pass)
    int32_t len;      // m >= 1
    int32_t strips;   // ceil(m / T)
};

// A work unit: one query against ng consecutive groups (one wave per group
// for the int16 kernel, two for the int32 kernel).
struct SearchUnit {
    int32_t q;
    int32_t g0;
    int32_t ng;
    int32_t qslot;    // which query slot of the boundary buffer this unit uses
};

struct SearchArgs {
    const uint2 *packed;
    const GroupInfo *grp;
    const int32_t *slot_target;   // original index or -1
    const int32_t *slot_len;
    const uint8_t *pair_dec;      // AP*AP*2: compact (lo, hi) codes of a pair code
    const uint8_t *inv_map;       // AP: compact code -> matrix code, 0xff = pad
    const uint8_t *q_codes;
    const QueryInfo *qinfo;
    const int8_t *subst;          // A*A
    const int8_t *pssm;           // position-specific profile (rows of A + 1), or null
    const SearchUnit *units;
    int32_t n_units;
    int32_t A, AP, o, e, ends;
    uint2 *bnd;                   // per column and lane: (H of the strip's last row, F leaving it)
    int64_t bnd_slot_stride;      // uint2 per query slot
    const uint32_t *prof;         // pair profiles (k_profile16)
    int32_t *out_score, *out_qend, *out_tend;
    uint8_t *out_status;
    int64_t n_t;                  // output row stride (targets per query)
    int32_t *unit_flags;          // per unit: 1 = rewrite saturated results, 2 = recompute all
    const int32_t *qflag;         // per query: int16 bound fails (global / semi-global)
    int32_t *counter;             // persistent-grid work counter
    // persistent form with wavefront units: the work list, longest first;
    // entry v in [0, kKsBase) is inter-sequence unit v, v >= kKsBase is
    // strip-pipelined unit v - kKsBase (an entry of units, one group), v < 0
    // is wavefront unit -v - 1
    const int32_t *order;
    int32_t n_order;
};

// Intra-sequence (wavefront) work: long targets of long queries.  Targets
// of the length-sorted groups from `long_group0` on are also stored as pairs
// (two consecutive sorted targets, the low and high int16 halves of a lane).
struct LongPair {
    int64_t off;      // first uint16 (low code | high code << 8 per column)
    int64_t bnd;      // first uint2 of the pair's boundary words in one query slot
    int32_t ncols;    // longer of the two lengths
    int32_t slot;     // sorted slot of the low target; the high one is slot + 1
};

struct IntraUnit {
    int32_t q;
    int32_t lp0;      // first long pair; one pair per wave
    int32_t np;       // pairs in this unit (<= waves per block)
    int32_t runit;    // int32 rerun unit (q, group of these pairs)
    int32_t qslot;
    int32_t pad;
};

struct IntraArgs {
    const LongPair *pairs;
    const uint16_t *lcodes;
    const IntraUnit *units;
    int32_t n_units;
    const QueryInfo *qinfo;       // strips counted in rows of kTI
    const uint8_t *q_codes;
    const int8_t *subst;
    const int8_t *pssm;           // position-specific profile (rows of A + 1), or null
    const uint8_t *inv_map;
    int32_t A, AP, o, e, ends;
    uint2 *bnd;
    int64_t bnd_slot_stride;      // uint2 per query slot
    int32_t *out_score, *out_qend, *out_tend;
    uint8_t *out_status;
    int64_t n_t;
    const int32_t *slot_target;
    const int32_t *slot_len;
    int32_t *unit_flags;          // indexed by IntraUnit.runit
    const int32_t *qflag;
};
constexpr int kTI = 16;           // rows per lane in the wavefront kernel
constexpr int kIntraWaves = 4;    // waves (pairs) per block
hipError_t launch_intra16(const IntraArgs &a, int mode, int n_blocks, size_t lds, hipStream_t s);
size_t intra16_lds_bytes(int AP, int A);

// Strip-pipelined unit (persistent local int16 search): LDS bytes with W
// waves and AP letters.
constexpr int kKsRowPad = 16;     // int16 of padding per letter row (bank shift)
__host__ __device__ constexpr size_t ks16_lds_bytes(int W, int AP) {
    return (size_t)2 * AP * (16 * W + kKsRowPad) * 2      // two round profiles, int16
           + (size_t)(W - 1) * 2 * 4 * kWave * 8           // hand-over ring, uint2
           + (size_t)AP * AP * 4;                           // pair code -> two letters' rows
}

// Pairwise alignment (query k against target k): one pair per lane, pairs
// sorted by (strips, target length) into groups of 64 so a wave's lanes share
// the strip count.
constexpr int kTP = 16;           // rows per strip in the pairwise kernel
constexpr int kPairWaves = 4;     // waves (groups) per block
constexpr int kWfBlock = 16;      // steps per lane per block of wavefront direction codes

struct PairInfo {
    int64_t q_off, t_off;         // into the query / target code buffers
    int64_t cig_off;              // first uint32 of this pair's CIGAR region
    int64_t pssm_row;             // position-specific profile: the query's first row
    int32_t m, n;
    int32_t res;                  // output index (caller order)
    int32_t cig_cap;              // CIGAR region capacity (uint32 runs)
};

struct PairGroup {
    int64_t tb;       // first uint32 of the group's direction codes (chunk-relative)
    int64_t bnd;      // first uint2 of the group's boundary words
    int64_t tpk;      // first uint32 of the group's interleaved target codes
    int32_t ncols;    // longest target, rounded up to 4
    int32_t strips;   // shared strip count
    int32_t p0;       // first pair slot
    int32_t np;       // pairs (<= 64)
};

// A pair filled by the wavefront kernel (one wave per pair).
struct WfPair {
    int64_t tb;       // first uint2 of its direction codes (chunk-relative)
    int64_t bnd;      // first uint2 of its boundary row between passes (n entries)
    int32_t slot;     // its PairInfo and end-cell slot
    int32_t seg;      // lanes per pair: 4, 8, 16, 32 or 64
};

// One wave of the wavefront pair kernel: pairs [p0, p0 + np) of the launch's
// wavefront pairs, each on a segment of `seg` lanes (np <= 64 / seg).
struct WfWave {
    int32_t p0, np, seg, pad;
};

struct PairArgs {
    const PairInfo *pairs;
    const PairGroup *groups;
    int32_t n_groups;
    const WfPair *wf;             // wavefront pairs of this launch (walk: one thread each)
    int32_t n_wf;
    const WfWave *waves;          // wavefront waves of this launch (fill)
    int32_t n_waves;
    const uint8_t *q_codes, *t_codes;
    const int8_t *subst;
    const int8_t *pssm;           // position-specific profile (PairInfo.pssm_row), or null
    int32_t A, o, e, ends;
    int32_t traceback;
    uint32_t *tb;                 // direction codes, 4 bits per cell
    uint2 *bnd;
    uint32_t *tpk;                // interleaved target codes (4 per uint32)
    int32_t *out_score, *out_qend, *out_tend, *out_qbeg, *out_tbeg;
    uint8_t *out_status;
    int32_t *end_i, *end_j;       // per slot: 1-based end cell for the walk
    int64_t *cig_off_out;
    int32_t *cig_len_out;
    uint32_t *cigar;
};
hipError_t launch_pack_targets(const PairArgs &a, int64_t n_words, hipStream_t s);
hipError_t launch_pair32(const PairArgs &a, int mode, hipStream_t s);
hipError_t launch_walk(const PairArgs &a, int mode, int64_t slot0, int64_t n_slots, hipStream_t s);
hipError_t launch_pairwf(const PairArgs &a, int mode, hipStream_t s);
hipError_t launch_walk_wf(const PairArgs &a, int mode, hipStream_t s);
size_t pair32_lds_bytes(int A);

struct TopkArgs {
    const int32_t *score, *qend, *tend;   // full results, n_q x n_t
    const uint8_t *status;
    int64_t n_t;
    int32_t n_q, K, positive_only;
    int32_t *out_score, *out_qend, *out_tend;
    int64_t *out_tindex;
    uint8_t *out_status;
    int32_t *hit_t;                       // n_q x K hit target indices (-1 = none)
};
hipError_t launch_topk(const TopkArgs &a, hipStream_t s);

// Launchers (kernels.hip).  Return hipSuccess or the launch error.
hipError_t launch_search16(const SearchArgs &a, const IntraArgs &w, int T, int mode, int waves_per_block,
                           int n_blocks, bool persistent, size_t lds_bytes, hipStream_t s);
hipError_t launch_search32(const SearchArgs &a, int mode, int waves_per_block,
                           int n_blocks, bool persistent, size_t lds_bytes, hipStream_t s,
                           int rerun_only);

// Per-query int16 safety for global / semi-global: qflag[q] = 1 when the sum
// of positive row maxima, or the most negative reachable value, leaves the
// int16 range.
struct BoundArgs {
    const uint8_t *q_codes;
    const QueryInfo *qinfo;
    int32_t n_q;
    const int8_t *subst;
    const int8_t *pssm;
    int32_t A;
    const uint8_t *inv_map;
    int32_t AP;
    int32_t o, e, min_s;
    int64_t n_max;
    int32_t *qflag;
};
hipError_t launch_bound16(const BoundArgs &a, hipStream_t s);

struct ProfileArgs {
    const uint8_t *q_codes;
    const QueryInfo *qinfo;       // prof offsets ascending
    int32_t n_q;
    const int8_t *subst;
    const int8_t *pssm;
    int32_t A, AP;
    const uint8_t *inv_map;
    const uint8_t *pair_dec;
    uint32_t *prof;
    int64_t total_dwords;
    int32_t add;                  // added to every real score (local: gap_extend)
};
hipError_t launch_profile16(const ProfileArgs &a, int T, hipStream_t s);
hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
size_t search16_lds_bytes(int T, int AP);
size_t search32_lds_bytes(int AP);

// Results for queries of length 0 (closed forms of the boundary rows).
struct EmptyArgs {
    int32_t mode, ends, o, e;
    int64_t n_t;
    const int64_t *t_len;       // per target (original order)
    const int32_t *q_rows;      // output rows (query indices) to fill
    int32_t n_rows;
    int32_t *out_score, *out_qend, *out_tend, *out_qbeg, *out_tbeg;
    uint8_t *out_status;
};
hipError_t launch_empty_queries(const EmptyArgs &a, hipStream_t s);

}  // namespace dsa
