// Packed int16 pairwise fill with checkpoints, and the walk that recomputes
// from them (pair16.hip); the exact int32 wavefront kernel takes the pairs
// this fill cannot hold exactly.
#pragma once
#include "internal.h"

namespace dsa {

constexpr int kCkCols = 16;  // columns between the stored left columns of a strip

// One segment of the packed fill: pairs a and b (indices into the launch's
// wavefront pairs; b < 0 when a is alone) share the segment's w lanes
// (lanes lane0 .. lane0 + w - 1 of its wave), a in the low half of every
// packed register, b in the high half.  Strip s of the pairs is on segment
// lane s % w in pass s / w.
struct Pk16Unit {
    int32_t a, b;
    int32_t nst;    // steps per pass, a multiple of kCkCols: both pairs' checkpoints use it
    int16_t lane0, w;
};

// One wave of the packed fill: units [u0, u0 + nu), side by side.
struct Pk16Wave {
    int32_t u0, nu;
};

// Per wavefront pair (same index as the pair's WfPair): how the packed fill
// holds it.  Values are kept as value + bias; bias covers the lowest value
// the pair's recurrence can reach and hlim is the largest H whose successors
// stay exact (see pk16_bias).
struct Pk16Pair {
    int32_t nst;   // its unit's steps per pass
    int32_t bias;
    int32_t hlim;
    int32_t w;     // its unit's lanes (the checkpoint layout's strips per pass)
};

struct Pk16Args {
    const Pk16Unit *units;
    const Pk16Wave *waves;
    const int8_t *lanemap;     // per wave and lane: its unit (from the wave's u0), -1 for none
    int32_t n_waves;
    const Pk16Pair *pk;        // indexed like PairArgs::wf
    int32_t *flag;             // per wavefront pair: 1 = left to the int32 kernel
};

// Checkpoints of one pair in its region, uint32 words holding two values +
// bias (low half, high half).  First the bottom row of every strip, (H, F)
// per step, pass by pass, a step's strips side by side (so that one step of
// a wave stores consecutive words); then every kCkCols steps every strip's
// column, 16 rows of (H, E), laid out the same way.  Strip s of a pair with
// S strips is lane s % seg of pass s / seg, whose pass has
// min(seg, S - pass * seg) strips.
__host__ __device__ inline int64_t pk16_words(int64_t strips, int64_t nst) { return 2 * strips * nst; }
__host__ __device__ inline int64_t pk16_bot_at(int s, int t, int S, int seg, int nst) {
    const int p = s / seg, l = s - p * seg, nsp = (S - p * seg < seg) ? S - p * seg : seg;
    return (int64_t)p * nst * seg + (int64_t)t * nsp + l;
}
__host__ __device__ inline int64_t pk16_left_at(int s, int q, int S, int seg, int nst) {
    const int p = s / seg, l = s - p * seg, nsp = (S - p * seg < seg) ? S - p * seg : seg;
    return (int64_t)S * nst + ((int64_t)p * (nst / kCkCols) * seg + (int64_t)q * nsp + l) * kTP;
}

size_t pk16_lds_bytes(int A);
hipError_t launch_pairpk(const PairArgs &a, const Pk16Args &x, int mode, hipStream_t s);
hipError_t launch_walk_ck(const PairArgs &a, const Pk16Args &x, int mode, hipStream_t s);
// The int32 wavefront fill and walk restricted to flagged pairs (only[k] != 0
// for wavefront pair k); the packed fill's flags select them.
hipError_t launch_pairwf_only(const PairArgs &a, int mode, const int32_t *only, hipStream_t s);
hipError_t launch_walk_wf_only(const PairArgs &a, int mode, const int32_t *only, hipStream_t s);

}  // namespace dsa
