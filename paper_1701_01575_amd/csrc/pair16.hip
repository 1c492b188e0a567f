// Pairwise alignment, packed int16 (Sections II.B.1 and II.C.2: global,
// semi-global and local alignment of query k against target k).
//
// Fill (k_pairpk): the wavefront layout of the int32 kernel (a segment of w
// lanes per unit, lane l owning the 16-row strips l, l + w, ... and computing
// column t - l + 1 at step t), with two pairs per segment: pair a in the low
// half of every packed register, pair b in the high half.  A segment has as
// many lanes as strips (passes of equal width beyond 64 strips) and sits at
// any lane of its wave beside the others.  Values
// are held as value + bias, with the bias chosen per pair so that every
// value the recurrence can reach is a positive normal binary16 pattern
// (pk16_bias in the runtime): one v_pk_maximum3_f16 then takes the three-way
// maximum of H for both pairs.  Scores come from an int8 copy of the matrix
// in LDS (code A pads rows past a query and columns past a target with 0,
// which keeps padding cells within the range of the real ones).
//
// Values are also held in a frame.  Global and semi-global: the cell of
// strip row r (0-15) and column j as value + bias + e (r + 1 + j).  There
// the gap-extend decrements of E and F vanish (both become a maximum with
// h - (o - e)), the diagonal gains 2e, which the score table carries (s +
// 2e), and a strip's bottom row reaches the strip below 16e lower, in that
// strip's frame.  Local: column j alone, value + bias + e j (a frame that
// grows down the rows would break the column maximum and the zero floor):
// E loses its decrement, F keeps it, the floor of both is bias + e (j + 1)
// and the table carries s + e.  Checkpoints keep the frame and the walk
// takes it off.
//
// Instead of direction codes the fill stores checkpoints, 0.5 byte per cell
// like the codes: the bottom row of each strip (H and the F entering the next
// strip, per step) and, every kCkCols steps, the strip's column (H and the E
// of the next column for its 16 rows).  The walk (k_walk_ck) recomputes from
// them, exactly, the direction codes of the 16 x 16 tile it stands in and
// follows them to the tile's edge.  The stored columns are staggered (strip s
// on lane l stores at columns c with c + l a multiple of kCkCols), so that
// all lanes of a wave store in the same step.
//
// Range: global and semi-global pairs whose H could exceed the limit (the
// query's sum of row maxima above hlim) and local pairs whose best score
// exceeds it are flagged; the exact int32 kernels then redo them (fill with
// direction codes in the same region, and their own walk).
#include <type_traits>
#include <utility>

#include "pair16.h"
#include "pk16.h"
#include "walk.h"

namespace dsa {

namespace {

// low halves of a and b as (a, b); high halves likewise (v_perm_b32)
__device__ __forceinline__ uint32_t lo_lo(uint32_t a, uint32_t b) { return __builtin_amdgcn_perm(b, a, 0x05040100u); }
__device__ __forceinline__ uint32_t hi_hi(uint32_t a, uint32_t b) { return __builtin_amdgcn_perm(b, a, 0x07060302u); }

// H[r] for a per-lane row r, by a uniform branch per distinct r (the
// registers stay registers).
__device__ __forceinline__ uint32_t row_of16(const uint32_t (&H)[kTP], int r) {
    uint32_t v = 0;
    for (;;) {
        int u = __builtin_amdgcn_readfirstlane(r);
        asm volatile("" : "+s"(u));
        uint32_t c;
#define DSA_ROW(k) case k: c = H[k]; asm volatile("" : "+v"(c)); break;
        switch (u) {
            DSA_ROW(0) DSA_ROW(1) DSA_ROW(2) DSA_ROW(3) DSA_ROW(4) DSA_ROW(5) DSA_ROW(6) DSA_ROW(7)
            DSA_ROW(8) DSA_ROW(9) DSA_ROW(10) DSA_ROW(11) DSA_ROW(12) DSA_ROW(13) DSA_ROW(14)
            default: c = H[15]; asm volatile("" : "+v"(c)); break;
        }
#undef DSA_ROW
        if (r == u) {
            v = c;
            break;
        }
    }
    return v;
}

// Reductions over a segment of w lanes starting at wave lane lane0 (lane =
// the segment lane): a tree towards the segment's first lane, whose result
// every lane of the segment then reads.
__device__ __forceinline__ uint64_t seg_max64(uint64_t k, int lane, int w, int lane0) {
    const int wl = lane0 + lane;
    for (int d = 1; d < w; d <<= 1) {
        const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)k, wl + d);
        const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(k >> 32), wl + d);
        if (lane + d < w) k = umax64(k, ((uint64_t)hi << 32) | lo);
    }
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)k, lane0), hi = (uint32_t)__shfl((int)(uint32_t)(k >> 32), lane0);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ int seg_sum(int v, int lane, int w, int lane0) {
    const int wl = lane0 + lane;
    for (int d = 1; d < w; d <<= 1) {
        const int x = __shfl(v, wl + d);
        if (lane + d < w) v += x;
    }
    return __shfl(v, lane0);
}

// the H of 1-based row i at column 0 (0 past the query: padding rows)
__device__ __forceinline__ int left_or_pad(int mode, int ends, int o, int e, int i, int m) {
    return i <= m ? left_value(mode, ends, o, e, i) : 0;
}

}  // namespace

// The fill's score table in LDS: the matrix as int8 with row and column A
// scoring 0, rows of kPkRow(A) entries (a multiple of 4), in kPkCopies
// copies interleaved by bank: entry e of copy c is byte e % 4 of dword
// (e / 4) * kPkCopies + c.  Lane L reads copy L % kPkCopies, so the 32 lanes
// the LDS serves at once read 32 different banks whatever their entries
// (random lookups into one copy collide several ways per read).  Then the
// row maxima of the matrix (int16).
constexpr int kPkCopies = 32;
__host__ __device__ inline int kPkRow(int A) { return (A + 1 + 3) & ~3; }
// Then, per target code 0..255 and 256 (past a target), the byte offset of
// its column in the table (uint16).
constexpr int kPkCodes = 257;
size_t pk16_lds_bytes(int A) {
    return (size_t)kPkCopies * (A + 1) * kPkRow(A) + (size_t)(A + 1) * 2 + 16 + kPkCodes * 2 + 16;
}

// SH: the row shift below, set by the launcher for semi-global calls with a
// free target begin (a template flag, so that the other instantiations keep
// no trace of it and this one none of the per-lane last-row select)
template <int MODE, bool TB, bool SH>
__global__ void __launch_bounds__(kPairWaves * kWave) __attribute__((amdgpu_waves_per_eu(3))) k_pairpk(PairArgs P, Pk16Args X) {
    constexpr int T = kTP;
    extern __shared__ uint32_t smw[];
    const int A = P.A, SS = P.A + 1, RW = kPkRow(A);
    const int nd = SS * RW / 4;  // dwords of one copy
    for (int k = threadIdx.x; k < nd * kPkCopies; k += blockDim.x) {
        const int d = k / kPkCopies;
        uint32_t v = 0;
#pragma unroll
        for (int x = 0; x < 4; x++) {
            const int en = 4 * d + x, r = en / RW, c = en - r * RW;
            int sc = (r < A && c < A) ? (int)P.subst[r * A + c] : 0;
            sc += (MODE == LOCAL ? 1 : 2) * P.e;  // the diagonal's step between frames
            v |= (uint32_t)(uint8_t)(int8_t)sc << (8 * x);
        }
        smw[k] = v;
    }
    uint16_t *rmx = reinterpret_cast<uint16_t *>(smw + nd * kPkCopies);
    uint16_t *coff = rmx + ((SS + 7) & ~7);
    for (int q = threadIdx.x; q < kPkCodes; q += blockDim.x) {
        const int b = q > 255 ? A : min(q, A - 1);  // code A (scores 0) past a target
        coff[q] = (uint16_t)((b >> 2) * (4 * kPkCopies) + (b & 3));
    }
    for (int q = threadIdx.x; q < SS; q += blockDim.x) {
        int mx = 0;
        if (q < A)
            for (int c = 0; c < A; c++) mx = max(mx, (int)P.subst[q * A + c]);
        rmx[q] = (uint16_t)mx;
    }
    __syncthreads();
    const int vw = blockIdx.x * kPairWaves + (threadIdx.x >> 6);
    if (vw >= X.n_waves) return;  // no block barrier below; segments never read another segment's lanes
    const Pk16Wave V = X.waves[vw];
    const int k_seg = X.lanemap[(int64_t)vw * kWave + (threadIdx.x & 63)];
    if (k_seg < 0) return;
    const Pk16Unit U = X.units[V.u0 + k_seg];
    const int SEG = U.w, lane0 = U.lane0;
    const int lane = (int)(threadIdx.x & 63) - lane0;
    const bool hasB = U.b >= 0;
    const int ub = hasB ? U.b : U.a;
    const WfPair WA = P.wf[U.a], WB = P.wf[ub];
    const PairInfo IA = P.pairs[WA.slot], IB = P.pairs[WB.slot];
    const Pk16Pair KA = X.pk[U.a], KB = X.pk[ub];
    const int o = P.o, e = P.e, ends = P.ends;
    const int mA = IA.m, nA = IA.n;
    const int mB = hasB ? IB.m : 0, nB = hasB ? IB.n : 0;
    const int SA = (mA + T - 1) / T, SB = (mB + T - 1) / T;
    const int S = max(SA, SB), passes = (S + SEG - 1) / SEG;
    const int nmax = max(nA, nB);
    const int NST = U.nst, Q = NST / kCkCols;
    const int nsteps = nmax + SEG - 1;
    const uint8_t *qA = P.q_codes + IA.q_off, *qB = P.q_codes + IB.q_off;
    const uint8_t *tA = P.t_codes + IA.t_off, *tB = P.t_codes + IB.t_off;
    uint32_t *ckA = P.tb + 2 * WA.tb, *ckB = P.tb + 2 * WB.tb;
    uint32_t *bdA = reinterpret_cast<uint32_t *>(P.bnd + WA.bnd), *bdB = reinterpret_cast<uint32_t *>(P.bnd + WB.bnd);
    // byte offsets into the score table: row q of this lane's copy at
    // q * RB + LB, column b at (b / 4) * 4 * kPkCopies + b % 4
    const int RB = RW / 4 * 4 * kPkCopies, LB = 4 * (int)(threadIdx.x % kPkCopies);
    const uint32_t bias2 = pack2(KA.bias, KB.bias);
    const uint32_t o2 = dup(o), e2 = dup(e), oe2 = dup(o - e), e16 = dup(16 * e);
    const char *smb = reinterpret_cast<const char *>(smw);

    // global and semi-global: H never exceeds the query's sum of positive row
    // maxima; a pair whose sum exceeds its limit goes to int32 at once
    int flagA = 0, flagB = 0;
    if (MODE != LOCAL) {
        int uA = 0, uB = 0;
        for (int i = lane; i < mA; i += SEG) uA += rmx[min((int)qA[i], A - 1)];
        for (int i = lane; i < mB; i += SEG) uB += rmx[min((int)qB[i], A - 1)];
        uA = seg_sum(uA, lane, SEG, lane0);
        uB = seg_sum(uB, lane, SEG, lane0);
        flagA = uA > KA.hlim;
        flagB = uB > KB.hlim;
    }
    const bool skip = flagA && (flagB || !hasB);

    uint64_t gkA = end_key(0, 0, 0), gkB = gkA;  // local: the lane's best over its strips
    int gsA = 0, gjA = 0, gsB = 0, gjB = 0;      // global / semi: held by the lane of the last strip
    const bool qe_free = (MODE == SEMIGLOBAL) && (ends & QE);
    // semi-global with a free target begin: each pair's rows sit pad = 16 S
    // - m strip rows down, below virtual rows of score 0 (code A) with H = 0
    // at column 0.  With the top row free those rows reproduce it exactly
    // (H stays 0 in them and the F entering row 1 is -o), and the query's
    // last row is row 15 of the pair's last strip, one register
    constexpr bool shifted = SH;
    const int padA = shifted ? SA * T - mA : 0, padB = shifted ? SB * T - mB : 0;
    int QsA = PAD32, QiA = 0, QsB = PAD32, QiB = 0;
    for (int pass = 0; pass < passes && !skip; pass++) {
        const int s = pass * SEG + lane;
        const int i0 = s * T;
        const int i0A = i0 - padA, i0B = i0 - padB;  // the rows above the strip, per pair
        const bool act = s < S;
        const bool lastA = (s == SA - 1), lastB = (s == SB - 1);
        const int rlastA = mA - 1 - i0A, rlastB = mB - 1 - i0B;
        uint32_t rowAB[T], H[T], E[T];
#pragma unroll
        for (int r = 0; r < T; r++) {
            const int iA = i0A + r, iB = i0B + r;  // 0-based query rows (virtual below 0)
            const int cA = (iA >= 0 && iA < mA) ? min((int)qA[iA], A - 1) : A;
            const int cB = (iB >= 0 && iB < mB) ? min((int)qB[iB], A - 1) : A;
            rowAB[r] = pack2(cA * RB + LB, cB * RB + LB);
            H[r] = addu(pack2(left_or_pad(MODE, ends, o, e, max(iA + 1, 0), mA),
                              left_or_pad(MODE, ends, o, e, max(iB + 1, 0), mB)),
                        bias2);
            if (MODE != LOCAL) H[r] = addu(H[r], dup((r + 1) * e));  // column 0's frame
            E[r] = (MODE == LOCAL) ? addu(bias2, e2) : subw(H[r], oe2);  // E of column 1, in its frame
        }
        uint32_t Hd_top = addu(pack2(left_or_pad(MODE, ends, o, e, max(i0A, 0), mA),
                                     left_or_pad(MODE, ends, o, e, max(i0B, 0), mB)),
                               bias2);
        // local: the strip's best in the frame of the lane's current column
        // (advanced by e every step, whether or not the lane is active),
        // its row and column, and phi = bias + e (j + 1), the floor of E and
        // F in that frame; column j = t - lane + 1 at step t
        uint32_t Bv = subw(bias2, mulu(dup(lane), e2)), Bi2 = 0, Bj2 = 0;
        uint32_t phi = addu(Bv, e2);
        int resA = 0, LsA = 0, LjA = 0, resB = 0, LsB = 0, LjB = 0;
        if (MODE != LOCAL) {
            if (lastA) { resA = left_value(MODE, ends, o, e, mA); LsA = resA; }
            if (lastB) { resB = left_value(MODE, ends, o, e, mB); LsB = resB; }
        }
        uint32_t outH = 0, outF = 0;
        // this lane's checkpoint words: step t of the bottom row at
        // bot + t * nsp, the q-th stored column at left + q * nsp * 16
        const int nspA = min(SEG, SA - pass * SEG), nspB = min(SEG, SB - pass * SEG);
        const int64_t botA = (int64_t)pass * NST * SEG + lane, botB = botA;
        const int64_t lftA = (int64_t)SA * NST + ((int64_t)pass * Q * SEG + lane) * T;
        const int64_t lftB = (int64_t)SB * NST + ((int64_t)pass * Q * SEG + lane) * T;
        // the previous pass's last strip (lane 0 reads it): column j of its
        // bottom row at prv + (j + SEG - 2) * SEG (with checkpoints), or bd[j - 1]
        const int prv = (pass - 1) * NST * SEG + (SEG - 1);
        const bool rdA = lane == 0 && pass > 0 && s < SA, rdB = lane == 0 && pass > 0 && s < SB;
        // one step ahead: the raw target codes of the lane's next column (256
        // past a target) and lane 0's next boundary words; a load is first
        // used one step after it is issued
        // A half with no such strip or column gets H = 0 and F = -o there,
        // which keeps its padding cells within range
        const uint32_t w0A = pack2(KA.bias, KA.bias - o), w0B = pack2(KB.bias, KB.bias - o);
        uint32_t ca = 256u, cb = 256u, wa = w0A, wb = w0B;
        auto fetch_col = [&](int j) {
            ca = 256u;
            cb = 256u;
            if (act && j >= 1 && j <= nA) ca = tA[j - 1];
            if (act && j >= 1 && j <= nB) cb = tB[j - 1];
            wa = w0A;
            wb = w0B;
            if (TB) {
                if (rdA && j >= 1 && j <= nA) wa = ckA[prv + (j + SEG - 2) * SEG];
                if (rdB && j >= 1 && j <= nB) wb = ckB[prv + (j + SEG - 2) * SEG];
            } else {
                if (rdA && j >= 1 && j <= nA) wa = bdA[j - 1];
                if (rdB && j >= 1 && j <= nB) wb = bdB[j - 1];
            }
        };
        fetch_col(1 - lane);
        // the column offsets of the codes in flight, looked up at the end of
        // the step that loaded them (their loads are back by then)
        uint32_t oa = coff[ca], ob = coff[cb];
        for (int t = 0; t < nsteps; t++) {
            if (MODE == LOCAL) {
                Bv = addu(Bv, e2);
                phi = addu(phi, e2);
            }
#pragma unroll
            for (int r = 0; r < T; r++) asm volatile("" : "+v"(rowAB[r]));  // the two row offsets stay one register
            uint32_t rH = (uint32_t)lane_above((int)outH);
            uint32_t rF = (uint32_t)lane_above((int)outF);
            const int j = t - lane + 1;
            const uint32_t oa0 = oa, ob0 = ob, wa0 = wa, wb0 = wb;
            fetch_col(j + 1);
            if (act && j >= 1 && j <= nmax) {
                if (lane == 0) {
                    if (pass == 0) {  // the top boundary row (0 past a target)
                        const int tv = top_value(MODE, ends, o, e, j);
                        rH = addu(pack2(j <= nA ? tv : 0, j <= nB ? tv : 0), bias2);
                        if (MODE == LOCAL) {
                            rH = subw(phi, e2);  // 0 in the frame: bias + e j
                            rF = subw(rH, o2);
                        } else {
                            rH = addu(rH, dup(e * j));
                            rF = subw(rH, oe2);
                        }
                    } else {
                        rH = lo_lo(wa0, wb0);
                        rF = hi_hi(wa0, wb0);
                    }
                }
                // the columns' offsets in the score table
                const int bA2 = (int)oa0, bB2 = (int)ob0;
                uint32_t Hd = Hd_top;
                Hd_top = rH;
                uint32_t F = rF;
                uint32_t cm = Bv, held = 0;
                // scores four rows ahead: the LDS reads of the next group of
                // four rows are in flight while the current group computes
                uint32_t na[4], nb[4], cur[4];
                auto fetch = [&](int g) {
#pragma unroll
                    for (int x = 0; x < 4; x++) {
                        const uint32_t ra = rowAB[4 * g + x];
                        na[x] = (uint32_t)(int)*reinterpret_cast<const int8_t *>(smb + (ra & 0xffffu) + bA2);
                        nb[x] = (uint32_t)(int)*reinterpret_cast<const int8_t *>(smb + (ra >> 16) + bB2);
                    }
                };
                fetch(0);
#pragma unroll
                for (int r = 0; r < T; r++) {
                    if ((r & 3) == 0) {
#pragma unroll
                        for (int x = 0; x < 4; x++) cur[x] = lo_lo(na[x], nb[x]);
                        if (r + 4 < T) fetch((r >> 2) + 1);
                        __builtin_amdgcn_sched_barrier(0);
                    }
                    const uint32_t t2 = addu(Hd, cur[r & 3]);
                    Hd = H[r];
                    const uint32_t h = max3h(t2, E[r], F);
                    if (MODE == LOCAL) {
                        if (r & 1) cm = max3h(cm, held, h);
                        else held = h;
                    }
                    const uint32_t hx = subw(h, oe2);  // in the frame E and F share h - (o - e)
                    if (MODE == LOCAL) {  // E loses its decrement, F (in this column's frame) keeps it
                        E[r] = max3h(E[r], hx, phi);
                        F = subw(max3h(F, hx, phi), e2);
                    } else {              // and in the row frame F loses it too
                        E[r] = maxu(E[r], hx);
                        F = maxu(F, hx);
                    }
                    H[r] = h;
                }
                // keep the E updates in the column's block, between the F
                // chain's steps, rather than sunk past the end-cell branches
#pragma unroll
                for (int r = 0; r < T; r++) asm volatile("" : "+v"(E[r]));
                if (MODE == LOCAL && TB) {
                    // with traceback only the column of the strip's best is
                    // kept, without a branch: the walk recomputes that tile
                    // and finds the row there.  A value past the finite
                    // binary16 range (the frame can take padding columns
                    // there before the best itself) flags the pair: shifting
                    // the best back out of the frame would hide it
                    Bj2 = bfi(nzmask(cm ^ Bv), dup(j), Bj2);
                    Bv = cm;
                    if (maxu(cm, 0x7bff7bffu) != 0x7bff7bffu) {
                        if ((cm & 0xffffu) >= 0x7c00u) flagA = 1;
                        if ((cm >> 16) >= 0x7c00u) flagB = 1;
                    }
                } else if (MODE == LOCAL) {
                    const uint32_t d = cm ^ Bv;  // nonzero in a half whose best grew
                    if (d) {
                        const uint32_t mk = nzmask(d);
                        const uint32_t row = first_row_of(H, cm);
                        Bi2 = bfi(mk, addu(row, dup(i0 + 1)), Bi2);
                        Bj2 = bfi(mk, dup(j), Bj2);
                        Bv = cm;
                        if ((cm & 0xffffu) >= 0x7c00u) flagA = 1;
                        if ((cm >> 16) >= 0x7c00u) flagB = 1;
                    }
                } else {
                    if (lastA && j <= nA && ((ends & TE) || j == nA)) {
                        const uint32_t hl = shifted ? H[T - 1] : row_of16(H, rlastA);
                        const int v = (int)(hl & 0xffffu) - KA.bias - e * (rlastA + 1 + j);
                        if (!(ends & TE)) resA = v;
                        else if (v > LsA) { LsA = v; LjA = j; }
                    }
                    if (lastB && j <= nB && ((ends & TE) || j == nB)) {
                        const uint32_t hl = shifted ? H[T - 1] : row_of16(H, rlastB);
                        const int v = (int)(hl >> 16) - KB.bias - e * (rlastB + 1 + j);
                        if (!(ends & TE)) resB = v;
                        else if (v > LsB) { LsB = v; LjB = j; }
                    }
                    if (qe_free) {
                        // running row and frame counters, made opaque so that
                        // no per-row constant is kept live through the step loop
                        if (j == nA && s < SA) {
                            int iA = mA - rlastA, fr = KA.bias + e * (1 + j);  // 1-based row of strip row 0
                            asm volatile("" : "+v"(iA), "+v"(fr));
#pragma unroll
                            for (int r = 0; r < T; r++, iA++, fr += e) {
                                const int v = (int)(H[r] & 0xffffu) - fr;
                                if (iA >= 1 && iA <= mA && v > QsA) { QsA = v; QiA = iA; }
                            }
                        }
                        if (j == nB && s < SB) {
                            int iB = mB - rlastB, fr = KB.bias + e * (1 + j);
                            asm volatile("" : "+v"(iB), "+v"(fr));
#pragma unroll
                            for (int r = 0; r < T; r++, iB++, fr += e) {
                                const int v = (int)(H[r] >> 16) - fr;
                                if (iB >= 1 && iB <= mB && v > QsB) { QsB = v; QiB = iB; }
                            }
                        }
                    }
                }
                // the bottom row in the frame of the strip below's row above
                // (16 rows up): H at e j, the F entering it at e (j + 1)
                outH = (MODE == LOCAL) ? H[T - 1] : subw(H[T - 1], e16);
                outF = (MODE == LOCAL) ? F : subw(F, e16);
                if (TB) {
                    // this step's bottom row, and every kCkCols steps the strip's column
                    if (s < SA) ckA[botA + (int64_t)t * nspA] = lo_lo(outH, outF);
                    if (s < SB) ckB[botB + (int64_t)t * nspB] = hi_hi(outH, outF);
                } else if (lane == SEG - 1 && pass + 1 < passes) {
                    if (j <= nA) bdA[j - 1] = lo_lo(outH, outF);
                    if (j <= nB) bdB[j - 1] = hi_hi(outH, outF);
                }
            }
            if (TB && ((t + 1) & (kCkCols - 1)) == 0) {
                const int q = (t + 1) / kCkCols - 1;
                if (s < SA) {
                    uint4 *d = reinterpret_cast<uint4 *>(ckA + lftA + (int64_t)q * nspA * T);
#pragma unroll
                    for (int x = 0; x < T / 4; x++)
                        d[x] = make_uint4(lo_lo(H[4 * x], E[4 * x]), lo_lo(H[4 * x + 1], E[4 * x + 1]),
                                          lo_lo(H[4 * x + 2], E[4 * x + 2]), lo_lo(H[4 * x + 3], E[4 * x + 3]));
                }
                if (s < SB) {
                    uint4 *d = reinterpret_cast<uint4 *>(ckB + lftB + (int64_t)q * nspB * T);
#pragma unroll
                    for (int x = 0; x < T / 4; x++)
                        d[x] = make_uint4(hi_hi(H[4 * x], E[4 * x]), hi_hi(H[4 * x + 1], E[4 * x + 1]),
                                          hi_hi(H[4 * x + 2], E[4 * x + 2]), hi_hi(H[4 * x + 3], E[4 * x + 3]));
                }
            }
            oa = coff[ca];
            ob = coff[cb];
        }
        if (act) {
            if (MODE == LOCAL) {
                // the best out of the frame of the last step's column
                const uint32_t Bu = subw(Bv, mulu(dup(nsteps - lane), e2));
                const int bA = (int)(Bu & 0xffffu), bB = (int)(Bu >> 16);
                if (bA > KA.bias + KA.hlim) flagA = 1;
                if (bB > KB.bias + KB.hlim) flagB = 1;
                // with traceback the strip's first row stands for its row (rows
                // of a lower strip all come later, and the walk finds the row)
                const int iA = TB ? i0 + 1 : (int)(Bi2 & 0xffffu), iB = TB ? i0 + 1 : (int)(Bi2 >> 16);
                if (bA > KA.bias) gkA = umax64(gkA, end_key(bA - KA.bias, (int)(Bj2 & 0xffffu), iA));
                if (bB > KB.bias) gkB = umax64(gkB, end_key(bB - KB.bias, (int)(Bj2 >> 16), iB));
            } else {
                if (lastA) {
                    if (ends & TE) { gsA = LsA; gjA = LjA; }
                    else { gsA = resA; gjA = nA; }
                }
                if (lastB) {
                    if (ends & TE) { gsB = LsB; gjB = LjB; }
                    else { gsB = resB; gjB = nB; }
                }
            }
        }
    }

    // per pair: the end cell over the segment's lanes
    int GsA, GjA, GiA, GsB, GjB, GiB;
    if (MODE == LOCAL) {
        flagA = seg_sum(flagA, lane, SEG, lane0) > 0;
        flagB = seg_sum(flagB, lane, SEG, lane0) > 0;
        gkA = seg_max64(gkA, lane, SEG, lane0);
        gkB = seg_max64(gkB, lane, SEG, lane0);
        GsA = key_score(gkA); GjA = key_j(gkA); GiA = key_i(gkA);
        GsB = key_score(gkB); GjB = key_j(gkB); GiB = key_i(gkB);
    } else {
        GsA = __shfl(gsA, lane0 + (SA > 0 ? (SA - 1) % SEG : 0));
        GjA = __shfl(gjA, lane0 + (SA > 0 ? (SA - 1) % SEG : 0));
        GsB = __shfl(gsB, lane0 + (SB > 0 ? (SB - 1) % SEG : 0));
        GjB = __shfl(gjB, lane0 + (SB > 0 ? (SB - 1) % SEG : 0));
        GiA = mA;
        GiB = mB;
        if (qe_free) {
            // the last column's best over the lanes (row 0 included), then
            // against the last row's candidate
            uint64_t qa = (lane == 0) ? end_key(top_value(MODE, ends, o, e, nA), nA, 0) : end_key(PAD32, nA, 0);
            uint64_t qb = (lane == 0) ? end_key(top_value(MODE, ends, o, e, nB), nB, 0) : end_key(PAD32, nB, 0);
            if (QsA > PAD32) qa = umax64(qa, end_key(QsA, nA, QiA));
            if (QsB > PAD32) qb = umax64(qb, end_key(QsB, nB, QiB));
            qa = seg_max64(qa, lane, SEG, lane0);
            qb = seg_max64(qb, lane, SEG, lane0);
            const uint64_t ka = umax64(end_key(GsA, GjA, GiA), qa), kb = umax64(end_key(GsB, GjB, GiB), qb);
            GsA = key_score(ka); GjA = key_j(ka); GiA = key_i(ka);
            GsB = key_score(kb); GjB = key_j(kb); GiB = key_i(kb);
        }
    }
    if (lane != 0) return;
    // the unit's records again, from memory: an opaque index keeps the
    // compiler from holding them in registers through the step loop
    int ui = V.u0 + k_seg;
    asm volatile("" : "+v"(ui));
    const Pk16Unit U2 = X.units[ui];
    for (int h = 0; h < (hasB ? 2 : 1); h++) {
        const int fl = h ? flagB : flagA;
        const int wk = h ? U2.b : U2.a;
        X.flag[wk] = fl;
        if (fl) continue;  // the int32 kernel writes this pair's results
        const int slot = P.wf[wk].slot;
        const PairInfo I = P.pairs[slot];
        int Gs = h ? GsB : GsA, Gj = h ? GjB : GjA, Gi = h ? GiB : GiA;
        const int m = I.m, n = I.n;
        if (m == 0) {  // empty query: the last row is the top boundary row
            if (MODE == LOCAL) { Gs = 0; }
            else if (MODE == SEMIGLOBAL && (ends & TE)) { Gs = 0; Gj = 0; }
            else { Gs = top_value(MODE, ends, o, e, n); Gj = n; }
            Gi = 0;
        }
        int qe, te;
        if (MODE == LOCAL) { qe = Gs > 0 ? Gi - 1 : -1; te = Gs > 0 ? Gj - 1 : -1; }
        else { qe = Gi - 1; te = Gj - 1; }
        P.out_score[I.res] = Gs;
        if (P.out_qend) P.out_qend[I.res] = qe;
        if (P.out_tend) P.out_tend[I.res] = te;
        if (P.out_status) P.out_status[I.res] = 0;  // exact in int16
        if (TB) {
            // local: -2 - the end cell's strip, whose row the walk finds (and
            // writes q_end); -1 for a score of 0
            P.end_i[slot] = (MODE == LOCAL) ? (Gs == 0 ? -1 : -2 - (Gi - 1) / T) : Gi;
            P.end_j[slot] = Gj;
        } else {
            if (P.out_qbeg) P.out_qbeg[I.res] = -1;
            if (P.out_tbeg) P.out_tbeg[I.res] = -1;
        }
    }
}

hipError_t launch_pairpk(const PairArgs &a, const Pk16Args &x, int mode, hipStream_t s) {
    if (x.n_waves <= 0) return hipSuccess;
    const int nb = (x.n_waves + kPairWaves - 1) / kPairWaves;
    const size_t lds = pk16_lds_bytes(a.A);
    // semi-global with a free target begin: the row-shifted fill (the walk
    // applies the same shift)
    const bool sh = mode == SEMIGLOBAL && (a.ends & Ends::TB);
#define LP(MODE, TBV, SHV) hipLaunchKernelGGL((k_pairpk<MODE, TBV, SHV>), dim3(nb), dim3(kPairWaves * kWave), lds, s, a, x)
    if (a.traceback) {
        if (mode == LOCAL) LP(LOCAL, true, false);
        else if (mode == GLOBAL) LP(GLOBAL, true, false);
        else if (sh) LP(SEMIGLOBAL, true, true);
        else LP(SEMIGLOBAL, true, false);
    } else {
        if (mode == LOCAL) LP(LOCAL, false, false);
        else if (mode == GLOBAL) LP(GLOBAL, false, false);
        else if (sh) LP(SEMIGLOBAL, false, true);
        else LP(SEMIGLOBAL, false, false);
    }
#undef LP
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Walk from checkpoints: 16 lanes per pair, four pairs per block.  At each
// step the pair stands in the tile of strip s = (i - 1) / 16 between the
// stored column c0 < j (or column 0) and column j.  The group recomputes the
// tile's rows (16 s, i] and columns (c0, j] as a wavefront over its lanes
// (lane r owns row 16 s + r + 1 and takes the row above from lane r - 1 by a
// DPP row shift), starting from the stored left column, the bottom row of
// strip s - 1 (or the top boundary) and the matrix; every lane keeps its
// row's 4-bit direction codes (those of the int32 kernels: bits 0-1 where H
// came from, 0 zero, 1 diagonal, 2 E, 3 F; bit 2 E extends; bit 3 F extends)
// and puts them in LDS.  All 16 lanes then follow the same codes out of the
// tile (one of them stores the CIGAR runs).
constexpr int kCkWalkThreads = 64;
constexpr int kCkGroup = 16;

__device__ __forceinline__ int row_above(int v) {  // lane r - 1 of the 16-lane row (0 for lane 0)
    return __builtin_amdgcn_update_dpp(0, v, 0x111 /* row_shr:1 */, 0xf, 0xf, false);
}
__device__ __forceinline__ int row_next(int v) {   // lane r + 1 of the 16-lane row (0 for lane 15)
    return __builtin_amdgcn_update_dpp(0, v, 0x101 /* row_shl:1 */, 0xf, 0xf, false);
}
// lane r - 1's v in the 16-lane row, `first` in lane 0
__device__ __forceinline__ int row_shr1(int first, int v) {
    return __builtin_amdgcn_update_dpp(first, v, 0x111 /* row_shr:1 */, 0xf, 0xf, false);
}
// One step of a prefix maximum down the 16 lanes of a row: max(v, lane r -
// K's v), v itself in lanes r < K.  The shifted-in value defaults to the
// maximum's identity, which lets the compiler fold the shift into the
// maximum (v_max_i32 with a DPP operand).
template <int K>
__device__ __forceinline__ int row_max_shr(int v) {
    return max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x110 + K /* row_shr:K */, 0xf, 0xf, false));
}
// f(integral_constant<int, X>) for X in the sequence, in order
template <int... X, class Fn>
__device__ __forceinline__ void for_cols(std::integer_sequence<int, X...>, Fn &&f) {
    (f(std::integral_constant<int, X>{}), ...);
}
// lane X's v in every lane of the 16-lane row
template <int X>
__device__ __forceinline__ int bcast16(int v) {
    return __builtin_amdgcn_update_dpp(0, v, 0x150 + X /* row_newbcast:X */, 0xf, 0xf, false);
}

template <int MODE>
__global__ void __launch_bounds__(kCkWalkThreads) k_walk_ck(PairArgs P, Pk16Args X) {
    // per lane: its row's 16 cells, one byte each (the 4-bit code, bit 4 = residues equal)
    __shared__ uint32_t tile[kCkWalkThreads * kCkCols / 4];
    __shared__ int16_t sm[(kMaxAlphabet16 + 1) * (kMaxAlphabet16 + 1)];
    const int A = P.A;
    for (int k = threadIdx.x; k < A * A; k += blockDim.x) sm[k] = (int16_t)P.subst[k];
    __syncthreads();
    const int r = threadIdx.x & (kCkGroup - 1);
    const int gbase = threadIdx.x & ~(kCkGroup - 1);  // the group's first thread
    const int k = blockIdx.x * (kCkWalkThreads / kCkGroup) + (threadIdx.x / kCkGroup);
    if (k >= P.n_wf) return;  // no block barrier below; groups never read another group's lanes
    if (X.flag[k]) return;    // walked by the int32 path
    const WfPair W = P.wf[k];
    const PairInfo I = P.pairs[W.slot];
    const Pk16Pair KP = X.pk[k];
    const int o = P.o, e = P.e, ends = P.ends;
    const int m = I.m, n = I.n, S = (m + kTP - 1) / kTP;
    const int seg = KP.w, NST = KP.nst, bias = KP.bias;
    const uint32_t *ck = P.tb + 2 * W.tb;
    const uint8_t *qc = P.q_codes + I.q_off, *tc = P.t_codes + I.t_off;
    RunWriter Wr{P.cigar, I.cig_off, I.cig_off + I.cig_cap};
    Wr.store = (r == 0);
    int i = P.end_i[W.slot], j = P.end_j[W.slot];
    if (i == -1) {  // local alignment of score 0: nothing to trace
        if (r == 0) {
            if (P.out_qbeg) P.out_qbeg[I.res] = -1;
            if (P.out_tbeg) P.out_tbeg[I.res] = -1;
            P.cig_off_out[I.res] = I.cig_off;
            P.cig_len_out[I.res] = 0;
        }
        return;
    }
    uint8_t *mine = reinterpret_cast<uint8_t *>(tile) + kCkCols * threadIdx.x;
    const uint8_t *grp = reinterpret_cast<const uint8_t *>(tile) + kCkCols * gbase;
    int state = 0;  // 0 = H, 1 = E, 2 = F
    int budget = 2 * (m + n) + 4;
    // local: the fill gave the end cell's strip (-2 - s) and column; its row
    // is the first of the strip whose H in that column is the score, found
    // in the first tile (until then i stands at the strip's last row)
    int rs = -1;
    if (MODE == LOCAL && i <= -2) {
        rs = -2 - i;
        i = min(rs * kTP + kTP, m);
    }
    // the fill's row shift (semi-global with a free target begin): rows sit
    // pad strip rows down, below virtual rows of score 0
    const int pad = (MODE == SEMIGLOBAL && (ends & Ends::TB)) ? S * kTP - m : 0;
    for (;;) {
        if (i == 0 || j == 0) {  // on the boundary, in state H
            if (MODE != LOCAL) {
                if (i == 0 && j > 0 && !(ends & TB)) { Wr.emit(OP_D, (uint32_t)j); j = 0; }
                else if (j == 0 && i > 0 && !(ends & QB)) { Wr.emit(OP_I, (uint32_t)i); i = 0; }
            }
            break;
        }
        if (--budget < 0) break;
        const int s = (i + pad - 1) / kTP, i0 = s * kTP - pad, l = s % seg;  // i0: the row above the tile
        int c0 = j - 1 - ((j - 1 + l) & (kCkCols - 1));
        if (c0 < 1) c0 = 0;
        const int nr = i - i0, nc = j - c0;  // 1 .. 16 each
        // lane r: row i0 + r + 1, its residue and left-column H and E;
        // lane x: column c0 + 1 + x, its residue and top-row H and F (the
        // bottom row of strip s - 1, or the top boundary)
        const int ri = i0 + r + 1;
        const bool virt = ri < 1;  // a virtual row: score 0, H 0 at column 0
        const int qcode = (r < nr && !virt) ? (int)qc[ri - 1] : 0;
        const int qrow = min(qcode, A - 1) * A;
        int Hl, El;
        if (c0 >= 1) {
            const uint32_t w = ck[pk16_left_at(s, (c0 + l) / kCkCols - 1, S, seg, NST) + r];
            Hl = (int)(w & 0xffffu) - bias;
            El = (int)(w >> 16) - bias;
            // the fill's frame: H(r, c0) at e (r + 1 + c0) (local: e c0), E of c0 + 1 one e above
            const int fr = e * ((MODE == LOCAL ? 0 : r + 1) + c0);
            Hl -= fr;
            El -= fr + e;
        } else {
            Hl = left_value(MODE, ends, o, e, max(ri, 0));
            El = (MODE == LOCAL) ? 0 : Hl - o;
        }
        const int lp = (s + seg - 1) % seg;  // lane of strip s - 1 in the fill
        int colH = 0, colF = 0, colT = 0;
        if (r < nc) {
            const int c = c0 + 1 + r;
            colT = (int)tc[c - 1];
            if (s == 0) {
                colH = top_value(MODE, ends, o, e, c);
                colF = colH - o;
            } else {
                const uint32_t w = ck[pk16_bot_at(s - 1, c + lp - 1, S, seg, NST)];
                colH = (int)(w & 0xffffu) - bias;
                colF = (int)(w >> 16) - bias;
                // the row above at e c, the F entering the strip at e (c + 1) (local: e c)
                colH -= e * c;
                colF -= e * (MODE == LOCAL ? c : c + 1);
            }
        }
        int corner;  // H(i0, c0), the diagonal of row i0 + 1 in column c0 + 1
        if (s == 0) corner = top_value(MODE, ends, o, e, c0);
        else if (c0 == 0) corner = left_value(MODE, ends, o, e, max(i0, 0));
        else corner = (int)(ck[pk16_bot_at(s - 1, c0 + lp - 1, S, seg, NST)] & 0xffffu) - bias - e * c0;
        // the tile column by column, all 16 rows at once.  F runs down a
        // column as a prefix maximum: with hp = max(diagonal + s, E[, 0]),
        // F(row r) = max(Ftop - r e, max over k < r of hp(k) - o - (r-1-k) e)
        // [, 0], since where F wins in a row H - o is below F - e (o >= e),
        // so the recurrence can drop F from the H it passes down.  The row
        // above comes from lane r - 1 by DPP row shifts, lane 0 takes the
        // strip above's row; a column's residue and top words are
        // broadcast from its lane
        int Hprev = Hl;   // H(i, c - 1)
        int E = El;       // E(i, c)
        int dtop = corner;  // H(i0, c - 1): lane 0's diagonal
        const int re = r * e;
        int hj = 0;  // this row's H in column j, the tile's last
        for_cols(std::make_integer_sequence<int, kCkCols>{}, [&](auto xc) {
            constexpr int x = decltype(xc)::value;
            if (x >= nc) return;  // uniform in a 16-lane group
            const int T = bcast16<x>(colT), htop = bcast16<x>(colH), ftop = bcast16<x>(colF);
            const int diag = row_shr1(dtop, Hprev);
            const int t = diag + (virt ? 0 : (int)sm[qrow + min(T, A - 1)]);
            int hp = max(t, E);
            if (MODE == LOCAL) hp = max(hp, 0);
            int Y = row_shr1(ftop - e, hp - o + re);  // lane r: row r - 1's term, lane 0: the top's
            Y = row_max_shr<1>(Y);
            Y = row_max_shr<2>(Y);
            Y = row_max_shr<4>(Y);
            Y = row_max_shr<8>(Y);
            int F = Y - re + e;
            if (MODE == LOCAL) F = max(F, 0);
            const int h = max(hp, F);
            const int hup = row_shr1(htop, h);  // H(i - 1, c)
            uint32_t code = (h == t) ? 1u : ((h == E) ? 2u : 3u);
            if (MODE == LOCAL && h == 0) code = 0u;
            code |= (E > Hprev - o) ? 4u : 0u;  // E(i, c) extends E(i, c - 1)
            code |= (F > hup - o) ? 8u : 0u;    // F(i, c) extends F(i - 1, c)
            code |= (qcode == T) ? 16u : 0u;    // residues equal (= or X on the diagonal)
            if (r < nr) mine[x] = (uint8_t)code;
            if (x == nc - 1) hj = h;
            int En = max(E - e, h - o);
            if (MODE == LOCAL) En = max(En, 0);
            E = En;
            Hprev = h;
            dtop = htop;
        });
        asm volatile("" ::: "memory");  // the codes are in LDS before any lane reads them
        if (MODE == LOCAL && rs >= 0) {  // the end cell's row (uniform in the group)
            const uint64_t bal = __ballot(r < nr && hj == P.out_score[I.res]);
            const uint32_t g = (uint32_t)(bal >> (gbase & 63)) & 0xffffu;
            if (g) i = i0 + __builtin_ctz(g) + 1;
            rs = -1;
            if (r == 0 && P.out_qend) P.out_qend[I.res] = i - 1;
        }
        // follow the codes out of the tile (every lane the same walk)
        bool stop = false;
        while (i > max(i0, 0) && j > c0) {
            if (--budget < 0) { stop = true; break; }
            const uint32_t code = grp[kCkCols * (i - i0 - 1) + (j - c0 - 1)];
            const uint32_t src = code & 3u;
            if (state == 0 && src == 0u) { stop = true; break; }
            // one move per step, the same for every lane and state: in H a
            // gap source moves on at once as that gap (E or F at this cell,
            // whose extend bit is in the same code)
            const int g = state == 0 ? (src == 1u ? 0 : (int)src - 1) : state;  // 0 diagonal, 1 E, 2 F
            Wr.emit(g == 0 ? ((code & 16u) ? OP_EQ : OP_X) : (g == 1 ? OP_D : OP_I), 1);
            i -= (g != 1);
            j -= (g != 2);
            state = g == 0 ? 0 : (g == 1 ? (int)((code >> 2) & 1u) : 2 * (int)((code >> 3) & 1u));
        }
        asm volatile("" ::: "memory");  // the next tile's codes are written after these reads
        if (stop) break;
    }
    Wr.flush();
    if (r != 0) return;
    if (P.out_qbeg) P.out_qbeg[I.res] = i;
    if (P.out_tbeg) P.out_tbeg[I.res] = j;
    P.cig_off_out[I.res] = Wr.pos;
    P.cig_len_out[I.res] = (int32_t)(I.cig_off + I.cig_cap - Wr.pos);
    if (Wr.truncated && P.out_status) P.out_status[I.res] |= 2;  // DSA_ST_TRUNCATED
}

hipError_t launch_walk_ck(const PairArgs &a, const Pk16Args &x, int mode, hipStream_t s) {
    if (a.n_wf <= 0) return hipSuccess;
    const int bs = kCkWalkThreads, per = kCkWalkThreads / kCkGroup;
    const unsigned nb = (unsigned)((a.n_wf + per - 1) / per);
    if (mode == LOCAL) hipLaunchKernelGGL(k_walk_ck<LOCAL>, dim3(nb), dim3(bs), 0, s, a, x);
    else if (mode == GLOBAL) hipLaunchKernelGGL(k_walk_ck<GLOBAL>, dim3(nb), dim3(bs), 0, s, a, x);
    else hipLaunchKernelGGL(k_walk_ck<SEMIGLOBAL>, dim3(nb), dim3(bs), 0, s, a, x);
    return hipGetLastError();
}

}  // namespace dsa
