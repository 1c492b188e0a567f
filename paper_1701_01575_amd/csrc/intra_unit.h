// The wavefront database-search unit, shared by the standalone wavefront
// kernel (intra.hip) and the persistent search kernel (search.hip), which
// takes both kinds of unit from one longest-first work list.
#pragma once
#include "internal.h"
#include "pk16.h"

namespace dsa {

constexpr int kPassRows = kWave * kTI;   // 1024 rows per pass
constexpr int kProfStride = kPassRows + 16;  // int16 per letter row (bank shift)

constexpr int kIntraShiftExtMax = 4;  // local units use the column frame up to this gap_extend

// One unit (a query against np long target pairs, one wave per pair) by the
// whole block; every thread of the block calls it.  lds4 holds the pass
// profile and the substitution matrix.  SHIFT (local mode): the column-shifted
// frame of the inter-sequence kernel, here per lane (each lane is at its own
// column): column j is held as value + kBias16 + ((j - 1) mod R) * e, R the
// largest power of two with R * e <= kShift16, and a lane takes its frame back
// by R * e when it enters column j = kR + 1.  Lanes hand rows to each other for
// the same column, so no value changes frame in transit.
template <int MODE, bool SHIFT>
__device__ __forceinline__ void intra16_run(const IntraArgs &P, const IntraUnit &U, uint4 *lds4) {
    constexpr int T = kTI;
    int16_t *qp = reinterpret_cast<int16_t *>(lds4);                 // [AP][kProfStride]
    int8_t *sub = reinterpret_cast<int8_t *>(qp + P.AP * kProfStride);  // A*A
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int o = P.o, e = P.e, ends = P.ends, A = P.A, AP = P.AP;
    const uint32_t o2 = dup(o), e2 = dup(e);
    const QueryInfo Q = P.qinfo[U.q];
    if (MODE != LOCAL && P.qflag[U.q]) {  // int16 unsafe: the int32 pass recomputes the group
        if (tid == 0) P.unit_flags[U.runit] = 2;
        return;
    }
    for (int k = tid; k < A * A; k += blockDim.x) sub[k] = P.subst[k];

    const bool active = wave < U.np;
    LongPair LP = {0, 0, 0, 0};
    if (active) LP = P.pairs[U.lp0 + wave];
    const int m = Q.len, S = Q.strips;  // strips of kTI rows
    const int passes = (S + kWave - 1) / kWave;
    const uint8_t *qc = P.q_codes + Q.off;
    const int ncols = LP.ncols;
    int n_lo = 0, n_hi = 0;
    if (active) {
        n_lo = P.slot_len[LP.slot];
        n_hi = P.slot_len[LP.slot + 1];
    }
    const uint32_t nn = pack2(n_lo, n_hi);
    const uint16_t *codes = P.lcodes + LP.off;
    uint2 *bnd = P.bnd + (int64_t)U.qslot * P.bnd_slot_stride + LP.bnd;

    // per-lane best over this lane's strips as end-cell keys (local), or the
    // result held by the lane of the last strip (global, semi)
    uint64_t gk[2] = {end_key(0, 0, 0), end_key(0, 0, 0)};
    int gs[2] = {NEG16, NEG16}, gj[2] = {0, 0};
    bool ovf = false;
    // local: every lane works on the same two targets, so a cell scoring
    // below the best any lane has seen cannot be the end cell.  Lanes record
    // a cell only above a threshold, and every 16 steps the thresholds rise
    // to one below the wave's best (ties stay recordable; the end-key merge
    // orders them).  This keeps the end-cell branch as rare as in the
    // inter-sequence kernel.  Wb: that floor carried across passes.
    uint32_t Wb = 0;
    const uint32_t K2 = dup(kBias16), oe2 = dup(o - e);
    const int R = e > 0 ? (1 << (31 - __builtin_clz(kShift16 / e))) : (1 << 30);
    const uint32_t back2 = dup(R * e);

    for (int pass = 0; pass < passes; pass++) {
        __syncthreads();
        // single-letter profile of rows [pass*1024, pass*1024 + 1024)
        for (int k = tid; k < AP * kPassRows; k += blockDim.x) {
            const int c = k / kPassRows, r = k - c * kPassRows;
            const int i = pass * kPassRows + r;
            int v = NEG16;
            const int mc = P.inv_map[c];
            if (i < m && mc != 0xff)
                v = (P.pssm ? (int)P.pssm[(Q.off + U.q + i) * (A + 1) + mc] : (int)sub[min((int)qc[i], A - 1) * A + mc]) +
                    (SHIFT ? e : 0);
            qp[c * kProfStride + r] = (int16_t)v;
        }
        __syncthreads();
        if (!active) continue;

        const int s = pass * kWave + lane;
        const bool act = s < S;
        const bool last = (s == S - 1);
        const int i0 = s * T;
        uint32_t H[T], E[T];
        // local: values offset by the bias (and, with SHIFT, column 0 one e
        // below column 1's frame), as in the inter-sequence kernel
        const int h0 = SHIFT ? kBias16 - e : kBias16;
#pragma unroll
        for (int r = 0; r < T; r++) {
            H[r] = (MODE == LOCAL) ? dup(h0) : dup(left_value(MODE, ends, o, e, i0 + r + 1));
            E[r] = (MODE == LOCAL) ? K2 : subs(H[r], o2);
        }
        uint32_t Hd_top = (MODE == LOCAL) ? dup(h0) : dup(left_value(MODE, ends, o, e, i0));
        uint32_t cj2 = K2;  // SHIFT: this lane's frame for its current column
        // B: the recording threshold; Bs, Bj, Bi: the best cell recorded in
        // this strip (Bs = 0: none); plain values
        uint32_t B = 0, Bs = 0, Bj = 0, Bi = 0;
        if (MODE == LOCAL)
            B = maxs(Wb, pack2(max(key_score(gk[0]) - 1, 0), max(key_score(gk[1]) - 1, 0)));
        const int rlast = m - 1 - i0;
        uint32_t res = 0, Ls = 0, Lj = 0;
        if (MODE != LOCAL && last) {
            res = dup(left_value(MODE, ends, o, e, m));
            Ls = res;
        }
        const int16_t *prow = qp + lane * T;
        uint32_t outH = 0, outF = 0;
        const int nsteps = ncols + kWave - 1;
        uint32_t cnext = (act && ncols > 0) ? codes[0] : 0;
        for (int t = 0; t < nsteps; t++) {
            // lane - 1's last row and the F leaving it, computed one step ago
            uint32_t rH = (uint32_t)lane_above((int)outH);
            uint32_t rF = (uint32_t)lane_above((int)outF);
            const int j = t - lane + 1;
            const bool colok = act && j >= 1 && j <= ncols;
            const uint32_t cc = cnext;
            if (colok && j < ncols) cnext = codes[j];
            if (colok) {
                if (SHIFT && j > 1) {
                    if (((j - 1) & (R - 1)) == 0) {  // take this lane's frame back
#pragma unroll
                        for (int r = 0; r < T; r++) {
                            H[r] = subw(H[r], back2);
                            E[r] = subw(E[r], back2);
                        }
                        Hd_top = subw(Hd_top, back2);
                        cj2 = K2;
                    } else {
                        cj2 = addu(cj2, e2);
                    }
                }
                if (lane == 0) {
                    if (pass == 0) {
                        rH = (MODE == LOCAL) ? cj2 : dup(top_value(MODE, ends, o, e, j));
                        rF = (MODE == LOCAL) ? cj2 : subs(rH, o2);
                    } else {
                        const uint2 b = bnd[j - 1];
                        rH = b.x;
                        rF = b.y;
                    }
                }
                const uint32_t Hd = Hd_top;
                Hd_top = rH;
                uint32_t F = rF;
                const int clo = cc & 0xff, chi = cc >> 8;
                const uint4 *plo = reinterpret_cast<const uint4 *>(prow + clo * kProfStride);
                const uint4 *phi = reinterpret_cast<const uint4 *>(prow + chi * kProfStride);
                uint32_t sc[T];
#pragma unroll
                for (int k = 0; k < T / 8; k++) {
                    const uint4 a = plo[k], b = phi[k];
                    const uint32_t la[4] = {a.x, a.y, a.z, a.w}, hb[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
                    for (int w = 0; w < 4; w++) {
                        sc[8 * k + 2 * w] = __builtin_amdgcn_perm(hb[w], la[w], 0x05040100u);
                        sc[8 * k + 2 * w + 1] = __builtin_amdgcn_perm(hb[w], la[w], 0x07060302u);
                    }
                }
                if (MODE == LOCAL) {
                    const uint32_t frame = SHIFT ? cj2 : K2;
                    const uint32_t Bc = addu(B, frame);
                    const uint32_t nb = SHIFT ? column16_local_cs<T>(sc, H, E, Hd, F, oe2, e2, addu(cj2, e2), Bc)
                                              : column16_local<T>(sc, H, E, Hd, F, o2, e2, Bc);
                    if (nb != Bc) {
                        // the integer maximum keeps B and Bs from falling if a
                        // cell beyond the exact range (flagged below) left a
                        // non-number pattern
                        const uint32_t mask = nzmask(nb ^ Bc);
                        const uint32_t idx = first_row_of<T>(H, nb);
                        B = maxs(B, subw(nb, frame));
                        Bs = bfi(mask, B, Bs);
                        Bi = bfi(mask, addu(idx, dup(i0 + 1)), Bi);
                        Bj = bfi(mask, dup(j), Bj);
                    }
                } else {
                    column16_global<T>(sc, H, E, Hd, F, o2, e2);
                    if (last) {
                        const uint32_t vl = pick_row<T>(H, rlast);
                        const uint32_t jj = dup(j);
                        if (!(ends & TE)) {
                            res = bfi(~nzmask(jj ^ nn), vl, res);
                        } else {
                            const uint32_t vm = bfi(nzmask(subu(jj, nn)), 0x80008000u, vl);
                            const uint32_t nb = maxs(Ls, vm);
                            Lj = bfi(nzmask(nb ^ Ls), jj, Lj);
                            Ls = nb;
                        }
                    }
                }
                outH = H[T - 1];
                outF = F;
                if (lane == kWave - 1 && pass + 1 < passes) bnd[j - 1] = make_uint2(outH, outF);
            }
            if (MODE == LOCAL && ((t & 15) == 15 || t == nsteps - 1)) {
                uint32_t w = B;
#pragma unroll
                for (int d = 1; d < kWave; d <<= 1) w = maxs(w, (uint32_t)__shfl_xor((int)w, d, kWave));
                Wb = subw(w, dup(1));
                B = maxs(B, Wb);
            }
        }
        if (act) {
            if (MODE == LOCAL) {
                const int b[2] = {lo16(Bs), hi16(Bs)};
                const int bj[2] = {(int)(Bj & 0xffff), (int)(Bj >> 16)};
                const int bi[2] = {(int)(Bi & 0xffff), (int)(Bi >> 16)};
#pragma unroll
                for (int h = 0; h < 2; h++) {
                    const uint64_t kk = end_key(b[h], bj[h], bi[h]);
                    gk[h] = (b[h] > 0) ? umax64(gk[h], kk) : gk[h];
                }
            } else if (last) {
                const uint32_t fs = (ends & TE) ? Ls : res;
                const uint32_t fj = (ends & TE) ? Lj : nn;
                gs[0] = lo16(fs); gs[1] = hi16(fs);
                gj[0] = (int)(fj & 0xffff); gj[1] = (int)(fj >> 16);
            }
        }
    }
    if (!active) return;

    // combine the lanes
    int gi[2] = {0, 0};
    if (MODE == LOCAL) {
#pragma unroll
        for (int h = 0; h < 2; h++) {
            for (int w = 1; w < kWave; w <<= 1) {
                const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)gk[h], w, kWave);
                const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(gk[h] >> 32), w, kWave);
                gk[h] = umax64(gk[h], ((uint64_t)hi << 32) | lo);
            }
            gs[h] = key_score(gk[h]);
            gj[h] = key_j(gk[h]);
            gi[h] = key_i(gk[h]);
        }
    } else {
        const int src = (S - 1) % kWave;
#pragma unroll
        for (int h = 0; h < 2; h++) {
            gs[h] = __shfl(gs[h], src, kWave);
            gj[h] = __shfl(gj[h], src, kWave);
        }
    }
    if (lane == 0) {
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const int t = P.slot_target[LP.slot + h];
            if (t < 0) continue;
            const int sc = gs[h];
            int qe, te;
            if (MODE == LOCAL) {
                qe = sc > 0 ? gi[h] - 1 : -1;
                te = sc > 0 ? gj[h] - 1 : -1;
                ovf |= sc > kLocal16Max;
            } else {
                qe = m - 1;
                te = gj[h] - 1;
                ovf |= (sc >= 32767) || (sc <= -32768);
            }
            const int64_t oi = (int64_t)U.q * P.n_t + t;
            P.out_score[oi] = sc;
            if (P.out_qend) P.out_qend[oi] = qe;
            if (P.out_tend) P.out_tend[oi] = te;
            if (P.out_status) P.out_status[oi] = 0;
        }
        if (ovf) P.unit_flags[U.runit] = 1;
    }
}

template <int MODE>
__device__ __forceinline__ void intra16_unit(const IntraArgs &P, const IntraUnit &U, uint4 *lds4) {
    if constexpr (MODE == LOCAL) {
        if (P.e <= kIntraShiftExtMax) {
            intra16_run<MODE, true>(P, U, lds4);
            return;
        }
    }
    intra16_run<MODE, false>(P, U, lds4);
}

}  // namespace dsa
