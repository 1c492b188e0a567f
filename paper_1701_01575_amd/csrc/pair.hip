// Pairwise alignment with traceback: query k against target k, the exact
// int32 kernels.  Pairs with short queries or few cells run here one pair per
// lane (k_pair32, k_walk); longer pairs take the packed int16 wavefront fill
// and checkpoint walk of pair16.hip, and the pairs that leave its exact int16
// range come back to the int32 wavefront kernels below (k_pairwf, k_walk_wf),
// which also serve every longer pair when int16 is not used (DSA_FORCE_INT32,
// position-specific profiles, alphabets above 32 letters).
//
// Lane-per-pair fill (k_pair32): one pair per lane, exact int32, the same recurrence, modes,
// boundaries and end-cell rule as the database kernels.  Pairs are sorted by
// strip count and target length into groups of 64 so that a wave's lanes
// share the strip count; the query is cut into 16-row strips held in VGPRs,
// the boundary row between strips goes through HBM, and each lane reads its
// substitution scores from an (A+1) x (A+1) copy of the matrix in LDS (the
// extra row and column score padding as -2^30).
//
// Traceback: while filling, every cell gets a 4-bit direction code
//   bits 0-1  where H came from, in the fixed priority
//             0 = zero (local, stop), 1 = diagonal, 2 = E (gap in query, D),
//             3 = F (gap in target, I)
//   bit 2     E[i][j] extends E[i][j-1] (it is not H[i][j-1] - o; open wins ties)
//   bit 3     F[i][j] extends F[i-1][j]
// packed 8 cells per uint32 per lane.  Two bits of H source alone do not
// determine an affine-gap path; the extend bits make the walk exact.  The
// walk (k_walk, one thread per pair) starts at the end cell in state H and
// follows the codes back, run-length encoding the CIGAR into the pair's
// region from its end backwards, so the runs read forward in order.
#include <algorithm>

#include "internal.h"
#include "pair16.h"
#include "pk16.h"
#include "walk.h"

namespace dsa {

size_t pair32_lds_bytes(int A) { return (size_t)(A + 1) * (A + 1) * 4 + 16; }

// Interleave target codes per group: word (c4, lane) holds columns
// 4*c4 .. 4*c4+3 of the lane's target (code A past its end).
__global__ void k_pack_targets(PairArgs P, int64_t n_words) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n_words;
         k += (int64_t)gridDim.x * blockDim.x) {
        int lo = 0, hi = P.n_groups - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (P.groups[mid].tpk <= k) lo = mid; else hi = mid - 1;
        }
        const PairGroup G = P.groups[lo];
        const int64_t rel = k - G.tpk;
        const int c4 = (int)(rel / kWave), lane = (int)(rel % kWave);
        uint32_t w = 0;
        const PairInfo I = P.pairs[(int64_t)lo * kWave + lane];
        for (int c = 0; c < 4; c++) {
            const int j = 4 * c4 + c;
            uint32_t code = (uint32_t)P.A;
            if (lane < G.np && j < I.n) code = min((uint32_t)P.t_codes[I.t_off + j], (uint32_t)(P.A - 1));
            w |= code << (8 * c);
        }
        P.tpk[k] = w;
    }
}

hipError_t launch_pack_targets(const PairArgs &a, int64_t n_words, hipStream_t s) {
    if (n_words <= 0) return hipSuccess;
    const int bs = 256;
    const int64_t nb = std::min<int64_t>((n_words + bs - 1) / bs, 65536);
    hipLaunchKernelGGL(k_pack_targets, dim3((unsigned)nb), dim3(bs), 0, s, a, n_words);
    return hipGetLastError();
}

// PS: scores from the position-specific profile (the pair's query rows, its
// padding row for rows past the query and column A past the target), read
// from global memory; otherwise from the (A+1) x (A+1) matrix in LDS.
template <int MODE, bool TB, bool PS>
__global__ void __launch_bounds__(kPairWaves * kWave) k_pair32(PairArgs P) {
    constexpr int T = kTP;
    extern __shared__ int32_t sm[];
    const int A = P.A, SS = P.A + 1;
    if (!PS) {
        for (int k = threadIdx.x; k < SS * SS; k += blockDim.x) {
            const int r = k / SS, c = k - r * SS;
            sm[k] = (r < A && c < A) ? (int)P.subst[r * A + c] : PAD32;
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = blockIdx.x * kPairWaves + wave;
    if (g >= P.n_groups) return;  // no block barrier below this point
    const PairGroup G = P.groups[g];
    const int slot = g * kWave + lane;
    const bool act = lane < G.np;
    PairInfo I = {0, 0, 0, 0, 0, -1, 0};
    if (act) I = P.pairs[slot];
    const int o = P.o, e = P.e, ends = P.ends;
    const int m = I.m, n = I.n, S = G.strips;
    const int Sl = (m + T - 1) / T;  // this lane's own strip count (<= S)
    const uint8_t *qc = P.q_codes + I.q_off;
    const int8_t *prow = PS ? P.pssm + I.pssm_row * SS : nullptr;
    const uint32_t *tw = P.tpk + G.tpk + lane;
    uint2 *bnd = P.bnd + G.bnd + lane;
    uint32_t *tb = P.tb + G.tb + lane;
    const int ncols = G.ncols;

    int Gs = (MODE == LOCAL) ? 0 : PAD32, Gj = 0, Gi = 0;
    // free query end: the last column's best, starting from row 0
    const bool qe_free = (MODE == SEMIGLOBAL) && (ends & QE);
    int Qs = top_value(MODE, ends, o, e, n), Qi = 0;
    for (int s = 0; s < S; s++) {
        const int i0 = s * T;
        const bool first = (s == 0), wave_last = (s == S - 1), last = (s == Sl - 1);
        int rowb[T], H[T], E[T];
#pragma unroll
        for (int r = 0; r < T; r++) {
            const int i = i0 + r;
            rowb[r] = PS ? min(i, m) * SS : (i < m ? min((int)qc[i], A - 1) : A) * SS;
            H[r] = left_value(MODE, ends, o, e, i + 1);
            E[r] = H[r] - o;
        }
        int Hd_top = left_value(MODE, ends, o, e, i0);
        int B = (MODE == LOCAL) ? max(Gs - 1, 0) : 0, Bj = 0, Bi = 0;
        const int rlast = m - 1 - i0;
        int res = 0, Ls = 0, Lj = 0;
        if (MODE != LOCAL && last) { res = left_value(MODE, ends, o, e, m); Ls = res; }
        // E-extend bits of the next column, known one column early
        uint32_t eN[2] = {0u, 0u};

        // software pipeline: the next 4 columns' target codes and boundary
        // words are in flight while the current 4 compute
        const int nblk4 = ncols >> 2;
        uint32_t w4n = 0;
        uint2 bn[4];
#pragma unroll
        for (int c = 0; c < 4; c++) bn[c] = make_uint2(0u, 0u);
        if (nblk4 > 0) {
            w4n = tw[0];
            if (!first) {
#pragma unroll
                for (int c = 0; c < 4; c++) bn[c] = bnd[(int64_t)c * kWave];
            }
        }
        for (int c4 = 0; c4 < nblk4; c4++) {
            const uint32_t w4 = w4n;
            uint2 bc[4];
#pragma unroll
            for (int c = 0; c < 4; c++) bc[c] = bn[c];
            if (c4 + 1 < nblk4) {
                w4n = tw[(int64_t)(c4 + 1) * kWave];
                if (!first) {
#pragma unroll
                    for (int c = 0; c < 4; c++) bn[c] = bnd[(int64_t)(4 * c4 + 4 + c) * kWave];
                }
            }
#pragma unroll
            for (int c = 0; c < 4; c++) {
                const int j = 4 * c4 + c + 1;
                const int b = (w4 >> (8 * c)) & 0xff;
                int Hup, F;
                if (first) {
                    Hup = top_value(MODE, ends, o, e, j);
                    F = Hup - o;
                } else {
                    Hup = (int)bc[c].x;
                    F = (int)bc[c].y;
                }
                int Hd = Hd_top;
                Hd_top = Hup;
                int ho_up = Hup - o;
                int cm = 0;
                uint32_t acc[2] = {eN[0], eN[1]};
                eN[0] = 0u;
                eN[1] = 0u;
#pragma unroll
                for (int r = 0; r < T; r++) {
                    const int t = Hd + (PS ? (int)prow[rowb[r] + b] : sm[rowb[r] + b]);
                    Hd = H[r];
                    const int Ein = E[r], Fin = F;
                    int h = max(max(t, Ein), Fin);
                    if (MODE == LOCAL) { h = max(h, 0); cm = max(cm, h); }
                    const int ho = h - o;
                    const int Ee = Ein - e;
                    E[r] = max(Ee, ho);
                    F = max(Fin - e, ho);
                    H[r] = h;
                    if (TB) {
                        const int sh = 4 * (r & 7);
                        uint32_t src = (h == t) ? (1u << sh) : ((h == Ein) ? (2u << sh) : (3u << sh));
                        if (MODE == LOCAL && h == 0) src = 0u;  // extend bits of a zero cell are never read
                        const uint32_t fext = (Fin != ho_up) ? (8u << sh) : 0u;
                        acc[r >> 3] |= src | fext;
                        // E of (i, j + 1) extends iff E - e beats H - o here (open wins ties)
                        eN[r >> 3] |= (Ee > ho) ? (4u << sh) : 0u;
                    }
                    ho_up = ho;
                }
                if (TB) {
                    tb[(((int64_t)s * ncols + (j - 1)) * 2) * kWave] = acc[0];
                    tb[(((int64_t)s * ncols + (j - 1)) * 2 + 1) * kWave] = acc[1];
                }
                if (MODE == LOCAL) {
                    if (cm > B) {
                        int rr = 0;
#pragma unroll
                        for (int r = T - 1; r >= 0; r--) rr = (H[r] == cm) ? r : rr;
                        B = cm; Bj = j; Bi = i0 + rr + 1;
                    }
                } else {
                    if (last && (j == n || ((ends & TE) && j < n))) {
                        int vl = H[0];
#pragma unroll
                        for (int k = 1; k < T; k++) vl = (k == rlast) ? H[k] : vl;
                        if (!(ends & TE)) {
                            res = vl;
                        } else if (vl > Ls) {
                            Ls = vl; Lj = j;
                        }
                    }
                    if (qe_free && j == n && s < Sl) last_column_scan<T>(H, i0, m, Qs, Qi);
                }
                if (!wave_last) bnd[(int64_t)(j - 1) * kWave] = make_uint2((uint32_t)H[T - 1], (uint32_t)F);
            }
        }
        if (MODE == LOCAL) {
            const uint64_t gk = umax64(end_key(Gs, Gj, Gi), end_key(B, Bj, Bi));
            if (B > 0) { Gs = key_score(gk); Gj = key_j(gk); Gi = key_i(gk); }
        } else if (last) {
            if (ends & TE) { Gs = Ls; Gj = Lj; }
            else { Gs = res; Gj = n; }
            Gi = m;
        }
    }
    if (!act) return;
    if (qe_free && Sl > 0) {  // the last row's candidate against the last column's
        const uint64_t gk = umax64(end_key(Gs, Gj, Gi), end_key(Qs, n, Qi));
        Gs = key_score(gk); Gj = key_j(gk); Gi = key_i(gk);
    }
    if (Sl == 0) {  // empty query: the last row is the top boundary row
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
    if (P.out_status) P.out_status[I.res] = 1;  // DSA_ST_INT32: exact int32 fill
    if (TB) {
        P.end_i[slot] = (MODE == LOCAL && Gs == 0) ? -1 : Gi;
        P.end_j[slot] = Gj;
    } else {
        if (P.out_qbeg) P.out_qbeg[I.res] = -1;
        if (P.out_tbeg) P.out_tbeg[I.res] = -1;
    }
}

hipError_t launch_pair32(const PairArgs &a, int mode, hipStream_t s) {
    if (a.n_groups <= 0) return hipSuccess;
    const int nb = (a.n_groups + kPairWaves - 1) / kPairWaves;
    const size_t lds = a.pssm ? 16 : pair32_lds_bytes(a.A);
#define LP(MODE, TBV, PSV) \
    hipLaunchKernelGGL((k_pair32<MODE, TBV, PSV>), dim3(nb), dim3(kPairWaves * kWave), lds, s, a)
#define LPM(TBV, PSV) \
    if (mode == LOCAL) LP(LOCAL, TBV, PSV); else if (mode == GLOBAL) LP(GLOBAL, TBV, PSV); else LP(SEMIGLOBAL, TBV, PSV)
    if (a.pssm) {
        if (a.traceback) { LPM(true, true); } else { LPM(false, true); }
    } else {
        if (a.traceback) { LPM(true, false); } else { LPM(false, false); }
    }
#undef LPM
#undef LP
    return hipGetLastError();
}

// Wavefront fill for large pairs: one segment of SEG lanes (4 to 64) per
// pair, 64 / SEG pairs per wave, SEG chosen per wave (the waves of one launch
// mix segment widths, longest first).  Segment lane l owns rows
// [16 s, 16 s + 16) of strip s = SEG * pass + l and at step t computes
// column t - l + 1, so the row above (lane l - 1's last row one step
// earlier) and the F leaving it arrive by a DPP wave shift (a segment's
// first lane takes the boundary instead); between passes the segment's last lane hands its last row over
// through the pair's boundary row in HBM.  Exact int32, the same
// recurrence, direction codes and end-cell rule as k_pair32.  A lane's 16
// codes of one step are 64 bits, stored in blocks of kWfBlock steps per lane
// ([pass][step / 16][lane][step % 16]): a diagonal or horizontal move of the
// traceback walk then stays inside one 128-byte line 15 times out of 16.
// H[r] for a per-lane row r: lanes that share r (one per segment at most)
// take it by a uniform index, one distinct r at a time.
template <int T>
__device__ __forceinline__ int row_of(const int (&H)[T], int r) {
    static_assert(T == 16, "row_of is written for 16-row strips");
    int v = 0;
    for (;;) {
        int u = __builtin_amdgcn_readfirstlane(r);
        asm volatile("" : "+s"(u));  // keep the index uniform: branch on it, do not select per lane
        // a branch per row on the uniform index; the empty asm keeps the
        // compiler from folding the cases into an indexed load of H, which
        // would move H out of registers
        int c;
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

// only: when set, the segments of the pairs k with only[k] == 0 do nothing.
template <int MODE, bool TB, bool PS>
__global__ void __launch_bounds__(kPairWaves * kWave) k_pairwf(PairArgs P, const int32_t *only) {
    constexpr int T = kTP;
    extern __shared__ int32_t sm[];
    const int A = P.A, SS = P.A + 1;
    if (!PS) {
        for (int k = threadIdx.x; k < SS * SS; k += blockDim.x) {
            const int r = k / SS, c = k - r * SS;
            sm[k] = (r < A && c < A) ? (int)P.subst[r * A + c] : PAD32;
        }
    }
    __syncthreads();
    const int vw = blockIdx.x * kPairWaves + (threadIdx.x >> 6);
    if (vw >= P.n_waves) return;  // no block barrier below; segments never read another segment's lanes
    const WfWave V = P.waves[vw];
    const int SEG = V.seg;        // uniform across the wave
    const int lane = threadIdx.x & (SEG - 1);
    const int k_seg = (threadIdx.x & 63) / SEG;
    if (k_seg >= V.np) return;
    if (only && !only[V.p0 + k_seg]) return;
    const WfPair W = P.wf[V.p0 + k_seg];
    const PairInfo I = P.pairs[W.slot];
    const int o = P.o, e = P.e, ends = P.ends;
    const int m = I.m, n = I.n;
    const int S = (m + T - 1) / T, passes = (S + SEG - 1) / SEG;
    const int nsteps = n + SEG - 1;
    const uint8_t *qc = P.q_codes + I.q_off, *tc = P.t_codes + I.t_off;
    const int8_t *prow = PS ? P.pssm + I.pssm_row * SS : nullptr;
    uint2 *bnd = P.bnd + W.bnd;
    uint2 *tb = reinterpret_cast<uint2 *>(P.tb) + W.tb + lane * kWfBlock;
    const int nblk = (nsteps + kWfBlock - 1) / kWfBlock;

    uint64_t gk = end_key(0, 0, 0);  // local: this lane's best over its strips
    int gs = 0, gj = 0;              // global / semi: held by the lane of the last strip
    // free query end: each lane's best of the last column over its strips
    const bool qe_free = (MODE == SEMIGLOBAL) && (ends & QE);
    int Qs = PAD32, Qi = 0;
    for (int pass = 0; pass < passes; pass++) {
        const int s = pass * SEG + lane;
        const bool act = s < S, last = (s == S - 1);
        const int i0 = s * T;
        int rowb[T], H[T], E[T];
#pragma unroll
        for (int r = 0; r < T; r++) {
            const int i = i0 + r;
            rowb[r] = PS ? min(i, m) * SS : (i < m ? min((int)qc[i], A - 1) : A) * SS;
            H[r] = left_value(MODE, ends, o, e, i + 1);
            E[r] = H[r] - o;
        }
        int Hd_top = left_value(MODE, ends, o, e, i0);
        int B = 0, Bj = 0, Bi = 0;
        const int rlast = m - 1 - i0;
        int res = 0, Ls = 0, Lj = 0;
        if (MODE != LOCAL && last) { res = left_value(MODE, ends, o, e, m); Ls = res; }
        int outH = 0, outF = 0;
        // E-extend bits of the lane's next column, known one column early
        uint32_t eN[2] = {0u, 0u};
        // the next step's target code, and lane 0's next boundary word
        int cnext = (lane == 0 && act && n > 0) ? (int)tc[0] : 0;
        uint2 bnext = make_uint2(0u, 0u);
        if (lane == 0 && pass > 0 && n > 0) bnext = bnd[0];
        for (int t = 0; t < nsteps; t++) {
            int rH = lane_above(outH);
            int rF = lane_above(outF);
            const int j = t - lane + 1;
            const int cc = cnext;
            const uint2 bc = bnext;
            if (act && j >= 0 && j < n) cnext = (int)tc[j];
            if (lane == 0 && pass > 0 && j < n) bnext = bnd[j];
            if (act && j >= 1 && j <= n) {
                if (lane == 0) {
                    if (pass == 0) {
                        rH = top_value(MODE, ends, o, e, j);
                        rF = rH - o;
                    } else {
                        rH = (int)bc.x;
                        rF = (int)bc.y;
                    }
                }
                const int b = min(cc, A - 1);
                int Hd = Hd_top;
                Hd_top = rH;
                int F = rF;
                int ho_up = rH - o;
                int cm = 0;
                uint32_t acc[2] = {eN[0], eN[1]};
                eN[0] = 0u;
                eN[1] = 0u;
#pragma unroll
                for (int r = 0; r < T; r++) {
                    const int tv = Hd + (PS ? (int)prow[rowb[r] + b] : sm[rowb[r] + b]);
                    Hd = H[r];
                    const int Ein = E[r], Fin = F;
                    int h = max(max(tv, Ein), Fin);
                    if (MODE == LOCAL) { h = max(h, 0); cm = max(cm, h); }
                    const int ho = h - o;
                    const int Ee = Ein - e;
                    E[r] = max(Ee, ho);
                    F = max(Fin - e, ho);
                    H[r] = h;
                    if (TB) {
                        const int sh = 4 * (r & 7);
                        uint32_t src = (h == tv) ? (1u << sh) : ((h == Ein) ? (2u << sh) : (3u << sh));
                        if (MODE == LOCAL && h == 0) src = 0u;  // extend bits of a zero cell are never read
                        const uint32_t fext = (Fin != ho_up) ? (8u << sh) : 0u;
                        acc[r >> 3] |= src | fext;
                        // E of (i, j + 1) extends iff E - e beats H - o here (open wins ties)
                        eN[r >> 3] |= (Ee > ho) ? (4u << sh) : 0u;
                    }
                    ho_up = ho;
                }
                if (TB)
                    tb[((int64_t)pass * nblk + t / kWfBlock) * (SEG * kWfBlock) + (t % kWfBlock)] =
                        make_uint2(acc[0], acc[1]);
                if (MODE == LOCAL) {
                    if (cm > B) {
                        int rr = 0;
#pragma unroll
                        for (int r = T - 1; r >= 0; r--) rr = (H[r] == cm) ? r : rr;
                        B = cm; Bj = j; Bi = i0 + rr + 1;
                    }
                } else {
                    if (last && ((ends & TE) || j == n)) {
                        const int vl = row_of<T>(H, rlast);
                        if (!(ends & TE)) {
                            res = vl;
                        } else if (vl > Ls) {
                            Ls = vl; Lj = j;
                        }
                    }
                    if (qe_free && j == n) last_column_scan<T>(H, i0, m, Qs, Qi);
                }
                outH = H[T - 1];
                outF = F;
                if (lane == SEG - 1 && pass + 1 < passes)
                    bnd[j - 1] = make_uint2((uint32_t)outH, (uint32_t)outF);
            }
        }
        if (act) {
            if (MODE == LOCAL) {
                if (B > 0) gk = umax64(gk, end_key(B, Bj, Bi));
            } else if (last) {
                if (ends & TE) { gs = Ls; gj = Lj; }
                else { gs = res; gj = n; }
            }
        }
    }
    int Gs, Gj, Gi;
    if (MODE == LOCAL) {
        for (int d = 1; d < SEG; d <<= 1) {
            const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)gk, d, SEG);
            const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(gk >> 32), d, SEG);
            gk = umax64(gk, ((uint64_t)hi << 32) | lo);
        }
        Gs = key_score(gk); Gj = key_j(gk); Gi = key_i(gk);
    } else {
        const int src = S > 0 ? (S - 1) % SEG : 0;
        Gs = __shfl(gs, src, SEG);
        Gj = __shfl(gj, src, SEG);
        Gi = m;
        if (qe_free) {
            // the last column's best over the lanes (row 0 included), then
            // against the last row's candidate
            uint64_t qk = (lane == 0) ? end_key(top_value(MODE, ends, o, e, n), n, 0) : end_key(PAD32, n, 0);
            if (Qs > PAD32) qk = umax64(qk, end_key(Qs, n, Qi));
            for (int d = 1; d < SEG; d <<= 1) {
                const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)qk, d, SEG);
                const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(qk >> 32), d, SEG);
                qk = umax64(qk, ((uint64_t)hi << 32) | lo);
            }
            const uint64_t gk2 = umax64(end_key(Gs, Gj, Gi), qk);
            Gs = key_score(gk2); Gj = key_j(gk2); Gi = key_i(gk2);
        }
    }
    if (lane != 0) return;
    if (S == 0) {  // empty query: the last row is the top boundary row
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
    if (P.out_status) P.out_status[I.res] = 1;  // DSA_ST_INT32: exact int32 fill
    if (TB) {
        P.end_i[W.slot] = (MODE == LOCAL && Gs == 0) ? -1 : Gi;
        P.end_j[W.slot] = Gj;
    } else {
        if (P.out_qbeg) P.out_qbeg[I.res] = -1;
        if (P.out_tbeg) P.out_tbeg[I.res] = -1;
    }
}

hipError_t launch_pairwf_only(const PairArgs &a, int mode, const int32_t *only, hipStream_t s) {
    if (a.n_waves <= 0) return hipSuccess;
    const int nb = (a.n_waves + kPairWaves - 1) / kPairWaves;
    const size_t lds = a.pssm ? 16 : pair32_lds_bytes(a.A);
#define LP(MODE, TBV, PSV) \
    hipLaunchKernelGGL((k_pairwf<MODE, TBV, PSV>), dim3(nb), dim3(kPairWaves * kWave), lds, s, a, only)
#define LPM(TBV, PSV) \
    if (mode == LOCAL) LP(LOCAL, TBV, PSV); else if (mode == GLOBAL) LP(GLOBAL, TBV, PSV); else LP(SEMIGLOBAL, TBV, PSV)
    if (a.pssm) {
        if (a.traceback) { LPM(true, true); } else { LPM(false, true); }
    } else {
        if (a.traceback) { LPM(true, false); } else { LPM(false, false); }
    }
#undef LPM
#undef LP
    return hipGetLastError();
}

hipError_t launch_pairwf(const PairArgs &a, int mode, hipStream_t s) {
    return launch_pairwf_only(a, mode, nullptr, s);
}

// ---------------------------------------------------------------------------
// Traceback walk: one thread per pair slot.


// Walk one pair back from its end cell (1-based i, j; i < 0 = nothing to
// trace) through the direction codes that code(i, j) returns.
// eq(i, j) tells whether query residue i and target residue j (1-based) are
// equal.  refill(i, j) runs before every 16th step from a cell with i, j >= 1:
// the next 16 steps read only rows (i - 16, i] and columns (j - 16, j].
template <int MODE, class Code, class Eq, class Refill>
__device__ void walk_pair(const PairArgs &P, const PairInfo &I, int i, int j, Code code, Eq eq, Refill refill) {
    const int ends = P.ends;
    RunWriter W{P.cigar, I.cig_off, I.cig_off + I.cig_cap};
    if (i < 0) {  // local alignment of score 0: nothing to trace
        if (P.out_qbeg) P.out_qbeg[I.res] = -1;
        if (P.out_tbeg) P.out_tbeg[I.res] = -1;
        P.cig_off_out[I.res] = I.cig_off;
        P.cig_len_out[I.res] = 0;
        return;
    }
    int state = 0;  // 0 = H, 1 = E, 2 = F
    const int max_steps = I.m + I.n + 2;
    for (int step = 0; step < max_steps; step++) {
        if ((step & 15) == 0 && i > 0 && j > 0) refill(i, j);
        if (state == 0) {
            if (i == 0 || j == 0) {
                if (MODE == LOCAL) break;
                if (i == 0 && j > 0 && !(ends & TB)) { W.emit(OP_D, (uint32_t)j); j = 0; }
                else if (j == 0 && i > 0 && !(ends & QB)) { W.emit(OP_I, (uint32_t)i); i = 0; }
                break;
            }
        }
        if (j <= 0 || i <= 0) break;  // in a gap: codes never lead here; keeps reads in bounds
        const uint32_t c = code(i, j), src = c & 3u;
        if (state == 0 && src == 0u) break;
        // one move per step, whatever the state: in H a gap source moves on
        // at once as that gap (E or F at this cell, whose extend bit is in
        // the same code), so lanes in different states stay on one path
        const int g = state == 0 ? (src == 1u ? 0 : (int)src - 1) : state;  // 0 diagonal, 1 E, 2 F
        W.emit(g == 0 ? (eq(i, j) ? OP_EQ : OP_X) : (g == 1 ? OP_D : OP_I), 1);
        const uint32_t ext = (c >> (g == 1 ? 2 : 3)) & 1u;
        i -= (g != 1);
        j -= (g != 2);
        state = (g != 0 && ext) ? g : 0;
    }
    W.flush();
    if (P.out_qbeg) P.out_qbeg[I.res] = i;
    if (P.out_tbeg) P.out_tbeg[I.res] = j;
    P.cig_off_out[I.res] = W.pos;
    P.cig_len_out[I.res] = (int32_t)(I.cig_off + I.cig_cap - W.pos);
    if (W.truncated && P.out_status) P.out_status[I.res] |= 2;  // DSA_ST_TRUNCATED
}

// Walk of the lane-per-pair kernel's pairs: one thread per pair slot.  Like
// the wavefront walk, it fetches every 16 steps the codes of the 16x16 cells
// it can reach next (two strips x 16 columns x 2 words, 64 independent
// loads) into LDS and the residues before its position into registers.
constexpr int kLaneWalkThreads = 64;
template <int MODE>
__global__ void __launch_bounds__(kLaneWalkThreads) k_walk(PairArgs P, int64_t slot0, int64_t n_slots) {
    __shared__ uint32_t cache[kLaneWalkThreads * 64];
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_slots) return;
    const int64_t slot = slot0 + k;
    const int g = (int)(slot / kWave), lane = (int)(slot % kWave);
    const PairGroup G = P.groups[g];
    if (lane >= G.np) return;
    const PairInfo I = P.pairs[slot];
    const uint32_t *tb = P.tb + G.tb + lane;
    const int ncols = G.ncols;
    const uint8_t *qc = P.q_codes + I.q_off, *tc = P.t_codes + I.t_off;
    uint32_t *mine = cache + threadIdx.x * 64;
    int s_lo = 0, jlo = 0, qbase = 0, tbase = 0;
    uint32_t qw[4] = {0u, 0u, 0u, 0u}, tw[4] = {0u, 0u, 0u, 0u};
    auto refill = [&](int i, int j) {
        s_lo = (i - 1) / kTP - 1;
        jlo = max(j - 16, 0);
        uint32_t v[64];
#pragma unroll
        for (int c = 0; c < 2; c++) {
            const int s = s_lo + c;
#pragma unroll
            for (int x = 0; x < 16; x++) {
                const int col = jlo + x;
                const bool ok = s >= 0 && col < ncols;
#pragma unroll
                for (int h = 0; h < 2; h++)
                    v[c * 32 + x * 2 + h] = ok ? tb[(((int64_t)s * ncols + col) * 2 + h) * kWave] : 0u;
            }
        }
        qbase = max(i - 16, 0);
        tbase = max(j - 16, 0);
        load_window(qc, I.m, qbase, qw);
        load_window(tc, I.n, tbase, tw);
#pragma unroll
        for (int x = 0; x < 64; x++) mine[x] = v[x];
    };
    walk_pair<MODE>(
        P, I, P.end_i[slot], P.end_j[slot],
        [&](int ii, int jj) -> uint32_t {
            const int s = (ii - 1) / kTP, r = (ii - 1) % kTP;
            const uint32_t w = mine[(s - s_lo) * 32 + (jj - 1 - jlo) * 2 + (r >> 3)];
            return (w >> (4 * (r & 7))) & 15u;
        },
        [&](int ii, int jj) { return byte_of(qw, ii - 1 - qbase) == byte_of(tw, jj - 1 - tbase); },
        refill);
}

// Walk of the wavefront kernel's pairs: one thread per pair.  The walk is a
// chain of dependent steps, so every 16 steps each thread fetches all it
// can need next in one batch of independent loads: the up to four 128-byte
// code blocks (16 steps of one lane) covering rows (i - 16, i] and columns
// (j - 16, j] into LDS, and the 16 query and target residues before i and j
// into registers.  The 16 steps then read only LDS and registers.
constexpr int kWalkThreads = 64;

// only: when set, the pairs k with only[k] == 0 are left alone.
template <int MODE>
__global__ void __launch_bounds__(kWalkThreads) k_walk_wf(PairArgs P, const int32_t *only) {
    __shared__ uint4 cache[kWalkThreads * 4 * 8];  // per thread: 4 blocks x 128 bytes
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P.n_wf) return;
    if (only && !only[k]) return;
    const WfPair W = P.wf[k];
    const PairInfo I = P.pairs[W.slot];
    const uint2 *tb = reinterpret_cast<const uint2 *>(P.tb) + W.tb;
    const int seg = W.seg;
    const int nblk = (I.n + seg - 1 + kWfBlock - 1) / kWfBlock;
    uint4 *mine = cache + threadIdx.x * 32;
    const uint2 *mine2 = reinterpret_cast<const uint2 *>(mine);
    const uint8_t *qc = P.q_codes + I.q_off, *tc = P.t_codes + I.t_off;
    int s_lo = 0, blo0 = 0, blo1 = 0, qbase = 0, tbase = 0;
    uint32_t qw[4] = {0u, 0u, 0u, 0u}, tw[4] = {0u, 0u, 0u, 0u};
    auto refill = [&](int i, int j) {
        const int s_hi = (i - 1) / kTP;
        s_lo = s_hi - 1;
        uint4 v[4][8];
        int bl[2] = {0, 0};
#pragma unroll
        for (int c = 0; c < 2; c++) {
            const int s = s_lo + c;
            const int pass = s / seg, lane = s % seg;
            bl[c] = (max(j - 16, 0) + lane) / kWfBlock;
#pragma unroll
            for (int q = 0; q < 2; q++) {
                const int b = bl[c] + q;
                if (s >= 0 && b < nblk) {
                    const uint4 *src = reinterpret_cast<const uint4 *>(
                        tb + (((int64_t)pass * nblk + b) * seg + lane) * kWfBlock);
#pragma unroll
                    for (int x = 0; x < 8; x++) v[2 * c + q][x] = src[x];
                }
            }
        }
        blo0 = bl[0];
        blo1 = bl[1];
        qbase = max(i - 16, 0);
        tbase = max(j - 16, 0);
        load_window(qc, I.m, qbase, qw);
        load_window(tc, I.n, tbase, tw);
#pragma unroll
        for (int c = 0; c < 4; c++)
#pragma unroll
            for (int x = 0; x < 8; x++) mine[c * 8 + x] = v[c][x];
    };
    walk_pair<MODE>(
        P, I, P.end_i[W.slot], P.end_j[W.slot],
        [&](int ii, int jj) -> uint32_t {
            const int s = (ii - 1) / kTP, r = (ii - 1) % kTP;
            const int c = s - s_lo;  // 0 or 1
            const int t = jj - 1 + s % seg;
            const int slot = 2 * c + (t / kWfBlock - (c ? blo1 : blo0));
            const uint2 v = mine2[slot * kWfBlock + t % kWfBlock];
            const uint32_t w = (r < 8) ? v.x : v.y;
            return (w >> (4 * (r & 7))) & 15u;
        },
        [&](int ii, int jj) { return byte_of(qw, ii - 1 - qbase) == byte_of(tw, jj - 1 - tbase); },
        refill);
}

hipError_t launch_walk_wf_only(const PairArgs &a, int mode, const int32_t *only, hipStream_t s) {
    if (a.n_wf <= 0) return hipSuccess;
    const int bs = kWalkThreads;
    const unsigned nb = (unsigned)((a.n_wf + bs - 1) / bs);
    if (mode == LOCAL) hipLaunchKernelGGL(k_walk_wf<LOCAL>, dim3(nb), dim3(bs), 0, s, a, only);
    else if (mode == GLOBAL) hipLaunchKernelGGL(k_walk_wf<GLOBAL>, dim3(nb), dim3(bs), 0, s, a, only);
    else hipLaunchKernelGGL(k_walk_wf<SEMIGLOBAL>, dim3(nb), dim3(bs), 0, s, a, only);
    return hipGetLastError();
}

hipError_t launch_walk_wf(const PairArgs &a, int mode, hipStream_t s) {
    return launch_walk_wf_only(a, mode, nullptr, s);
}

hipError_t launch_walk(const PairArgs &a, int mode, int64_t slot0, int64_t n_slots, hipStream_t s) {
    if (n_slots <= 0) return hipSuccess;
    const int bs = kLaneWalkThreads;
    const unsigned nb = (unsigned)((n_slots + bs - 1) / bs);
    if (mode == LOCAL) hipLaunchKernelGGL(k_walk<LOCAL>, dim3(nb), dim3(bs), 0, s, a, slot0, n_slots);
    else if (mode == GLOBAL) hipLaunchKernelGGL(k_walk<GLOBAL>, dim3(nb), dim3(bs), 0, s, a, slot0, n_slots);
    else hipLaunchKernelGGL(k_walk<SEMIGLOBAL>, dim3(nb), dim3(bs), 0, s, a, slot0, n_slots);
    return hipGetLastError();
}

}  // namespace dsa
