// Database-search kernels: one query against groups of length-sorted targets.
//
// Recurrence (affine gaps, Gotoh; local / global / semi-global as in the
// paper's three algorithms, Section II.C.2):
//   E[i][j] = max(E[i][j-1] - e, H[i][j-1] - o)
//   F[i][j] = max(F[i-1][j] - e, H[i-1][j] - o)
//   H[i][j] = max([0 if local], H[i-1][j-1] + S[a_i][b_j], E[i][j], F[i][j])
//
// Mapping (inter-sequence): a wave owns one group of 128 targets; lane l
// carries target l in the low int16 half and target l+64 in the high half
// of every 32-bit register, so each v_pk_* instruction advances two cells.
// The query is cut into strips of T rows; the T rows' H and E live in
// VGPRs while the wave sweeps the target columns left to right, carrying F
// and the diagonal down each column.  The last row's H and the F leaving
// the strip are written to a boundary buffer and read back by the next
// strip.  Substitution scores come from a pair profile in LDS:
// QP[p][r] = (S[a_r][lo(p)], S[a_r][hi(p)]) for the pair code p the packed
// database stores for each lane and column, so one 4-byte LDS word feeds a
// packed add.  All waves of a workgroup share the strip's profile.
//
// Local mode holds each value as value + kBias16 in a column-shifted frame
// (column j adds (j - 1) e, taken back every few column blocks), where the
// E decrement disappears and E and F share one subtraction.  The bias keeps
// every reachable pattern a positive normal binary16 number, on which
// v_pk_maximum3_f16 is the integer maximum, so the H maximum, the zero
// floors and the running best are three-way maxima: 6.5 packed
// instructions per two cells (pk16.h).  Global and semi-global use signed
// saturating int16.  A unit whose int16 best passes the exact range is
// flagged, and the exact int32 kernel recomputes it (the int32 kernel also
// serves DSA_FORCE_INT32).
//
// Persistent form: one launch pulls units from a longest-first work list on
// an atomic counter.  Besides the inter-sequence units it runs, with the
// whole block, the wavefront units of long targets (intra_unit.h) and the
// strip-pipelined units that share one group's strips among the block's
// waves (ks_unit.h).
//
// End cell (smallest target end j, then smallest query end i, among cells
// reaching the best score): each strip scans its columns in order and keeps
// a strictly-greater running best; when a column improves it, the first row
// reaching the column maximum is located.  Strips are then merged
// lexicographically (score desc, j asc, i asc).
#include <algorithm>
#include <type_traits>

#include "internal.h"
#include "intra_unit.h"
#include "ks_unit.h"
#include "pk16.h"

namespace dsa {

template <int T>
__device__ __forceinline__ void load_profile(const uint32_t *lds, uint32_t off, uint32_t (&sc)[T]) {
    const uint4 *prow = reinterpret_cast<const uint4 *>(lds + off);
#pragma unroll
    for (int k = 0; k < T / 4; k++) {
        const uint4 v = prow[k];
        sc[4 * k + 0] = v.x; sc[4 * k + 1] = v.y; sc[4 * k + 2] = v.z; sc[4 * k + 3] = v.w;
    }
}

size_t search16_lds_bytes(int T, int AP) { return (size_t)AP * AP * (T + 4) * 4; }
size_t search32_lds_bytes(int AP) { return (size_t)AP * (kT32 + 4) * 4 + (size_t)AP * AP * 2 + 16; }

// Pair profile of every strip of every query, built once per call in the
// same padded layout the search kernel keeps in LDS, so each strip is a
// straight 16-byte copy: prof[Q.prof + s*AP*AP*SP + p*SP + r].
template <int T>
__global__ void k_profile16(ProfileArgs a) {
    constexpr int SP = T + 4;
    const int AP = a.AP, A = a.A;
    const int64_t per_strip = (int64_t)AP * AP * SP;
    const int64_t total = a.total_dwords;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
         k += (int64_t)gridDim.x * blockDim.x) {
        // locate the query: strip_base is ascending
        int lo = 0, hi = a.n_q - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.qinfo[mid].prof <= k) lo = mid; else hi = mid - 1;
        }
        const QueryInfo Q = a.qinfo[lo];
        const int64_t rel = k - Q.prof;
        const int s = (int)(rel / per_strip);
        const int w = (int)(rel - (int64_t)s * per_strip);
        const int p = w / SP, r = w - p * SP;
        const int i = s * T + r;
        int slo = NEG16, shi = NEG16;
        if (r < T && i < Q.len) {
            // query codes >= A are caller errors; qscore clamps them
            const int clo = a.inv_map[a.pair_dec[2 * p]], chi = a.inv_map[a.pair_dec[2 * p + 1]];
            if (clo != 0xff) slo = qscore(a.pssm, a.subst, a.q_codes, A, Q.off + i, lo, clo) + a.add;
            if (chi != 0xff) shi = qscore(a.pssm, a.subst, a.q_codes, A, Q.off + i, lo, chi) + a.add;
        }
        a.prof[k] = pack2(slo, shi);
    }
}

hipError_t launch_profile16(const ProfileArgs &a, int T, hipStream_t s) {
    if (a.total_dwords <= 0) return hipSuccess;
    const int bs = 256;
    const int64_t nb = std::min<int64_t>((a.total_dwords + bs - 1) / bs, 65536);
    if (T == 16) hipLaunchKernelGGL(k_profile16<16>, dim3((unsigned)nb), dim3(bs), 0, s, a);
    else hipLaunchKernelGGL(k_profile16<32>, dim3((unsigned)nb), dim3(bs), 0, s, a);
    return hipGetLastError();
}

template <int T, int MODE, bool PERSIST>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(T <= 16 ? 4 : 2)))
k_search16(SearchArgs P, IntraArgs W) {
    extern __shared__ uint4 lds4[];
    uint32_t *lds = reinterpret_cast<uint32_t *>(lds4);
    constexpr int SP = T + 4;  // dwords per profile row, a 16-byte multiple
    __shared__ int s_unit;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int o = P.o, e = P.e, ends = P.ends, AP = P.AP;
    const uint32_t o2 = dup(o), e2 = dup(e);
    const int strip4 = AP * AP * SP / 4;  // uint4 per strip profile
    // local mode, column-shifted frame: column j (1-based) holds value +
    // kBias16 + ((j - 1) mod 4*rb) * e; every 4*rb columns the frame is taken
    // back by 4*rb*e (at most kShift16)
    const uint32_t oe2 = dup(o - e);
    const int rb = e > 0 ? max(1, (kShift16 / 4) / e) : (1 << 28);
    const uint32_t back2 = dup(4 * rb * e);

    for (int iter = 0;; iter++) {
        int u;
        if (PERSIST) {
            if (tid == 0) s_unit = atomicAdd(P.counter, 1);
            __syncthreads();
            u = s_unit;
            __syncthreads();
            if (u >= (P.order ? P.n_order : P.n_units)) return;
            if (P.order) {
                const int v = P.order[u];
                if (v < 0) {  // a wavefront unit: the whole block takes it
                    intra16_unit<MODE>(W, W.units[-v - 1], lds4);
                    __syncthreads();
                    continue;
                }
                if (v >= kKsBase) {  // a strip-pipelined unit: the whole block takes it
                    if (MODE == LOCAL && T == 16) ks16_unit(P, P.units[v - kKsBase], v - kKsBase, lds4);
                    __syncthreads();
                    continue;
                }
                u = v;
            }
        } else {
            if (iter > 0) return;
            u = blockIdx.x;
        }
        const SearchUnit U = P.units[u];
        const QueryInfo Q = P.qinfo[U.q];
        if (MODE != LOCAL && P.qflag[U.q]) {  // int16 unsafe: leave it to the int32 pass
            if (tid == 0) P.unit_flags[u] = 2;
            continue;
        }
        const bool active = wave < U.ng;
        GroupInfo G = {0, 0, 0, 0};
        if (active) G = P.grp[U.g0 + wave];
        const int m = Q.len, S = Q.strips;
        int n_lo = 0, n_hi = 0;
        if (active) {
            n_lo = P.slot_len[G.slot0 + lane];
            n_hi = P.slot_len[G.slot0 + 64 + lane];
        }
        const uint32_t nn = pack2(n_lo, n_hi);
        const uint2 *pk = P.packed + G.off + lane;
        uint2 *bnd = P.bnd + (int64_t)U.qslot * P.bnd_slot_stride + G.bnd + lane;
        const uint4 *qprof = reinterpret_cast<const uint4 *>(P.prof + Q.prof);

        // best so far over finished strips (local), or the result (global / semi)
        uint32_t Gs = 0, Gj = 0, Gi = 0;

        for (int s = 0; s < S; s++) {
            const int i0 = s * T;
            __syncthreads();
            {
                const uint4 *src = qprof + (int64_t)s * strip4;
                for (int k = tid; k < strip4; k += blockDim.x) lds4[k] = src[k];
            }
            __syncthreads();
            if (!active) continue;

            const bool first = (s == 0), last = (s == S - 1);
            uint32_t H[T], E[T];
#pragma unroll
            for (int r = 0; r < T; r++) {
                // local: column 0 sits one e below column 1's frame
                H[r] = (MODE == LOCAL) ? dup(kBias16 - e) : dup(left_value(MODE, ends, o, e, i0 + r + 1));
                E[r] = (MODE == LOCAL) ? dup(kBias16) : subs(H[r], o2);
            }
            uint32_t Hd_top = (MODE == LOCAL) ? dup(kBias16 - e) : dup(left_value(MODE, ends, o, e, i0));

            // strip-local running best (local mode, plain values): starts
            // just below the best of earlier strips so only cells that can
            // still win are recorded.
            uint32_t B = 0, Bj = 0, Bi = 0;
            if (MODE == LOCAL) B = maxs(subs(Gs, dup(1)), 0u);
            // last-strip capture (global / semi-global)
            const int rlast = m - 1 - i0;
            uint32_t res = 0, Ls = 0, Lj = 0;
            if (MODE != LOCAL && last) {
                res = dup(left_value(MODE, ends, o, e, m));
                Ls = res;
            }

            const int nblk = G.ncols >> 2;
            // one 4-column block; on the first strip the row above is the
            // top boundary (a compile-time case, so the other strips carry
            // no selects for it)
            auto block = [&](auto first_strip, const int c4, const uint2 cd, const uint2 (&hf)[4]) {
                constexpr bool FIRST = decltype(first_strip)::value;
                if (MODE == LOCAL && c4 > 0 && c4 % rb == 0) {  // take the column frame back
#pragma unroll
                    for (int r = 0; r < T; r++) {
                        H[r] = subw(H[r], back2);
                        E[r] = subw(E[r], back2);
                    }
                    Hd_top = subw(Hd_top, back2);
                }
                const int cbase = kBias16 + (c4 % rb) * 4 * e;  // frame of the block's first column
#pragma unroll
                for (int c = 0; c < 4; c++) {
                    const int j = c4 * 4 + c + 1;
                    const uint32_t p = ((c < 2 ? cd.x : cd.y) >> ((c & 1) * 16)) & 0xffffu;
                    uint32_t Hup, F;
                    const int cj = cbase + c * e;  // local: this column's frame
                    if constexpr (FIRST) {
                        Hup = (MODE == LOCAL) ? dup(cj) : dup(top_value(MODE, ends, o, e, j));
                        F = (MODE == LOCAL) ? dup(cj) : subs(Hup, o2);
                    } else {
                        Hup = hf[c].x;
                        F = hf[c].y;
                    }
                    const uint32_t Hd = Hd_top;
                    Hd_top = Hup;
                    uint32_t sc[T];
                    load_profile<T>(lds, p * SP, sc);
                    if (MODE == LOCAL) {
                        const uint32_t Bc = addu(B, dup(cj));
                        const uint32_t nb = column16_local_cs<T>(sc, H, E, Hd, F, oe2, e2, dup(cj + e), Bc);
                        if (nb != Bc) {
                            // some half improved: find the first row reaching
                            // the column maximum.  The integer maximum keeps B
                            // from falling if a cell beyond the exact range
                            // (flagged below) left a non-number pattern.
                            const uint32_t mask = nzmask(nb ^ Bc);
                            const uint32_t idx = first_row_of<T>(H, nb);
                            Bi = bfi(mask, addu(idx, dup(i0 + 1)), Bi);
                            Bj = bfi(mask, dup(j), Bj);
                            B = maxs(B, subw(nb, dup(cj)));
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
                    if (!last) bnd[(int64_t)(j - 1) * 64] = make_uint2(H[T - 1], F);
                }
            };
            // software pipeline: the next block's codes and boundary words
            // are in flight while the current block computes
            auto sweep = [&](auto first_strip) {
                constexpr bool FIRST = decltype(first_strip)::value;
                uint2 cd_n = make_uint2(0, 0), hf_n[4];
#pragma unroll
                for (int c = 0; c < 4; c++) hf_n[c] = make_uint2(0, 0);
                auto fetch = [&](const int c4) {
                    cd_n = pk[(int64_t)c4 * 64];
                    if constexpr (!FIRST) {
#pragma unroll
                        for (int c = 0; c < 4; c++) hf_n[c] = bnd[(int64_t)(4 * c4 + c) * 64];
                    }
                };
                if (nblk > 0) fetch(0);
                for (int c4 = 0; c4 < nblk; c4++) {
                    const uint2 cd = cd_n;
                    uint2 hf[4];
#pragma unroll
                    for (int c = 0; c < 4; c++) hf[c] = hf_n[c];
                    if (c4 + 1 < nblk) fetch(c4 + 1);
                    block(first_strip, c4, cd, hf);
                }
            };
            if (first) sweep(std::true_type{});
            else sweep(std::false_type{});

            if (MODE == LOCAL) {
                const int b[2] = {lo16(B), hi16(B)};
                const int bj[2] = {(int)(Bj & 0xffff), (int)(Bj >> 16)};
                const int bi[2] = {(int)(Bi & 0xffff), (int)(Bi >> 16)};
                uint64_t gk[2] = {end_key(lo16(Gs), (int)(Gj & 0xffff), (int)(Gi & 0xffff)),
                                  end_key(hi16(Gs), (int)(Gj >> 16), (int)(Gi >> 16))};
#pragma unroll
                for (int h = 0; h < 2; h++) {
                    const uint64_t kk = end_key(b[h], bj[h], bi[h]);
                    gk[h] = (b[h] > 0) ? umax64(gk[h], kk) : gk[h];
                }
                Gs = pack2(key_score(gk[0]), key_score(gk[1]));
                Gj = pack2(key_j(gk[0]), key_j(gk[1]));
                Gi = pack2(key_i(gk[0]), key_i(gk[1]));
            } else if (last) {
                if (ends & TE) { Gs = Ls; Gj = Lj; }
                else { Gs = res; Gj = nn; }
            }
        }

        if (active) {
            bool ovf = false;
#pragma unroll
            for (int h = 0; h < 2; h++) {
                const int slot = G.slot0 + h * 64 + lane;
                const int t = P.slot_target[slot];
                if (t < 0) continue;
                const int sc = h ? hi16(Gs) : lo16(Gs);
                const int jj = h ? (int)(Gj >> 16) : (int)(Gj & 0xffff);
                int qe, te;
                if (MODE == LOCAL) {
                    const int ii = h ? (int)(Gi >> 16) : (int)(Gi & 0xffff);
                    qe = sc > 0 ? ii - 1 : -1;
                    te = sc > 0 ? jj - 1 : -1;
                    ovf |= sc > kLocal16Max;
                } else {
                    qe = m - 1;
                    te = jj - 1;
                    ovf |= (sc >= 32767) || (sc <= -32768);
                }
                const int64_t oi = (int64_t)U.q * P.n_t + t;
                P.out_score[oi] = sc;
                if (P.out_qend) P.out_qend[oi] = qe;
                if (P.out_tend) P.out_tend[oi] = te;
                if (P.out_status) P.out_status[oi] = 0;
            }
            if (ovf) P.unit_flags[u] = 1;
        }
        if (PERSIST) __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Exact int32 kernel: one target per lane, two waves per group (low halves,
// then high halves).  Same strips, boundary layout and end-cell rule; the
// profile is the single-letter QP[c][r] = S[a_r][c].  With rerun_only it
// visits only flagged units and rewrites only results whose int16 value
// saturated.
// ---------------------------------------------------------------------------
template <int MODE, bool PERSIST>
__global__ void __launch_bounds__(1024) k_search32(SearchArgs P, int rerun_only) {
    constexpr int T = kT32;
    constexpr int SP = T + 4;
    extern __shared__ uint4 lds4[];
    int32_t *prof = reinterpret_cast<int32_t *>(lds4);
    uint8_t *dec = reinterpret_cast<uint8_t *>(prof + P.AP * SP);
    __shared__ int s_unit;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int o = P.o, e = P.e, ends = P.ends, A = P.A, AP = P.AP;
    for (int k = tid; k < AP * AP * 2; k += blockDim.x) dec[k] = P.pair_dec[k];

    for (int iter = 0;; iter++) {
        int u;
        if (PERSIST) {
            if (tid == 0) s_unit = atomicAdd(P.counter, 1);
            __syncthreads();
            u = s_unit;
            __syncthreads();
            if (u >= P.n_units) return;
        } else {
            if (iter > 0) return;
            u = blockIdx.x;
        }
        const int uflag = rerun_only ? P.unit_flags[u] : 2;
        if (uflag == 0) continue;  // uniform per block
        const SearchUnit U = P.units[u];
        const QueryInfo Q = P.qinfo[U.q];
        const int half = wave & 1;
        const bool active = (wave >> 1) < U.ng;
        GroupInfo G = {0, 0, 0, 0};
        if (active) G = P.grp[U.g0 + (wave >> 1)];
        const int m = Q.len, S = Q.strips;
        const uint8_t *qc = P.q_codes + Q.off;
        const int slot = G.slot0 + half * 64 + lane;
        const int nt = active ? P.slot_len[slot] : 0;
        const uint2 *pk = P.packed + G.off + lane;
        uint2 *bnd = P.bnd + (int64_t)U.qslot * P.bnd_slot_stride + G.bnd +
                     (int64_t)half * G.ncols * 64 + lane;

        int Gs = (MODE == LOCAL) ? 0 : PAD32, Gj = 0, Gi = 0;
        // free query end: the last column's best, starting from row 0
        const bool qe_free = (MODE == SEMIGLOBAL) && (ends & QE);
        int Qs = top_value(MODE, ends, o, e, nt), Qi = 0;
        for (int s = 0; s < S; s++) {
            const int i0 = s * T;
            __syncthreads();
            for (int idx = tid; idx < AP * T; idx += blockDim.x) {
                const int c = idx / T, r = idx - c * T;
                const int i = i0 + r;
                int v = PAD32;
                if (i < m && P.inv_map[c] != 0xff) v = qscore(P.pssm, P.subst, P.q_codes, A, Q.off + i, U.q, P.inv_map[c]);
                prof[c * SP + r] = v;
            }
            __syncthreads();
            if (!active) continue;

            const bool first = (s == 0), last = (s == S - 1);
            int H[T], E[T];
#pragma unroll
            for (int r = 0; r < T; r++) {
                H[r] = left_value(MODE, ends, o, e, i0 + r + 1);
                E[r] = H[r] - o;
            }
            int Hd_top = left_value(MODE, ends, o, e, i0);
            int B = 0, Bj = 0, Bi = 0;
            if (MODE == LOCAL) B = Gs > 0 ? Gs - 1 : 0;
            const int rlast = m - 1 - i0;
            int res = 0, Ls = 0, Lj = 0;
            if (MODE != LOCAL && last) { res = left_value(MODE, ends, o, e, m); Ls = res; }

            const int nblk = G.ncols >> 2;
            for (int c4 = 0; c4 < nblk; c4++) {
                const uint2 cd = pk[(int64_t)c4 * 64];
                int hf[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                if (!first) {
#pragma unroll
                    for (int c = 0; c < 4; c++) {
                        const uint2 b = bnd[(int64_t)(4 * c4 + c) * 64];
                        hf[2 * c] = (int)b.x;
                        hf[2 * c + 1] = (int)b.y;
                    }
                }
#pragma unroll
                for (int c = 0; c < 4; c++) {
                    const int j = c4 * 4 + c + 1;
                    const uint32_t p = ((c < 2 ? cd.x : cd.y) >> ((c & 1) * 16)) & 0xffffu;
                    const int code = dec[p * 2 + half];
                    int Hup, F;
                    if (first) {
                        Hup = top_value(MODE, ends, o, e, j);
                        F = Hup - o;
                    } else {
                        Hup = hf[2 * c];
                        F = hf[2 * c + 1];
                    }
                    int Hd = Hd_top;
                    Hd_top = Hup;
                    const int32_t *prow = prof + code * SP;
                    int cm = 0;
#pragma unroll
                    for (int r = 0; r < T; r++) {
                        const int t = Hd + prow[r];
                        Hd = H[r];
                        int h = max(max(t, E[r]), F);
                        if (MODE == LOCAL) { h = max(h, 0); cm = max(cm, h); }
                        const int ho = h - o;
                        E[r] = max(E[r] - e, ho);
                        F = max(F - e, ho);
                        H[r] = h;
                    }
                    if (MODE == LOCAL) {
                        if (cm > B) {
                            int rr = 0;
#pragma unroll
                            for (int r = T - 1; r >= 0; r--) rr = (H[r] == cm) ? r : rr;
                            B = cm; Bj = j; Bi = i0 + rr + 1;
                        }
                    } else {
                        if (last) {
                            int vl = H[0];
#pragma unroll
                            for (int k = 1; k < T; k++) vl = (k == rlast) ? H[k] : vl;
                            if (!(ends & TE)) {
                                if (j == nt) res = vl;
                            } else if (j <= nt && vl > Ls) {
                                Ls = vl; Lj = j;
                            }
                        }
                        if (qe_free && j == nt) last_column_scan<T>(H, i0, m, Qs, Qi);
                    }
                    if (!last) bnd[(int64_t)(j - 1) * 64] = make_uint2((uint32_t)H[T - 1], (uint32_t)F);
                }
            }
            if (MODE == LOCAL) {
                const uint64_t gk = umax64(end_key(Gs, Gj, Gi), end_key(B, Bj, Bi));
                if (B > 0) { Gs = key_score(gk); Gj = key_j(gk); Gi = key_i(gk); }
            } else if (last) {
                if (ends & TE) { Gs = Ls; Gj = Lj; }
                else { Gs = res; Gj = nt; }
                Gi = m;
            }
        }
        if (qe_free) {  // the last row's candidate against the last column's
            const uint64_t gk = umax64(end_key(Gs, Gj, Gi), end_key(Qs, nt, Qi));
            Gs = key_score(gk); Gj = key_j(gk); Gi = key_i(gk);
        }

        if (active) {
            const int t = P.slot_target[slot];
            if (t >= 0) {
                const int64_t oi = (int64_t)U.q * P.n_t + t;
                bool write = true;
                if (uflag == 1) {
                    const int prev = P.out_score[oi];
                    write = (MODE == LOCAL) ? prev > kLocal16Max : (prev >= 32767) || (prev <= -32768);
                }
                if (write) {
                    int qe, te;
                    if (MODE == LOCAL) { qe = Gs > 0 ? Gi - 1 : -1; te = Gs > 0 ? Gj - 1 : -1; }
                    else { qe = Gi - 1; te = Gj - 1; }
                    P.out_score[oi] = Gs;
                    if (P.out_qend) P.out_qend[oi] = qe;
                    if (P.out_tend) P.out_tend[oi] = te;
                    if (P.out_status) P.out_status[oi] = 1;  // DSA_ST_INT32
                }
            }
        }
        if (PERSIST) __syncthreads();
    }
}

// ---------------------------------------------------------------------------
template <int T>
static hipError_t launch16_T(const SearchArgs &a, const IntraArgs &w, int mode, int wpb, int nb, bool persist,
                             size_t lds, hipStream_t s) {
    dim3 grid(nb), block(wpb * kWave);
#define L16(MODE, PER)                                                                  \
    do {                                                                                \
        auto kfn = k_search16<T, MODE, PER>;                                            \
        hipError_t err = hipFuncSetAttribute((const void *)kfn,                         \
                                             hipFuncAttributeMaxDynamicSharedMemorySize, \
                                             (int)lds);                                 \
        if (err != hipSuccess) return err;                                              \
        hipLaunchKernelGGL(kfn, grid, block, lds, s, a, w);                             \
        return hipGetLastError();                                                       \
    } while (0)
    if (mode == LOCAL) { if (persist) L16(LOCAL, true); else L16(LOCAL, false); }
    if (mode == GLOBAL) { if (persist) L16(GLOBAL, true); else L16(GLOBAL, false); }
    if (persist) L16(SEMIGLOBAL, true); else L16(SEMIGLOBAL, false);
#undef L16
}

hipError_t launch_search16(const SearchArgs &a, const IntraArgs &w, int T, int mode, int wpb, int nb,
                           bool persist, size_t lds, hipStream_t s) {
    switch (T) {
        case 16: return launch16_T<16>(a, w, mode, wpb, nb, persist, lds, s);
        case 32: return launch16_T<32>(a, w, mode, wpb, nb, persist, lds, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_search32(const SearchArgs &a, int mode, int wpb, int nb, bool persist,
                           size_t lds, hipStream_t s, int rerun_only) {
    dim3 grid(nb), block(wpb * kWave);
#define L32(MODE, PER)                                                                  \
    do {                                                                                \
        auto kfn = k_search32<MODE, PER>;                                               \
        hipError_t err = hipFuncSetAttribute((const void *)kfn,                         \
                                             hipFuncAttributeMaxDynamicSharedMemorySize, \
                                             (int)lds);                                 \
        if (err != hipSuccess) return err;                                              \
        hipLaunchKernelGGL(kfn, grid, block, lds, s, a, rerun_only);                    \
        return hipGetLastError();                                                       \
    } while (0)
    if (mode == LOCAL) { if (persist) L32(LOCAL, true); else L32(LOCAL, false); }
    if (mode == GLOBAL) { if (persist) L32(GLOBAL, true); else L32(GLOBAL, false); }
    if (persist) L32(SEMIGLOBAL, true); else L32(SEMIGLOBAL, false);
#undef L32
}

// ---------------------------------------------------------------------------
// int16 safety of a query for global / semi-global: every H is at most the
// sum over its rows of the best positive substitution score, and at least
// -(2o + (m+n)e) - |min S| (the E / F values one more open below).
__global__ void k_bound16(BoundArgs a) {
    const int q = blockIdx.x;
    if (q >= a.n_q) return;
    const QueryInfo Q = a.qinfo[q];
    int64_t sum = 0;
    for (int i = threadIdx.x; i < Q.len; i += blockDim.x) {
        int best = 0;
        for (int k = 0; k < a.AP; k++) {
            const int t = a.inv_map[k];
            if (t != 0xff) best = max(best, qscore(a.pssm, a.subst, a.q_codes, a.A, Q.off + i, q, t));
        }
        sum += best;
    }
    __shared__ int64_t red[256];
    red[threadIdx.x] = sum;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t low = 3LL * a.o + (int64_t)(Q.len + 64 + a.n_max) * a.e + a.min_s;
        a.qflag[q] = (red[0] >= 32000 || low >= 32000) ? 1 : 0;
    }
}

hipError_t launch_bound16(const BoundArgs &a, hipStream_t s) {
    if (a.n_q <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bound16, dim3(a.n_q), dim3(256), 0, s, a);
    return hipGetLastError();
}

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int bs = 256;
    const int64_t nb = (n + bs - 1) / bs;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)nb), dim3(bs), 0, s, p, v, n);
    return hipGetLastError();
}

// Results of empty queries: the last row is the top boundary row.
__global__ void k_empty(EmptyArgs a) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)a.n_rows * a.n_t) return;
    const int row = (int)(k / a.n_t);
    const int64_t t = k - (int64_t)row * a.n_t;
    const int64_t oi = (int64_t)a.q_rows[row] * a.n_t + t;
    const int n = (int)a.t_len[t];
    int sc, te;
    if (a.mode == LOCAL) {
        sc = 0; te = -1;
    } else if (a.mode == SEMIGLOBAL && (a.ends & TE)) {
        sc = 0; te = -1;  // (0, 0) reaches the maximum 0 at the smallest column
    } else {
        sc = top_value(a.mode, a.ends, a.o, a.e, n);
        te = n - 1;
    }
    a.out_score[oi] = sc;
    if (a.out_qend) a.out_qend[oi] = -1;
    if (a.out_tend) a.out_tend[oi] = te;
    if (a.out_qbeg) a.out_qbeg[oi] = -1;
    if (a.out_tbeg) a.out_tbeg[oi] = -1;
    if (a.out_status) a.out_status[oi] = 0;
}

hipError_t launch_empty_queries(const EmptyArgs &a, hipStream_t s) {
    const int64_t n = (int64_t)a.n_rows * a.n_t;
    if (n <= 0) return hipSuccess;
    const int bs = 256;
    hipLaunchKernelGGL(k_empty, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s, a);
    return hipGetLastError();
}

}  // namespace dsa
