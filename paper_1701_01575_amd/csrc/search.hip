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
// Local mode uses unsigned saturating subtractions for E and F, which
// clamps them at 0 and makes the explicit 0 in the H maximum redundant:
// 9 packed instructions per two cells.  An int16 result that reached 32767
// may have saturated; its unit is flagged and the exact int32 kernel
// recomputes it (the int32 kernel also serves DSA_FORCE_INT32).
//
// End cell (smallest target end j, then smallest query end i, among cells
// reaching the best score): each strip scans its columns in order and keeps
// a strictly-greater running best; when a column improves it, the first row
// reaching the column maximum is located.  Strips are then merged
// lexicographically (score desc, j asc, i asc).
#include "internal.h"

namespace dsa {

typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ s16x2 S2(uint32_t x) { return __builtin_bit_cast(s16x2, x); }
__device__ __forceinline__ u16x2 U2(uint32_t x) { return __builtin_bit_cast(u16x2, x); }
__device__ __forceinline__ uint32_t Bs(s16x2 x) { return __builtin_bit_cast(uint32_t, x); }
__device__ __forceinline__ uint32_t Bu(u16x2 x) { return __builtin_bit_cast(uint32_t, x); }

__device__ __forceinline__ uint32_t adds(uint32_t a, uint32_t b) { return Bs(__builtin_elementwise_add_sat(S2(a), S2(b))); }
__device__ __forceinline__ uint32_t subs(uint32_t a, uint32_t b) { return Bs(__builtin_elementwise_sub_sat(S2(a), S2(b))); }
__device__ __forceinline__ uint32_t maxs(uint32_t a, uint32_t b) { return Bs(__builtin_elementwise_max(S2(a), S2(b))); }
__device__ __forceinline__ uint32_t subu(uint32_t a, uint32_t b) { return Bu(__builtin_elementwise_sub_sat(U2(a), U2(b))); }
__device__ __forceinline__ uint32_t maxu(uint32_t a, uint32_t b) { return Bu(__builtin_elementwise_max(U2(a), U2(b))); }
__device__ __forceinline__ uint32_t minu(uint32_t a, uint32_t b) { return Bu(__builtin_elementwise_min(U2(a), U2(b))); }
__device__ __forceinline__ uint32_t addu(uint32_t a, uint32_t b) { return Bu(U2(a) + U2(b)); }
__device__ __forceinline__ uint32_t mulu(uint32_t a, uint32_t b) { return Bu(U2(a) * U2(b)); }

__device__ __forceinline__ uint32_t pack2(int lo, int hi) {
    return (uint32_t)(uint16_t)lo | ((uint32_t)(uint16_t)hi << 16);
}
__device__ __forceinline__ uint32_t dup(int v) { return pack2(v, v); }
__device__ __forceinline__ int lo16(uint32_t x) { return (int)(short)(x & 0xffffu); }
__device__ __forceinline__ int hi16(uint32_t x) { return (int)(short)(x >> 16); }
__device__ __forceinline__ uint32_t bfi(uint32_t mask, uint32_t a, uint32_t b) { return (a & mask) | (b & ~mask); }
// 0xffff in each half of x that is nonzero, 0 elsewhere
__device__ __forceinline__ uint32_t nzmask(uint32_t x) {
    return Bu((u16x2)0 - __builtin_elementwise_min(U2(x), (u16x2)1));
}

constexpr int NEG16 = -32768;
constexpr int PAD32 = -(1 << 30);

// H[i][0]: the left boundary column (i >= 0).
__device__ __forceinline__ int left_value(int mode, int ends, int o, int e, int i) {
    if (i == 0 || mode == LOCAL || (ends & QB)) return 0;
    return -(o + (i - 1) * e);
}
// H[0][j]: the top boundary row (j >= 0).
__device__ __forceinline__ int top_value(int mode, int ends, int o, int e, int j) {
    if (j == 0 || mode == LOCAL || (ends & TB)) return 0;
    return -(o + (j - 1) * e);
}

template <int T>
__device__ __forceinline__ uint32_t pick_row(const uint32_t (&H)[T], int r) {
    uint32_t v = H[0];
#pragma unroll
    for (int k = 1; k < T; k++) v = (k == r) ? H[k] : v;
    return v;
}

template <int T>
__device__ __forceinline__ void load_profile(const uint32_t *lds, uint32_t off, uint32_t (&sc)[T]) {
    const uint4 *prow = reinterpret_cast<const uint4 *>(lds + off);
#pragma unroll
    for (int k = 0; k < T / 4; k++) {
        const uint4 v = prow[k];
        sc[4 * k + 0] = v.x; sc[4 * k + 1] = v.y; sc[4 * k + 2] = v.z; sc[4 * k + 3] = v.w;
    }
}

// One column of a strip, local mode, packed int16 (E, F clamped at 0).
// Returns the column maximum.
template <int T>
__device__ __forceinline__ uint32_t column16_local(const uint32_t (&sc)[T], uint32_t (&H)[T],
                                                   uint32_t (&E)[T], uint32_t Hd, uint32_t &F,
                                                   uint32_t o2, uint32_t e2) {
    uint32_t cm = 0;
#pragma unroll
    for (int r = 0; r < T; r++) {
        const uint32_t t = adds(Hd, sc[r]);
        Hd = H[r];
        const uint32_t h = maxs(maxs(t, E[r]), F);
        cm = maxs(cm, h);
        const uint32_t ho = subu(h, o2);
        E[r] = maxu(subu(E[r], e2), ho);
        F = maxu(subu(F, e2), ho);
        H[r] = h;
    }
    return cm;
}

// One column, global / semi-global, packed int16 with signed saturation.
template <int T>
__device__ __forceinline__ void column16_global(const uint32_t (&sc)[T], uint32_t (&H)[T],
                                                uint32_t (&E)[T], uint32_t Hd, uint32_t &F,
                                                uint32_t o2, uint32_t e2) {
#pragma unroll
    for (int r = 0; r < T; r++) {
        const uint32_t t = adds(Hd, sc[r]);
        Hd = H[r];
        const uint32_t h = maxs(maxs(t, E[r]), F);
        const uint32_t ho = subs(h, o2);
        E[r] = maxs(subs(E[r], e2), ho);
        F = maxs(subs(F, e2), ho);
        H[r] = h;
    }
}

size_t search16_lds_bytes(int T, int AP) { return (size_t)AP * AP * (T + 4) * 4; }
size_t search32_lds_bytes(int AP) { return (size_t)AP * (kT32 + 4) * 4 + (size_t)AP * AP * 2 + 16; }

template <int T, int MODE, bool PERSIST>
__global__ void __launch_bounds__(512) k_search16(SearchArgs P) {
    extern __shared__ uint4 lds4[];
    uint32_t *lds = reinterpret_cast<uint32_t *>(lds4);
    constexpr int SP = T + 4;  // dwords per profile row, a 16-byte multiple
    __shared__ int s_unit;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int o = P.o, e = P.e, ends = P.ends, A = P.A, AP = P.AP;
    const uint32_t o2 = dup(o), e2 = dup(e);
    const int nprof = AP * AP * T;

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
        const uint8_t *qc = P.q_codes + Q.off;
        int n_lo = 0, n_hi = 0;
        if (active) {
            n_lo = P.slot_len[G.slot0 + lane];
            n_hi = P.slot_len[G.slot0 + 64 + lane];
        }
        const uint32_t nn = pack2(n_lo, n_hi);
        const uint2 *pk = P.packed + G.off + lane;
        uint4 *bnd = P.bnd + (int64_t)U.qslot * P.bnd_slot_stride + G.bnd + 2 * lane;

        // best so far over finished strips (local), or the result (global / semi)
        uint32_t Gs = 0, Gj = 0, Gi = 0;

        for (int s = 0; s < S; s++) {
            const int i0 = s * T;
            __syncthreads();
            for (int idx = tid; idx < nprof; idx += blockDim.x) {
                const int p = idx / T, r = idx - p * T;
                const int i = i0 + r;
                int slo = NEG16, shi = NEG16;
                if (i < m) {
                    const int a = min((int)qc[i], A - 1);  // codes >= A are caller errors
                    const int clo = P.inv_map[p / AP], chi = P.inv_map[p % AP];
                    if (clo != 0xff) slo = P.subst[a * A + clo];
                    if (chi != 0xff) shi = P.subst[a * A + chi];
                }
                lds[p * SP + r] = pack2(slo, shi);
            }
            __syncthreads();
            if (!active) continue;

            const bool first = (s == 0), last = (s == S - 1);
            uint32_t H[T], E[T];
#pragma unroll
            for (int r = 0; r < T; r++) {
                H[r] = dup(left_value(MODE, ends, o, e, i0 + r + 1));
                E[r] = (MODE == LOCAL) ? 0u : subs(H[r], o2);
            }
            uint32_t Hd_top = dup(left_value(MODE, ends, o, e, i0));

            // strip-local running best (local mode): starts just below the
            // best of earlier strips so only cells that can still win are
            // recorded.
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
            for (int c4 = 0; c4 < nblk; c4++) {
                const uint2 cd = pk[(int64_t)c4 * 64];
                uint32_t hf[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                if (!first) {
                    const uint4 b0 = bnd[(int64_t)c4 * 128], b1 = bnd[(int64_t)c4 * 128 + 1];
                    hf[0] = b0.x; hf[1] = b0.y; hf[2] = b0.z; hf[3] = b0.w;
                    hf[4] = b1.x; hf[5] = b1.y; hf[6] = b1.z; hf[7] = b1.w;
                }
                uint32_t ob[8];
#pragma unroll
                for (int c = 0; c < 4; c++) {
                    const int j = c4 * 4 + c + 1;
                    const uint32_t p = ((c < 2 ? cd.x : cd.y) >> ((c & 1) * 16)) & 0xffffu;
                    uint32_t Hup, F;
                    if (first) {
                        const int tv = top_value(MODE, ends, o, e, j);
                        Hup = dup(tv);
                        F = (MODE == LOCAL) ? 0u : subs(Hup, o2);
                    } else {
                        Hup = hf[2 * c];
                        F = hf[2 * c + 1];
                    }
                    const uint32_t Hd = Hd_top;
                    Hd_top = Hup;
                    uint32_t sc[T];
                    load_profile<T>(lds, p * SP, sc);
                    if (MODE == LOCAL) {
                        const uint32_t cm = column16_local<T>(sc, H, E, Hd, F, o2, e2);
                        const uint32_t nb = maxs(B, cm);
                        if (nb != B) {
                            // some half improved: find the first row reaching
                            // the column maximum
                            const uint32_t mask = nzmask(nb ^ B);
                            uint32_t idx = 0xffffffffu;
#pragma unroll
                            for (int r = 0; r < T; r++) {
                                const uint32_t z = minu(H[r] ^ cm, 0x00010001u);
                                idx = minu(idx, addu(mulu(z, 0x80008000u), dup(r)));
                            }
                            Bi = bfi(mask, addu(idx, dup(i0 + 1)), Bi);
                            Bj = bfi(mask, dup(j), Bj);
                            B = nb;
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
                    ob[2 * c] = H[T - 1];
                    ob[2 * c + 1] = F;
                }
                if (!last) {
                    bnd[(int64_t)c4 * 128] = make_uint4(ob[0], ob[1], ob[2], ob[3]);
                    bnd[(int64_t)c4 * 128 + 1] = make_uint4(ob[4], ob[5], ob[6], ob[7]);
                }
            }

            if (MODE == LOCAL) {
                int g[2] = {lo16(Gs), hi16(Gs)};
                int gj[2] = {(int)(Gj & 0xffff), (int)(Gj >> 16)};
                int gi[2] = {(int)(Gi & 0xffff), (int)(Gi >> 16)};
                const int b[2] = {lo16(B), hi16(B)};
                const int bj[2] = {(int)(Bj & 0xffff), (int)(Bj >> 16)};
                const int bi[2] = {(int)(Bi & 0xffff), (int)(Bi >> 16)};
#pragma unroll
                for (int h = 0; h < 2; h++) {
                    if (b[h] > 0 && (b[h] > g[h] || (b[h] == g[h] && bj[h] < gj[h]))) {
                        g[h] = b[h]; gj[h] = bj[h]; gi[h] = bi[h];
                    }
                }
                Gs = pack2(g[0], g[1]);
                Gj = pack2(gj[0], gj[1]);
                Gi = pack2(gi[0], gi[1]);
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
                    ovf |= sc >= 32767;
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
        uint4 *bnd = P.bnd + (int64_t)U.qslot * P.bnd_slot_stride + G.bnd +
                     (int64_t)half * (G.ncols >> 2) * 128 + 2 * lane;

        int Gs = (MODE == LOCAL) ? 0 : PAD32, Gj = 0, Gi = 0;
        for (int s = 0; s < S; s++) {
            const int i0 = s * T;
            __syncthreads();
            for (int idx = tid; idx < AP * T; idx += blockDim.x) {
                const int c = idx / T, r = idx - c * T;
                const int i = i0 + r;
                int v = PAD32;
                if (i < m && P.inv_map[c] != 0xff) v = P.subst[min((int)qc[i], A - 1) * A + P.inv_map[c]];
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
                    const uint4 b0 = bnd[(int64_t)c4 * 128], b1 = bnd[(int64_t)c4 * 128 + 1];
                    hf[0] = b0.x; hf[1] = b0.y; hf[2] = b0.z; hf[3] = b0.w;
                    hf[4] = b1.x; hf[5] = b1.y; hf[6] = b1.z; hf[7] = b1.w;
                }
                int ob[8];
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
                    } else if (last) {
                        int vl = H[0];
#pragma unroll
                        for (int k = 1; k < T; k++) vl = (k == rlast) ? H[k] : vl;
                        if (!(ends & TE)) {
                            if (j == nt) res = vl;
                        } else if (j <= nt && vl > Ls) {
                            Ls = vl; Lj = j;
                        }
                    }
                    ob[2 * c] = H[T - 1];
                    ob[2 * c + 1] = F;
                }
                if (!last) {
                    bnd[(int64_t)c4 * 128] = make_uint4(ob[0], ob[1], ob[2], ob[3]);
                    bnd[(int64_t)c4 * 128 + 1] = make_uint4(ob[4], ob[5], ob[6], ob[7]);
                }
            }
            if (MODE == LOCAL) {
                if (B > 0 && (B > Gs || (B == Gs && Bj < Gj))) { Gs = B; Gj = Bj; Gi = Bi; }
            } else if (last) {
                if (ends & TE) { Gs = Ls; Gj = Lj; }
                else { Gs = res; Gj = nt; }
            }
        }

        if (active) {
            const int t = P.slot_target[slot];
            if (t >= 0) {
                const int64_t oi = (int64_t)U.q * P.n_t + t;
                bool write = true;
                if (uflag == 1) {
                    const int prev = P.out_score[oi];
                    write = (prev >= 32767) || (prev <= -32768);
                }
                if (write) {
                    int qe, te;
                    if (MODE == LOCAL) { qe = Gs > 0 ? Gi - 1 : -1; te = Gs > 0 ? Gj - 1 : -1; }
                    else { qe = m - 1; te = Gj - 1; }
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
static hipError_t launch16_T(const SearchArgs &a, int mode, int wpb, int nb, bool persist,
                             size_t lds, hipStream_t s) {
    dim3 grid(nb), block(wpb * kWave);
#define L16(MODE, PER)                                                                  \
    do {                                                                                \
        auto kfn = k_search16<T, MODE, PER>;                                            \
        hipError_t err = hipFuncSetAttribute((const void *)kfn,                         \
                                             hipFuncAttributeMaxDynamicSharedMemorySize, \
                                             (int)lds);                                 \
        if (err != hipSuccess) return err;                                              \
        hipLaunchKernelGGL(kfn, grid, block, lds, s, a);                                \
        return hipGetLastError();                                                       \
    } while (0)
    if (mode == LOCAL) { if (persist) L16(LOCAL, true); else L16(LOCAL, false); }
    if (mode == GLOBAL) { if (persist) L16(GLOBAL, true); else L16(GLOBAL, false); }
    if (persist) L16(SEMIGLOBAL, true); else L16(SEMIGLOBAL, false);
#undef L16
}

hipError_t launch_search16(const SearchArgs &a, int T, int mode, int wpb, int nb, bool persist,
                           size_t lds, hipStream_t s) {
    switch (T) {
        case 16: return launch16_T<16>(a, mode, wpb, nb, persist, lds, s);
        case 32: return launch16_T<32>(a, mode, wpb, nb, persist, lds, s);
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
        const int c = min((int)a.q_codes[Q.off + i], a.A - 1);
        int best = 0;
        for (int k = 0; k < a.AP; k++) {
            const int t = a.inv_map[k];
            if (t != 0xff) best = max(best, (int)a.subst[c * a.A + t]);
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
