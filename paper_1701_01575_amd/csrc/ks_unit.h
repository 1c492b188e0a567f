// The strip-pipelined database-search unit (local mode): one query against
// one 128-target group, taken by the whole block of the persistent search
// kernel.  An inter-sequence unit walks all strips of the query over the
// group with one wave; on a long query and a wide group that single
// dependency chain outlasts the rest of the search.  Here the block's W waves
// share the strips: wave w takes strips w, w + W, w + 2W, ... and, one
// 4-column block behind the wave above it, fills the same group columns, so
// W strips are in flight at once.  Waves step in lockstep, one 4-column block
// per tick between block barriers:
//   - wave w hands the bottom row of each block to wave w + 1 through a
//     two-slot ring in LDS (written at tick t, read at tick t + 1);
//   - the last wave hands its strip to wave 0's next strip through the
//     group's boundary row in HBM (read nblk - W + 1 ticks later, so wave 0
//     prefetches it one block ahead);
//   - each round of W strips has a single-letter profile of its 16 W rows in
//     LDS (two buffers: round r + 1's is built while round r runs), packed per
//     target pair with v_perm like the wavefront units.
// Arithmetic, frame, end-cell rule and overflow flag are those of the
// inter-sequence kernel.
#pragma once
#include <type_traits>

#include "internal.h"
#include "pk16.h"

namespace dsa {

// Boundary words written by another wave of the block: loaded past the
// vector L1 (an agent-scope relaxed atomic load), so that a line this CU
// cached in an earlier round is never read stale.
__device__ __forceinline__ uint2 load_handover(const uint2 *p) {
    const uint64_t v = __hip_atomic_load(reinterpret_cast<const uint64_t *>(p), __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    return make_uint2((uint32_t)v, (uint32_t)(v >> 32));
}

__device__ __forceinline__ void ks16_unit(const SearchArgs &P, const SearchUnit &U, int u, uint4 *lds4) {
    constexpr int T = 16;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int W = blockDim.x >> 6;
    const int o = P.o, e = P.e, AP = P.AP, A = P.A;
    const int stride = 16 * W + kKsRowPad;  // int16 per letter row of a round profile
    int16_t *qp = reinterpret_cast<int16_t *>(lds4);                          // [2][AP][stride]
    uint2 *ring = reinterpret_cast<uint2 *>(qp + 2 * AP * stride);            // [W-1][2][4][64]
    // per pair code: byte offsets of its two letters' rows in a round profile
    uint32_t *rows = reinterpret_cast<uint32_t *>(ring + (W - 1) * 2 * 4 * kWave);  // [AP*AP]

    const QueryInfo Q = P.qinfo[U.q];
    const GroupInfo G = P.grp[U.g0];
    const int m = Q.len, S = (m + T - 1) / T, R = (S + W - 1) / W;
    const int nblk = G.ncols >> 2;
    const uint8_t *qc = P.q_codes + Q.off;
    for (int k = tid; k < AP * AP; k += blockDim.x)
        rows[k] = (uint32_t)(P.pair_dec[2 * k] * stride * 2) | ((uint32_t)(P.pair_dec[2 * k + 1] * stride * 2) << 16);

    // single-letter profile of round r (rows 16 W r ...), scores + e (the frame)
    auto build = [&](int r) {
        int16_t *b = qp + (r & 1) * AP * stride;
        const int rows = 16 * W;
        for (int k = tid; k < AP * rows; k += blockDim.x) {
            const int c = k / rows, rr = k - c * rows;
            const int i = r * rows + rr;
            int v = NEG16;
            const int mc = P.inv_map[c];
            if (i < m && mc != 0xff) v = qscore(P.pssm, P.subst, P.q_codes, A, Q.off + i, U.q, mc) + e;
            b[c * stride + rr] = (int16_t)v;
        }
    };
    build(0);
    __syncthreads();

    const uint32_t o2e = dup(o - e), e2 = dup(e);
    const int rb = e > 0 ? max(1, (kShift16 / 4) / e) : (1 << 28);
    const uint32_t back2 = dup(4 * rb * e);
    const uint2 *pk = P.packed + G.off + lane;
    uint2 *bnd = P.bnd + (int64_t)U.qslot * P.bnd_slot_stride + G.bnd + lane;

    // this wave's best over its finished strips, per half (plain values)
    uint32_t Gs = 0, Gj = 0, Gi = 0;
    uint32_t H[T], E[T], Hd_top = 0, B = 0, Bj = 0, Bi = 0;
    uint2 hf_n[4];
#pragma unroll
    for (int c = 0; c < 4; c++) hf_n[c] = make_uint2(0, 0);
    // a wave's active ticks take the blocks of its strips in order, block
    // nblk - 1 of one strip followed by block 0 of the next: the codes of the
    // next block are loaded one tick ahead
    uint2 cd_n = pk[0];

    const int ticks = R * nblk + W - 1;
    // the step loop, specialised by the wave's role: wave 0 reads the row
    // above from the boundary row (or the top boundary), the others from
    // the ring; the last wave writes its bottom row to the boundary row,
    // the others to the ring
    auto steps = [&](auto role) {
        constexpr int ROLE = decltype(role)::value;  // 0: first wave, 1: middle, 2: last
        for (int t = 0; t < ticks; t++) {
            // round r + 1's profile while round r is under way (its buffer was
            // last read at tick (r - 1) nblk + W - 2 and is first read at tick
            // (r + 1) nblk; nblk > W)
            if (t >= W && (t - W) % nblk == 0) {
                const int r1 = (t - W) / nblk + 1;
                if (r1 < R) build(r1);
            }
            const int tt = t - wave;
            const int r = tt >= 0 ? tt / nblk : 0, c4 = tt >= 0 ? tt - r * nblk : 0;
            const int s = r * W + wave;
            if (tt >= 0 && r < R && s < S) {
                const int i0 = s * T;
                if (c4 == 0) {  // a new strip: column 0 sits one e below column 1's frame
#pragma unroll
                    for (int x = 0; x < T; x++) {
                        H[x] = dup(kBias16 - e);
                        E[x] = dup(kBias16);
                    }
                    Hd_top = dup(kBias16 - e);
                    B = maxs(subs(Gs, dup(1)), 0u);
                    Bj = 0;
                    Bi = 0;
                } else if (c4 % rb == 0) {  // take the column frame back
#pragma unroll
                    for (int x = 0; x < T; x++) {
                        H[x] = subw(H[x], back2);
                        E[x] = subw(E[x], back2);
                    }
                    Hd_top = subw(Hd_top, back2);
                }
                const int cbase = kBias16 + (c4 % rb) * 4 * e;
                // the row above this block: the strip above's bottom row
                uint2 hf[4];
                if (ROLE == 0 && s == 0) {
#pragma unroll
                    for (int c = 0; c < 4; c++) hf[c] = make_uint2(dup(cbase + c * e), dup(cbase + c * e));
                } else if (ROLE != 0) {
                    const uint2 *src = ring + ((wave - 1) * 2 + ((t - 1) & 1)) * 4 * kWave + lane;
#pragma unroll
                    for (int c = 0; c < 4; c++) hf[c] = src[c * kWave];
                } else {
                    if (c4 == 0) {
#pragma unroll
                        for (int c = 0; c < 4; c++) hf_n[c] = load_handover(bnd + (int64_t)c * 64);
                    }
#pragma unroll
                    for (int c = 0; c < 4; c++) hf[c] = hf_n[c];
                    if (c4 + 1 < nblk) {
#pragma unroll
                        for (int c = 0; c < 4; c++) hf_n[c] = load_handover(bnd + (int64_t)(4 * c4 + 4 + c) * 64);
                    }
                }
                const uint2 cd = cd_n;
                cd_n = pk[(int64_t)(c4 + 1 < nblk ? c4 + 1 : 0) * 64];
                const char *prow = reinterpret_cast<const char *>(qp + (r & 1) * AP * stride + wave * 16);
                // the four columns' letter-row offsets up front, so that a
                // column's profile reads wait for one LDS round trip, not two
                uint32_t rw4[4];
#pragma unroll
                for (int c = 0; c < 4; c++) rw4[c] = rows[((c < 2 ? cd.x : cd.y) >> ((c & 1) * 16)) & 0xffffu];
                uint2 out[4];
#pragma unroll
                for (int c = 0; c < 4; c++) {
                    const int j = c4 * 4 + c + 1;
                    const uint32_t rw = rw4[c];
                    const uint4 *plo = reinterpret_cast<const uint4 *>(prow + (rw & 0xffffu));
                    const uint4 *phi = reinterpret_cast<const uint4 *>(prow + (rw >> 16));
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
                    const int cj = cbase + c * e;
                    const uint32_t Hup = hf[c].x;
                    uint32_t F = hf[c].y;
                    const uint32_t Hd = Hd_top;
                    Hd_top = Hup;
                    const uint32_t Bc = addu(B, dup(cj));
                    const uint32_t nb = column16_local_cs<T>(sc, H, E, Hd, F, o2e, e2, dup(cj + e), Bc);
                    if (nb != Bc) {
                        const uint32_t mask = nzmask(nb ^ Bc);
                        const uint32_t idx = first_row_of<T>(H, nb);
                        Bi = bfi(mask, addu(idx, dup(i0 + 1)), Bi);
                        Bj = bfi(mask, dup(j), Bj);
                        B = maxs(B, subw(nb, dup(cj)));
                    }
                    out[c] = make_uint2(H[T - 1], F);
                }
                // hand the block's bottom row on
                if (ROLE != 2) {
                    uint2 *dst = ring + (wave * 2 + (t & 1)) * 4 * kWave + lane;
#pragma unroll
                    for (int c = 0; c < 4; c++) dst[c * kWave] = out[c];
                } else if (s + 1 < S) {
#pragma unroll
                    for (int c = 0; c < 4; c++) bnd[(int64_t)(4 * c4 + c) * 64] = out[c];
                }
                if (c4 == nblk - 1) {  // strip done: merge its best into the wave's
                    const int b2[2] = {lo16(B), hi16(B)};
                    const int bj[2] = {(int)(Bj & 0xffff), (int)(Bj >> 16)};
                    const int bi[2] = {(int)(Bi & 0xffff), (int)(Bi >> 16)};
                    uint64_t gk[2] = {end_key(lo16(Gs), (int)(Gj & 0xffff), (int)(Gi & 0xffff)),
                                      end_key(hi16(Gs), (int)(Gj >> 16), (int)(Gi >> 16))};
#pragma unroll
                    for (int h = 0; h < 2; h++) {
                        const uint64_t kk = end_key(b2[h], bj[h], bi[h]);
                        gk[h] = (b2[h] > 0) ? umax64(gk[h], kk) : gk[h];
                    }
                    Gs = pack2(key_score(gk[0]), key_score(gk[1]));
                    Gj = pack2(key_j(gk[0]), key_j(gk[1]));
                    Gi = pack2(key_i(gk[0]), key_i(gk[1]));
                }
            }
            __syncthreads();
        }
    };
    if (wave == 0) steps(std::integral_constant<int, 0>{});
    else if (wave == W - 1) steps(std::integral_constant<int, 2>{});
    else steps(std::integral_constant<int, 1>{});

    // merge the waves' bests per target: end keys through LDS
    uint64_t *keys = reinterpret_cast<uint64_t *>(lds4);  // [W][2][64]
    keys[(wave * 2 + 0) * kWave + lane] = end_key(lo16(Gs), (int)(Gj & 0xffff), (int)(Gi & 0xffff));
    keys[(wave * 2 + 1) * kWave + lane] = end_key(hi16(Gs), (int)(Gj >> 16), (int)(Gi >> 16));
    __syncthreads();
    if (wave == 0) {
        bool ovf = false;
#pragma unroll
        for (int h = 0; h < 2; h++) {
            uint64_t k = keys[h * kWave + lane];
            for (int w = 1; w < W; w++) k = umax64(k, keys[(w * 2 + h) * kWave + lane]);
            const int slot = G.slot0 + h * 64 + lane;
            const int tg = P.slot_target[slot];
            if (tg < 0) continue;
            const int sc = key_score(k);
            const int64_t oi = (int64_t)U.q * P.n_t + tg;
            P.out_score[oi] = sc;
            if (P.out_qend) P.out_qend[oi] = sc > 0 ? key_i(k) - 1 : -1;
            if (P.out_tend) P.out_tend[oi] = sc > 0 ? key_j(k) - 1 : -1;
            if (P.out_status) P.out_status[oi] = 0;
            ovf |= sc > kLocal16Max;
        }
        if (__builtin_amdgcn_ballot_w64(ovf) && lane == 0) P.unit_flags[u] = 1;
    }
    __syncthreads();
}

}  // namespace dsa
