// Per-query top-K selection over database-search results (Section II.B.2:
// the K most similar alignments by score, sorted).  One block per query; K
// passes, each a block-wide maximum of the 64-bit key
//   (score << 32) | ~target_index
// restricted to keys below the previous winner, so equal scores come out in
// ascending original target order.  Local alignments qualify only with a
// positive score.  Unused slots get t_index = -1, score 0, coordinates -1.
#include "internal.h"

namespace dsa {

__global__ void __launch_bounds__(256) k_topk(TopkArgs a) {
    const int q = blockIdx.x;
    if (q >= a.n_q) return;
    __shared__ uint64_t red[256];
    __shared__ uint64_t s_prev;
    const int tid = threadIdx.x;
    const int32_t *sc = a.score + (int64_t)q * a.n_t;
    if (tid == 0) s_prev = ~0ull;
    __syncthreads();
    for (int k = 0; k < a.K; k++) {
        const uint64_t prev = s_prev;
        uint64_t best = 0;
        for (int64_t t = tid; t < a.n_t; t += blockDim.x) {
            const int s = sc[t];
            if (a.positive_only && s <= 0) continue;
            const uint64_t key = ((uint64_t)(uint32_t)(s + 0x40000000) << 32) | (uint32_t)~(uint32_t)t;
            best = (key < prev && key > best) ? key : best;
        }
        red[tid] = best;
        __syncthreads();
        for (int w = blockDim.x / 2; w > 0; w >>= 1) {
            if (tid < w) red[tid] = red[tid] > red[tid + w] ? red[tid] : red[tid + w];
            __syncthreads();
        }
        const uint64_t win = red[0];
        const int64_t oi = (int64_t)q * a.K + k;
        if (tid == 0) {
            if (win == 0) {
                a.out_tindex[oi] = -1;
                a.out_score[oi] = 0;
                if (a.out_qend) a.out_qend[oi] = -1;
                if (a.out_tend) a.out_tend[oi] = -1;
                if (a.out_status) a.out_status[oi] = 0;
                a.hit_t[oi] = -1;
            } else {
                const int64_t t = (int64_t)(~(uint32_t)(win & 0xffffffffu));
                const int64_t fi = (int64_t)q * a.n_t + t;
                a.out_tindex[oi] = t;
                a.out_score[oi] = (int)(uint32_t)(win >> 32) - 0x40000000;
                if (a.out_qend) a.out_qend[oi] = a.qend[fi];
                if (a.out_tend) a.out_tend[oi] = a.tend[fi];
                if (a.out_status) a.out_status[oi] = a.status[fi];
                a.hit_t[oi] = (int32_t)t;
            }
            s_prev = win == 0 ? 0 : win;
        }
        __syncthreads();
    }
}

hipError_t launch_topk(const TopkArgs &a, hipStream_t s) {
    if (a.n_q <= 0 || a.K <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_topk, dim3(a.n_q), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace dsa
