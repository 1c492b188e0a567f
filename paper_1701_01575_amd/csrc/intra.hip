// Intra-sequence (wavefront) database-search kernel for long targets of long
// queries.
//
// The inter-sequence kernel gives one wave a whole (query, 128-target group)
// problem, so a long query against long targets becomes one long sequential
// task.  Here a wave works on one pair of long targets (low and high int16
// halves) and spreads the query over its lanes: lane l owns rows
// [16 s, 16 s + 16) for strip s = 64 * pass + l.  The lanes sweep the target
// columns on an anti-diagonal: at step t lane l computes column t - l + 1, so
// the row above it (lane l - 1's last row, one step earlier) arrives through
// a DPP row shift (wave_shr:1) together with the F leaving it.  Between passes lane 63's
// last row goes through a boundary buffer in HBM.  Same recurrence, modes,
// saturation rules and end-cell rule as the inter-sequence kernel; strips
// track their own strictly-greater best, merged lexicographically (score
// desc, target end asc, query end asc) across passes and lanes.
//
// Scores come from a single-letter query profile of the pass's 1024 rows in
// LDS, shared by the block's waves; the two targets' rows are interleaved
// into packed pairs with v_perm_b32.
#include "intra_unit.h"

namespace dsa {

size_t intra16_lds_bytes(int AP, int A) {
    return (size_t)AP * kProfStride * 2 + (size_t)A * A + 64;
}

template <int MODE>
__global__ void __launch_bounds__(kIntraWaves * kWave) k_intra16(IntraArgs P) {
    extern __shared__ uint4 lds4[];
    const int u = blockIdx.x;
    if (u >= P.n_units) return;
    intra16_unit<MODE>(P, P.units[u], lds4);
}

hipError_t launch_intra16(const IntraArgs &a, int mode, int nb, size_t lds, hipStream_t s) {
    if (nb <= 0) return hipSuccess;
    dim3 grid(nb), block(kIntraWaves * kWave);
#define LI(MODE)                                                                        \
    do {                                                                                \
        auto kfn = k_intra16<MODE>;                                                     \
        hipError_t err = hipFuncSetAttribute((const void *)kfn,                         \
                                             hipFuncAttributeMaxDynamicSharedMemorySize, \
                                             (int)lds);                                 \
        if (err != hipSuccess) return err;                                              \
        hipLaunchKernelGGL(kfn, grid, block, lds, s, a);                                \
        return hipGetLastError();                                                       \
    } while (0)
    if (mode == LOCAL) LI(LOCAL);
    if (mode == GLOBAL) LI(GLOBAL);
    LI(SEMIGLOBAL);
#undef LI
}

}  // namespace dsa
