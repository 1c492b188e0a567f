// Peak probes: measured issue rate of the VALU instructions the alignment
// kernels are built from (packed int16 add/sub with clamp, packed max,
// packed binary16 three-way maximum, plain 32-bit ops) and an HBM stream
// copy.  They give the measured ceilings the roofline fractions are
// compared against.  One more probe checks, over every operand the offset
// local-mode search can produce, that the binary16 three-way maximum orders
// bit patterns as that search assumes.
#include <algorithm>

#include "dsa.h"
#include "internal.h"
#include "pk16.h"
#include "swar8.h"

namespace dsa {

template <int OP>
__device__ __forceinline__ uint32_t probe_op(uint32_t a, uint32_t b) {
    if (OP == 0) return __builtin_bit_cast(uint32_t, __builtin_elementwise_add_sat(
                                              __builtin_bit_cast(s16x2, a), __builtin_bit_cast(s16x2, b)));
    if (OP == 1) return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(
                                              __builtin_bit_cast(s16x2, a), __builtin_bit_cast(s16x2, b)));
    if (OP == 2) return __builtin_bit_cast(uint32_t, __builtin_elementwise_sub_sat(
                                              __builtin_bit_cast(u16x2, a), __builtin_bit_cast(u16x2, b)));
    if (OP == 3) return a + b;
    if (OP == 5) return max3h(a, b, 0x3c003c00u);
    return (uint32_t)max((int)a, (int)b);
}

// 16 independent chains per lane so dependency latency never limits issue.
template <int OP>
__global__ void __launch_bounds__(256) k_probe(uint32_t *out, int iters, uint32_t seed) {
    uint32_t acc[16];
#pragma unroll
    for (int k = 0; k < 16; k++) acc[k] = seed * (threadIdx.x + 1) + k;
    uint32_t b = seed ^ blockIdx.x;
    for (int it = 0; it < iters; it++) {
#pragma unroll
        for (int k = 0; k < 16; k++) acc[k] = probe_op<OP>(acc[k], b);
        b += 0x00010001u;
    }
    uint32_t r = 0;
#pragma unroll
    for (int k = 0; k < 16; k++) r ^= acc[k];
    if (r == 0x12345678u) out[blockIdx.x] = r;  // keeps the chains alive
}

// Order of a binary16 bit pattern as an integer (sign and magnitude).
__device__ __forceinline__ int h_order(uint32_t p) { return p < 0x8000u ? (int)p : 0x7fff - (int)p; }

// Every a in [0x0400, 0x7bff] and its negative, every b in [0x0400, 0x7bff],
// c = the offset floor: max3h must return the operand of greatest order in
// both halves (the high half gets b and a swapped).  Counts the failures.
__global__ void k_max3_order(unsigned long long *bad) {
    const uint32_t c = kBias16;
    unsigned long long nbad = 0;
    const int64_t na = 2 * 0x7800, nb = 0x7800, total = na * nb;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int ia = (int)(k / nb), ib = (int)(k - (int64_t)ia * nb);
        const uint32_t a = (ia < 0x7800 ? 0x0400u : 0x8400u) + (uint32_t)(ia % 0x7800);
        const uint32_t b = 0x0400u + (uint32_t)ib;
        const uint32_t r = max3h(a | (b << 16), b | (a << 16), c | (c << 16));
        uint32_t want = h_order(a) > h_order(b) ? a : b;
        want = h_order(want) > h_order(c) ? want : c;
        nbad += ((r & 0xffffu) != want) + ((r >> 16) != want);
    }
    if (nbad) atomicAdd(bad, nbad);
}

// Cell-rate probes: the local recurrence of one 16-row strip column after
// column, scores from a profile in LDS (a random profile row per column),
// nothing else (no boundary rows, no end-cell bookkeeping).  k_cells16: two
// targets per lane, packed int16, the search kernel's column (offset
// binary16 three-way maxima in the column-shifted frame); k_cells8: four
// targets per lane, 8-bit lanes in 32-bit ALU operations (swar8.h), the two
// 8-bit pairs of a row's scores from two profile reads, as an int8 first
// pass over the same database layout would fetch them.  Values are not kept
// in range (the profile favours matches); only the instruction stream
// matters here.
__global__ void __launch_bounds__(256) k_cells16(uint32_t *out, int cols, uint32_t seed) {
    __shared__ uint32_t prof[64 * 16];
    for (int k = threadIdx.x; k < 64 * 16; k += blockDim.x) prof[k] = dup((int)((k * 2654435761u) >> 28) - 3);
    __syncthreads();
    uint32_t H[16], E[16];
#pragma unroll
    for (int r = 0; r < 16; r++) {
        H[r] = dup(kBias16);
        E[r] = dup(kBias16);
    }
    uint32_t B = dup(kBias16), code = seed * (threadIdx.x + 1u);
    const uint32_t oe2 = dup(10), e2 = dup(1), phi = dup(kBias16);
    for (int c = 0; c < cols; c++) {
        code = code * 1664525u + 1013904223u;
        const uint32_t *pr = prof + ((code >> 26) << 4);
        uint32_t sc[16];
#pragma unroll
        for (int r = 0; r < 16; r++) sc[r] = pr[r];
        uint32_t F = dup(kBias16);
        B = column16_local_cs<16>(sc, H, E, dup(kBias16), F, oe2, e2, phi, B);
    }
    out[blockIdx.x * blockDim.x + threadIdx.x] = B ^ H[15] ^ E[15];
}

struct SpreadPerm {  // bit 7 of each byte over the byte: one v_perm_b32 (see swar8.h)
    __device__ uint32_t operator()(uint32_t d) const { return __builtin_amdgcn_perm(d << 8, d, 0x090B080Au); }
};

__global__ void __launch_bounds__(256) k_cells8(uint32_t *out, int cols, uint32_t seed) {
    __shared__ uint16_t prof[64 * 16];  // two targets' scores + p per entry
    for (int k = threadIdx.x; k < 64 * 16; k += blockDim.x)
        prof[k] = (uint16_t)(((k * 2654435761u) >> 28) | (((k * 40503u) >> 12) & 15u) << 8);
    __syncthreads();
    Swar8Gaps g;
    g.o4 = 0x0a0a0a0au;
    g.e4 = 0x01010101u;
    g.z4 = 0x0b0b0b0bu;
    g.np4 = 0u - 0x04040404u;
    uint32_t H[16], E[16];
#pragma unroll
    for (int r = 0; r < 16; r++) {
        H[r] = g.z4;
        E[r] = g.z4 - g.o4 + g.e4;
    }
    uint32_t B = g.z4, ovf = 0, code = seed * (threadIdx.x + 1u);
    for (int c = 0; c < cols; c++) {
        code = code * 1664525u + 1013904223u;
        const uint16_t *pa = prof + ((code >> 26) << 4), *pb = prof + (((code >> 20) & 63u) << 4);
        uint32_t sc[16];
#pragma unroll
        for (int r = 0; r < 16; r++) sc[r] = (uint32_t)pa[r] | ((uint32_t)pb[r] << 16);
        uint32_t F = g.z4 - g.o4 + g.e4;
        B = column8_local(sc, H, E, g.z4, F, g, B, ovf, SpreadPerm());
    }
    out[blockIdx.x * blockDim.x + threadIdx.x] = B ^ H[15] ^ E[15] ^ ovf;
}

// SpreadPerm against its definition on 2^26 hashed words (every pattern of
// the four sign bits with varied low bits).  Counts the failures.
__global__ void k_spread_check(unsigned long long *bad) {
    unsigned long long nbad = 0;
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < (1u << 26); k += gridDim.x * blockDim.x) {
        const uint32_t d = (k * 2654435761u) ^ (k << 7) ^ (k >> 11);
        uint32_t want = 0;
        for (int i = 0; i < 4; i++) want |= ((d >> (8 * i + 7)) & 1u) ? 0xffu << (8 * i) : 0u;
        nbad += SpreadPerm()(d) != want;
    }
    if (nbad) atomicAdd(bad, nbad);
}

__global__ void k_stream_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

}  // namespace dsa

using namespace dsa;

// which: 0 = v_pk_add_i16 clamp, 1 = v_pk_max_i16, 2 = v_pk_sub_u16 clamp,
// 3 = v_add_u32, 4 = v_max_i32, 6 = v_pk_maximum3_f16 (result: instructions
// per second summed over lanes); 5 = HBM copy of `bytes` (result: bytes read
// + written per second); 7 = the three-way maximum order check (result: the
// number of wrong results); 8 = local cells per second, packed int16 (two
// targets per lane), 9 = the same with four 8-bit targets per lane, each
// over `size` columns; 10 = the byte sign-spread check of the 8-bit probe
// (result: the number of wrong results); 11..14 = 8 with 1..4 waves per
// SIMD instead of 8 (how many waves the column needs to keep a SIMD busy).
extern "C" int dsa_probe(int which, int64_t size, double *rate) {
    if (!rate || which < 0 || which > 14 || size <= 0) return DSA_E_INVAL;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess) return DSA_E_DEVICE;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    hipEvent_t a = nullptr, b = nullptr;
    void *p0 = nullptr, *p1 = nullptr;
    int rc = DSA_OK;
    auto ok = [&](hipError_t e) {
        if (e != hipSuccess && rc == DSA_OK) rc = DSA_E_DEVICE;
        return rc == DSA_OK;
    };
    if (ok(hipEventCreate(&a)) && ok(hipEventCreate(&b))) {
        float ms = 0.f;
        if (which == 8 || which == 9 || (which >= 11 && which <= 14)) {
            // 8 x 256-thread blocks per CU (8 waves per SIMD), or for 11..14
            // the int16 column with 1..4 waves per SIMD
            const int blocks = cus * (which >= 11 ? which - 10 : 8);
            const int cols = (int)std::min<int64_t>(size, 1 << 24);
            if (ok(hipMalloc(&p0, (size_t)blocks * 256 * sizeof(uint32_t)))) {
                uint32_t *out = (uint32_t *)p0;
                auto launch = [&]() {
                    if (which == 9) hipLaunchKernelGGL(k_cells8, dim3(blocks), dim3(256), 0, 0, out, cols, 7u);
                    else hipLaunchKernelGGL(k_cells16, dim3(blocks), dim3(256), 0, 0, out, cols, 7u);
                    return hipGetLastError();
                };
                if (ok(launch()) && ok(hipEventRecord(a, 0)) && ok(launch()) && ok(hipEventRecord(b, 0)) &&
                    ok(hipEventSynchronize(b)) && ok(hipEventElapsedTime(&ms, a, b)))
                    *rate = (double)blocks * 256.0 * (which == 9 ? 4.0 : 2.0) * 16.0 * cols / (ms * 1e-3);
            }
        } else if (which == 7 || which == 10) {
            unsigned long long bad = 0;
            if (ok(hipMalloc(&p0, sizeof(bad))) && ok(hipMemset(p0, 0, sizeof(bad)))) {
                if (which == 7) hipLaunchKernelGGL(k_max3_order, dim3(cus * 8), dim3(256), 0, 0, (unsigned long long *)p0);
                else hipLaunchKernelGGL(k_spread_check, dim3(cus * 8), dim3(256), 0, 0, (unsigned long long *)p0);
                if (ok(hipGetLastError()) && ok(hipMemcpy(&bad, p0, sizeof(bad), hipMemcpyDeviceToHost)))
                    *rate = (double)bad;
            }
        } else if (which != 5) {
            const int blocks = cus * 8;  // 8 x 4 waves per CU
            const int iters = (int)std::min<int64_t>(size, 1 << 30);
            uint32_t *out = nullptr;
            if (ok(hipMalloc(&p0, blocks * sizeof(uint32_t)))) {
                out = (uint32_t *)p0;
                auto launch = [&]() {
                    switch (which) {
                        case 0: hipLaunchKernelGGL(k_probe<0>, dim3(blocks), dim3(256), 0, 0, out, iters, 7u); break;
                        case 1: hipLaunchKernelGGL(k_probe<1>, dim3(blocks), dim3(256), 0, 0, out, iters, 7u); break;
                        case 2: hipLaunchKernelGGL(k_probe<2>, dim3(blocks), dim3(256), 0, 0, out, iters, 7u); break;
                        case 3: hipLaunchKernelGGL(k_probe<3>, dim3(blocks), dim3(256), 0, 0, out, iters, 7u); break;
                        case 6: hipLaunchKernelGGL(k_probe<5>, dim3(blocks), dim3(256), 0, 0, out, iters, 7u); break;
                        default: hipLaunchKernelGGL(k_probe<4>, dim3(blocks), dim3(256), 0, 0, out, iters, 7u); break;
                    }
                    return hipGetLastError();
                };
                if (ok(launch()) && ok(hipEventRecord(a, 0)) && ok(launch()) && ok(hipEventRecord(b, 0)) &&
                    ok(hipEventSynchronize(b)) && ok(hipEventElapsedTime(&ms, a, b)))
                    *rate = (double)blocks * 256.0 * 16.0 * iters / (ms * 1e-3);
            }
        } else {
            const int64_t n = size / 16;
            if (ok(hipMalloc(&p0, n * 16)) && ok(hipMalloc(&p1, n * 16)) && ok(hipMemset(p0, 1, n * 16))) {
                const uint4 *src = (const uint4 *)p0;
                uint4 *dst = (uint4 *)p1;
                hipLaunchKernelGGL(k_stream_copy, dim3(cus * 16), dim3(256), 0, 0, src, dst, n);
                if (ok(hipGetLastError()) && ok(hipEventRecord(a, 0))) {
                    for (int r = 0; r < 5; r++)
                        hipLaunchKernelGGL(k_stream_copy, dim3(cus * 16), dim3(256), 0, 0, src, dst, n);
                    if (ok(hipGetLastError()) && ok(hipEventRecord(b, 0)) && ok(hipEventSynchronize(b)) &&
                        ok(hipEventElapsedTime(&ms, a, b)))
                        *rate = 5.0 * 2.0 * (double)n * 16.0 / (ms * 1e-3);
                }
            }
        }
    }
    if (p0) (void)hipFree(p0);
    if (p1) (void)hipFree(p1);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    return rc;
}
