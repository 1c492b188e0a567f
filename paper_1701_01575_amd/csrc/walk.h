// Pieces shared by the traceback walks: the CIGAR run writer and the
// residue windows a walk keeps in registers.
#pragma once
#include "internal.h"

namespace dsa {

struct RunWriter {
    uint32_t *out;
    int64_t lo, pos;  // region [lo, hi); runs are written downwards from hi
    uint32_t op = 0, len = 0;
    bool truncated = false;
    bool store = true;  // lanes that follow the same walk keep the state; one stores
    __device__ void flush() {
        if (len == 0) return;
        if (pos > lo) {
            --pos;
            if (store) out[pos] = (len << 4) | op;
        } else {
            truncated = true;
        }
        len = 0;
    }
    __device__ void emit(uint32_t o, uint32_t count) {
        if (count == 0) return;
        if (o != op) { flush(); op = o; }
        len += count;
    }
};

constexpr uint32_t OP_I = 1, OP_D = 2, OP_EQ = 7, OP_X = 8;

// Residue k (0..15) of a 16-residue window held as four uint32.
// (Two 64-bit halves and a shift: a select over the four words would be
// turned into an indexed copy of the array in scratch memory.)
__device__ __forceinline__ int byte_of(const uint32_t (&w)[4], int k) {
    const uint64_t lo = (uint64_t)w[0] | ((uint64_t)w[1] << 32), hi = (uint64_t)w[2] | ((uint64_t)w[3] << 32);
    return (int)(((k < 8 ? lo : hi) >> (8 * (k & 7))) & 0xffu);
}

// Residues [base, base + 16) of a sequence of `len` (zero past its end),
// as 16 independent byte loads.
__device__ __forceinline__ void load_window(const uint8_t *seq, int len, int base, uint32_t (&w)[4]) {
    uint32_t v[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int k = 0; k < 16; k++)
        if (base + k < len) v[k >> 2] |= (uint32_t)seq[base + k] << (8 * (k & 3));
#pragma unroll
    for (int k = 0; k < 4; k++) w[k] = v[k];
}

}  // namespace dsa
