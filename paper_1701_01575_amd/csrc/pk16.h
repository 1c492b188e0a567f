// Packed int16 helpers shared by the alignment kernels.  A uint32 register
// holds two independent int16 lanes; every helper maps to one VOP3P
// instruction (v_pk_add_i16 / v_pk_sub_i16 / v_pk_sub_u16 with clamp,
// v_pk_max_i16 / v_pk_max_u16 / v_pk_min_u16, v_pk_add_u16, v_pk_mul_lo_u16).
#pragma once
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
__device__ __forceinline__ uint32_t subw(uint32_t a, uint32_t b) { return Bu(U2(a) - U2(b)); }
// Three-way maximum of two binary16 pairs (v_pk_maximum3_f16).  On positive
// normal patterns it is the unsigned integer maximum of the bit patterns.
__device__ __forceinline__ uint32_t max3h(uint32_t a, uint32_t b, uint32_t c) {
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    const h2 x = __builtin_bit_cast(h2, a), y = __builtin_bit_cast(h2, b), z = __builtin_bit_cast(h2, c);
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_maximum(__builtin_elementwise_maximum(x, y), z));
}

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


// End-cell order as one integer: a larger key is a better end cell (higher
// score, then smaller target end j, then smaller query end i; j, i < 65536).
// Comparing keys with a plain maximum keeps the merges free of the nested
// short-circuit conditions the compiler if-converted incorrectly.
__device__ __forceinline__ uint64_t end_key(int score, int j, int i) {
    return ((uint64_t)(uint32_t)(score + 0x40000000) << 32) |
           ((uint64_t)(uint32_t)(0xffff - j) << 16) | (uint64_t)(uint32_t)(0xffff - i);
}
__device__ __forceinline__ int key_score(uint64_t k) { return (int)(uint32_t)(k >> 32) - 0x40000000; }
__device__ __forceinline__ int key_j(uint64_t k) { return 0xffff - (int)((k >> 16) & 0xffff); }
__device__ __forceinline__ int key_i(uint64_t k) { return 0xffff - (int)(k & 0xffff); }
__device__ __forceinline__ uint64_t umax64(uint64_t a, uint64_t b) { return a > b ? a : b; }

// Free query end (semi-global QE): the best cell of the last column, over
// rows i0 + 1 .. of one strip that are real (i <= m); strictly greater, rows
// in order, so the smallest i wins ties (strips are visited in order too).
template <int T>
__device__ __forceinline__ void last_column_scan(const int (&H)[T], int i0, int m, int &Qs, int &Qi) {
#pragma unroll
    for (int r = 0; r < T; r++) {
        if (i0 + r < m && H[r] > Qs) {
            Qs = H[r];
            Qi = i0 + r + 1;
        }
    }
}

template <int T>
__device__ __forceinline__ uint32_t pick_row(const uint32_t (&H)[T], int r) {
    uint32_t v = H[0];
#pragma unroll
    for (int k = 1; k < T; k++) v = (k == r) ? H[k] : v;
    return v;
}

// One column of a strip, local mode, packed int16 held as value + kBias16.
// E and F are floored at the bias (a zero floor on the values), which
// implies the 0 of the H maximum.  The floors and the H maximum are binary16
// three-way maxima; the additions and subtractions are integer.  Returns the
// maximum of B and the column, also a three-way maximum chain.
template <int T>
__device__ __forceinline__ uint32_t column16_local(const uint32_t (&sc)[T], uint32_t (&H)[T],
                                                   uint32_t (&E)[T], uint32_t Hd, uint32_t &F,
                                                   uint32_t o2, uint32_t e2, uint32_t B) {
    static_assert(T % 2 == 0, "rows are taken in pairs by the maximum chain");
    const uint32_t K2 = dup(kBias16);
    uint32_t cm = B, held = 0;
#pragma unroll
    for (int r = 0; r < T; r++) {
        const uint32_t t = addu(Hd, sc[r]);
        Hd = H[r];
        const uint32_t h = max3h(t, E[r], F);
        if (r & 1) cm = max3h(cm, held, h);
        else held = h;
        const uint32_t ho = subw(h, o2);
        E[r] = max3h(subw(E[r], e2), ho, K2);
        F = max3h(subw(F, e2), ho, K2);
        H[r] = h;
    }
    return cm;
}

// One column, local mode, in the column-shifted frame of the inter-sequence
// kernel: every value of column j is held as value + c_j, where c_j grows by
// e from column to column (the caller takes a multiple of e back between
// column blocks).  In that frame the gap-extend decrement of E disappears,
// E[j+1] = max(E[j], H[j] - (o - e)), and F is formed as X = max(F, H - (o -
// e)), the next row's F being X - e, so E and F share one subtraction.
// phi = c_j + e is the floor of E[j+1] and of X (a zero floor on E and F,
// which implies the 0 of the H maximum); the profile carries s + e, which
// moves the diagonal term into this column's frame.  oe2 = o - e.  Returns
// max(Bc, column), Bc being the running best in this column's frame.
template <int T>
__device__ __forceinline__ uint32_t column16_local_cs(const uint32_t (&sc)[T], uint32_t (&H)[T],
                                                      uint32_t (&E)[T], uint32_t Hd, uint32_t &F,
                                                      uint32_t oe2, uint32_t e2, uint32_t phi,
                                                      uint32_t Bc) {
    static_assert(T % 2 == 0, "rows are taken in pairs by the maximum chain");
    uint32_t cm = Bc, held = 0;
#pragma unroll
    for (int r = 0; r < T; r++) {
        const uint32_t t = addu(Hd, sc[r]);
        Hd = H[r];
        const uint32_t h = max3h(t, E[r], F);
        if (r & 1) cm = max3h(cm, held, h);
        else held = h;
        const uint32_t hx = subw(h, oe2);
        E[r] = max3h(E[r], hx, phi);
        F = subw(max3h(F, hx, phi), e2);
        H[r] = h;
    }
    // keep the E updates in this column's block, where they fill the gaps
    // of the F chain, rather than sunk past the caller's end-cell branch
#pragma unroll
    for (int r = 0; r < T; r++) asm volatile("" : "+v"(E[r]));
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

// First row r (0-based) whose H equals the column maximum cm, per half,
// as a packed uint16 pair.
template <int T>
__device__ __forceinline__ uint32_t first_row_of(const uint32_t (&H)[T], uint32_t cm) {
    // per half: a stays 1 while every row so far differs from cm, and idx
    // counts those rows, which is the index of the first equal row (T when
    // there is none): three packed ops per row
    uint32_t a = 0x00010001u, idx = 0;
#pragma unroll
    for (int r = 0; r < T; r++) {
        a = minu(a, H[r] ^ cm);
        idx = addu(idx, a);
    }
    return idx;
}

}  // namespace dsa
