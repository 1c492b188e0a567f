// Local-mode affine-gap recurrence on four 8-bit lanes of a 32-bit register
// (four targets per register), in plain 32-bit ALU operations: gfx950 has
// packed 16-bit and binary16 maxima but no packed 8-bit maximum or
// saturating 8-bit add.  Only the cell-rate probe uses it; it measures what
// an int8 first pass of the database search would issue per cell.
//
// Values are held as value + z, z >= gap_open + gap_extend and z >= the
// largest penalty of the matrix, in the low 7 bits of each byte; bit 7 is a
// guard.  Subtracting gap_open or gap_extend then never borrows across
// bytes, the diagonal sum takes the score + p profile entry and subtracts p
// in the same add, and a sum that passes 127 sets its byte's guard bit,
// which the caller collects as that target's overflow (its result must be
// computed again in a wider type).
#pragma once
#include <cstdint>

namespace dsa {

// Bit 7 of each byte spread over its byte, three ALU operations (0x7f per
// byte, which is enough below 128).  The probe passes a one-instruction
// byte-permute spreader instead.
struct SpreadShift {
    __host__ __device__ uint32_t operator()(uint32_t d) const {
        const uint32_t m = d & 0x80808080u;
        return m - (m >> 7);
    }
};

// Per byte, the larger of a and b (bytes below 128): a + 128 - b keeps bit
// 7 where a >= b and never borrows; the spread bit picks a or b.
template <class Spread>
__host__ __device__ inline uint32_t smax8(uint32_t a, uint32_t b, Spread sp) {
    const uint32_t m = sp((a | 0x80808080u) - b);
    return (a & m) | (b & ~m);
}

struct Swar8Gaps {
    uint32_t o4, e4, z4, np4;  // gap_open, gap_extend, z in every byte; -p as a 32-bit addend
};

// One column of 16 rows for four targets.  sc[r]: the four targets'
// scores + p for row r (bytes); H, E: the rows' state (E of this column on
// entry, of the next on exit); Hd: H of the row above in the previous
// column; F: F entering row 0.  Returns the maximum of B and the column's
// H; ovf collects guard bits.
template <class Spread>
__host__ __device__ inline uint32_t column8_local(const uint32_t (&sc)[16], uint32_t (&H)[16], uint32_t (&E)[16],
                                                  uint32_t Hd, uint32_t &F, const Swar8Gaps &g, uint32_t B,
                                                  uint32_t &ovf, Spread sp) {
#pragma unroll
    for (int r = 0; r < 16; r++) {
        uint32_t t = Hd + sc[r] + g.np4;  // value + z + s, borrow-free per byte
        ovf |= t;
        t &= 0x7f7f7f7fu;                 // an overflowed byte stays in its own lane
        Hd = H[r];
        const uint32_t h = smax8(smax8(smax8(t, E[r], sp), F, sp), g.z4, sp);  // the 0 of local mode
        B = smax8(B, h, sp);
        const uint32_t ho = h - g.o4;
        E[r] = smax8(E[r] - g.e4, ho, sp);
        F = smax8(F - g.e4, ho, sp);
        H[r] = h;
    }
    return B;
}

}  // namespace dsa
