// CPU check of the 8-bit-lane recurrence used by the cell-rate probe:
// smax8 against a per-byte maximum, the byte-permute sign spread (emulated
// from its selector definition) against its definition, and column8_local
// against an exact per-target local recurrence (Gotoh, with the floor at
// zero), including the guard bits against an exact overflow test.  Prints
// "ok", or the first failure and exits non-zero.
#include <cstdint>
#include <cstdio>
#include <random>

#include "swar8.h"

using namespace dsa;

// v_perm_b32: byte i of the result is chosen by byte i of sel from the
// eight bytes of {hi, lo} (lo = bytes 0-3); selectors 8-11 spread the sign
// bit of byte 1, 3, 5, 7 over the byte, 12 gives 0x00, 13 and up 0xff.
static uint32_t perm_emul(uint32_t hi, uint32_t lo, uint32_t sel) {
    const uint64_t v = ((uint64_t)hi << 32) | lo;
    uint32_t r = 0;
    for (int i = 0; i < 4; i++) {
        const uint32_t s = (sel >> (8 * i)) & 0xffu;
        uint32_t b;
        if (s < 8) b = (uint32_t)(v >> (8 * s)) & 0xffu;
        else if (s < 12) b = ((v >> (8 * (2 * (s - 8) + 1) + 7)) & 1u) ? 0xffu : 0u;
        else b = s == 12 ? 0u : 0xffu;
        r |= b << (8 * i);
    }
    return r;
}

// The spreader the probe builds from __builtin_amdgcn_perm.
struct SpreadPermEmul {
    uint32_t operator()(uint32_t d) const { return perm_emul(d << 8, d, 0x090B080Au); }
};

static int fail(const char *what, long k) {
    std::printf("FAIL %s at %ld\n", what, k);
    return 1;
}

static int byte(uint32_t w, int t) { return (int)((w >> (8 * t)) & 0xffu); }

int main() {
    std::mt19937 rng(1701);
    // smax8: every byte pair below 128 in a varying position, the other
    // bytes random
    for (uint32_t a = 0; a < 128; a++)
        for (uint32_t b = 0; b < 128; b++) {
            const int pos = (int)((a * 131 + b) & 3);
            const uint32_t keep = ~(0xffu << (8 * pos));
            const uint32_t A = ((uint32_t)rng() & 0x7f7f7f7fu & keep) | (a << (8 * pos));
            const uint32_t B = ((uint32_t)rng() & 0x7f7f7f7fu & keep) | (b << (8 * pos));
            const uint32_t r1 = smax8(A, B, SpreadShift()), r2 = smax8(A, B, SpreadPermEmul());
            for (int i = 0; i < 4; i++) {
                const int x = byte(A, i), y = byte(B, i), m = x > y ? x : y;
                if (byte(r1, i) != m) return fail("smax8 shift", (long)(a * 128 + b));
                if (byte(r2, i) != m) return fail("smax8 perm", (long)(a * 128 + b));
            }
        }
    // the permute spread: 0xff in each byte whose bit 7 is set, else 0
    for (long k = 0; k < (1L << 22); k++) {
        const uint32_t d = (uint32_t)rng();
        uint32_t want = 0;
        for (int i = 0; i < 4; i++) want |= (d >> (8 * i + 7)) & 1u ? 0xffu << (8 * i) : 0u;
        if (SpreadPermEmul()(d) != want) return fail("perm spread", k);
        if (SpreadShift()(d) != (want & 0x7f7f7f7fu)) return fail("shift spread", k);
    }
    // column8_local against the exact recurrence, four targets per word.
    // Scores in [-4, hi]: small hi keeps scores bounded, large hi drives
    // them past the 8-bit range (the guard bit must then be set).
    const int o = 10, e = 1, z = 11, p = 4, NEG = -100000;
    Swar8Gaps g;
    g.o4 = 0x01010101u * o;
    g.e4 = 0x01010101u * e;
    g.z4 = 0x01010101u * z;
    g.np4 = 0u - 0x01010101u * p;
    const uint32_t entry = 0x01010101u * (uint32_t)(z - o + e);  // an E or F that cannot win
    long checked = 0, overflowed = 0;
    for (int trial = 0; trial < 600; trial++) {
        const int cols = 1 + (int)(rng() % 200), hi = 1 + (int)(rng() % 11);
        int h[4][16], E[4][16], best[4], ovf_exact[4];
        uint32_t Hw[16], Ew[16], Bw = g.z4, ovf = 0;
        for (int t = 0; t < 4; t++) {
            best[t] = 0;
            ovf_exact[t] = 0;
            for (int r = 0; r < 16; r++) h[t][r] = 0, E[t][r] = NEG;
        }
        for (int r = 0; r < 16; r++) Hw[r] = g.z4, Ew[r] = entry;
        for (int c = 0; c < cols; c++) {
            uint32_t sc[16];
            int s[4][16];
            for (int r = 0; r < 16; r++) {
                sc[r] = 0;
                for (int t = 0; t < 4; t++) {
                    s[t][r] = (int)(rng() % (uint32_t)(hi + 5)) - 4;
                    sc[r] |= (uint32_t)(s[t][r] + p) << (8 * t);
                }
            }
            // the row above the strip: H in [0, 8 hi], F in [-o, H - o] (as a
            // strip below another would see), or the matrix edge (0, none)
            const bool edge = rng() % 3 == 0;
            int top_h[4], top_f[4];
            uint32_t Hd = 0, F = 0;
            for (int t = 0; t < 4; t++) {
                top_h[t] = edge ? 0 : (int)(rng() % (uint32_t)(8 * hi + 1));
                top_f[t] = edge ? NEG : -o + (int)(rng() % (uint32_t)(top_h[t] + 1));
                Hd |= (uint32_t)(top_h[t] + z) << (8 * t);
                F |= edge ? (entry & 0xffu) << (8 * t) : (uint32_t)(top_f[t] + z) << (8 * t);
            }
            Bw = column8_local(sc, Hw, Ew, Hd, F, g, Bw, ovf, SpreadShift());
            for (int t = 0; t < 4; t++) {
                int above = top_h[t], f = top_f[t];
                for (int r = 0; r < 16; r++) {
                    const int diag = above + s[t][r];
                    if (diag + z > 127) ovf_exact[t] = 1;
                    above = h[t][r];
                    int v = diag > E[t][r] ? diag : E[t][r];
                    v = v > f ? v : f;
                    v = v > 0 ? v : 0;
                    best[t] = best[t] > v ? best[t] : v;
                    E[t][r] = E[t][r] - e > v - o ? E[t][r] - e : v - o;
                    f = f - e > v - o ? f - e : v - o;
                    h[t][r] = v;
                }
                const int guard = (int)((ovf >> (8 * t + 7)) & 1u);
                if (guard != ovf_exact[t]) return fail("guard bit", trial * 1000L + c);
                if (ovf_exact[t]) continue;
                for (int r = 0; r < 16; r++) {
                    if (byte(Hw[r], t) != h[t][r] + z) return fail("H", trial * 1000L + c);
                    if (byte(Ew[r], t) != E[t][r] + z) return fail("E", trial * 1000L + c);
                }
                if (byte(Bw, t) != best[t] + z) return fail("best", trial * 1000L + c);
                checked++;
            }
        }
        for (int t = 0; t < 4; t++) overflowed += ovf_exact[t];
    }
    if (checked < 50000 || overflowed < 200) return fail("too few cases of one kind", checked * 10000 + overflowed);
    std::printf("ok %ld exact columns, %ld overflowed targets\n", checked, overflowed);
    return 0;
}
