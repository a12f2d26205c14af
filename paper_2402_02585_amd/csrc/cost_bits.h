// Bit-sliced clause counting: the word layout, clause records and counter
// arithmetic used by the cost-table kernels. Host and device share these
// definitions (the host packs the records, the device evaluates them).
//
// One 32-bit word carries 32 assignments. Word w covers z in [32w, 32w+32);
// word bit j = 8q + r (q in [0,4), r in [0,8)) holds z = 32w + 4r + q. With
// this order the 8x8 bit transposes at the end leave, in transposed row r,
// the byte-packed costs of z = 32w + 4r .. 32w + 4r + 3, ready to store.
//
// Within a wave of 64 lanes, lane l handles word 64*W + l, so z bits 5..10
// are the lane index and z bits >= 11 are the same for the whole wave.
// A clause's unsatisfied-mask on a word is
//     P  (the AND of the false-masks of its literals on bits 0..4)
//   & L[lane]   (its literals on bits 5..10 are all false for this lane)
//   & H(wave)   (its literals on bits >= 11 are all false for this wave).
// P and L depend only on the clause and are packed once on the host.
#pragma once

#include <cstdint>

#ifndef GQ_HD
#include <hip/hip_runtime.h>
#define GQ_HD __host__ __device__ __forceinline__
#endif

namespace gqaoa {

constexpr int kLowBits = 5;    // z bits inside a word
constexpr int kLaneBits = 6;   // z bits across the 64 lanes of a wave
constexpr int kHighBit0 = kLowBits + kLaneBits;  // first wave-uniform bit (11)
constexpr int kGroup = 16;     // clauses per carry-save-adder block

struct alignas(32) ClauseRec {
    uint32_t P;       // false-mask over the 32 word bits of the low literals
    uint32_t pad;
    uint64_t L;       // bit l set iff the literals on bits 5..10 are false in lane l
    uint64_t hivar;   // variables >= 11 of the clause (bit v)
    uint64_t hineg;   // their neg flags (bit v)
};

struct alignas(16) UniformRec {  // clause with all variables >= 11
    uint64_t hivar;
    uint64_t hineg;
};

// z offset (bits 0..4) held by word bit j.
GQ_HD uint32_t word_bit_to_zlow(int j) { return 4u * (uint32_t)(j & 7) + (uint32_t)(j >> 3); }

// Word whose bit j is set iff bit v of word_bit_to_zlow(j) is 1 (v < 5).
GQ_HD uint32_t low_var_pattern(int v) {
    uint32_t p = 0;
    for (int j = 0; j < 32; ++j)
        if ((word_bit_to_zlow(j) >> v) & 1u) p |= 1u << j;
    return p;
}

// low_var_pattern(v) in closed form: z bit 0 <-> word bit 3, bit 1 <-> 4, bit 2 <-> 0,
// bit 3 <-> 1, bit 4 <-> 2.
constexpr uint32_t kLowVarPattern[kLowBits] = {0xFF00FF00u, 0xFFFF0000u, 0xAAAAAAAAu, 0xCCCCCCCCu, 0xF0F0F0F0u};
// Lanes whose lane-index bit b is 1 (b = v - 5 for a variable on z bits 5..10).
constexpr uint64_t kLaneBitPattern[kLaneBits] = {
    0xAAAAAAAAAAAAAAAAull, 0xCCCCCCCCCCCCCCCCull, 0xF0F0F0F0F0F0F0F0ull,
    0xFF00FF00FF00FF00ull, 0xFFFF0000FFFF0000ull, 0xFFFFFFFF00000000ull};

// Record of one clause (validated literals: lit = 2*var + neg, distinct vars).
// Sets *uniform when every variable sits at z bits >= 11.
GQ_HD ClauseRec make_record(int32_t l0, int32_t l1, int32_t l2, bool *uniform) {
    ClauseRec r{0xFFFFFFFFu, 0u, ~0ull, 0ull, 0ull};
    bool uni = true;
    const int32_t lits[3] = {l0, l1, l2};
    for (int j = 0; j < 3; ++j) {
        const int v = lits[j] >> 1, neg = lits[j] & 1;
        if (v < kLowBits) {
            const uint32_t pat = kLowVarPattern[v];
            r.P &= neg ? pat : ~pat;     // false iff bit v == neg
            uni = false;
        } else if (v < kHighBit0) {
            const uint64_t ones = kLaneBitPattern[v - kLowBits];
            r.L &= neg ? ones : ~ones;   // false iff the lane's bit equals neg
            uni = false;
        } else {
            r.hivar |= 1ull << v;
            r.hineg |= (uint64_t)neg << v;
        }
    }
    if (uniform) *uniform = uni;
    return r;
}

// A clause is active for a wave when its high literals are all false there.
GQ_HD bool high_literals_false(uint64_t zwave, uint64_t hivar, uint64_t hineg) {
    return ((zwave ^ hineg) & hivar) == 0;
}

// Carry-save adder: a + b + c = 2*hi + lo, bitwise. On the device each output
// is one v_bitop3_b32 (truth tables 0x96 = three-input XOR, 0xE8 = majority).
GQ_HD void csa(uint32_t &hi, uint32_t &lo, uint32_t a, uint32_t b, uint32_t c) {
#if defined(__HIP_DEVICE_COMPILE__)
    hi = __builtin_amdgcn_bitop3_b32(a, b, c, 0xE8);
    lo = __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
#else
    const uint32_t u = a ^ b;
    hi = (a & b) | (u & c);
    lo = u ^ c;
#endif
}

// Bit-sliced 8-bit counters, one per word bit: count = sum_b plane[b] << b.
struct SlicedCounter {
    uint32_t p[8];
    GQ_HD void clear() {
        for (int b = 0; b < 8; ++b) p[b] = 0;
    }
    // Add 16 one-bit inputs per word bit (Harley-Seal style adder tree into
    // the ones/twos/fours/eights planes, then a ripple of the sixteens).
    GQ_HD void add16(const uint32_t (&f)[kGroup]) {
        uint32_t twosA, twosB, foursA, foursB, eightsA, eightsB, sixteens;
        csa(twosA, p[0], p[0], f[0], f[1]);
        csa(twosB, p[0], p[0], f[2], f[3]);
        csa(foursA, p[1], p[1], twosA, twosB);
        csa(twosA, p[0], p[0], f[4], f[5]);
        csa(twosB, p[0], p[0], f[6], f[7]);
        csa(foursB, p[1], p[1], twosA, twosB);
        csa(eightsA, p[2], p[2], foursA, foursB);
        csa(twosA, p[0], p[0], f[8], f[9]);
        csa(twosB, p[0], p[0], f[10], f[11]);
        csa(foursA, p[1], p[1], twosA, twosB);
        csa(twosA, p[0], p[0], f[12], f[13]);
        csa(twosB, p[0], p[0], f[14], f[15]);
        csa(foursB, p[1], p[1], twosA, twosB);
        csa(eightsB, p[2], p[2], foursA, foursB);
        csa(sixteens, p[3], p[3], eightsA, eightsB);
        uint32_t c = sixteens;
        for (int b = 4; b < 8; ++b) {  // counts never exceed 255
            const uint32_t t = p[b] & c;
            p[b] ^= c;
            c = t;
        }
    }
    // Add the same value u (< 256) to every word bit's count, bit-sliced:
    // plane b gets p_b ^ u_b ^ carry and the carry becomes maj(p_b, u_b, carry).
    GQ_HD void add_scalar(uint32_t u) {
        uint32_t c = 0;
        for (int b = 0; b < 8; ++b) {
            const uint32_t ub = ((u >> b) & 1u) ? 0xFFFFFFFFu : 0u;
            uint32_t s, carry;
            csa(carry, s, p[b], ub, c);
            p[b] = s;
            c = carry;
        }
    }
    // Transpose: afterwards p[r] byte q = count of word bit 8q + r.
    GQ_HD void transpose_to_bytes() {
        for (int b = 0; b < 4; ++b) {
            const uint32_t t = ((p[b] >> 4) ^ p[b + 4]) & 0x0F0F0F0Fu;
            p[b + 4] ^= t;
            p[b] ^= t << 4;
        }
        for (int b0 = 0; b0 < 8; b0 += 4)
            for (int b = b0; b < b0 + 2; ++b) {
                const uint32_t t = ((p[b] >> 2) ^ p[b + 2]) & 0x33333333u;
                p[b + 2] ^= t;
                p[b] ^= t << 2;
            }
        for (int b = 0; b < 8; b += 2) {
            const uint32_t t = ((p[b] >> 1) ^ p[b + 1]) & 0x55555555u;
            p[b + 1] ^= t;
            p[b] ^= t << 1;
        }
    }
};

}  // namespace gqaoa

#include <vector>

namespace gqaoa {

// Pack validated clauses (lit = 2*var + neg, 3 distinct vars) into the records
// above. Clauses with all three variables at bits >= 11 go to `uni`; the rest
// go to `vec`, padded with empty records to a multiple of kGroup. Fixed-capacity
// form: for m clauses vec needs room for m rounded up to kGroup records, uni for m.
inline void pack_clauses(int m, const int32_t *lits, ClauseRec *vec, int *nvec, UniformRec *uni, int *nuni) {
    int nv = 0, nu = 0;
    for (int i = 0; i < m; ++i) {
        bool uniform = false;
        const ClauseRec r = make_record(lits[3 * i], lits[3 * i + 1], lits[3 * i + 2], &uniform);
        if (uniform)
            uni[nu++] = UniformRec{r.hivar, r.hineg};
        else
            vec[nv++] = r;
    }
    while (nv % kGroup) vec[nv++] = ClauseRec{0u, 0u, 0ull, 0ull, 0ull};
    *nvec = nv;
    *nuni = nu;
}

inline void pack_clauses(int m, const int32_t *lits, std::vector<ClauseRec> &vec,
                         std::vector<UniformRec> &uni) {
    vec.resize((size_t)(m + kGroup - 1) / kGroup * kGroup);
    uni.resize((size_t)m);
    int nv = 0, nu = 0;
    pack_clauses(m, lits, vec.data(), &nv, uni.data(), &nu);
    vec.resize((size_t)nv);
    uni.resize((size_t)nu);
}

}  // namespace gqaoa
