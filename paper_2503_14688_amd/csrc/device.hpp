// Device building blocks for gfx950: Philox4x32-10, the lazy bit-plane
// Metropolis test, bit-sliced counters and block reductions.
//
// Every lattice word holds 32 sites of one colour of one row (multispin
// coding, paper Introduction); all logic below works on 32 sites at once,
// one bit per site.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spin {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 products, round key bumped by the Weyl constants.
constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

struct Block4 {
    uint32_t v[4];
};

// a ^ b ^ k in one VALU instruction: gfx950's three-input bitwise operation
// with truth table 0x96 (odd parity); the compiler otherwise emits two XORs.
// k is a wave-uniform round key held in a scalar register.
__device__ __forceinline__ uint32_t xor3_key(uint32_t a, uint32_t b, uint32_t k)
{
    uint32_t d;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(d) : "v"(a), "v"(b), "s"(k));
    return d;
}

// One Philox4x32-10 block.  The key (k0, k1) must be uniform across the
// wavefront: the round keys live in scalar registers.
//
// The sweep index and stream tag (words 2 and 3) are wave-uniform at every
// call, so the first two rounds are plain C, grouped so that the compiler
// combines their uniform parts in scalar registers (one vector XOR each
// instead of a register copy and a three-input XOR); from round 3 on every
// word is per lane.
__device__ __forceinline__ Block4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                uint32_t k0, uint32_t k1)
{
    k0 = __builtin_amdgcn_readfirstlane(k0);
    k1 = __builtin_amdgcn_readfirstlane(k1);
    uint64_t p0, p1;
    uint32_t n0, n2;
    // round 1: words 2 and 3 uniform, so are the product of word 2 and the
    // key parts XORed with them
    p0 = (uint64_t)kPhiloxM0 * c0;
    p1 = (uint64_t)kPhiloxM1 * c2;
    n0 = ((uint32_t)(p1 >> 32) ^ k0) ^ c1;
    n2 = (uint32_t)(p0 >> 32) ^ (c3 ^ k1);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
    // round 2: word 1 (the low half of round 1's uniform product) uniform
    p0 = (uint64_t)kPhiloxM0 * c0;
    p1 = (uint64_t)kPhiloxM1 * c2;
    n0 = (uint32_t)(p1 >> 32) ^ (c1 ^ k0);
    n2 = xor3_key((uint32_t)(p0 >> 32), c3, k1);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
#pragma unroll
    for (int round = 2; round < 10; ++round) {
        p0 = (uint64_t)kPhiloxM0 * c0;
        p1 = (uint64_t)kPhiloxM1 * c2;
        n0 = xor3_key((uint32_t)(p1 >> 32), c1, k0);
        n2 = xor3_key((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
    Block4 r;
    r.v[0] = c0;
    r.v[1] = c1;
    r.v[2] = c2;
    r.v[3] = c3;
    return r;
}

// philox4x32_10 with every round on the vector unit (the scalar unit only
// bumps the round keys).  For the per-word two-group test on row-uniform
// counters, where the form above would put most of the first two rounds on
// the scalar unit and make it the busier one (measured 3-4% slower there).
__device__ __forceinline__ Block4 philox4x32_10_vec(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                    uint32_t k0, uint32_t k1)
{
    k0 = __builtin_amdgcn_readfirstlane(k0);
    k1 = __builtin_amdgcn_readfirstlane(k1);
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = (uint64_t)kPhiloxM0 * c0;
        const uint64_t p1 = (uint64_t)kPhiloxM1 * c2;
        const uint32_t n0 = xor3_key((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = xor3_key((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
    Block4 r;
    r.v[0] = c0;
    r.v[1] = c1;
    r.v[2] = c2;
    r.v[3] = c3;
    return r;
}

// philox4x32_10 for a counter whose words 0, 2 and 3 are wave-uniform (row,
// sweep index, stream tag) while word 1 (the word column) varies by lane.
// The first rounds are written so that every value that is still uniform
// stays in scalar registers (the compiler places plain C by divergence):
// round 1 needs one vector operation, round 2 two, round 3 three, and only
// from round 4 on is the whole state per lane.  Same result as philox4x32_10.
__device__ __forceinline__ Block4 philox4x32_10_ru(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                   uint32_t k0, uint32_t k1)
{
    k0 = __builtin_amdgcn_readfirstlane(k0);
    k1 = __builtin_amdgcn_readfirstlane(k1);
    c0 = __builtin_amdgcn_readfirstlane(c0);
    c2 = __builtin_amdgcn_readfirstlane(c2);
    c3 = __builtin_amdgcn_readfirstlane(c3);
    uint64_t p0, p1;
    uint32_t n0, n2;
    // round 1: words 0, 2, 3 uniform
    p0 = (uint64_t)kPhiloxM0 * c0;
    p1 = (uint64_t)kPhiloxM1 * c2;
    n0 = ((uint32_t)(p1 >> 32) ^ k0) ^ c1;
    n2 = ((uint32_t)(p0 >> 32) ^ k1) ^ c3;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
    // round 2: words 1, 2, 3 uniform
    p0 = (uint64_t)kPhiloxM0 * c0;
    p1 = (uint64_t)kPhiloxM1 * c2;
    n0 = ((uint32_t)(p1 >> 32) ^ k0) ^ c1;
    n2 = (uint32_t)(p0 >> 32) ^ (k1 ^ c3);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
    // round 3: words 0 and 1 uniform
    p0 = (uint64_t)kPhiloxM0 * c0;
    p1 = (uint64_t)kPhiloxM1 * c2;
    n0 = (uint32_t)(p1 >> 32) ^ (k0 ^ c1);
    n2 = ((uint32_t)(p0 >> 32) ^ k1) ^ c3;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
    // round 4: word 3 uniform
    p0 = (uint64_t)kPhiloxM0 * c0;
    p1 = (uint64_t)kPhiloxM1 * c2;
    n0 = xor3_key((uint32_t)(p1 >> 32), c1, k0);
    n2 = (uint32_t)(p0 >> 32) ^ (k1 ^ c3);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
#pragma unroll
    for (int round = 4; round < 10; ++round) {
        p0 = (uint64_t)kPhiloxM0 * c0;
        p1 = (uint64_t)kPhiloxM1 * c2;
        n0 = xor3_key((uint32_t)(p1 >> 32), c1, k0);
        n2 = xor3_key((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
    Block4 r;
    r.v[0] = c0;
    r.v[1] = c1;
    r.v[2] = c2;
    r.v[3] = c3;
    return r;
}

// The Philox block of counter (row, word, t, tag): row-uniform form when
// the caller knows the row is the same across the wavefront.
template <bool ROW_UNIFORM>
__device__ __forceinline__ Block4 philox_block(uint32_t row, uint32_t word, uint32_t t, uint32_t tag, uint32_t k0,
                                               uint32_t k1)
{
    if constexpr (ROW_UNIFORM)
        return philox4x32_10_ru(row, word, t, tag, k0, k1);
    else
        return philox4x32_10(row, word, t, tag, k0, k1);
}

// Stream purposes, placed in bits 16.. of counter word 3.
constexpr uint32_t kPurposeInit = 0u;
constexpr uint32_t kPurposeAccept = 1u;
constexpr uint32_t kPurposePropose = 2u;

__device__ __forceinline__ uint32_t stream_tag(uint32_t purpose, uint32_t colour, uint32_t blk)
{
    return (purpose << 16) | (colour << 8) | blk;
}

// One plane of the lazy test in two three-input operations: the sites of
// `und` whose bit is 0 against a threshold bit 1 are accepted (und & tb & ~u,
// truth table 0x40), and those whose bits agree stay undecided
// (und & ~(tb ^ u), truth table 0x90).
__device__ __forceinline__ uint32_t newly_accepted(uint32_t und, uint32_t tb, uint32_t u)
{
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x40" : "=v"(r) : "v"(und), "v"(tb), "v"(u));
    return r;
}

__device__ __forceinline__ uint32_t still_tied(uint32_t und, uint32_t tb, uint32_t u)
{
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x90" : "=v"(r) : "v"(und), "v"(tb), "v"(u));
    return r;
}

// Bit-sliced "u < thr" over the 32 sites of a word, evaluated lazily.
//
// Site b's uniform u_b is read plane by plane from the most significant bit
// (plane k = word k & 3 of Philox block k >> 2).  A site is decided at the
// first plane where its bit differs from its threshold's bit: 0 against 1
// accepts, 1 against 0 rejects.  Blocks are drawn only while some site of the
// word is undecided, which gives the same answer as drawing all 32 planes;
// sites still tied after 32 planes have u == thr and are rejected.
//
// need[g]: sites whose move needs a random number and whose threshold is
// thr[g]; always: sites accepted outright.  Returns the accepted sites.
//
// apply_block consumes the four planes of block blk; metropolis_accept runs
// the whole lazy test for one word.
//
// The plane's threshold bit of each group is the same for every lane.  With
// two groups it enters as a scalar mask (one vector AND-OR per group); with
// the Blume-Capel group counts (6 or 13) each group whose bit is set adds
// its sites under a wave-uniform branch, so the vector unit does one OR per
// set bit and the scalar unit, otherwise idle there, does the tests.
template <int NG>
__device__ __forceinline__ void apply_block(const Block4 &r, uint32_t blk, const uint32_t (&need)[NG],
                                            const uint32_t (&thr)[NG], uint32_t &undecided, uint32_t &accepted)
{
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t shift = 31u - (4u * blk + (uint32_t)q);
        uint32_t tb = 0;
        if constexpr (NG > 2) {
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                if ((thr[g] >> shift) & 1u) {  // wave-uniform
                    tb |= need[g];
                    asm volatile("" : "+v"(tb));  // keeps the branch (no vector select)
                }
            }
        } else {
#pragma unroll
            for (int g = 0; g < NG; ++g)
                tb |= need[g] & (0u - ((thr[g] >> shift) & 1u));
        }
        const uint32_t ub = r.v[q];
        accepted |= newly_accepted(undecided, tb, ub);
        undecided = still_tied(undecided, tb, ub);
    }
}

// Six-group form of apply_block (Blume-Capel at Delta = 0).  pat4 holds the
// plane's group pattern byte by byte (bit g of byte q: group g's threshold
// bit in plane 4 blk + q is 1).  A wave-uniform switch over the 64 patterns
// gives each its own code: the threshold word is the OR of just the groups
// in the pattern (none, one register, or one or two three-input ORs), fed
// straight into the two three-input updates, so no copy or per-group test
// runs on the vector unit.
// The ORs are volatile: they must stay inside their case (the masks are the
// same for every block of a word, and the compiler would otherwise compute
// every case's OR once per word, ahead of the block loop).
__device__ __forceinline__ uint32_t or2_here(uint32_t a, uint32_t b)
{
    uint32_t d;
    asm volatile("v_or_b32 %0, %1, %2" : "=v"(d) : "v"(a), "v"(b));
    return d;
}

__device__ __forceinline__ uint32_t or3_here(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t d;
    asm volatile("v_or3_b32 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
    return d;
}

// t | need[g] over the groups g in M (M != 0), two more groups per
// three-input OR.
template <uint32_t M>
__device__ __forceinline__ uint32_t or_more(uint32_t t, const uint32_t (&need)[6])
{
    constexpr int a = __builtin_ctz(M);
    constexpr uint32_t M1 = M & (M - 1u);
    if constexpr (M1 == 0u) {
        return or2_here(t, need[a]);
    } else {
        constexpr int b = __builtin_ctz(M1);
        constexpr uint32_t M2 = M1 & (M1 - 1u);
        const uint32_t r = or3_here(t, need[a], need[b]);
        if constexpr (M2 == 0u)
            return r;
        else
            return or_more<M2>(r, need);
    }
}

// OR of need[g] over the groups g in M (M != 0): the register itself for
// one group, else as few two- and three-input ORs as the count allows.
template <uint32_t M>
__device__ __forceinline__ uint32_t or_groups(const uint32_t (&need)[6])
{
    constexpr int a = __builtin_ctz(M);
    constexpr uint32_t M1 = M & (M - 1u);
    if constexpr (M1 == 0u) {
        return need[a];
    } else {
        constexpr int b = __builtin_ctz(M1);
        constexpr uint32_t M2 = M1 & (M1 - 1u);
        if constexpr (M2 == 0u) {
            return or2_here(need[a], need[b]);
        } else {
            constexpr int c = __builtin_ctz(M2);
            constexpr uint32_t M3 = M2 & (M2 - 1u);
            const uint32_t r = or3_here(need[a], need[b], need[c]);
            if constexpr (M3 == 0u)
                return r;
            else
                return or_more<M3>(r, need);
        }
    }
}

template <uint32_t M>
__device__ __forceinline__ void plane6(const uint32_t (&need)[6], uint32_t u, uint32_t &und, uint32_t &newly)
{
    if constexpr (M == 0u) {
        newly = 0u;
        und &= ~u;
    } else {
        const uint32_t tb = or_groups<M>(need);
        newly = newly_accepted(und, tb, u);
        und = still_tied(und, tb, u);
    }
}

__device__ __forceinline__ void plane6_switch(uint32_t m, const uint32_t (&need)[6], uint32_t u, uint32_t &und,
                                              uint32_t &newly)
{
#define SPIN_P1(n) case n: plane6<n>(need, u, und, newly); break;
#define SPIN_P4(n) SPIN_P1(n) SPIN_P1(n + 1) SPIN_P1(n + 2) SPIN_P1(n + 3)
#define SPIN_P16(n) SPIN_P4(n) SPIN_P4(n + 4) SPIN_P4(n + 8) SPIN_P4(n + 12)
    switch (m) {
        SPIN_P16(0u) SPIN_P16(16u) SPIN_P16(32u) SPIN_P16(48u)
    default: break;
    }
#undef SPIN_P16
#undef SPIN_P4
#undef SPIN_P1
}

__device__ __forceinline__ void apply_block6(const Block4 &r, uint32_t pat4, const uint32_t (&need)[6],
                                             uint32_t &undecided, uint32_t &accepted)
{
    uint32_t n[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
        plane6_switch((pat4 >> (8 * q)) & 63u, need, r.v[q], undecided, n[q]);
    accepted |= (n[0] | n[1]) | (n[2] | n[3]);
}

// apply_block for any group count; the six-group form reads its plane
// patterns from pats (GroupTable::plane_groups, uniform).
template <int NG>
__device__ __forceinline__ void apply_block_any(const Block4 &r, uint32_t blk, const uint32_t (&need)[NG],
                                                const uint32_t (&thr)[NG], const uint32_t *pats,
                                                uint32_t &undecided, uint32_t &accepted)
{
    if constexpr (NG == 6)
        apply_block6(r, __builtin_amdgcn_readfirstlane(pats[blk]), need, undecided, accepted);
    else
        apply_block<NG>(r, blk, need, thr, undecided, accepted);
}

// ROW_UNIFORM: the row is the same across the wavefront (the row-uniform
// Philox form; used by the six-group test).
template <int NG, bool ROW_UNIFORM = false>
__device__ __forceinline__ uint32_t metropolis_accept(const uint32_t (&need)[NG], const uint32_t (&thr)[NG],
                                                      uint32_t always, uint32_t row, uint32_t word,
                                                      uint32_t t, uint32_t colour, uint32_t k0, uint32_t k1,
                                                      const uint32_t *pats = nullptr)
{
    uint32_t undecided = 0;
#pragma unroll
    for (int g = 0; g < NG; ++g)
        undecided |= need[g];
    uint32_t accepted = always;
    for (uint32_t blk = 0; blk < 8u && undecided != 0u; ++blk) {
        const uint32_t tag = stream_tag(kPurposeAccept, colour, blk);
        Block4 r;
        if constexpr (ROW_UNIFORM)
            r = philox4x32_10_ru(row, word, t, tag, k0, k1);
        else if constexpr (NG == 2)
            r = philox4x32_10_vec(row, word, t, tag, k0, k1);
        else
            r = philox4x32_10(row, word, t, tag, k0, k1);
        apply_block_any<NG>(r, blk, need, thr, pats, undecided, accepted);
    }
    return accepted;
}

// Two-group form of apply_block (Ising: dE = 4J and 8J).  need[1] marks
// the undecided sites of group 1, the others are in group 0.  The two
// threshold bits of a plane are the same for every lane: as masks m0, m1
// (all ones or zero, scalar), a site's threshold bit is
// m0 ^ (H & (m0 ^ m1)) with H = group-1 sites, two vector operations per
// plane and no branch.  (A wave-uniform four-way branch per plane needs
// fewer vector but many more scalar instructions, and measured 5% slower.)
__device__ __forceinline__ void apply_block_2g(const Block4 &r, uint32_t blk, const uint32_t (&need)[2],
                                               const uint32_t (&thr)[2], uint32_t &undecided, uint32_t &accepted)
{
    const uint32_t H = need[1];
    const uint32_t dthr = thr[0] ^ thr[1];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t shift = 31u - (4u * blk + (uint32_t)q);
        const uint32_t m0 = 0u - ((thr[0] >> shift) & 1u);
        const uint32_t d = 0u - ((dthr >> shift) & 1u);
        const uint32_t tb = (H & d) ^ m0;
        const uint32_t u = r.v[q];
        accepted |= newly_accepted(undecided, tb, u);
        undecided = still_tied(undecided, tb, u);
    }
}

// Threshold bits of the two Ising groups for planes 0..7 (the planes every
// word draws in place), prepared once per tile: the group-0 bit of plane k
// as a scalar mask m0[k], and the difference of the two groups' bits as a
// vector mask d[k] (all ones or zero in every lane).  Kept in vector
// registers and opaque to the compiler, d[k] lets the plane's threshold
// word m0 ^ (H & d) be one three-input bitwise operation (the compiler
// otherwise turns H & d into a select and adds an XOR).
struct PlaneMasks2 {
    uint32_t m0[8];
    uint32_t d[8];
};

__device__ __forceinline__ PlaneMasks2 plane_masks_2g(const uint32_t (&thr)[2])
{
    PlaneMasks2 pm;
    const uint32_t dthr = thr[0] ^ thr[1];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        pm.m0[k] = 0u - ((thr[0] >> (31 - k)) & 1u);
        uint32_t d = 0u - ((dthr >> (31 - k)) & 1u);
        asm volatile("v_mov_b32 %0, %1" : "=v"(d) : "s"(d));
        pm.d[k] = d;
    }
    return pm;
}

// (h & d) ^ m: gfx950's three-input bitwise operation, truth table 0x6A
// (operands in order h, d, m); m is wave-uniform.
__device__ __forceinline__ uint32_t and_xor_s(uint32_t h, uint32_t d, uint32_t m)
{
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x6a" : "=v"(r) : "v"(h), "v"(d), "s"(m));
    return r;
}

// apply_block_2g for block 0 or 1 (planes 0..7) with prepared plane masks:
// three vector operations per plane (and one OR per two planes).
template <int BLK>
__device__ __forceinline__ void apply_block_2g_pm(const Block4 &r, const PlaneMasks2 &pm, uint32_t H,
                                                  uint32_t &undecided, uint32_t &accepted)
{
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t tb = and_xor_s(H, pm.d[4 * BLK + q], pm.m0[4 * BLK + q]);
        const uint32_t u = r.v[q];
        accepted |= newly_accepted(undecided, tb, u);
        undecided = still_tied(undecided, tb, u);
    }
}

// apply_block_2g for block 0 or 1 (planes 0..7) with a wave-uniform branch
// per plane on its two threshold bits (pg: GroupTable::plane_groups word of
// the block, byte q = plane 4 BLK + q, bit 0 group 0, bit 1 group 1).  H =
// the group-1 (dE = 8J) sites, the other undecided sites are group 0.  Each
// case is two vector operations (one when neither bit is set):
//   neither: none accepted, und &= ~u
//   group 0: accepted und & ~H & ~u, still tied und & (u ^ H)
//   group 1: accepted und & H & ~u, still tied und & ~(u ^ H)
//   both:    accepted und & ~u, still tied und & u
// The operations are volatile so that no case is evaluated outside its
// branch.
template <int BLK>
__device__ __forceinline__ void apply_block_2g_sw(const Block4 &r, uint32_t pg, uint32_t H, uint32_t &undecided,
                                                  uint32_t &accepted)
{
    uint32_t n[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t u = r.v[q];
        uint32_t und = undecided, nw, nu;
        switch ((pg >> (8 * q)) & 3u) {
        case 0u:
            nw = 0u;
            asm volatile("v_bitop3_b32 %0, %1, %2, %2 bitop3:0x10" : "=v"(nu) : "v"(und), "v"(u));
            break;
        case 1u:
            asm volatile("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x10" : "=v"(nw) : "v"(und), "v"(H), "v"(u));
            asm volatile("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x60" : "=v"(nu) : "v"(und), "v"(H), "v"(u));
            break;
        case 2u:
            asm volatile("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x40" : "=v"(nw) : "v"(und), "v"(H), "v"(u));
            asm volatile("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x90" : "=v"(nu) : "v"(und), "v"(H), "v"(u));
            break;
        default:
            asm volatile("v_bitop3_b32 %0, %1, %2, %2 bitop3:0x10" : "=v"(nw) : "v"(und), "v"(u));
            asm volatile("v_bitop3_b32 %0, %1, %2, %2 bitop3:0x80" : "=v"(nu) : "v"(und), "v"(u));
            break;
        }
        n[q] = nw;
        undecided = nu;
    }
    accepted |= (n[0] | n[1]) | (n[2] | n[3]);
}

// Full adder and half adder on bit-sliced operands.
__device__ __forceinline__ void full_add(uint32_t a, uint32_t b, uint32_t c, uint32_t &s, uint32_t &carry)
{
    const uint32_t x = a ^ b;
    s = x ^ c;
    carry = (a & b) | (c & x);
}

// Bit-sliced count of eight one-bit inputs per site: v = b0 + 2 b1 + 4 b2 + 8 b3.
__device__ __forceinline__ void count8(const uint32_t (&a)[8], uint32_t &b0, uint32_t &b1, uint32_t &b2,
                                       uint32_t &b3)
{
    uint32_t s1, c1, s2, c2, c4, t1, d1;
    full_add(a[0], a[1], a[2], s1, c1);
    full_add(a[3], a[4], a[5], s2, c2);
    const uint32_t s3 = a[6] ^ a[7];
    const uint32_t c3 = a[6] & a[7];
    full_add(s1, s2, s3, b0, c4);
    full_add(c1, c2, c3, t1, d1);
    b1 = t1 ^ c4;
    const uint32_t d2 = t1 & c4;
    b2 = d1 ^ d2;
    b3 = d1 & d2;
}

// 64-bit wave reduction (wave64) followed by one atomic per block.
template <int N>
__device__ __forceinline__ void block_reduce_atomic(unsigned long long (&v)[N], unsigned long long *dst)
{
    __shared__ unsigned long long part[N][16];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < N; ++q) {
        unsigned long long x = v[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
            x += __shfl_xor(x, off, 64);
        if (lane == 0)
            part[q][wave] = x;
    }
    __syncthreads();
    const int nwaves = (blockDim.x + 63) >> 6;
    if (threadIdx.x < N) {
        unsigned long long s = 0;
        for (int w = 0; w < nwaves; ++w)
            s += part[threadIdx.x][w];
        if (s)
            atomicAdd(dst + threadIdx.x, s);
    }
}

// A copy of *p in scalar registers (p is the same for the whole wavefront):
// a descriptor that a block reads from memory instead of its kernel
// arguments, kept where the arguments would be.
template <typename T>
__device__ __forceinline__ T wave_uniform_copy(const T *p)
{
    static_assert(sizeof(T) % 4 == 0, "whole 32-bit words");
    T out;
    const uint32_t *src = reinterpret_cast<const uint32_t *>(p);
    uint32_t *dst = reinterpret_cast<uint32_t *>(&out);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(T) / 4); ++k)
        dst[k] = __builtin_amdgcn_readfirstlane(src[k]);
    return out;
}

} // namespace spin
