// Sweep tiles shared by the single-lattice half-sweep kernels (kernels.hip)
// and the batched half-sweep (batch_kernels.hip): the Ising and Blume-Capel
// tile functions, their wavefront work lists and the tile geometry.  Device
// code only; each translation unit that includes it gets its own copy.
//
// Layout (one colour plane per checkerboard colour, paper Introduction):
// site (i, j) has colour c = (i + j) & 1 and sits at m = j >> 1 of row i of
// plane c, word w = m >> 5, bit b = m & 31.  Its vertical neighbours are at
// the same (w, b) in rows i -+ 1 of the other plane; its horizontal
// neighbours are (i, m) and (i, m - 1) of the other plane when (i + c) is
// even, (i, m) and (i, m + 1) when it is odd.
#pragma once

#include <type_traits>

#include "device.hpp"
#include "kernels.hpp"

namespace spin {

namespace {

constexpr int kBlock = 256;

// Horizontal neighbour word: bit b holds the site at m -+ 1 of the other
// plane, built from the same-row word and the word to its left or right.
__device__ __forceinline__ uint32_t side_word(uint32_t cur, uint32_t nb, uint32_t odd)
{
    return odd ? ((cur >> 1) | (nb << 31)) : ((cur << 1) | (nb >> 31));
}

// Row group of a lane's work item g: g / W.  Items of one lattice plane number
// fewer than 2^32 for every L up to 65536 (and for most larger ones), and then
// the quotient is taken in 32 bits: far fewer vector instructions than the
// 64-bit division, which the rest keep.  nitems is wave-uniform, so is the
// branch.  (Where the row is wave-uniform the division runs on the scalar
// unit and stays 64-bit.)
__device__ __forceinline__ uint32_t row_group(uint64_t g, uint32_t W, uint64_t nitems)
{
    if (nitems <= 0xFFFFFFFFull)
        return (uint32_t)g / W;
    return (uint32_t)(g / W);
}

// ------------------------------------------------------------ sweeps --
//
// Work unit: a tile of kBlock items; with R rows per thread, item g of a
// lattice is word column w = g mod W over the R rows starting at R (g / W),
// and thread tid of a block takes item tile * kBlock + tid.  Single-lattice kernels walk the
// tiles of one lattice; the batched kernel walks a flat list of the tiles of
// many lattices.

// Ising half-sweep, compacting form.  Every word gets its classes and the
// first two Philox blocks (planes 0-7) in place, which settles all sites of
// about nine words in ten.  The rest go to a work list owned by the
// wavefront (ballot ranks, no block barrier); the wavefront then drains the
// list with one word per lane, so the later blocks are drawn for the few
// words that need them and not for every word of a wavefront that holds one
// slow word.  New words collect in LDS and go to HBM as whole rows at the end
// of the tile.  Every site ends with the outcome that all 32 planes define.
constexpr int kWaves = kBlock / 64;

// One wavefront's list: CAP slots; words past the last slot finish in place.
// A block holds one per wavefront, each a contiguous region, so wavefronts
// that are at different tiles never touch each other's storage, whichever
// list type each tile uses.
template <int CAP>
struct WaveList {
    static constexpr int kCap = CAP;
    uint32_t und[CAP], acc[CAP];
    uint32_t m3[CAP], m4[CAP];
    uint16_t slot[CAP];  // row offset << 6 | owning lane
    uint32_t i0[64], w[64];
    // new words of the tile, stored to HBM in whole rows once the list is
    // drained (listed words hold the old word until then)
    uint32_t stage[8][64];
};

// Orders the LDS accesses of one wavefront's lanes (no cross-wave effect).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct IsingNbrs {
    uint32_t up, dn, cur, side;
};

__device__ __forceinline__ IsingNbrs ising_nbrs(const uint32_t *oth, uint32_t L, uint32_t W, uint32_t c,
                                                uint32_t i, uint32_t w)
{
    const uint32_t iu = i == 0 ? L - 1 : i - 1, id = i + 1 == L ? 0 : i + 1;
    const uint32_t odd = (i + c) & 1u;
    const uint32_t wn = odd ? (w + 1u == W ? 0u : w + 1u) : (w == 0 ? W : w) - 1u;
    IsingNbrs n;
    n.up = oth[(size_t)iu * W + w];
    n.dn = oth[(size_t)id * W + w];
    n.cur = oth[(size_t)i * W + w];
    n.side = side_word(n.cur, oth[(size_t)i * W + wn], odd);
    return n;
}

// Energy/magnetisation counters of one updated word (see kEmCounters): the
// word's 32 sites and the 32 other-colour sites at the same position, and
// the four bonds of each updated site.
__device__ __forceinline__ void ising_em(unsigned long long (&e)[kEmCounters], uint32_t ns, uint32_t up,
                                         uint32_t dn, uint32_t cur, uint32_t side)
{
    e[0] += 64;
    e[1] += __popc(ns) + __popc(cur);
    e[2] += 128;
    e[3] += __popc(ns ^ up) + __popc(ns ^ dn) + __popc(ns ^ cur) + __popc(ns ^ side);
}

// Q is the calling wavefront's own list.
// PLAIN: both Ising groups draw random numbers and neither is never
// accepted (every finite T > 0), so the classification needs no selects.
template <bool MEASURE, int R, bool UNIFORM, typename List, bool PLAIN = false>
__device__ __forceinline__ void ising_tile_compact(const Lattice &lat, uint32_t c, uint32_t t, const GroupTable &gt,
                                                   uint64_t tile, List &Q, unsigned long long (&e)[kEmCounters])
{
    constexpr int kListCap = List::kCap;
    const uint32_t L = lat.L, W = lat.W;
    uint32_t *own = lat.planes + (c ? lat.plane_u32 : 0);
    const uint32_t *oth = lat.planes + (c ? 0 : lat.plane_u32);
    const uint64_t nitems = (uint64_t)(L / R) * W;
    const uint32_t thr[2] = {gt.thr[0], gt.thr[1]};
    PlaneMasks2 pm;
    if constexpr (!UNIFORM)
        pm = plane_masks_2g(thr);
    const bool rng3 = gt.rng_bits & 1u, rng4 = gt.rng_bits & 2u;
    const bool nev3 = gt.never_bits & 1u, nev4 = gt.never_bits & 2u;
    const uint32_t k0 = lat.key0, k1 = lat.key1;
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t g = tile * kBlock + threadIdx.x;
    // W % 64 == 0 makes L a multiple of 4096, so the items fill whole tiles:
    // with UNIFORM no lane is past the end, and the test is compiled out
    const bool valid = UNIFORM || g < nitems;
    uint32_t rg, w;
    if (UNIFORM) {
        // W % 64 == 0: the wavefront's 64 items lie in one row group
        const uint32_t wave0 = __builtin_amdgcn_readfirstlane(threadIdx.x) & ~63u;
        rg = __builtin_amdgcn_readfirstlane((uint32_t)((tile * kBlock + wave0) / W));
        w = (uint32_t)(g - (uint64_t)rg * W);
    } else {
        rg = valid ? row_group(g, W, nitems) : 0u;
        w = valid ? (uint32_t)(g - (uint64_t)rg * W) : 0u;
    }
    const uint32_t i0 = rg * R;
    Q.i0[lane] = i0;
    Q.w[lane] = w;
    uint32_t n = 0;
    const uint32_t wl = (w == 0 ? W : w) - 1u;
    const uint32_t wr = (w + 1u == W) ? 0u : w + 1u;
    // Words of row i0 and its vertical neighbours; each row below loads the
    // next row's words before it draws random planes, so the loads are in
    // flight while the Philox rounds run.  Lanes past the end of the lattice
    // (rg = w = 0) load rows 0..R of column 0, which exist, and never use the
    // values: the loads stay unconditional, so the wait before a row covers
    // only that row's words.
    uint32_t up = oth[(size_t)(i0 == 0 ? L - 1 : i0 - 1) * W + w];
    uint32_t cur = oth[(size_t)i0 * W + w];
    uint32_t dn = oth[(size_t)(i0 + 1u == L ? 0u : i0 + 1u) * W + w];
    uint32_t nbw = oth[(size_t)i0 * W + (((i0 + c) & 1u) ? wr : wl)];
    uint32_t sv = own[(size_t)i0 * W + w];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t i = i0 + (uint32_t)r;
        uint32_t dn2 = 0, nbw2 = 0, sv2 = 0;
        if (r + 1 < R) {
            const uint32_t i1 = i + 1u;  // i0 + R <= L: still in the tile
            dn2 = oth[(size_t)(i1 + 1u == L ? 0u : i1 + 1u) * W + w];
            nbw2 = oth[(size_t)i1 * W + (((i1 + c) & 1u) ? wr : wl)];
            sv2 = own[(size_t)i1 * W + w];
        }
        const uint32_t odd = (i + c) & 1u;
        const uint32_t side = side_word(cur, nbw, odd);
        // every lane runs the word it holds (lanes past the end hold words that
        // exist and drop out with an empty undecided set afterwards), so no
        // lane state needs zeroing first
        uint32_t acc, und, need[2];
        {
            // aligned-neighbour indicators; a = number aligned, dE = J (4a - 8)
            const uint32_t e1 = ~(sv ^ up), e2 = ~(sv ^ dn), e3 = ~(sv ^ cur), e4 = ~(sv ^ side);
            const uint32_t a1 = e1 & e2, x1 = e1 ^ e2, a2 = e3 & e4, x2 = e3 ^ e4;
            const uint32_t m4 = a1 & a2;                // a = 4: dE = 8J
            const uint32_t m3 = (a1 & x2) | (a2 & x1);  // a = 3: dE = 4J
            if constexpr (PLAIN) {
                need[0] = m3;
                need[1] = m4;
                und = m3 | m4;
                acc = ~und;
            } else {
                need[0] = rng3 ? m3 : 0u;
                need[1] = rng4 ? m4 : 0u;
                const uint32_t never = (nev3 ? m3 : 0u) | (nev4 ? m4 : 0u);
                acc = ~(need[0] | need[1] | never);
                und = need[0] | need[1];
            }
            // blocks 0 and 1 for every word: the wavefront would run them
            // anyway unless all 64 of its words were settled, which is rare
            const Block4 b0 = philox_block<UNIFORM>(i, w, t, stream_tag(kPurposeAccept, c, 0), k0, k1);
            // row-uniform tiles (the large lattices): one branch per plane on
            // its two threshold bits; otherwise the prepared masks (measured
            // faster there, in the batched kernel)
            if constexpr (UNIFORM)
                apply_block_2g_sw<0>(b0, gt.plane_groups[0], need[1], und, acc);
            else
                apply_block_2g_pm<0>(b0, pm, need[1], und, acc);
            const Block4 b1 = philox_block<UNIFORM>(i, w, t, stream_tag(kPurposeAccept, c, 1), k0, k1);
            if constexpr (UNIFORM)
                apply_block_2g_sw<1>(b1, gt.plane_groups[1], need[1], und, acc);
            else
                apply_block_2g_pm<1>(b1, pm, need[1], und, acc);
            und = valid ? und : 0u;
        }
        const unsigned long long bal = __ballot(und != 0u);
        bool listed = false;
        if (und != 0u) {
            const uint32_t p = n + __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                             __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
            if (p < (uint32_t)kListCap) {
                Q.und[p] = und;
                Q.acc[p] = acc;
                Q.m3[p] = need[0];
                Q.m4[p] = need[1];
                Q.slot[p] = (uint16_t)(((uint32_t)r << 6) | lane);
                Q.stage[r][lane] = sv;
                listed = true;
            } else {
                for (uint32_t blk = 2; blk < 8u && und != 0u; ++blk) {
                    const Block4 b = philox4x32_10(i, w, t, stream_tag(kPurposeAccept, c, blk), k0, k1);
                    apply_block_2g(b, blk, need, thr, und, acc);
                }
            }
        }
        if (valid && !listed) {
            // sites still tied after 32 planes have u == thr: rejected
            const uint32_t ns = sv ^ acc;
            Q.stage[r][lane] = ns;
            if (MEASURE)
                ising_em(e, ns, up, dn, cur, side);
        }
        n += (uint32_t)__popcll(bal);
        up = cur;
        cur = dn;
        dn = dn2;
        nbw = nbw2;
        sv = sv2;
    }
    if (n > (uint32_t)kListCap)
        n = kListCap;
    wave_sync();
    for (uint32_t k = lane; k < n; k += 64u) {
        const uint32_t slot = Q.slot[k], owner = slot & 63u;
        const uint32_t i = Q.i0[owner] + (slot >> 6), wq = Q.w[owner];
        const uint32_t need[2] = {Q.m3[k], Q.m4[k]};
        uint32_t und = Q.und[k], acc = Q.acc[k];
        for (uint32_t blk = 2; blk < 8u && und != 0u; ++blk) {
            const Block4 b = philox4x32_10(i, wq, t, stream_tag(kPurposeAccept, c, blk), k0, k1);
            apply_block_2g(b, blk, need, thr, und, acc);
        }
        const uint32_t ns = Q.stage[slot >> 6][owner] ^ acc;
        Q.stage[slot >> 6][owner] = ns;
        if (MEASURE) {
            const IsingNbrs nb = ising_nbrs(oth, L, W, c, i, wq);
            ising_em(e, ns, nb.up, nb.dn, nb.cur, nb.side);
        }
    }
    wave_sync();
    // whole rows to HBM: every line of the tile is written once and complete
    if (valid) {
#pragma unroll
        for (int r = 0; r < R; ++r)
            own[(size_t)(i0 + (uint32_t)r) * W + w] = Q.stage[r][lane];
    }
    wave_sync();  // the list and the stage are refilled by the next tile
}

// Ising half-sweep of one tile, one word at a time: each thread runs the
// lazy Metropolis test of its word to completion (no list, no LDS).
// UNIFORM: W is a multiple of 64, so a wavefront's 64 items share one row
// group; the row index is then wave-uniform and the counter words that
// depend only on it and on t start the Philox rounds in scalar registers.
template <bool MEASURE, int R, bool UNIFORM>
__device__ __forceinline__ void ising_tile_lazy(const Lattice &lat, uint32_t c, uint32_t t, const GroupTable &gt,
                                                uint64_t tile, unsigned long long (&e)[kEmCounters])
{
    const uint32_t L = lat.L, W = lat.W;
    uint32_t *own = lat.planes + (c ? lat.plane_u32 : 0);
    const uint32_t *oth = lat.planes + (c ? 0 : lat.plane_u32);
    const uint64_t nitems = (uint64_t)(L / R) * W;
    const uint64_t g = tile * kBlock + threadIdx.x;
    if (!UNIFORM && g >= nitems)  // UNIFORM: whole tiles (see ising_tile_compact)
        return;
    const uint32_t thr[2] = {gt.thr[0], gt.thr[1]};
    const bool rng3 = gt.rng_bits & 1u, rng4 = gt.rng_bits & 2u;
    const bool nev3 = gt.never_bits & 1u, nev4 = gt.never_bits & 2u;
    uint32_t rg, w;
    if (UNIFORM) {
        // W % 64 == 0: the wavefront's 64 items lie in one row group (and L is
        // a multiple of 4096, so the items fill whole tiles: no lane is past
        // the end)
        const uint32_t wave0 = __builtin_amdgcn_readfirstlane(threadIdx.x) & ~63u;
        rg = __builtin_amdgcn_readfirstlane((uint32_t)((tile * kBlock + wave0) / W));
        w = (uint32_t)(g - (uint64_t)rg * W);
    } else {
        rg = row_group(g, W, nitems);
        w = (uint32_t)(g - (uint64_t)rg * W);
    }
    const uint32_t i0 = rg * R;
    const uint32_t wl = (w == 0 ? W : w) - 1u;
    const uint32_t wr = (w + 1u == W) ? 0u : w + 1u;
    // row i0's words; each row loads the next row's words before its random
    // planes are drawn
    uint32_t up = oth[(size_t)(i0 == 0 ? L - 1 : i0 - 1) * W + w];
    uint32_t cur = oth[(size_t)i0 * W + w];
    uint32_t dn = oth[(size_t)(i0 + 1u == L ? 0u : i0 + 1u) * W + w];
    uint32_t nbw = oth[(size_t)i0 * W + (((i0 + c) & 1u) ? wr : wl)];
    uint32_t sv = own[(size_t)i0 * W + w];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t i = i0 + (uint32_t)r;
        uint32_t dn2 = 0, nbw2 = 0, sv2 = 0;
        if (r + 1 < R) {
            const uint32_t i1 = i + 1u;  // i0 + R <= L: still in the tile
            dn2 = oth[(size_t)(i1 + 1u == L ? 0u : i1 + 1u) * W + w];
            nbw2 = oth[(size_t)i1 * W + (((i1 + c) & 1u) ? wr : wl)];
            sv2 = own[(size_t)i1 * W + w];
        }
        const uint32_t odd = (i + c) & 1u;
        const uint32_t side = side_word(cur, nbw, odd);
        const size_t idx = (size_t)i * W + w;
        // aligned-neighbour indicators; a = number aligned, dE = J (4a - 8)
        const uint32_t e1 = ~(sv ^ up), e2 = ~(sv ^ dn), e3 = ~(sv ^ cur), e4 = ~(sv ^ side);
        const uint32_t a1 = e1 & e2, x1 = e1 ^ e2, a2 = e3 & e4, x2 = e3 ^ e4;
        const uint32_t m4 = a1 & a2;                // a = 4: dE = 8J
        const uint32_t m3 = (a1 & x2) | (a2 & x1);  // a = 3: dE = 4J
        const uint32_t need[2] = {rng3 ? m3 : 0u, rng4 ? m4 : 0u};
        const uint32_t never = (nev3 ? m3 : 0u) | (nev4 ? m4 : 0u);
        const uint32_t always = ~(need[0] | need[1] | never);
        const uint32_t flip = metropolis_accept<2>(need, thr, always, i, w, t, c, lat.key0, lat.key1);
        const uint32_t ns = sv ^ flip;
        own[idx] = ns;
        if (MEASURE)
            ising_em(e, ns, up, dn, cur, side);
        up = cur;
        cur = dn;
        dn = dn2;
        nbw = nbw2;
        sv = sv2;
    }
}

struct Pair {
    uint32_t z, s;  // z: s != 0, s: s < 0
};

__device__ __forceinline__ Pair load_pair(const uint32_t *plane, size_t word)
{
    const uint2 v = reinterpret_cast<const uint2 *>(plane)[word];
    return Pair{v.x, v.y};
}

// Blume-Capel site classes of one word.  X is the proposal plane (plane 0 of
// the proposal stream): the bit-sliced y = s_eff * h (neighbour sum seen from
// the sign that the move carries) and the move family give each site its
// acceptance group; need[q] are the sites of group q that need a random
// number, never the sites that are always rejected (T = 0); the rest are
// accepted outright.
template <int NG, bool PLAIN = false>
__device__ __forceinline__ void bc_classify(const GroupTable &gt, const Pair &s, const Pair (&nbr)[4], uint32_t X,
                                            uint32_t (&need)[NG], uint32_t &never)
{
    uint32_t mask[NG];
    if constexpr (NG == kBcGroups) {
        // sign carried by y: that of s when s != 0, of the proposed s' when s = 0
        const uint32_t neg = (s.z & s.s) | (~s.z & X);
        uint32_t bits[8];
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            const uint32_t anti = nbr[n].s ^ neg;
            bits[n] = nbr[n].z & ~anti;        // neighbour contributes +1 to y
            bits[4 + n] = ~(nbr[n].z & anti);  // neighbour does not contribute -1
        }
        uint32_t b0, b1, b2, b3;
        count8(bits, b0, b1, b2, b3);  // v = y + 4 in [0, 8]
        uint32_t Y[9];
        {
            const uint32_t nb3 = ~b3;
            const uint32_t t0 = ~b1 & ~b0, t1 = ~b1 & b0, t2 = b1 & ~b0, t3 = b1 & b0;
            const uint32_t h0 = nb3 & ~b2, h1 = nb3 & b2;
            Y[0] = h0 & t0; Y[1] = h0 & t1; Y[2] = h0 & t2; Y[3] = h0 & t3;
            Y[4] = h1 & t0; Y[5] = h1 & t1; Y[6] = h1 & t2; Y[7] = h1 & t3;
            Y[8] = b3;
        }
        const uint32_t famA = s.z & ~X;  // s -> 0:   dE = J y - Delta
        const uint32_t famB = ~s.z;      // 0 -> s':  dE = -J y + Delta
        const uint32_t famC = s.z & X;   // s -> -s:  dE = 2 J y
        // general Delta: for each y one of {s -> 0, 0 -> s'} can have dE > 0
        // (sel_a picks it); s -> -s has dE > 0 for y > 0
#pragma unroll
        for (int q = 0; q < NG; ++q)
            mask[q] = q < 9 ? ((((gt.sel_a_bits >> q) & 1u) ? famA : famB) & Y[q]) : (famC & Y[q - 4]);
    } else {
        // Delta = 0.  With the sign carried by y taken as that of s when
        // s != 0 and as the opposite of the proposed s' when s = 0, every move
        // has dE = J y (s -> 0 and 0 -> s') or 2 J y (s -> -s): only
        // y = 1..4 (v = y + 4 = 5..8) falls in a group, and the two families
        // with dE = J y share their masks.
        const uint32_t neg = (s.z & s.s) | (~s.z & ~X);
        uint32_t bits[8];
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            const uint32_t anti = nbr[n].s ^ neg;
            bits[n] = nbr[n].z & ~anti;        // neighbour contributes +1 to y
            bits[4 + n] = ~(nbr[n].z & anti);  // neighbour does not contribute -1
        }
        uint32_t b0, b1, b2, b3;
        count8(bits, b0, b1, b2, b3);  // v in [0, 8]
        const uint32_t h1 = b2 & ~b3;  // v in 4..7
        const uint32_t Y5 = h1 & ~b1 & b0, Y6 = h1 & b1 & ~b0, Y7 = h1 & b1 & b0, Y8 = b3;
        const uint32_t famC = s.z & X;  // s -> -s (the rest: dE = J y)
        mask[0] = ~famC & Y5;                   // dE = J
        mask[1] = (famC & Y5) | (~famC & Y6);   // 2J
        mask[2] = ~famC & Y7;                   // 3J
        mask[3] = (famC & Y6) | (~famC & Y8);   // 4J
        mask[4] = famC & Y7;                    // 6J
        mask[5] = famC & Y8;                    // 8J
    }
    never = 0;
#pragma unroll
    for (int q = 0; q < NG; ++q) {
        if constexpr (PLAIN) {
            need[q] = mask[q];
        } else {
            need[q] = ((gt.rng_bits >> q) & 1u) ? mask[q] : 0u;
            never |= ((gt.never_bits >> q) & 1u) ? mask[q] : 0u;
        }
    }
}

// Every one of the NG groups draws random numbers and none is never accepted
// (every finite T > 0): the classification then needs no selects.
template <int NG>
__host__ __device__ __forceinline__ bool bc_plain(const GroupTable &gt)
{
    constexpr uint32_t all = (1u << NG) - 1u;
    return (gt.rng_bits & all) == all && (gt.never_bits & all) == 0u;
}

// New state of a word: accepted sites (F) take the proposed value.
__device__ __forceinline__ Pair bc_new_state(uint32_t F, const Pair &s, uint32_t X)
{
    const uint32_t zp = ~s.z | X;          // proposed s' != 0
    const uint32_t sp = X & ~(s.z & s.s);  // proposed s' < 0
    return Pair{(F & zp) | (~F & s.z), (F & sp) | (~F & s.s)};
}

__device__ __forceinline__ void bc_store(uint32_t *own, size_t idx, const Pair &p)
{
    uint2 out;
    out.x = p.z;
    out.y = p.s;
    reinterpret_cast<uint2 *>(own)[idx] = out;
}

// Energy/magnetisation counters of one updated word and the other-colour word
// at its position (see kEmCounters).
__device__ __forceinline__ void bc_em(unsigned long long (&e)[kEmCounters], const Pair &n, const Pair &cur,
                                      const Pair (&nbr)[4])
{
    e[0] += __popc(n.z) + __popc(cur.z);
    e[1] += __popc(n.s) + __popc(cur.s);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t both = n.z & nbr[k].z;
        e[2] += __popc(both);
        e[3] += __popc(both & (n.s ^ nbr[k].s));
    }
}

// Neighbour pairs of word (i, w) of the other plane: up, down, same, side.
__device__ __forceinline__ void bc_nbrs(const uint32_t *oth, uint32_t L, uint32_t W, uint32_t c, uint32_t i,
                                        uint32_t w, Pair (&nbr)[4])
{
    const uint32_t iu = i == 0 ? L - 1 : i - 1, id = i + 1 == L ? 0 : i + 1;
    const uint32_t odd = (i + c) & 1u;
    const uint32_t wn = odd ? (w + 1u == W ? 0u : w + 1u) : (w == 0 ? W : w) - 1u;
    nbr[0] = load_pair(oth, (size_t)iu * W + w);
    nbr[1] = load_pair(oth, (size_t)id * W + w);
    nbr[2] = load_pair(oth, (size_t)i * W + w);
    const Pair nb = load_pair(oth, (size_t)i * W + wn);
    nbr[3] = Pair{side_word(nbr[2].z, nb.z, odd), side_word(nbr[2].s, nb.s, odd)};
}

// Blume-Capel half-sweep of one tile, one word at a time: each thread runs
// the lazy Metropolis test of its word to completion.  Each row loads the
// next row's words before it draws random planes.
// pats: the table's plane_groups, read with uniform loads (the kernel
// argument's, or the batch table's in global memory).
// UNIFORM: W is a multiple of 64, so a wavefront's 64 items share one row
// group (and fill whole tiles): the row is wave-uniform and the Philox rounds
// start in scalar registers, as in ising_tile_lazy.
template <bool MEASURE, int R, int NG, bool PLAIN = false, bool UNIFORM = false>
__device__ __forceinline__ void bc_tile(const Lattice &lat, uint32_t c, uint32_t t, const GroupTable &gt,
                                        const uint32_t *pats, uint64_t tile, unsigned long long (&e)[kEmCounters])
{
    const uint32_t L = lat.L, W = lat.W;
    uint32_t *own = lat.planes + (c ? lat.plane_u32 : 0);
    const uint32_t *oth = lat.planes + (c ? 0 : lat.plane_u32);
    const uint64_t nitems = (uint64_t)(L / R) * W;
    const uint64_t g = tile * kBlock + threadIdx.x;
    if (!UNIFORM && g >= nitems)
        return;
    uint32_t thr[NG];
#pragma unroll
    for (int q = 0; q < NG; ++q)
        thr[q] = gt.thr[q];
    uint32_t rg;
    if (UNIFORM) {
        const uint32_t wave0 = __builtin_amdgcn_readfirstlane(threadIdx.x) & ~63u;
        rg = __builtin_amdgcn_readfirstlane((uint32_t)((tile * kBlock + wave0) / W));
    } else {
        rg = row_group(g, W, nitems);
    }
    const uint32_t w = (uint32_t)(g - (uint64_t)rg * W);
    const uint32_t i0 = rg * R;
    const uint32_t wl = (w == 0 ? W : w) - 1u;
    const uint32_t wr = (w + 1u == W) ? 0u : w + 1u;
    Pair up = load_pair(oth, (size_t)(i0 == 0 ? L - 1 : i0 - 1) * W + w);
    Pair cur = load_pair(oth, (size_t)i0 * W + w);
    Pair dn = load_pair(oth, (size_t)(i0 + 1u == L ? 0u : i0 + 1u) * W + w);
    Pair nbw = load_pair(oth, (size_t)i0 * W + (((i0 + c) & 1u) ? wr : wl));
    Pair s = load_pair(own, (size_t)i0 * W + w);
#pragma unroll 2
    for (int r = 0; r < R; ++r) {
        const uint32_t i = i0 + (uint32_t)r;
        Pair dn2{0u, 0u}, nbw2{0u, 0u}, s2{0u, 0u};
        if (r + 1 < R) {
            const uint32_t i1 = i + 1u;  // i0 + R <= L: still in the tile
            dn2 = load_pair(oth, (size_t)(i1 + 1u == L ? 0u : i1 + 1u) * W + w);
            nbw2 = load_pair(oth, (size_t)i1 * W + (((i1 + c) & 1u) ? wr : wl));
            s2 = load_pair(own, (size_t)i1 * W + w);
        }
        const uint32_t odd = (i + c) & 1u;
        const Pair side{side_word(cur.z, nbw.z, odd), side_word(cur.s, nbw.s, odd)};
        const Pair nbr[4] = {up, dn, cur, side};
        const uint32_t X =
            philox_block<UNIFORM>(i, w, t, stream_tag(kPurposePropose, c, 0), lat.key0, lat.key1).v[0];
        uint32_t need[NG], never;
        bc_classify<NG, PLAIN>(gt, s, nbr, X, need, never);
        uint32_t any = 0;
#pragma unroll
        for (int q = 0; q < NG; ++q)
            any |= need[q];
        const uint32_t F =
            metropolis_accept<NG, UNIFORM>(need, thr, ~(any | never), i, w, t, c, lat.key0, lat.key1, pats);
        const Pair n = bc_new_state(F, s, X);
        bc_store(own, (size_t)i * W + w, n);
        if (MEASURE)
            bc_em(e, n, cur, nbr);
        up = cur;
        cur = dn;
        dn = dn2;
        nbw = nbw2;
        s = s2;
    }
}

// Blume-Capel half-sweep, compacting form (as ising_tile_compact): proposal
// plane and acceptance blocks 0 and 1 in place, words still undecided after
// eight planes to the wavefront's list, drained one word per lane, new words
// staged in LDS and stored as whole rows.
template <int NG, int CAP, int R>
struct BcList {
    static constexpr int kCap = CAP;
    uint32_t und[CAP], acc[CAP], x[CAP];
    uint32_t need[NG][CAP];
    uint16_t slot[CAP];  // row offset << 6 | owning lane
    uint32_t i0[64], w[64];
    // new (Z, S) words of the tile, stored to HBM in whole rows once the
    // list is drained (listed words hold the old pair until then)
    uint2 stage[R][64];
};

template <bool MEASURE, int R, int NG, typename List, bool PLAIN = false, bool UNIFORM = false>
__device__ __forceinline__ void bc_tile_compact(const Lattice &lat, uint32_t c, uint32_t t, const GroupTable &gt,
                                                const uint32_t *pats, uint64_t tile, List &Q,
                                                unsigned long long (&e)[kEmCounters])
{
    constexpr int kListCap = List::kCap;
    const uint32_t L = lat.L, W = lat.W;
    uint32_t *own = lat.planes + (c ? lat.plane_u32 : 0);
    const uint32_t *oth = lat.planes + (c ? 0 : lat.plane_u32);
    const uint64_t nitems = (uint64_t)(L / R) * W;
    uint32_t thr[NG];
#pragma unroll
    for (int q = 0; q < NG; ++q)
        thr[q] = gt.thr[q];
    const uint32_t k0 = lat.key0, k1 = lat.key1;
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t g = tile * kBlock + threadIdx.x;
    const bool valid = UNIFORM || g < nitems;  // UNIFORM: whole tiles (see bc_tile)
    uint32_t rg, w;
    if (UNIFORM) {
        const uint32_t wave0 = __builtin_amdgcn_readfirstlane(threadIdx.x) & ~63u;
        rg = __builtin_amdgcn_readfirstlane((uint32_t)((tile * kBlock + wave0) / W));
        w = (uint32_t)(g - (uint64_t)rg * W);
    } else {
        rg = valid ? row_group(g, W, nitems) : 0u;
        w = valid ? (uint32_t)(g - (uint64_t)rg * W) : 0u;
    }
    const uint32_t i0 = rg * R;
    Q.i0[lane] = i0;
    Q.w[lane] = w;
    uint32_t n = 0;
    const uint32_t wl = (w == 0 ? W : w) - 1u;
    const uint32_t wr = (w + 1u == W) ? 0u : w + 1u;
    // lanes past the end (rg = w = 0) load existing words and never use them
    Pair up = load_pair(oth, (size_t)(i0 == 0 ? L - 1 : i0 - 1) * W + w);
    Pair cur = load_pair(oth, (size_t)i0 * W + w);
    Pair dn = load_pair(oth, (size_t)(i0 + 1u == L ? 0u : i0 + 1u) * W + w);
    Pair nbw = load_pair(oth, (size_t)i0 * W + (((i0 + c) & 1u) ? wr : wl));
    Pair s = load_pair(own, (size_t)i0 * W + w);
#pragma unroll 2
    for (int r = 0; r < R; ++r) {
        const uint32_t i = i0 + (uint32_t)r;
        Pair dn2{0u, 0u}, nbw2{0u, 0u}, s2{0u, 0u};
        if (r + 1 < R) {
            const uint32_t i1 = i + 1u;  // i0 + R <= L: still in the tile
            dn2 = load_pair(oth, (size_t)(i1 + 1u == L ? 0u : i1 + 1u) * W + w);
            nbw2 = load_pair(oth, (size_t)i1 * W + (((i1 + c) & 1u) ? wr : wl));
            s2 = load_pair(own, (size_t)i1 * W + w);
        }
        const uint32_t odd = (i + c) & 1u;
        const Pair side{side_word(cur.z, nbw.z, odd), side_word(cur.s, nbw.s, odd)};
        const Pair nbr[4] = {up, dn, cur, side};
        uint32_t X = 0, acc = 0, und = 0, need[NG];
#pragma unroll
        for (int q = 0; q < NG; ++q)
            need[q] = 0;
        if (valid) {
            X = philox_block<UNIFORM>(i, w, t, stream_tag(kPurposePropose, c, 0), k0, k1).v[0];
            uint32_t never;
            bc_classify<NG, PLAIN>(gt, s, nbr, X, need, never);
#pragma unroll
            for (int q = 0; q < NG; ++q)
                und |= need[q];
            acc = ~(und | never);
            if (und != 0u) {
                const Block4 b = philox_block<UNIFORM>(i, w, t, stream_tag(kPurposeAccept, c, 0), k0, k1);
                apply_block_any<NG>(b, 0u, need, thr, pats, und, acc);
            }
            if (und != 0u) {
                const Block4 b = philox_block<UNIFORM>(i, w, t, stream_tag(kPurposeAccept, c, 1), k0, k1);
                apply_block_any<NG>(b, 1u, need, thr, pats, und, acc);
            }
        }
        const unsigned long long bal = __ballot(und != 0u);
        bool listed = false;
        if (und != 0u) {
            const uint32_t p = n + __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                             __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
            if (p < (uint32_t)kListCap) {
                Q.und[p] = und;
                Q.acc[p] = acc;
                Q.x[p] = X;
                Q.stage[r][lane] = make_uint2(s.z, s.s);
#pragma unroll
                for (int q = 0; q < NG; ++q)
                    Q.need[q][p] = need[q];
                Q.slot[p] = (uint16_t)(((uint32_t)r << 6) | lane);
                listed = true;
            } else {
                for (uint32_t blk = 2; blk < 8u && und != 0u; ++blk) {
                    const Block4 b = philox4x32_10(i, w, t, stream_tag(kPurposeAccept, c, blk), k0, k1);
                    apply_block_any<NG>(b, blk, need, thr, pats, und, acc);
                }
            }
        }
        if (valid && !listed) {
            const Pair ns = bc_new_state(acc, s, X);  // ties after 32 planes (u == thr) rejected
            Q.stage[r][lane] = make_uint2(ns.z, ns.s);
            if (MEASURE)
                bc_em(e, ns, cur, nbr);
        }
        n += (uint32_t)__popcll(bal);
        up = cur;
        cur = dn;
        dn = dn2;
        nbw = nbw2;
        s = s2;
    }
    if (n > (uint32_t)kListCap)
        n = kListCap;
    wave_sync();
    for (uint32_t k = lane; k < n; k += 64u) {
        const uint32_t slot = Q.slot[k], owner = slot & 63u;
        const uint32_t i = Q.i0[owner] + (slot >> 6), wq = Q.w[owner];
        uint32_t need[NG];
#pragma unroll
        for (int q = 0; q < NG; ++q)
            need[q] = Q.need[q][k];
        uint32_t und = Q.und[k], acc = Q.acc[k];
        for (uint32_t blk = 2; blk < 8u && und != 0u; ++blk) {
            const Block4 b = philox4x32_10(i, wq, t, stream_tag(kPurposeAccept, c, blk), k0, k1);
            apply_block_any<NG>(b, blk, need, thr, pats, und, acc);
        }
        const uint2 old = Q.stage[slot >> 6][owner];
        const Pair ns = bc_new_state(acc, Pair{old.x, old.y}, Q.x[k]);
        Q.stage[slot >> 6][owner] = make_uint2(ns.z, ns.s);
        if (MEASURE) {
            Pair nbr[4];
            bc_nbrs(oth, L, W, c, i, wq, nbr);
            bc_em(e, ns, nbr[2], nbr);
        }
    }
    wave_sync();
    // whole rows to HBM: every line of the tile is written once and complete
    if (valid) {
#pragma unroll
        for (int r = 0; r < R; ++r)
            reinterpret_cast<uint2 *>(own)[(size_t)(i0 + (uint32_t)r) * W + w] = Q.stage[r][lane];
    }
    wave_sync();  // the list and the stage are refilled by the next tile
}

template <int R>
__host__ __device__ inline uint64_t tiles_of(const Lattice &lat)
{
    return ((uint64_t)(lat.L / R) * lat.W + kBlock - 1) / kBlock;
}

// Blume-Capel list slots per wavefront: 8 per row of the tile (about 6% of
// the words are still undecided after eight planes).
constexpr int bc_list_cap(int v) { return v == 4 ? 16 : 8 * variant_rows(v); }

} // namespace

} // namespace spin
