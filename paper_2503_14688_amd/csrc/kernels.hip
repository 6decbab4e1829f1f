// gfx950 kernels: initial state, checkerboard half-sweeps (Ising 1 bit per
// spin, Blume-Capel 2 bit planes), the energy/magnetisation reduction, the
// axis correlation sums C(r), and the window decoder.
//
// Layout (one colour plane per checkerboard colour, paper Introduction):
// site (i, j) has colour c = (i + j) & 1 and sits at m = j >> 1 of row i of
// plane c, word w = m >> 5, bit b = m & 31.  Its vertical neighbours are at
// the same (w, b) in rows i -+ 1 of the other plane; its horizontal
// neighbours are (i, m) and (i, m - 1) of the other plane when (i + c) is
// even, (i, m) and (i, m + 1) when it is odd.
#include <type_traits>

#include "device.hpp"
#include "kernels.hpp"

namespace spin {

namespace {

constexpr int kBlock = 256;

inline unsigned grid_for(uint64_t items)
{
    uint64_t b = (items + kBlock - 1) / kBlock;
    if (b > 65536)
        b = 65536;
    if (b == 0)
        b = 1;
    return (unsigned)b;
}

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

// ---------------------------------------------------------------- init --

__global__ __launch_bounds__(kBlock) void k_init_ising(uint32_t *planes, uint32_t L, uint32_t W,
                                                       uint64_t plane_u32, uint32_t k0, uint32_t k1)
{
    const uint64_t n = 2 * plane_u32;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n;
         g += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t c = g >= plane_u32;
        const uint64_t rem = g - (c ? plane_u32 : 0);
        const uint32_t i = (uint32_t)(rem / W);
        const uint32_t w = (uint32_t)(rem - (uint64_t)i * W);
        // plane 0 of the stream is the sign bit: u >= 2^31 <=> s = -1
        planes[g] = philox4x32_10(i, w, 0u, stream_tag(kPurposeInit, c, 0), k0, k1).v[0];
    }
}

__global__ __launch_bounds__(kBlock) void k_init_bc(uint32_t *planes, uint32_t L, uint32_t W,
                                                    uint64_t plane_u32, uint32_t k0, uint32_t k1)
{
    // s = floor(3u / 2^32) - 1: s = -1 iff u < 1431655766, s = 0 iff
    // 1431655766 <= u < 2863311531, else +1; both comparisons bit-sliced.
    constexpr uint32_t kThird = 1431655766u, kTwoThirds = 2863311531u;
    const uint64_t words = plane_u32;  // two uint32 per site word in BC planes
    const uint64_t n = words;          // (Z, S) pairs over both colours
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n;
         g += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t per_plane = plane_u32 / 2;
        const uint32_t c = g >= per_plane;
        const uint64_t rem = g - (c ? per_plane : 0);
        const uint32_t i = (uint32_t)(rem / W);
        const uint32_t w = (uint32_t)(rem - (uint64_t)i * W);
        uint32_t lt1 = 0, eq1 = ~0u, lt2 = 0, eq2 = ~0u;
        for (uint32_t blk = 0; blk < 8; ++blk) {
            const Block4 r = philox4x32_10(i, w, 0u, stream_tag(kPurposeInit, c, blk), k0, k1);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t sh = 31u - (4u * blk + (uint32_t)q);
                const uint32_t ub = r.v[q];
                const uint32_t a = 0u - ((kThird >> sh) & 1u);
                const uint32_t b = 0u - ((kTwoThirds >> sh) & 1u);
                lt1 |= eq1 & a & ~ub;
                eq1 &= ~(a ^ ub);
                lt2 |= eq2 & b & ~ub;
                eq2 &= ~(b ^ ub);
            }
        }
        uint2 v;
        v.x = lt1 | ~lt2;  // nonzero: u < 1/3 or u >= 2/3
        v.y = lt1;         // negative: u < 1/3
        reinterpret_cast<uint2 *>(planes)[g] = v;
    }
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
    const PlaneMasks2 pm = plane_masks_2g(thr);
    const bool rng3 = gt.rng_bits & 1u, rng4 = gt.rng_bits & 2u;
    const bool nev3 = gt.never_bits & 1u, nev4 = gt.never_bits & 2u;
    const uint32_t k0 = lat.key0, k1 = lat.key1;
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t g = tile * kBlock + threadIdx.x;
    const bool valid = g < nitems;
    uint32_t rg, w;
    if (UNIFORM) {
        // W % 64 == 0: the wavefront's 64 items lie in one row group (and L is
        // a multiple of 4096, so the items fill whole tiles: no lane is past
        // the end)
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
        uint32_t acc = 0, und = 0, need[2] = {0u, 0u};
        if (valid) {
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
            apply_block_2g_pm<0>(b0, pm, need[1], und, acc);
            const Block4 b1 = philox_block<UNIFORM>(i, w, t, stream_tag(kPurposeAccept, c, 1), k0, k1);
            apply_block_2g_pm<1>(b1, pm, need[1], und, acc);
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
    if (g >= nitems)
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
template <int NG>
__device__ __forceinline__ void bc_classify(const GroupTable &gt, const Pair &s, const Pair (&nbr)[4], uint32_t X,
                                            uint32_t (&need)[NG], uint32_t &never)
{
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
    uint32_t mask[NG];
    if constexpr (NG == kBcGroups) {
        // general Delta: for each y one of {s -> 0, 0 -> s'} can have dE > 0
        // (sel_a picks it); s -> -s has dE > 0 for y > 0
#pragma unroll
        for (int q = 0; q < NG; ++q)
            mask[q] = q < 9 ? ((((gt.sel_a_bits >> q) & 1u) ? famA : famB) & Y[q]) : (famC & Y[q - 4]);
    } else {
        // Delta = 0: dE = J y (s -> 0), -J y (0 -> s'), 2 J y (s -> -s); v = y + 4
        mask[0] = (famA & Y[5]) | (famB & Y[3]);                 // dE = J
        mask[1] = (famA & Y[6]) | (famB & Y[2]) | (famC & Y[5]);  // 2J
        mask[2] = (famA & Y[7]) | (famB & Y[1]);                 // 3J
        mask[3] = (famA & Y[8]) | (famB & Y[0]) | (famC & Y[6]);  // 4J
        mask[4] = famC & Y[7];                                   // 6J
        mask[5] = famC & Y[8];                                   // 8J
    }
    never = 0;
#pragma unroll
    for (int q = 0; q < NG; ++q) {
        need[q] = ((gt.rng_bits >> q) & 1u) ? mask[q] : 0u;
        never |= ((gt.never_bits >> q) & 1u) ? mask[q] : 0u;
    }
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
template <bool MEASURE, int R, int NG>
__device__ __forceinline__ void bc_tile(const Lattice &lat, uint32_t c, uint32_t t, const GroupTable &gt,
                                        uint64_t tile, unsigned long long (&e)[kEmCounters])
{
    const uint32_t L = lat.L, W = lat.W;
    uint32_t *own = lat.planes + (c ? lat.plane_u32 : 0);
    const uint32_t *oth = lat.planes + (c ? 0 : lat.plane_u32);
    const uint64_t nitems = (uint64_t)(L / R) * W;
    const uint64_t g = tile * kBlock + threadIdx.x;
    if (g >= nitems)
        return;
    uint32_t thr[NG];
#pragma unroll
    for (int q = 0; q < NG; ++q)
        thr[q] = gt.thr[q];
    const uint32_t rg = row_group(g, W, nitems);
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
        const uint32_t X = philox4x32_10(i, w, t, stream_tag(kPurposePropose, c, 0), lat.key0, lat.key1).v[0];
        uint32_t need[NG], never;
        bc_classify<NG>(gt, s, nbr, X, need, never);
        uint32_t any = 0;
#pragma unroll
        for (int q = 0; q < NG; ++q)
            any |= need[q];
        const uint32_t F = metropolis_accept<NG>(need, thr, ~(any | never), i, w, t, c, lat.key0, lat.key1);
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

template <bool MEASURE, int R, int NG, typename List>
__device__ __forceinline__ void bc_tile_compact(const Lattice &lat, uint32_t c, uint32_t t, const GroupTable &gt,
                                                uint64_t tile, List &Q, unsigned long long (&e)[kEmCounters])
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
    const bool valid = g < nitems;
    const uint32_t rg = valid ? row_group(g, W, nitems) : 0u;
    const uint32_t w = valid ? (uint32_t)(g - (uint64_t)rg * W) : 0u;
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
            X = philox4x32_10(i, w, t, stream_tag(kPurposePropose, c, 0), k0, k1).v[0];
            uint32_t never;
            bc_classify<NG>(gt, s, nbr, X, need, never);
#pragma unroll
            for (int q = 0; q < NG; ++q)
                und |= need[q];
            acc = ~(und | never);
            if (und != 0u) {
                const Block4 b = philox4x32_10(i, w, t, stream_tag(kPurposeAccept, c, 0), k0, k1);
                apply_block<NG>(b, 0u, need, thr, und, acc);
            }
            if (und != 0u) {
                const Block4 b = philox4x32_10(i, w, t, stream_tag(kPurposeAccept, c, 1), k0, k1);
                apply_block<NG>(b, 1u, need, thr, und, acc);
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
                    apply_block<NG>(b, blk, need, thr, und, acc);
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
            apply_block<NG>(b, blk, need, thr, und, acc);
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

// LDS of the compacting tiles, per wavefront: one list per model and group
// count, sharing that wavefront's storage (a tile uses one of them).
// Blume-Capel list slots per wavefront: 8 per row of the tile (about 6% of
// the words are still undecided after eight planes).
constexpr int bc_list_cap(int v) { return v == 4 ? 16 : 8 * variant_rows(v); }

template <int V>
union BcListUnion {
    BcList<kBcGroupsDelta0, bc_list_cap(V), variant_rows(V)> d0;
    BcList<kBcGroups, bc_list_cap(V), variant_rows(V)> gen;
};

template <int V>
union AnyList {
    WaveList<variant_list_cap(V)> ising;
    BcList<kBcGroupsDelta0, bc_list_cap(V), variant_rows(V)> d0;
    BcList<kBcGroups, bc_list_cap(V), variant_rows(V)> gen;
};

template <int V>
struct IsingList {
    WaveList<variant_list_cap(V)> ising;
};

// LDS of the batched kernel, per wavefront: only the lists of the models the
// batch holds and of the strategies it runs them with (an Ising-only batch
// keeps the Ising kernel's smaller LDS, so as many blocks fit on a CU as in
// the single-lattice launch; a per-word strategy needs no list).
template <int BV, int MODELS>
union BatchList {
    static constexpr int VI = batch_ising_variant(BV), VB = batch_bc_variant(BV);
    static constexpr bool kIsingList = (MODELS & kBatchIsing) != 0 && variant_compact(VI);
    static constexpr bool kBcList = (MODELS & kBatchBc) != 0 && variant_compact(VB);
    std::conditional_t<kIsingList, WaveList<variant_list_cap(VI)>, char> ising;
    std::conditional_t<kBcList, BcList<kBcGroupsDelta0, bc_list_cap(VB), variant_rows(VB)>, char> d0;
    std::conditional_t<kBcList, BcList<kBcGroups, bc_list_cap(VB), variant_rows(VB)>, char> gen;
};

template <bool MEASURE, int V>
__global__ __launch_bounds__(kBlock) void k_sweep_ising(Lattice lat, uint32_t c, uint32_t t, GroupTable gt,
                                                        unsigned long long *acc)
{
    constexpr int R = variant_rows(V);
    unsigned long long e[kEmCounters] = {0, 0, 0, 0};
    const uint64_t ntiles = tiles_of<R>(lat);
    if constexpr (variant_compact(V)) {
        __shared__ WaveList<variant_list_cap(V)> Q[kWaves];
        using QL = WaveList<variant_list_cap(V)>;
        const bool plain = (gt.rng_bits & 3u) == 3u && (gt.never_bits & 3u) == 0u;
        if (lat.W % 64 == 0 && plain) {
            for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x)
                ising_tile_compact<MEASURE, R, true, QL, true>(lat, c, t, gt, tile, Q[threadIdx.x >> 6], e);
        } else if (lat.W % 64 == 0) {
            for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x)
                ising_tile_compact<MEASURE, R, true>(lat, c, t, gt, tile, Q[threadIdx.x >> 6], e);
        } else {
            for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x)
                ising_tile_compact<MEASURE, R, false>(lat, c, t, gt, tile, Q[threadIdx.x >> 6], e);
        }
    } else if (lat.W % 64 == 0) {
        for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x)
            ising_tile_lazy<MEASURE, R, true>(lat, c, t, gt, tile, e);
    } else {
        for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x)
            ising_tile_lazy<MEASURE, R, false>(lat, c, t, gt, tile, e);
    }
    if (MEASURE)
        block_reduce_atomic<kEmCounters>(e, acc);
}

template <bool MEASURE, int V>
__global__ __launch_bounds__(kBlock) void k_sweep_bc(Lattice lat, uint32_t c, uint32_t t, GroupTable gt,
                                                     unsigned long long *acc)
{
    constexpr int R = variant_rows(V);
    unsigned long long e[kEmCounters] = {0, 0, 0, 0};
    const uint64_t ntiles = tiles_of<R>(lat);
    if constexpr (variant_compact(V)) {
        __shared__ BcListUnion<V> Q[kWaves];
        if (lat.bc_groups == kBcGroupsDelta0) {
            for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x)
                bc_tile_compact<MEASURE, R, kBcGroupsDelta0>(lat, c, t, gt, tile, Q[threadIdx.x >> 6].d0, e);
        } else {
            for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x)
                bc_tile_compact<MEASURE, R, kBcGroups>(lat, c, t, gt, tile, Q[threadIdx.x >> 6].gen, e);
        }
    } else if (lat.bc_groups == kBcGroupsDelta0) {
        for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x)
            bc_tile<MEASURE, R, kBcGroupsDelta0>(lat, c, t, gt, tile, e);
    } else {
        for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x)
            bc_tile<MEASURE, R, kBcGroups>(lat, c, t, gt, tile, e);
    }
    if (MEASURE)
        block_reduce_atomic<kEmCounters>(e, acc);
}

// Batched half-sweep: one launch advances colour c of every replica.  The
// flat tile list maps each global tile to (replica, local tile); replica r's
// thresholds for this sweep are tables[sched(r) * stride + step] and its
// random stream runs at sweep index t0(r) + step.
// A copy of *p in scalar registers (p is the same for the whole wavefront).
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

template <int BV, int MODELS>
__global__ __launch_bounds__(kBlock) void k_batch_half_sweep(const BatchReplica *__restrict__ reps,
                                                             const uint32_t *__restrict__ tile_rep, uint64_t ntiles,
                                                             const GroupTable *__restrict__ tables, uint32_t stride,
                                                             const uint32_t *__restrict__ step_base, uint32_t step_off,
                                                             uint32_t c)
{
    constexpr int VI = batch_ising_variant(BV), VB = batch_bc_variant(BV);
    constexpr int RI = variant_rows(VI), RB = variant_rows(VB);
    // schedule step: the batch's device step counter (advanced at the end of
    // every run) plus this launch's offset in the run, so that a captured
    // run can be replayed for the next steps unchanged
    const uint32_t step = __builtin_amdgcn_readfirstlane(*step_base) + step_off;
    __shared__ BatchList<BV, MODELS> Q[kWaves];
    unsigned long long e[kEmCounters] = {0, 0, 0, 0};
    for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        // The tile, hence its replica, is the same for the whole block: keep
        // the descriptor and thresholds in scalar registers, as the
        // single-lattice kernel has them (its arguments), so that addresses,
        // keys and the row-uniform Philox rounds stay scalar.
        const uint32_t rid = __builtin_amdgcn_readfirstlane(tile_rep[tile]);
        const BatchReplica rep = wave_uniform_copy(reps + rid);
        const GroupTable gt = wave_uniform_copy(tables + (size_t)rep.sched * stride + step);
        const uint64_t local = tile - rep.tile0;
        const uint32_t t = rep.t0 + step;
        if (rep.lat.model == kIsing) {
            if constexpr ((MODELS & kBatchIsing) != 0) {
                if constexpr (variant_compact(VI)) {
                    using QL = WaveList<variant_list_cap(VI)>;
                    const bool plain = (gt.rng_bits & 3u) == 3u && (gt.never_bits & 3u) == 0u;
                    if (rep.lat.W % 64 == 0 && plain)
                        ising_tile_compact<false, RI, true, QL, true>(rep.lat, c, t, gt, local,
                                                                      Q[threadIdx.x >> 6].ising, e);
                    else if (rep.lat.W % 64 == 0)
                        ising_tile_compact<false, RI, true>(rep.lat, c, t, gt, local, Q[threadIdx.x >> 6].ising, e);
                    else
                        ising_tile_compact<false, RI, false>(rep.lat, c, t, gt, local, Q[threadIdx.x >> 6].ising, e);
                } else if (rep.lat.W % 64 == 0) {
                    ising_tile_lazy<false, RI, true>(rep.lat, c, t, gt, local, e);
                } else {
                    ising_tile_lazy<false, RI, false>(rep.lat, c, t, gt, local, e);
                }
            }
        } else if constexpr ((MODELS & kBatchBc) != 0) {
            if constexpr (variant_compact(VB)) {
                if (rep.lat.bc_groups == kBcGroupsDelta0)
                    bc_tile_compact<false, RB, kBcGroupsDelta0>(rep.lat, c, t, gt, local, Q[threadIdx.x >> 6].d0, e);
                else
                    bc_tile_compact<false, RB, kBcGroups>(rep.lat, c, t, gt, local, Q[threadIdx.x >> 6].gen, e);
            } else if (rep.lat.bc_groups == kBcGroupsDelta0) {
                bc_tile<false, RB, kBcGroupsDelta0>(rep.lat, c, t, gt, local, e);
            } else {
                bc_tile<false, RB, kBcGroups>(rep.lat, c, t, gt, local, e);
            }
        }
    }
}

// ------------------------------------------ energy / magnetisation sums --

template <int MODEL>
__global__ __launch_bounds__(kBlock) void k_measure_em(Lattice lat, unsigned long long *acc)
{
    // Walks the colour-1 plane: every bond has exactly one colour-1 end, and
    // word (i, w) of plane 0 is counted once as the same-row word.
    const uint32_t L = lat.L, W = lat.W;
    const uint32_t *p1 = lat.planes + lat.plane_u32;
    const uint32_t *p0 = lat.planes;
    const uint64_t nitems = (uint64_t)L * W;
    unsigned long long e[kEmCounters] = {0, 0, 0, 0};
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < nitems;
         g += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t i = (uint32_t)(g / W);
        const uint32_t w = (uint32_t)(g - (uint64_t)i * W);
        const uint32_t iu = i == 0 ? L - 1 : i - 1, id = i + 1 == L ? 0 : i + 1;
        const uint32_t odd = (i + 1u) & 1u;
        const uint32_t wn = odd ? (w + 1 == W ? 0 : w + 1) : (w == 0 ? W : w) - 1;
        Pair s, up, dn, cur, nbw;
        if (MODEL == kIsing) {
            s = Pair{~0u, p1[g]};
            up = Pair{~0u, p0[(size_t)iu * W + w]};
            dn = Pair{~0u, p0[(size_t)id * W + w]};
            cur = Pair{~0u, p0[g]};
            nbw = Pair{~0u, p0[(size_t)i * W + wn]};
        } else {
            s = load_pair(p1, g);
            up = load_pair(p0, (size_t)iu * W + w);
            dn = load_pair(p0, (size_t)id * W + w);
            cur = load_pair(p0, g);
            nbw = load_pair(p0, (size_t)i * W + wn);
        }
        const Pair side{side_word(cur.z, nbw.z, odd), side_word(cur.s, nbw.s, odd)};
        const Pair nbr[4] = {up, dn, cur, side};
        e[0] += __popc(s.z) + __popc(cur.z);
        e[1] += __popc(s.s) + __popc(cur.s);
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            const uint32_t both = s.z & nbr[n].z;
            e[2] += __popc(both);
            e[3] += __popc(both & (s.s ^ nbr[n].s));
        }
    }
    block_reduce_atomic<kEmCounters>(e, acc);
}

// ------------------------------------------------------- correlations --

struct RList {
    uint32_t r[kCorrChunk];
};

template <int MODEL, bool VERTICAL>
__global__ __launch_bounds__(kBlock) void k_corr(Lattice lat, RList rl, int n_r, unsigned long long *acc)
{
    const uint32_t L = lat.L, W = lat.W, half = L / 2;
    const uint64_t per_plane = (uint64_t)L * W;
    const uint64_t nitems = 2 * per_plane;
    unsigned long long cnt[2 * kCorrChunk];
#pragma unroll
    for (int q = 0; q < 2 * kCorrChunk; ++q)
        cnt[q] = 0;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < nitems;
         g += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t c = g >= per_plane;
        const uint64_t rem = g - (c ? per_plane : 0);
        const uint32_t i = (uint32_t)(rem / W);
        const uint32_t w = (uint32_t)(rem - (uint64_t)i * W);
        const uint32_t *pc = lat.planes + (c ? lat.plane_u32 : 0);
        Pair a;
        if (MODEL == kIsing)
            a = Pair{~0u, pc[rem]};
        else
            a = load_pair(pc, rem);
#pragma unroll
        for (int q = 0; q < kCorrChunk; ++q) {
            if (q >= n_r)
                break;
            const uint32_t r = rl.r[q];
            const uint32_t tc = c ^ (r & 1u);
            const uint32_t *pt = lat.planes + (tc ? lat.plane_u32 : 0);
            Pair b;
            if (VERTICAL) {
                // partner (i + r, j): same m in row i + r of plane c ^ (r & 1)
                uint32_t ti = i + r;
                if (ti >= L)
                    ti -= L;
                const size_t word = (size_t)ti * W + w;
                b = MODEL == kIsing ? Pair{~0u, pt[word]} : load_pair(pt, word);
            } else {
                // partner (i, j + r): m + r/2 in the same plane for even r,
                // m + (r - 1)/2 + ((i + c) & 1) in the other plane for odd r
                uint32_t sh = (r >> 1) + ((r & 1u) & ((i + c) & 1u));
                if (sh >= half)
                    sh -= half;
                uint32_t wa = w + (sh >> 5);
                if (wa >= W)
                    wa -= W;
                const uint32_t wb = wa + 1 == W ? 0 : wa + 1;
                const uint32_t rr = sh & 31u;
                const size_t base = (size_t)i * W;
                Pair x, y;
                if (MODEL == kIsing) {
                    x = Pair{~0u, pt[base + wa]};
                    y = Pair{~0u, pt[base + wb]};
                } else {
                    x = load_pair(pt, base + wa);
                    y = load_pair(pt, base + wb);
                }
                if (rr) {
                    b.z = (x.z >> rr) | (y.z << (32u - rr));
                    b.s = (x.s >> rr) | (y.s << (32u - rr));
                } else {
                    b = x;
                }
            }
            const uint32_t both = a.z & b.z;
            cnt[2 * q] += __popc(both);
            cnt[2 * q + 1] += __popc(both & (a.s ^ b.s));
        }
    }
    block_reduce_atomic<2 * kCorrChunk>(cnt, acc);
}

// ------------------------------------------------------------- helpers --

__global__ void k_advance_step(uint32_t *step, uint32_t n)
{
    if (blockIdx.x == 0 && threadIdx.x == 0)
        *step += n;
}

__global__ void k_fill_u64(unsigned long long *p, uint64_t n, unsigned long long v)
{
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n;
         g += (uint64_t)gridDim.x * blockDim.x)
        p[g] = v;
}

template <int MODEL>
__global__ __launch_bounds__(kBlock) void k_window(Lattice lat, uint32_t i0, uint32_t j0, uint32_t rows,
                                                   uint32_t cols, int8_t *out)
{
    const uint32_t L = lat.L, W = lat.W;
    const uint64_t n = (uint64_t)rows * cols;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n;
         g += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t a = (uint32_t)(g / cols);
        const uint32_t b = (uint32_t)(g - (uint64_t)a * cols);
        uint32_t i = i0 + a, j = j0 + b;
        if (i >= L)
            i -= L;
        if (j >= L)
            j -= L;
        const uint32_t c = (i + j) & 1u;
        const uint32_t m = j >> 1;
        const size_t word = (size_t)i * W + (m >> 5);
        const uint32_t bit = m & 31u;
        const uint32_t *pc = lat.planes + (c ? lat.plane_u32 : 0);
        int8_t v;
        if (MODEL == kIsing) {
            v = ((pc[word] >> bit) & 1u) ? -1 : 1;
        } else {
            const Pair p = load_pair(pc, word);
            v = ((p.z >> bit) & 1u) ? (((p.s >> bit) & 1u) ? -1 : 1) : 0;
        }
        out[g] = v;
    }
}

} // namespace

hipError_t launch_init(const Lattice &lat, hipStream_t st)
{
    if (lat.model == kIsing) {
        hipLaunchKernelGGL(k_init_ising, dim3(grid_for(2 * lat.plane_u32)), dim3(kBlock), 0, st, lat.planes,
                           lat.L, lat.W, lat.plane_u32, lat.key0, lat.key1);
    } else {
        hipLaunchKernelGGL(k_init_bc, dim3(grid_for(lat.plane_u32)), dim3(kBlock), 0, st, lat.planes, lat.L,
                           lat.W, lat.plane_u32, lat.key0, lat.key1);
    }
    return hipGetLastError();
}

template <bool M, int V>
hipError_t launch_half_sweep_v(const Lattice &lat, uint32_t colour, uint32_t t, const GroupTable &gt,
                               unsigned long long *em_acc, hipStream_t st)
{
    constexpr int R = variant_rows(V);
    const uint64_t tiles = tiles_of<R>(lat);
    const dim3 block(kBlock);
    // many more blocks than fit at once: the hardware keeps every CU full
    // while a block's grid-stride loop walks its tiles
    if (lat.model == kIsing) {
        static const unsigned g = 65536u;
        hipLaunchKernelGGL((k_sweep_ising<M, V>), dim3(g < tiles ? g : (unsigned)tiles), block, 0, st, lat, colour,
                           t, gt, em_acc);
    } else {
        static const unsigned g = 65536u;
        hipLaunchKernelGGL((k_sweep_bc<M, V>), dim3(g < tiles ? g : (unsigned)tiles), block, 0, st, lat, colour, t,
                           gt, em_acc);
    }
    return hipGetLastError();
}

hipError_t launch_half_sweep(const Lattice &lat, uint32_t colour, uint32_t t, const GroupTable &gt,
                             unsigned long long *em_acc, hipStream_t st)
{
    const bool m = em_acc != nullptr;
    switch (lat.variant) {
    case 0: return m ? launch_half_sweep_v<true, 0>(lat, colour, t, gt, em_acc, st)
                     : launch_half_sweep_v<false, 0>(lat, colour, t, gt, em_acc, st);
    case 1: return m ? launch_half_sweep_v<true, 1>(lat, colour, t, gt, em_acc, st)
                     : launch_half_sweep_v<false, 1>(lat, colour, t, gt, em_acc, st);
    case 2: return m ? launch_half_sweep_v<true, 2>(lat, colour, t, gt, em_acc, st)
                     : launch_half_sweep_v<false, 2>(lat, colour, t, gt, em_acc, st);
    case 3: return m ? launch_half_sweep_v<true, 3>(lat, colour, t, gt, em_acc, st)
                     : launch_half_sweep_v<false, 3>(lat, colour, t, gt, em_acc, st);
    case 4: return m ? launch_half_sweep_v<true, 4>(lat, colour, t, gt, em_acc, st)
                     : launch_half_sweep_v<false, 4>(lat, colour, t, gt, em_acc, st);
    default: return hipErrorInvalidValue;
    }
}

uint64_t sweep_tiles(const Lattice &lat, int rows)
{
    return rows == 4 ? tiles_of<4>(lat) : tiles_of<8>(lat);
}

template <int V, int MODELS>
hipError_t launch_batch_vm(const BatchReplica *reps, const uint32_t *tile_rep, uint64_t ntiles,
                           const GroupTable *tables, uint32_t stride, const uint32_t *step_base, uint32_t step,
                           uint32_t colour, hipStream_t st)
{
    // The single-lattice launch's grid: up to 65536 blocks, a block walks
    // tiles by grid stride.  (A grid of only the resident blocks, each walking
    // dozens of tiles, measured about 25% slower on large replicas: the
    // hardware's block dispatch overlaps one tile's start with another's end
    // better than a persistent block does.)
    constexpr unsigned g = 65536u;
    hipLaunchKernelGGL((k_batch_half_sweep<V, MODELS>), dim3(g < ntiles ? g : (unsigned)ntiles), dim3(kBlock), 0,
                       st, reps, tile_rep, ntiles, tables, stride, step_base, step, colour);
    return hipGetLastError();
}

template <int V>
hipError_t launch_batch_v(int models, const BatchReplica *reps, const uint32_t *tile_rep, uint64_t ntiles,
                          const GroupTable *tables, uint32_t stride, const uint32_t *step_base, uint32_t step,
                          uint32_t colour, hipStream_t st)
{
    switch (models) {
    case kBatchIsing: return launch_batch_vm<V, kBatchIsing>(reps, tile_rep, ntiles, tables, stride, step_base, step, colour, st);
    case kBatchBc: return launch_batch_vm<V, kBatchBc>(reps, tile_rep, ntiles, tables, stride, step_base, step, colour, st);
    case kBatchMixed: return launch_batch_vm<V, kBatchMixed>(reps, tile_rep, ntiles, tables, stride, step_base, step, colour, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batch_half_sweep(int variant, int models, const BatchReplica *reps, const uint32_t *tile_rep,
                                   uint64_t ntiles, const GroupTable *tables, uint32_t stride,
                                   const uint32_t *step_base, uint32_t step, uint32_t colour, hipStream_t st)
{
    switch (variant) {
    case 0: return launch_batch_v<0>(models, reps, tile_rep, ntiles, tables, stride, step_base, step, colour, st);
    case 1: return launch_batch_v<1>(models, reps, tile_rep, ntiles, tables, stride, step_base, step, colour, st);
    case 2: return launch_batch_v<2>(models, reps, tile_rep, ntiles, tables, stride, step_base, step, colour, st);
    case 3: return launch_batch_v<3>(models, reps, tile_rep, ntiles, tables, stride, step_base, step, colour, st);
    case 4: return launch_batch_v<4>(models, reps, tile_rep, ntiles, tables, stride, step_base, step, colour, st);
    case 5: return launch_batch_v<5>(models, reps, tile_rep, ntiles, tables, stride, step_base, step, colour, st);
    case 6: return launch_batch_v<6>(models, reps, tile_rep, ntiles, tables, stride, step_base, step, colour, st);
    case 7: return launch_batch_v<7>(models, reps, tile_rep, ntiles, tables, stride, step_base, step, colour, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_measure_em(const Lattice &lat, unsigned long long *em_acc, hipStream_t st)
{
    const dim3 grid(grid_for((uint64_t)lat.L * lat.W)), block(kBlock);
    if (lat.model == kIsing)
        hipLaunchKernelGGL(k_measure_em<kIsing>, grid, block, 0, st, lat, em_acc);
    else
        hipLaunchKernelGGL(k_measure_em<kBlumeCapel>, grid, block, 0, st, lat, em_acc);
    return hipGetLastError();
}

hipError_t launch_corr(const Lattice &lat, bool vertical, const uint32_t *r, int n_r,
                       unsigned long long *acc, hipStream_t st)
{
    if (n_r <= 0 || n_r > kCorrChunk)
        return hipErrorInvalidValue;
    RList rl;
    for (int q = 0; q < kCorrChunk; ++q)
        rl.r[q] = q < n_r ? r[q] : 0u;
    const dim3 grid(grid_for(2ull * lat.L * lat.W)), block(kBlock);
    if (lat.model == kIsing) {
        if (vertical)
            hipLaunchKernelGGL((k_corr<kIsing, true>), grid, block, 0, st, lat, rl, n_r, acc);
        else
            hipLaunchKernelGGL((k_corr<kIsing, false>), grid, block, 0, st, lat, rl, n_r, acc);
    } else {
        if (vertical)
            hipLaunchKernelGGL((k_corr<kBlumeCapel, true>), grid, block, 0, st, lat, rl, n_r, acc);
        else
            hipLaunchKernelGGL((k_corr<kBlumeCapel, false>), grid, block, 0, st, lat, rl, n_r, acc);
    }
    return hipGetLastError();
}

hipError_t launch_advance_step(uint32_t *step, uint32_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_advance_step, dim3(1), dim3(64), 0, st, step, n);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, uint64_t n, unsigned long long v, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n)), dim3(kBlock), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_window(const Lattice &lat, uint32_t i0, uint32_t j0, uint32_t rows, uint32_t cols,
                         int8_t *out, hipStream_t st)
{
    const dim3 grid(grid_for((uint64_t)rows * cols)), block(kBlock);
    if (lat.model == kIsing)
        hipLaunchKernelGGL(k_window<kIsing>, grid, block, 0, st, lat, i0, j0, rows, cols, out);
    else
        hipLaunchKernelGGL(k_window<kBlumeCapel>, grid, block, 0, st, lat, i0, j0, rows, cols, out);
    return hipGetLastError();
}

} // namespace spin
