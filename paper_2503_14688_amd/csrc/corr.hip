// Correlation sums S_x(r), S_y(r) (paper Eq. 2, App. C) for the sparse
// separation set r in {1..16} u {round(16 * 2^(k/4)), k = 1..32}, i.e. up to
// r = 4096, on gfx950.
//
// Horizontal (k_corr_x_sparse): a block stages one row segment of both
// colour planes in LDS with a 66-word halo; every separation is a fixed bit
// shift of the partner plane (r even: same colour, m + r/2; r odd: other
// colour, m + (r-1)/2 + ((i + c) & 1)), so with the set known at compile time
// each pair costs one funnel shift, one XOR and one accumulating popcount.
// The two halves of a block take 24 separations each.  When a row is a whole
// number of 1024-word segments, k_corr_x_runs gives each lane a run of 8
// consecutive words (nine LDS reads per separation instead of sixteen).
//
// Vertical (k_corr_y_ring): a block owns a 4-word (Ising) or 2-word
// (Blume-Capel) column strip of both planes and walks down the lattice once,
// keeping the last r_max + 512 rows in an LDS ring; each new row meets its
// 48 partners above it in the ring (four threads per row, twelve
// separations each), so the lattice is read from HBM about once for all
// separations.  The ring stores 16-row blocks plane by plane so that the
// 16-byte LDS loads of neighbouring lanes never share a bank, the four
// separation groups take turns at loading the rows four chunks ahead, and
// one barrier per 256-row chunk suffices.
//
// A batch of lattices is measured by one launch per kernel kind: grid y
// picks the lattice, grid x walks its tiles or strips as in the launch for
// one lattice.
#include "device.hpp"
#include "kernels.hpp"

namespace spin {

namespace {

constexpr int kBlock = 256;
constexpr int kSparseN = 48;

__host__ __device__ constexpr uint32_t sparse_r(int q)
{
    if (q < 16)
        return (uint32_t)q + 1u;
    switch (q) {
    case 16: return 19;   case 17: return 23;   case 18: return 27;   case 19: return 32;
    case 20: return 38;   case 21: return 45;   case 22: return 54;   case 23: return 64;
    case 24: return 76;   case 25: return 91;   case 26: return 108;  case 27: return 128;
    case 28: return 152;  case 29: return 181;  case 30: return 215;  case 31: return 256;
    case 32: return 304;  case 33: return 362;  case 34: return 431;  case 35: return 512;
    case 36: return 609;  case 37: return 724;  case 38: return 861;  case 39: return 1024;
    case 40: return 1218; case 41: return 1448; case 42: return 1722; case 43: return 2048;
    case 44: return 2435; case 45: return 2896; case 46: return 3444; default: return 4096;
    }
}

// ------------------------------------------------------------ horizontal --

constexpr int kTileW = 1024;  // words of a row segment per block iteration
constexpr int kHalo = 66;     // (4096 / 2 + 1) / 32 + 2 words of shifted partners

template <int MODEL>
struct XTile {
    static constexpr int E = MODEL == kIsing ? 1 : 2;  // uint32 per word (S) or (Z, S)
    uint32_t w[2][(kTileW + kHalo) * E];
};

// Separation groups: each half of a block pairs the words of the staged
// segment with 24 of the 48 separations (counters for 24 only, so the kernel
// keeps fewer registers per lane and more wavefronts per CU).
constexpr int kXGroups = 2;
constexpr int kXPer = kSparseN / kXGroups;

// Pairs of one own word (plane C, row parity P) with separations Q0 .. Q0 +
// kXPer - 1.  Every separation of the group is computed (no per-r branch, so
// the LDS reads pipeline); counters past the requested prefix are dropped at
// the end.
template <int MODEL, int C, int P, int Q0, int Q>
__device__ __forceinline__ void x_pairs(const XTile<MODEL> &t, int k, uint32_t oz, uint32_t os,
                                        uint32_t (&ca)[kXPer], uint32_t (&cb)[kXPer])
{
    if constexpr (Q < Q0 + kXPer) {
        {
            constexpr uint32_t r = sparse_r(Q);
            constexpr int tc = C ^ (int)(r & 1u);
            constexpr uint32_t s = (r >> 1) + ((r & 1u) & (uint32_t)P);
            constexpr int qw = (int)(s >> 5);
            constexpr uint32_t rr = s & 31u;
            constexpr int E = XTile<MODEL>::E;
            if constexpr (MODEL == kIsing) {
                const uint32_t x = t.w[tc][k + qw], y = t.w[tc][k + qw + 1];
                const uint32_t b = rr ? __builtin_amdgcn_alignbit(y, x, rr) : x;
                cb[Q - Q0] += __popc(os ^ b);
            } else {
                const uint32_t xz = t.w[tc][(k + qw) * E], yz = t.w[tc][(k + qw + 1) * E];
                const uint32_t xs = t.w[tc][(k + qw) * E + 1], ys = t.w[tc][(k + qw + 1) * E + 1];
                const uint32_t bz = rr ? __builtin_amdgcn_alignbit(yz, xz, rr) : xz;
                const uint32_t bs = rr ? __builtin_amdgcn_alignbit(ys, xs, rr) : xs;
                const uint32_t both = oz & bz;
                ca[Q - Q0] += __popc(both);
                cb[Q - Q0] += __popc(both & (os ^ bs));
            }
        }
        x_pairs<MODEL, C, P, Q0, Q + 1>(t, k, oz, os, ca, cb);
    }
}

// Every word of the staged segment against the group's separations; P0 is
// the row parity of colour 0 (colour 1 has the other).
template <int MODEL, int P0, int Q0>
__device__ __forceinline__ void x_segment(const XTile<MODEL> &t, int tw, uint32_t (&ca)[kXPer],
                                          uint32_t (&cb)[kXPer])
{
    constexpr int E = XTile<MODEL>::E;
#pragma unroll 1
    for (int k = (int)(threadIdx.x % (kBlock / kXGroups)); k < tw; k += kBlock / kXGroups) {
#pragma unroll
        for (int C = 0; C < 2; ++C) {
            const uint32_t oz = MODEL == kIsing ? ~0u : t.w[C][k * E];
            const uint32_t os = t.w[C][k * E + (E - 1)];
            if (C == 0)
                x_pairs<MODEL, 0, P0, Q0, Q0>(t, k, oz, os, ca, cb);
            else
                x_pairs<MODEL, 1, P0 ^ 1, Q0, Q0>(t, k, oz, os, ca, cb);
        }
    }
}

template <int MODEL, int P0>
__device__ __forceinline__ void x_group(int sg, const XTile<MODEL> &t, int tw, uint32_t (&ca)[kXPer],
                                        uint32_t (&cb)[kXPer])
{
    static_assert(kXGroups == 2, "one branch per group");
    if (sg == 0)  // wave-uniform
        x_segment<MODEL, P0, 0>(t, tw, ca, cb);
    else
        x_segment<MODEL, P0, kXPer>(t, tw, ca, cb);
}

// Whole-segment form (rows that are a whole number of kTileW-word segments):
// each lane walks a run of kXRun consecutive own words, so one separation
// costs nine LDS reads for eight pairs instead of two per pair.  The staged
// words of both planes sit side by side (E uint32 per word and plane) with
// one spare uint32 after every 8 words: neighbouring lanes' runs start an
// odd number of uint32 apart (distinct banks), and a run's partners stay
// within the offset range of one LDS instruction.
constexpr int kXRun = 8;

template <int MODEL>
struct XRunTile {
    static constexpr int E = MODEL == kIsing ? 1 : 2;
    __host__ __device__ static constexpr int idx(int e, int plane, int part)
    {
        return (e * 2 + plane) * E + part + (e >> 3);
    }
    uint32_t w[idx(kTileW + kHalo, 0, 0) + 1];
};

// acc + popcount(x) as one v_bcnt_u32_b32, kept in program order (the
// compiler would otherwise re-associate a run's sum into a tree of partial
// counts, all live at once).
__device__ __forceinline__ uint32_t popc_acc(uint32_t x, uint32_t acc)
{
    uint32_t d;
    asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(d) : "v"(x), "v"(acc));
    return d;
}

// One lane's run of kXRun own words (plane C, row parity P, staged from
// index base) against separations Q0 .. Q0 + kXPer - 1.  A separation is a
// shift of s bits in plane tc, so the run's partners are the kXRun + 1 words
// from s / 32 on, funnel-shifted by s % 32.
template <int MODEL, int C, int P, int Q0, int Q>
__device__ __forceinline__ void x_run_pairs(const XRunTile<MODEL> &t, int base, const uint32_t (&oz)[kXRun],
                                            const uint32_t (&os)[kXRun], uint32_t (&ca)[kXPer],
                                            uint32_t (&cb)[kXPer])
{
    if constexpr (Q < Q0 + kXPer) {
        {
            constexpr uint32_t r = sparse_r(Q);
            constexpr int tc = C ^ (int)(r & 1u);
            constexpr uint32_t s = (r >> 1) + ((r & 1u) & (uint32_t)P);
            constexpr int qw = (int)(s >> 5);
            constexpr uint32_t rr = s & 31u;
            constexpr int E = XRunTile<MODEL>::E;
            uint32_t xz[kXRun + 1], xs[kXRun + 1];
#pragma unroll
            for (int m = 0; m <= kXRun; ++m) {
                // the run's first word is a multiple of 8: idx(e0 + c) = base + idx(c)
                xs[m] = t.w[base + XRunTile<MODEL>::idx(qw + m, tc, E - 1)];
                xz[m] = MODEL == kIsing ? ~0u : t.w[base + XRunTile<MODEL>::idx(qw + m, tc, 0)];
            }
            uint32_t na = ca[Q - Q0], nb = cb[Q - Q0];
#pragma unroll
            for (int j = 0; j < kXRun; ++j) {
                const uint32_t bs = rr ? __builtin_amdgcn_alignbit(xs[j + 1], xs[j], rr) : xs[j];
                if constexpr (MODEL == kIsing) {
                    nb = popc_acc(os[j] ^ bs, nb);
                } else {
                    const uint32_t bz = rr ? __builtin_amdgcn_alignbit(xz[j + 1], xz[j], rr) : xz[j];
                    const uint32_t both = oz[j] & bz;
                    na = popc_acc(both, na);
                    nb = popc_acc(both & (os[j] ^ bs), nb);
                }
            }
            ca[Q - Q0] = na;
            cb[Q - Q0] = nb;
        }
        __builtin_amdgcn_sched_barrier(0);  // one separation's partners at a time
        x_run_pairs<MODEL, C, P, Q0, Q + 1>(t, base, oz, os, ca, cb);
    }
}

template <int MODEL, int P0, int Q0>
__device__ __forceinline__ void x_runs(const XRunTile<MODEL> &t, uint32_t (&ca)[kXPer], uint32_t (&cb)[kXPer])
{
    constexpr int E = XRunTile<MODEL>::E;
    const int base = XRunTile<MODEL>::idx((int)(threadIdx.x % (kBlock / kXGroups)) * kXRun, 0, 0);
#pragma unroll
    for (int C = 0; C < 2; ++C) {
        uint32_t oz[kXRun], os[kXRun];
#pragma unroll
        for (int j = 0; j < kXRun; ++j) {
            os[j] = t.w[base + XRunTile<MODEL>::idx(j, C, E - 1)];
            oz[j] = MODEL == kIsing ? ~0u : t.w[base + XRunTile<MODEL>::idx(j, C, 0)];
        }
        if (C == 0)
            x_run_pairs<MODEL, 0, P0, Q0, Q0>(t, base, oz, os, ca, cb);
        else
            x_run_pairs<MODEL, 1, P0 ^ 1, Q0, Q0>(t, base, oz, os, ca, cb);
    }
}

// Block sums of per-group counters: each wavefront adds its group's counters
// (one LDS atomic per counter and wavefront), then one atomic per counter and
// block to HBM.  acc[2q] takes ca, acc[2q + 1] takes cb.
template <bool WITH_A, int PER>
__device__ __forceinline__ void flush_groups(const uint32_t (&ca)[PER], const uint32_t (&cb)[PER], int sg,
                                             int n_r, unsigned long long *acc)
{
    __shared__ unsigned long long part[2][kSparseN];
    __syncthreads();
    for (int q = threadIdx.x; q < 2 * kSparseN; q += blockDim.x)
        part[q / kSparseN][q % kSparseN] = 0;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        unsigned long long a = ca[q], b = cb[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            if (WITH_A)
                a += __shfl_xor(a, off, 64);
            b += __shfl_xor(b, off, 64);
        }
        if ((threadIdx.x & 63) == 0) {
            if (WITH_A)
                atomicAdd(&part[0][sg * PER + q], a);
            atomicAdd(&part[1][sg * PER + q], b);
        }
        __builtin_amdgcn_sched_barrier(0);  // one counter at a time: few live registers
    }
    __syncthreads();
    for (int q = threadIdx.x; q < n_r; q += blockDim.x) {
        if (WITH_A && part[0][q])
            atomicAdd(acc + 2 * q, part[0][q]);
        if (part[1][q])
            atomicAdd(acc + 2 * q + 1, part[1][q]);
    }
}

template <int MODEL>
__device__ __forceinline__ void corr_x_sparse(const Lattice &lat, int n_r, unsigned long long *acc)
{
    __shared__ XTile<MODEL> t;
    constexpr int E = XTile<MODEL>::E;
    const uint32_t L = lat.L, W = lat.W;
    const uint32_t tiles_per_row = (W + kTileW - 1) / kTileW;
    const uint64_t ntiles = (uint64_t)L * tiles_per_row;
    const int sg = (int)(threadIdx.x / (kBlock / kXGroups));  // separation group (wave-uniform)
    uint32_t ca[kXPer], cb[kXPer];
#pragma unroll
    for (int q = 0; q < kXPer; ++q) {
        ca[q] = 0;
        cb[q] = 0;
    }
    for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const uint32_t i = (uint32_t)(tile / tiles_per_row);
        const uint32_t w0 = (uint32_t)(tile - (uint64_t)i * tiles_per_row) * kTileW;
        const int tw = (int)(W - w0 < (uint32_t)kTileW ? W - w0 : (uint32_t)kTileW);
        __syncthreads();
        for (int k = threadIdx.x; k < (tw + kHalo) * E; k += kBlock) {
            const int e = k / E, part = k - e * E;
            uint32_t wk = w0 + (uint32_t)e;
            if (wk >= W)
                wk = W >= kTileW + kHalo ? wk - W : wk % W;
            const size_t off = ((size_t)i * W + wk) * E + part;
            t.w[0][k] = lat.planes[off];
            t.w[1][k] = lat.planes[lat.plane_u32 + off];
        }
        __syncthreads();
        if (i & 1u)
            x_group<MODEL, 1>(sg, t, tw, ca, cb);
        else
            x_group<MODEL, 0>(sg, t, tw, ca, cb);
    }
    flush_groups<MODEL != kIsing, kXPer>(ca, cb, sg, n_r, acc);
}

template <int MODEL>
__device__ __forceinline__ void corr_x_runs(const Lattice &lat, int n_r, unsigned long long *acc)
{
    __shared__ XRunTile<MODEL> t;
    constexpr int E = XRunTile<MODEL>::E;
    static_assert(kXRun * (kBlock / kXGroups) == kTileW, "a group's runs cover the segment");
    const uint32_t L = lat.L, W = lat.W;
    const uint32_t tiles_per_row = W / kTileW;  // W is a multiple of kTileW
    const uint64_t ntiles = (uint64_t)L * tiles_per_row;
    const int sg = (int)(threadIdx.x / (kBlock / kXGroups));  // separation group (wave-uniform)
    uint32_t ca[kXPer], cb[kXPer];
#pragma unroll
    for (int q = 0; q < kXPer; ++q) {
        ca[q] = 0;
        cb[q] = 0;
    }
    for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const uint32_t i = (uint32_t)(tile / tiles_per_row);
        const uint32_t w0 = (uint32_t)(tile - (uint64_t)i * tiles_per_row) * kTileW;
        __syncthreads();
        for (int k = threadIdx.x; k < (kTileW + kHalo) * E; k += kBlock) {
            const int e = k / E, part = k - e * E;
            uint32_t wk = w0 + (uint32_t)e;
            if (wk >= W)
                wk -= W;  // W >= kTileW > kHalo
            const size_t off = ((size_t)i * W + wk) * E + part;
            t.w[XRunTile<MODEL>::idx(e, 0, part)] = lat.planes[off];
            t.w[XRunTile<MODEL>::idx(e, 1, part)] = lat.planes[lat.plane_u32 + off];
        }
        __syncthreads();
        if (i & 1u) {
            if (sg == 0)
                x_runs<MODEL, 1, 0>(t, ca, cb);
            else
                x_runs<MODEL, 1, kXPer>(t, ca, cb);
        } else {
            if (sg == 0)
                x_runs<MODEL, 0, 0>(t, ca, cb);
            else
                x_runs<MODEL, 0, kXPer>(t, ca, cb);
        }
    }
    flush_groups<MODEL != kIsing, kXPer>(ca, cb, sg, n_r, acc);
}

template <int MODEL>
__global__ __launch_bounds__(kBlock) void k_corr_x_sparse(Lattice lat, int n_r, unsigned long long *acc)
{
    corr_x_sparse<MODEL>(lat, n_r, acc);
}

template <int MODEL>
__global__ __launch_bounds__(kBlock) void k_corr_x_runs(Lattice lat, int n_r, unsigned long long *acc)
{
    corr_x_runs<MODEL>(lat, n_r, acc);
}

// The same sums for lattice items[ids[blockIdx.y]] of a batch, one launch
// for all lattices of one kind (its horizontal counters follow its E/M
// counters; blocks past a smaller lattice's tiles find none).
template <int MODEL, bool RUNS>
__global__ __launch_bounds__(kBlock) void k_corr_x_batch(const MeasItem *__restrict__ items,
                                                         const uint32_t *__restrict__ ids, int n_r)
{
    const MeasItem it = wave_uniform_copy(items + __builtin_amdgcn_readfirstlane(ids[blockIdx.y]));
    if (RUNS)
        corr_x_runs<MODEL>(it.lat, n_r, it.acc + kEmCounters);
    else
        corr_x_sparse<MODEL>(it.lat, n_r, it.acc + kEmCounters);
}

// -------------------------------------------------------------- vertical --

// A ring row is 8 uint32 (32 bytes): a 16-byte half of plane 0 (Ising words
// [w0, w0 + 4), Blume-Capel (Z, S) of words [w0, w0 + 2)) and the same half
// of plane 1.  Thread jr of a block owns ring row j0 + jr of every chunk: it
// reads its own row once and, for each separation, the row r above it with
// two 16-byte LDS loads, pairing all 8 words at once.
constexpr int kRingCols = 8;
constexpr int kChunk = kBlock;  // ring rows per chunk, one per thread
static_assert(kChunk % 16 == 0, "chunks start on a 16-row block of the ring");

// Rows are stored in blocks of 16: the plane-0 halves of the block's 16 rows
// (256 bytes), then their plane-1 halves.  Consecutive lanes read consecutive
// rows, so one 16-byte load of 16 neighbouring lanes covers 256 contiguous
// bytes modulo the block boundary: every bank once.  (With whole 32-byte
// rows side by side, lanes 16 bytes apart in bank space would collide two by
// two, which halves the LDS read rate.)  A row's plane-1 half is always 256
// bytes past its plane-0 half: one immediate offset.
constexpr uint32_t kHalfStep = 64;  // uint32 from a row's plane-0 half to its plane-1 half

__host__ __device__ constexpr uint32_t ring_index(uint32_t s)
{
    return (s + (s & ~15u)) * 4u;
}

template <int MODEL>
struct YShape {
    static constexpr int SW = MODEL == kIsing ? 4 : 2;  // words per plane in the strip
};

struct Row8 {
    uint32_t v[8];
};

__device__ __forceinline__ Row8 lds_row(const uint32_t *p)
{
    const uint4 a = *reinterpret_cast<const uint4 *>(p);
    const uint4 b = *reinterpret_cast<const uint4 *>(p + kHalfStep);
    Row8 r;
    r.v[0] = a.x; r.v[1] = a.y; r.v[2] = a.z; r.v[3] = a.w;
    r.v[4] = b.x; r.v[5] = b.y; r.v[6] = b.z; r.v[7] = b.w;
    return r;
}

__device__ __forceinline__ void lds_store_row(uint32_t *p, const uint4 &h0, const uint4 &h1)
{
    *reinterpret_cast<uint4 *>(p) = h0;
    *reinterpret_cast<uint4 *>(p + kHalfStep) = h1;
}

// Separation groups of the vertical kernel: a block has kYGroups threads per
// ring row, each pairing the row with kYPer of the 48 separations, so four
// times as many wavefronts share one LDS ring (the ring, not the thread
// count, limits a CU to one block).
constexpr int kYGroups = 4;
constexpr int kYPer = kSparseN / kYGroups;
constexpr int kYThreads = kChunk * kYGroups;

// Row r above row j0 + jr of the chunk at ring slot slot0.  Its slot is
// base + jr, base = (slot0 - r) mod RING the same for the whole block (rows
// RING .. RING + kChunk - 1 mirror rows 0 .. kChunk - 1, so base + jr needs
// no second wrap).  slot0 and RING are multiples of 16, so base % 16 = bl is
// fixed by r, and ring_index(base + jr) = ring_index(bl + jr) + 8 (base - bl):
// a per-lane part that is the same for every chunk plus a scalar, one vector
// add per pair.
template <uint32_t r>
__device__ __forceinline__ Row8 y_row(const uint32_t *ring, int jr, uint32_t slot0, uint32_t RING)
{
    constexpr uint32_t bl = (16u - (r & 15u)) & 15u;
    uint32_t base = slot0 + RING - (r % RING);
    if (base >= RING)
        base -= RING;
    // the whole scalar part in one scalar register (base >= bl: base % 16 ==
    // bl), so the lane's address is one vector add and both 16-byte halves
    // are reached by non-negative immediate offsets of the LDS loads
    uint32_t sb = (base - bl) * kRingCols;
    asm("" : "+s"(sb));  // keeps the constant part inside the scalar
    return lds_row(ring + ring_index(bl + (uint32_t)jr) + sb);
}

// Counts of one pair, added to the running counters (b: base row j - r,
// x: partner row j; base plane c pairs with partner plane c ^ (r & 1), same
// words): Ising nb += #antiparallel; Blume-Capel na += #both nonzero,
// nb += #both nonzero and opposite.
template <int MODEL, int Q>
__device__ __forceinline__ void y_count(const Row8 &b, const Row8 &x, uint32_t &na, uint32_t &nb)
{
    constexpr uint32_t r = sparse_r(Q);
    constexpr int flip = (r & 1u) ? 4 : 0;  // partner column of base column k: k ^ flip
    if constexpr (MODEL == kIsing) {
#pragma unroll
        for (int k = 0; k < 8; ++k)
            nb = popc_acc(b.v[k] ^ x.v[k ^ flip], nb);
    } else {
#pragma unroll
        for (int k = 0; k < 8; k += 2) {
            const uint32_t both = b.v[k] & x.v[k ^ flip];
            na = popc_acc(both, na);
            nb = popc_acc(both & (b.v[k + 1] ^ x.v[(k ^ flip) + 1]), nb);
        }
    }
}

// Chunks whose pairs are all inside the lattice: the counters themselves
// accumulate.
template <int MODEL, int Q0, int Q>
__device__ __forceinline__ void y_pairs_inner(const uint32_t *ring, int jr, uint32_t slot0, uint32_t RING,
                                              const Row8 &x, uint32_t (&ca)[kYPer], uint32_t (&cb)[kYPer])
{
    if constexpr (Q < Q0 + kYPer) {
        const Row8 b = y_row<sparse_r(Q)>(ring, jr, slot0, RING);
        y_count<MODEL, Q>(b, x, ca[Q - Q0], cb[Q - Q0]);
        y_pairs_inner<MODEL, Q0, Q + 1>(ring, jr, slot0, RING, x, ca, cb);
    }
}

// Chunks at the top and bottom of the walk: a pair counts only when both
// rows are lattice rows (j - r >= 0 and j < L).
template <int MODEL, int Q0, int Q>
__device__ __forceinline__ void y_pairs_edge(const uint32_t *ring, int jr, uint32_t slot0, uint32_t RING,
                                             const Row8 &x, int64_t j, uint32_t L, uint32_t (&ca)[kYPer],
                                             uint32_t (&cb)[kYPer])
{
    if constexpr (Q < Q0 + kYPer) {
        constexpr uint32_t r = sparse_r(Q);
        const Row8 b = y_row<r>(ring, jr, slot0, RING);
        uint32_t na = 0, nb = 0;
        y_count<MODEL, Q>(b, x, na, nb);
        const int64_t i = j - (int64_t)r;
        const bool ok = i >= 0 && i < (int64_t)L;
        ca[Q - Q0] += ok ? na : 0u;
        cb[Q - Q0] += ok ? nb : 0u;
        y_pairs_edge<MODEL, Q0, Q + 1>(ring, jr, slot0, RING, x, j, L, ca, cb);
    }
}

// One separation group's walk over the block's strips (Q0: the group's first
// separation).  Each group has its own copy of the loop, so the per-lane
// address parts of its separations stay in registers for the whole walk.
template <int MODEL, int Q0>
__device__ __forceinline__ void y_walk(const Lattice &lat, int n_r, uint32_t RING, uint32_t *ring, int jr,
                                       uint32_t (&ca)[kYPer], uint32_t (&cb)[kYPer])
{
    constexpr int SW = YShape<MODEL>::SW;
    constexpr int E = MODEL == kIsing ? 1 : 2;
    constexpr int sg = Q0 / kYPer;  // this group
    const uint32_t L = lat.L, W = lat.W;
    const uint32_t strips = W / SW;
    const uint32_t r_max = sparse_r(n_r - 1);
    const int64_t rows_total = (int64_t)L + r_max;  // partner rows j = 0 .. L + r_max - 1
    const int64_t nchunks = (rows_total + kChunk - 1) / kChunk;
    // A strip row is 16 bytes of each plane, an eighth of a 128-byte line.
    // Blocks are dealt round-robin to the eight XCDs (block b on XCD b % 8),
    // so when the strips are a whole number of lines and the grid a multiple
    // of 64, the eight strips of one line go to eight blocks of the same XCD
    // that walk down the lattice together: each line is fetched into that
    // XCD's L2 once and read by all eight.  Otherwise strips are dealt out
    // one by one.
    const bool lines = strips % 8u == 0 && gridDim.x % 64u == 0;
    const uint32_t per_iter = lines ? gridDim.x / 8u : gridDim.x;  // lines, or strips, per pass
    const uint32_t total = lines ? strips / 8u : strips;
    const uint32_t xcd = blockIdx.x % 8u, m = blockIdx.x / 8u;
    const uint32_t first = lines ? xcd * (gridDim.x / 64u) + m / 8u : blockIdx.x;
    // each group loads its chunks four chunks ahead of the chunk being paired
    for (uint32_t unit = first; unit < total; unit += per_iter) {
        const uint32_t strip = lines ? unit * 8u + m % 8u : unit;
        const uint32_t w0 = strip * SW;
        auto load_row = [&](int64_t j, uint4 &p0, uint4 &p1) {
            const uint32_t jg = (uint32_t)(j % (int64_t)L);
            const size_t off = ((size_t)jg * W + w0) * E;  // 16 bytes per plane
            p0 = *reinterpret_cast<const uint4 *>(lat.planes + off);
            p1 = *reinterpret_cast<const uint4 *>(lat.planes + lat.plane_u32 + off);
        };
        // The groups take turns at loading: group g holds chunk ch in registers
        // for ch % kYGroups == g, read kYGroups chunks before it is stored.
        uint4 n0{}, n1{};
        __syncthreads();
        if (sg < nchunks)
            load_row((int64_t)sg * kChunk + jr, n0, n1);
        uint32_t slot0 = 0;  // ring slot of the chunk's first row: j0 mod RING
        int turn = 0;        // ch % kYGroups
        for (int64_t ch = 0; ch < nchunks; ++ch) {
            const int64_t j0 = ch * kChunk;
            const bool loader = turn == sg;  // wave-uniform
            if (loader) {
                lds_store_row(ring + ring_index(slot0 + (uint32_t)jr), n0, n1);
                if (slot0 == 0)
                    lds_store_row(ring + ring_index(RING + (uint32_t)jr), n0, n1);
            }
            __syncthreads();
            if (loader && ch + kYGroups < nchunks)
                load_row(j0 + kYGroups * kChunk + jr, n0, n1);
            turn = turn + 1 == kYGroups ? 0 : turn + 1;
            const Row8 x = lds_row(ring + ring_index(slot0 + (uint32_t)jr));
            // every pair of the chunk is valid when j0 - r >= 0 for the largest r
            // of the set and j0 + kChunk - 1 - r < L for r = 1
            if (j0 >= (int64_t)sparse_r(kSparseN - 1) && j0 + kChunk - 1 < (int64_t)L + 1)
                y_pairs_inner<MODEL, Q0, Q0>(ring, jr, slot0, RING, x, ca, cb);
            else
                y_pairs_edge<MODEL, Q0, Q0>(ring, jr, slot0, RING, x, j0 + jr, L, ca, cb);
            // No barrier here: a wave that finishes early may store the next
            // chunk while others still pair this one.  The next chunk's slots
            // hold rows at least RING - 2 kChunk + 1 > r_max above this
            // chunk's first row (RING >= r_max + 2 kChunk), which no pair of
            // this chunk reads, and this chunk never reads the mirror rows
            // that a store at slot 0 rewrites (it sits at slot RING - kChunk
            // then, and its partner slots do not wrap).
            slot0 += kChunk;
            if (slot0 == RING)
                slot0 = 0;
        }
    }
}

// Ring rows (a multiple of kChunk): room for the r_max rows above a chunk,
// the chunk itself and the next chunk, which an early wave may store while
// the others still pair this one.  With r_max = 4096 the ring and its
// kChunk mirror rows take 152 KiB of LDS.
static uint32_t y_ring_rows(int n_r)
{
    const uint32_t r_max = sparse_r(n_r - 1);
    return (r_max + 2u * kChunk + kChunk - 1u) / kChunk * kChunk;
}

template <int MODEL>
__device__ __forceinline__ void corr_y_ring(const Lattice &lat, int n_r, uint32_t RING, unsigned long long *acc)
{
    extern __shared__ uint32_t ring[];  // (RING + kChunk) rows of kRingCols words
    const int jr = threadIdx.x % kChunk;  // ring row of the chunk
    const int sg = threadIdx.x / kChunk;  // separation group (wave-uniform)
    uint32_t ca[kYPer], cb[kYPer];
#pragma unroll
    for (int q = 0; q < kYPer; ++q) {
        ca[q] = 0;
        cb[q] = 0;
    }
    static_assert(kYGroups == 4, "one case per group");
    switch (sg) {  // every group passes the same barriers the same number of times
    case 0: y_walk<MODEL, 0>(lat, n_r, RING, ring, jr, ca, cb); break;
    case 1: y_walk<MODEL, kYPer>(lat, n_r, RING, ring, jr, ca, cb); break;
    case 2: y_walk<MODEL, 2 * kYPer>(lat, n_r, RING, ring, jr, ca, cb); break;
    default: y_walk<MODEL, 3 * kYPer>(lat, n_r, RING, ring, jr, ca, cb); break;
    }
    flush_groups<MODEL != kIsing, kYPer>(ca, cb, sg, n_r, acc);
}

template <int MODEL>
__global__ __launch_bounds__(kYThreads) void k_corr_y_ring(Lattice lat, int n_r, uint32_t RING,
                                                           unsigned long long *acc)
{
    corr_y_ring<MODEL>(lat, n_r, RING, acc);
}

// The same sums for lattice items[ids[blockIdx.y]] of a batch, one launch
// for all lattices of one model (its vertical counters follow its E/M and
// horizontal counters; blocks past a smaller lattice's strips find none).
template <int MODEL>
__global__ __launch_bounds__(kYThreads) void k_corr_y_batch(const MeasItem *__restrict__ items,
                                                            const uint32_t *__restrict__ ids, int n_r, uint32_t RING)
{
    const MeasItem it = wave_uniform_copy(items + __builtin_amdgcn_readfirstlane(ids[blockIdx.y]));
    corr_y_ring<MODEL>(it.lat, n_r, RING, it.acc + kEmCounters + 2 * n_r);
}

} // namespace

bool sparse_prefix(const uint32_t *r, int n_r)
{
    if (n_r <= 0 || n_r > kSparseN)
        return false;
    for (int q = 0; q < n_r; ++q)
        if (r[q] != sparse_r(q))
            return false;
    return true;
}

bool corr_sparse_x_ok(const Lattice &lat, const uint32_t *r, int n_r)
{
    (void)lat;
    return sparse_prefix(r, n_r);
}

bool corr_sparse_y_ok(const Lattice &lat, const uint32_t *r, int n_r)
{
    const uint32_t sw = lat.model == kIsing ? YShape<kIsing>::SW : YShape<kBlumeCapel>::SW;
    return sparse_prefix(r, n_r) && lat.W % sw == 0;
}

static unsigned corr_grid(uint64_t items, unsigned cap)
{
    uint64_t g = items < cap ? items : cap;
    return (unsigned)(g ? g : 1);
}

int corr_sparse_kind(const Lattice &lat, bool vertical)
{
    const int m = lat.model == kIsing ? 0 : 1;
    if (!vertical)
        return 2 * m + (lat.W % kTileW == 0 ? 1 : 0);
    const uint32_t sw = m == 0 ? YShape<kIsing>::SW : YShape<kBlumeCapel>::SW;
    return lat.W % sw == 0 ? m : -1;
}

uint32_t corr_sparse_blocks(const Lattice &lat, bool vertical)
{
    if (!vertical)
        return corr_grid((uint64_t)lat.L * ((lat.W + kTileW - 1) / kTileW), 2048);
    return corr_grid(lat.W / (lat.model == kIsing ? YShape<kIsing>::SW : YShape<kBlumeCapel>::SW), 256);
}

hipError_t launch_corr_sparse_batch(int kind, bool vertical, const MeasItem *items, const uint32_t *ids, uint32_t n,
                                    uint32_t blocks, int n_r, hipStream_t st)
{
    if (n == 0)
        return hipSuccess;
    if (n > 65535u || blocks == 0 || n_r <= 0 || n_r > kSparseN || kind < 0 || kind > (vertical ? 1 : 3))
        return hipErrorInvalidValue;
    if (!vertical) {
        const dim3 grid(blocks, n), block(kBlock);
        switch (kind) {
        case 0: hipLaunchKernelGGL((k_corr_x_batch<kIsing, false>), grid, block, 0, st, items, ids, n_r); break;
        case 1: hipLaunchKernelGGL((k_corr_x_batch<kIsing, true>), grid, block, 0, st, items, ids, n_r); break;
        case 2: hipLaunchKernelGGL((k_corr_x_batch<kBlumeCapel, false>), grid, block, 0, st, items, ids, n_r); break;
        default: hipLaunchKernelGGL((k_corr_x_batch<kBlumeCapel, true>), grid, block, 0, st, items, ids, n_r); break;
        }
        return hipGetLastError();
    }
    const uint32_t RING = y_ring_rows(n_r);
    const size_t lds = (size_t)(RING + kChunk) * kRingCols * sizeof(uint32_t);
    const dim3 grid(blocks, n), block(kYThreads);
    if (kind == 0) {
        (void)hipFuncSetAttribute((const void *)k_corr_y_batch<kIsing>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds);
        hipLaunchKernelGGL(k_corr_y_batch<kIsing>, grid, block, lds, st, items, ids, n_r, RING);
    } else {
        (void)hipFuncSetAttribute((const void *)k_corr_y_batch<kBlumeCapel>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(k_corr_y_batch<kBlumeCapel>, grid, block, lds, st, items, ids, n_r, RING);
    }
    return hipGetLastError();
}

hipError_t launch_corr_sparse(const Lattice &lat, bool vertical, int n_r, unsigned long long *acc, hipStream_t st)
{
    if (!vertical) {
        const uint64_t tiles = (uint64_t)lat.L * ((lat.W + kTileW - 1) / kTileW);
        const dim3 grid(corr_grid(tiles, 2048)), block(kBlock);
        const bool runs = lat.W % kTileW == 0;
        if (lat.model == kIsing) {
            if (runs)
                hipLaunchKernelGGL(k_corr_x_runs<kIsing>, grid, block, 0, st, lat, n_r, acc);
            else
                hipLaunchKernelGGL(k_corr_x_sparse<kIsing>, grid, block, 0, st, lat, n_r, acc);
        } else {
            if (runs)
                hipLaunchKernelGGL(k_corr_x_runs<kBlumeCapel>, grid, block, 0, st, lat, n_r, acc);
            else
                hipLaunchKernelGGL(k_corr_x_sparse<kBlumeCapel>, grid, block, 0, st, lat, n_r, acc);
        }
        return hipGetLastError();
    }
    const uint32_t RING = y_ring_rows(n_r);
    const size_t lds = (size_t)(RING + kChunk) * kRingCols * sizeof(uint32_t);
    if (lat.model == kIsing) {
        const dim3 grid(corr_grid(lat.W / YShape<kIsing>::SW, 256)), block(kYThreads);
        (void)hipFuncSetAttribute((const void *)k_corr_y_ring<kIsing>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(k_corr_y_ring<kIsing>, grid, block, lds, st, lat, n_r, RING, acc);
    } else {
        const dim3 grid(corr_grid(lat.W / YShape<kBlumeCapel>::SW, 256)), block(kYThreads);
        (void)hipFuncSetAttribute((const void *)k_corr_y_ring<kBlumeCapel>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(k_corr_y_ring<kBlumeCapel>, grid, block, lds, st, lat, n_r, RING, acc);
    }
    return hipGetLastError();
}


} // namespace spin
