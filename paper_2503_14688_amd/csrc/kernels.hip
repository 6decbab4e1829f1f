// gfx950 kernels: initial state, checkerboard half-sweeps of one lattice
// (Ising 1 bit per spin, Blume-Capel 2 bit planes; the tile functions are in
// sweep_tiles.hpp), the energy/magnetisation reduction, the generic axis
// correlation sums C(r), and the window decoder.
#include "sweep_tiles.hpp"

namespace spin {

namespace {

inline unsigned grid_for(uint64_t items)
{
    uint64_t b = (items + kBlock - 1) / kBlock;
    if (b > 65536)
        b = 65536;
    if (b == 0)
        b = 1;
    return (unsigned)b;
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

// Occupancy target of a sweep kernel: the row-uniform tiles without the
// fused measurement are compiled for eight wavefronts per SIMD (they fit in
// 64 vector registers without spills, and the tighter schedule measured 1%
// (Ising) and 3% (Blume-Capel, compacting) faster); the others keep the
// compiler's own target (at eight wavefronts they would spill).
template <bool MEASURE, bool UNIFORM>
constexpr int sweep_waves()
{
    return !MEASURE && UNIFORM ? 8 : 1;
}

// One kernel per tile form: row-uniform or not (rows a multiple of 64
// words), select-free classification or not, so that each keeps only its
// own path's values in registers.
template <bool MEASURE, int V, bool UNIFORM, bool PLAIN>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(sweep_waves<MEASURE, UNIFORM>()))) void k_sweep_ising(Lattice lat, uint32_t c, uint32_t t, GroupTable gt,
                                                        unsigned long long *acc)
{
    constexpr int R = variant_rows(V);
    unsigned long long e[kEmCounters] = {0, 0, 0, 0};
    const uint64_t ntiles = tiles_of<R>(lat);
    if constexpr (variant_compact(V)) {
        using QL = WaveList<variant_list_cap(V)>;
        __shared__ QL Q[kWaves];
        for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x)
            ising_tile_compact<MEASURE, R, UNIFORM, QL, PLAIN>(lat, c, t, gt, tile, Q[threadIdx.x >> 6], e);
    } else {
        for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x)
            ising_tile_lazy<MEASURE, R, UNIFORM>(lat, c, t, gt, tile, e);
    }
    if (MEASURE)
        block_reduce_atomic<kEmCounters>(e, acc);
}

// One kernel per group count and classification form, so that each keeps
// only its own thresholds and masks in registers (one kernel with both group
// counts spills scalar registers in the loops of either).
template <bool MEASURE, int V, int NG, bool PLAIN, bool UNIFORM = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(sweep_waves<MEASURE, UNIFORM>()))) void k_sweep_bc(Lattice lat, uint32_t c, uint32_t t, GroupTable gt,
                                                     unsigned long long *acc)
{
    constexpr int R = variant_rows(V);
    unsigned long long e[kEmCounters] = {0, 0, 0, 0};
    const uint64_t ntiles = tiles_of<R>(lat);
    if constexpr (variant_compact(V)) {
        using QB = BcList<NG, bc_list_cap(V), R>;
        __shared__ QB Q[kWaves];
        for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x)
            bc_tile_compact<MEASURE, R, NG, QB, PLAIN, UNIFORM>(lat, c, t, gt, gt.plane_groups, tile,
                                                                Q[threadIdx.x >> 6], e);
    } else {
        for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x)
            bc_tile<MEASURE, R, NG, PLAIN, UNIFORM>(lat, c, t, gt, gt.plane_groups, tile, e);
    }
    if (MEASURE)
        block_reduce_atomic<kEmCounters>(e, acc);
}

// ------------------------------------------ energy / magnetisation sums --

template <int MODEL>
__device__ __forceinline__ void measure_em(const Lattice &lat, unsigned long long *acc)
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

template <int MODEL>
__global__ __launch_bounds__(kBlock) void k_measure_em(Lattice lat, unsigned long long *acc)
{
    measure_em<MODEL>(lat, acc);
}

// The same for lattice ids[blockIdx.y] of a batch.
template <int MODEL>
__global__ __launch_bounds__(kBlock) void k_measure_em_batch(const MeasItem *__restrict__ items,
                                                             const uint32_t *__restrict__ ids)
{
    const MeasItem it = wave_uniform_copy(items + __builtin_amdgcn_readfirstlane(ids[blockIdx.y]));
    measure_em<MODEL>(it.lat, it.acc);
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
        const dim3 grid(g < tiles ? g : (unsigned)tiles);
        const bool uniform = lat.W % 64 == 0;
        // the select-free classification matters for the compacting tiles only
        const bool plain = variant_compact(V) && (gt.rng_bits & 3u) == 3u && (gt.never_bits & 3u) == 0u;
        if (uniform && plain)
            hipLaunchKernelGGL((k_sweep_ising<M, V, true, variant_compact(V)>), grid, block, 0, st, lat, colour, t, gt,
                               em_acc);
        else if (uniform)
            hipLaunchKernelGGL((k_sweep_ising<M, V, true, false>), grid, block, 0, st, lat, colour, t, gt, em_acc);
        else if (plain)
            hipLaunchKernelGGL((k_sweep_ising<M, V, false, variant_compact(V)>), grid, block, 0, st, lat, colour, t,
                               gt, em_acc);
        else
            hipLaunchKernelGGL((k_sweep_ising<M, V, false, false>), grid, block, 0, st, lat, colour, t, gt, em_acc);
    } else {
        static const unsigned g = 65536u;
        const dim3 grid(g < tiles ? g : (unsigned)tiles);
        if (lat.bc_groups == kBcGroupsDelta0 && bc_plain<kBcGroupsDelta0>(gt) && lat.W % 64 == 0)
            hipLaunchKernelGGL((k_sweep_bc<M, V, kBcGroupsDelta0, true, true>), grid, block, 0, st, lat, colour, t,
                               gt, em_acc);
        else if (lat.bc_groups == kBcGroupsDelta0 && bc_plain<kBcGroupsDelta0>(gt))
            hipLaunchKernelGGL((k_sweep_bc<M, V, kBcGroupsDelta0, true>), grid, block, 0, st, lat, colour, t, gt, em_acc);
        else if (lat.bc_groups == kBcGroupsDelta0)
            hipLaunchKernelGGL((k_sweep_bc<M, V, kBcGroupsDelta0, false>), grid, block, 0, st, lat, colour, t, gt,
                               em_acc);
        else
            hipLaunchKernelGGL((k_sweep_bc<M, V, kBcGroups, false>), grid, block, 0, st, lat, colour, t, gt, em_acc);
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

uint32_t measure_em_blocks(const Lattice &lat) { return grid_for((uint64_t)lat.L * lat.W); }

hipError_t launch_measure_em_batch(int model, const MeasItem *items, const uint32_t *ids, uint32_t n,
                                   uint32_t blocks, hipStream_t st)
{
    if (n == 0)
        return hipSuccess;
    if (n > 65535u || blocks == 0)
        return hipErrorInvalidValue;
    const dim3 grid(blocks, n), block(kBlock);
    if (model == kIsing)
        hipLaunchKernelGGL(k_measure_em_batch<kIsing>, grid, block, 0, st, items, ids);
    else
        hipLaunchKernelGGL(k_measure_em_batch<kBlumeCapel>, grid, block, 0, st, items, ids);
    return hipGetLastError();
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
