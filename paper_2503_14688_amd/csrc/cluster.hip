// Equilibrium kernels of the Blume-Capel critical-temperature study (paper
// App. B): the Swendsen-Wang cluster step restricted to the sites with
// s = +-1 (for Ising: every site), and the row and column sums of the spin
// field from which the host forms the Fourier moments M(0) and M(k_min).
//
// Swendsen-Wang step at sweep index t (Swendsen and Wang 1987, on the signs
// of the non-zero spins, which with s^2 fixed form an Ising model on the
// bonds between non-zero sites):
//   1. every bond between two equal non-zero spins is active iff its uniform
//      u < thr = floor(2^32 (1 - exp(-2J/T))) (all such bonds when the
//      probability rounds to one); u is word 0 (bond to the right) or word 1
//      (bond below) of Philox4x32-10 at counter (i, j, t, 3 << 16); the two
//      ends of an active bond are merged in a union-find forest whose roots
//      only ever hook onto smaller roots (site index i L + j), so every
//      cluster ends with its smallest site index as root whatever the order
//      of merges: first inside 16 x 64 tiles in LDS, then across tile edges
//      in the global forest with lock-free compare-and-swap;
//   2. each non-zero site flips iff its cluster's root n draws word 0 >= 2^31
//      from Philox4x32-10 at counter (n, 0, t, 4 << 16).
// The result depends only on the stream, never on the schedule of the
// merges, so it is reproducible bit for bit.
#include "kernels.hpp"
#include "device.hpp"

namespace spin {

namespace {

constexpr int kBlock = 256;
constexpr uint32_t kPurposeSwBond = 3u;
constexpr uint32_t kPurposeSwFlip = 4u;

inline unsigned grid_for(uint64_t items)
{
    uint64_t b = (items + kBlock - 1) / kBlock;
    if (b > 65536)
        b = 65536;
    return (unsigned)(b ? b : 1);
}

// Spin at (i, j) from the colour planes: +1, -1, or 0 (Blume-Capel vacancy).
__device__ __forceinline__ int site_spin(const Lattice &lat, uint32_t i, uint32_t j)
{
    const uint32_t c = (i + j) & 1u, m = j >> 1;
    const size_t word = (size_t)i * lat.W + (m >> 5);
    const uint32_t bit = m & 31u;
    const uint32_t *pc = lat.planes + (c ? lat.plane_u32 : 0);
    if (lat.model == kIsing)
        return ((pc[word] >> bit) & 1u) ? -1 : 1;
    const uint32_t z = pc[2 * word], s = pc[2 * word + 1];
    return ((z >> bit) & 1u) ? (((s >> bit) & 1u) ? -1 : 1) : 0;
}

// Parent links are read and written by many workgroups at once (on every
// XCD), so they go through device-coherent relaxed atomics.
__device__ __forceinline__ uint32_t load_parent(const uint32_t *P, uint32_t x)
{
    return __hip_atomic_load(P + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x with path halving: each visited node is pointed at its
// grandparent, which is also an ancestor with a smaller index, so any
// interleaving of these stores keeps the forest valid.
__device__ uint32_t find_root(uint32_t *P, uint32_t x)
{
    uint32_t p = load_parent(P, x);
    while (p != x) {
        const uint32_t g = load_parent(P, p);
        if (g != p)
            __hip_atomic_store(P + x, g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        x = p;
        p = g;
    }
    return x;
}

// Merge the trees of a and b: the larger root is hooked onto the smaller one
// by compare-and-swap, retried from the new roots when another merge got
// there first.  Parents always have smaller indices than their children, so
// every walk ends.
__device__ void unite(uint32_t *P, uint32_t a, uint32_t b)
{
    a = find_root(P, a);
    b = find_root(P, b);
    while (a != b) {
        if (a < b) {
            const uint32_t x = a;
            a = b;
            b = x;
        }
        uint32_t expected = a;
        if (__hip_atomic_compare_exchange_strong(P + a, &expected, b, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT))
            return;
        a = find_root(P, expected);
        b = find_root(P, b);
    }
}

// Tiled linking: a block first merges the bonds inside its 16 x 64 tile in an
// LDS forest (the same hooking rule on tile-local indices, whose order is the
// global order within the tile), then writes every site's parent as the
// global index of its tile-local root; a second kernel merges the bonds that
// cross tile edges in the global forest.  Only about one bond in sixteen then
// touches global atomics.
constexpr uint32_t kTileRows = 16, kTileCols = 64, kTileSites = kTileRows * kTileCols;

__device__ uint32_t lds_find(uint32_t *lab, uint32_t x)
{
    uint32_t p = __hip_atomic_load(lab + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    while (p != x) {
        const uint32_t g = __hip_atomic_load(lab + p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (g != p)
            __hip_atomic_store(lab + x, g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        x = p;
        p = g;
    }
    return x;
}

__device__ void lds_unite(uint32_t *lab, uint32_t a, uint32_t b)
{
    a = lds_find(lab, a);
    b = lds_find(lab, b);
    while (a != b) {
        if (a < b) {
            const uint32_t x = a;
            a = b;
            b = x;
        }
        uint32_t expected = a;
        if (__hip_atomic_compare_exchange_strong(lab + a, &expected, b, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_WORKGROUP))
            return;
        a = lds_find(lab, expected);
        b = lds_find(lab, b);
    }
}

// Whether the bond from (i, j) to its right (dir 0) or lower (dir 1)
// neighbour is active, given both spins.
__device__ __forceinline__ bool bond_active(const Lattice &lat, uint32_t i, uint32_t j, uint32_t t, int dir, int s,
                                            int s_nb, uint32_t thr, uint32_t always)
{
    if (s == 0 || s != s_nb)
        return false;
    if (always)
        return true;
    const Block4 u = philox4x32_10(i, j, t, kPurposeSwBond << 16, lat.key0, lat.key1);
    return (dir == 0 ? u.v[0] : u.v[1]) < thr;
}

__global__ __launch_bounds__(kBlock) void k_sw_link_tiles(Lattice lat, uint32_t t, uint32_t thr, uint32_t always,
                                                          uint32_t *P)
{
    __shared__ uint32_t lab[kTileSites];
    __shared__ int8_t spin[kTileSites];
    const uint32_t L = lat.L;
    const uint32_t tiles_x = L / kTileCols;
    const uint64_t ntiles = (uint64_t)(L / kTileRows) * tiles_x;
    for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const uint32_t i0 = (uint32_t)(tile / tiles_x) * kTileRows;
        const uint32_t j0 = (uint32_t)(tile % tiles_x) * kTileCols;
        __syncthreads();  // the previous tile is done with lab and spin
        for (uint32_t q = threadIdx.x; q < kTileSites; q += kBlock) {
            lab[q] = q;
            spin[q] = (int8_t)site_spin(lat, i0 + q / kTileCols, j0 + q % kTileCols);
        }
        __syncthreads();
        for (uint32_t q = threadIdx.x; q < kTileSites; q += kBlock) {
            const uint32_t li = q / kTileCols, lj = q % kTileCols;
            const int s = spin[q];
            if (s == 0)
                continue;
            const bool in_r = lj + 1 < kTileCols, in_d = li + 1 < kTileRows;
            const bool need_r = in_r && spin[q + 1] == s, need_d = in_d && spin[q + kTileCols] == s;
            if (!need_r && !need_d)
                continue;
            bool act_r = need_r, act_d = need_d;
            if (!always) {
                const Block4 u = philox4x32_10(i0 + li, j0 + lj, t, kPurposeSwBond << 16, lat.key0, lat.key1);
                act_r = need_r && u.v[0] < thr;
                act_d = need_d && u.v[1] < thr;
            }
            if (act_r)
                lds_unite(lab, q, q + 1);
            if (act_d)
                lds_unite(lab, q, q + kTileCols);
        }
        __syncthreads();
        for (uint32_t q = threadIdx.x; q < kTileSites; q += kBlock) {
            const uint32_t r = lds_find(lab, q);
            const uint32_t gi = i0 + q / kTileCols, gj = j0 + q % kTileCols;
            P[(size_t)gi * L + gj] = (i0 + r / kTileCols) * L + (j0 + r % kTileCols);
        }
    }
}

// The bonds that leave a tile: from its last column to the right and from its
// last row downwards (periodic), one thread per such site.
__global__ __launch_bounds__(kBlock) void k_sw_link_edges(Lattice lat, uint32_t t, uint32_t thr, uint32_t always,
                                                          uint32_t *P)
{
    const uint32_t L = lat.L;
    const uint32_t tiles_x = L / kTileCols;
    const uint64_t ntiles = (uint64_t)(L / kTileRows) * tiles_x;
    constexpr uint32_t per_tile = kTileRows + kTileCols;  // last column, then last row
    const uint64_t n = ntiles * per_tile;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n; g += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t tile = g / per_tile;
        const uint32_t k = (uint32_t)(g - tile * per_tile);
        const uint32_t i0 = (uint32_t)(tile / tiles_x) * kTileRows;
        const uint32_t j0 = (uint32_t)(tile % tiles_x) * kTileCols;
        const int dir = k < kTileRows ? 0 : 1;
        const uint32_t i = dir == 0 ? i0 + k : i0 + kTileRows - 1;
        const uint32_t j = dir == 0 ? j0 + kTileCols - 1 : j0 + (k - kTileRows);
        const uint32_t in = dir == 0 ? i : (i + 1 == L ? 0u : i + 1);
        const uint32_t jn = dir == 0 ? (j + 1 == L ? 0u : j + 1) : j;
        const int s = site_spin(lat, i, j);
        if (bond_active(lat, i, j, t, dir, s, site_spin(lat, in, jn), thr, always))
            unite(P, i * L + j, in * L + jn);
    }
}

// One thread per lattice word: flip the non-zero sites whose cluster root
// draws a flip.  Every merge has finished, so the roots are plain reads.
__global__ __launch_bounds__(kBlock) void k_sw_flip(Lattice lat, uint32_t t, const uint32_t *P)
{
    const uint32_t L = lat.L, W = lat.W, half = L / 2;
    const uint64_t words = 2ull * L * W;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < words;
         g += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t c = (uint32_t)(g / ((uint64_t)L * W));
        const uint64_t rest = g - (uint64_t)c * L * W;
        const uint32_t i = (uint32_t)(rest / W), w = (uint32_t)(rest - (uint64_t)i * W);
        uint32_t *pc = lat.planes + (c ? lat.plane_u32 : 0);
        const size_t word = (size_t)i * W + w;
        const uint32_t z = lat.model == kIsing ? 0xFFFFFFFFu : pc[2 * word];
        uint32_t flip = 0;
        for (uint32_t b = 0; b < 32; ++b) {
            const uint32_t m = 32 * w + b;
            if (m >= half || !((z >> b) & 1u))
                continue;
            const uint32_t j = 2 * m + ((i + c) & 1u);
            uint32_t x = i * L + j, p = P[x];
            while (p != x) {
                x = p;
                p = P[x];
            }
            const Block4 r = philox4x32_10(x, 0u, t, kPurposeSwFlip << 16, lat.key0, lat.key1);
            flip |= (r.v[0] >> 31) << b;
        }
        if (lat.model == kIsing)
            pc[word] ^= flip;
        else
            pc[2 * word + 1] ^= flip;
    }
}

// Row sums: one wavefront per row, both colour planes.  |sum| <= L < 2^31,
// so the wavefront reduction runs on 32-bit integers.
__global__ __launch_bounds__(kBlock) void k_row_sums(Lattice lat, long long *row)
{
    const uint32_t L = lat.L, W = lat.W;
    const uint32_t lane = threadIdx.x & 63u;
    for (uint32_t i = blockIdx.x * (kBlock / 64) + threadIdx.x / 64; i < L; i += gridDim.x * (kBlock / 64)) {
        int acc = 0;
        for (uint32_t q = lane; q < 2 * W; q += 64) {
            const uint32_t c = q >= W, w = q - c * W;
            const uint32_t *pc = lat.planes + (c ? lat.plane_u32 : 0);
            const size_t word = (size_t)i * W + w;
            if (lat.model == kIsing)
                acc += 32 - 2 * __popc(pc[word]);
            else
                acc += __popc(pc[2 * word]) - 2 * __popc(pc[2 * word + 1]);
        }
        for (int off = 32; off > 0; off >>= 1)
            acc += __shfl_xor(acc, off, 64);
        if (lane == 0)
            row[i] = (long long)acc;
    }
}

// Column sums: one thread per (column, block of rows), accumulated with
// 64-bit atomics into col (zeroed beforehand).
__global__ __launch_bounds__(kBlock) void k_col_sums(Lattice lat, uint32_t rows_per, long long *col)
{
    const uint32_t L = lat.L;
    const uint32_t j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= L)
        return;
    const uint32_t i0 = blockIdx.y * rows_per;
    const uint32_t i1 = i0 + rows_per < L ? i0 + rows_per : L;
    long long acc = 0;
    for (uint32_t i = i0; i < i1; ++i)
        acc += site_spin(lat, i, j);
    atomicAdd((unsigned long long *)(col + j), (unsigned long long)acc);
}

} // namespace

hipError_t launch_sw_step(const Lattice &lat, uint32_t t, uint32_t thr, bool always, uint32_t *labels,
                          hipStream_t st)
{
    const uint64_t ntiles = (uint64_t)(lat.L / kTileRows) * (lat.L / kTileCols);
    const unsigned gt = (unsigned)(ntiles < 65536 ? ntiles : 65536);
    hipLaunchKernelGGL(k_sw_link_tiles, dim3(gt), dim3(kBlock), 0, st, lat, t, thr, always ? 1u : 0u, labels);
    hipLaunchKernelGGL(k_sw_link_edges, dim3(grid_for(ntiles * (kTileRows + kTileCols))), dim3(kBlock), 0, st, lat,
                       t, thr, always ? 1u : 0u, labels);
    hipLaunchKernelGGL(k_sw_flip, dim3(grid_for(2ull * lat.L * lat.W)), dim3(kBlock), 0, st, lat, t,
                       (const uint32_t *)labels);
    return hipGetLastError();
}

hipError_t launch_line_sums(const Lattice &lat, long long *row, long long *col, hipStream_t st)
{
    hipLaunchKernelGGL(k_row_sums, dim3(grid_for((uint64_t)lat.L * 64)), dim3(kBlock), 0, st, lat, row);
    const uint32_t rows_per = 64;
    const dim3 grid((lat.L + kBlock - 1) / kBlock, (lat.L + rows_per - 1) / rows_per);
    hipLaunchKernelGGL(k_col_sums, grid, dim3(kBlock), 0, st, lat, rows_per, col);
    return hipGetLastError();
}

} // namespace spin
