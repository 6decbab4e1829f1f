// Equilibrium kernels of the Blume-Capel critical-temperature study (paper
// App. B): the Swendsen-Wang cluster step restricted to the sites with
// s = +-1 (for Ising: every site), and the row and column sums of the spin
// field from which the host forms the Fourier moments M(0) and M(k_min).
//
// Swendsen-Wang step at sweep index t (Swendsen and Wang 1987, on the signs
// of the non-zero spins, which with s^2 fixed form an Ising model on the
// bonds between non-zero sites):
//   1. every site starts as its own cluster (label = linear index i L + j);
//   2. every bond between two equal non-zero spins is active iff its uniform
//      u < thr = floor(2^32 (1 - exp(-2J/T))) (all such bonds when the
//      probability rounds to one); u is word 0 (bond to the right) or word 1
//      (bond below) of Philox4x32-10 at counter (i, j, t, 3 << 16); the two
//      ends of an active bond are merged in a lock-free union-find forest
//      whose roots only ever hook onto smaller roots, so every cluster ends
//      with its smallest site index as root whatever the order of merges;
//   3. each non-zero site flips iff its cluster's root n draws word 0 >= 2^31
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

__global__ __launch_bounds__(kBlock) void k_sw_init(uint32_t *P, uint64_t n)
{
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n; g += (uint64_t)gridDim.x * blockDim.x)
        P[g] = (uint32_t)g;
}

// One thread per site: its bonds to the right and below.
__global__ __launch_bounds__(kBlock) void k_sw_link(Lattice lat, uint32_t t, uint32_t thr, uint32_t always,
                                                    uint32_t *P)
{
    const uint32_t L = lat.L;
    const uint64_t n = (uint64_t)L * L;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n; g += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t i = (uint32_t)(g / L), j = (uint32_t)(g - (uint64_t)i * L);
        const int s = site_spin(lat, i, j);
        if (s == 0)
            continue;
        const uint32_t jr = j + 1 == L ? 0u : j + 1, id = i + 1 == L ? 0u : i + 1;
        const Block4 u = philox4x32_10(i, j, t, kPurposeSwBond << 16, lat.key0, lat.key1);
        if (site_spin(lat, i, jr) == s && (always || u.v[0] < thr))
            unite(P, (uint32_t)g, i * L + jr);
        if (site_spin(lat, id, j) == s && (always || u.v[1] < thr))
            unite(P, (uint32_t)g, id * L + j);
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
    const uint64_t n = (uint64_t)lat.L * lat.L;
    hipLaunchKernelGGL(k_sw_init, dim3(grid_for(n)), dim3(kBlock), 0, st, labels, n);
    hipLaunchKernelGGL(k_sw_link, dim3(grid_for(n)), dim3(kBlock), 0, st, lat, t, thr, always ? 1u : 0u, labels);
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
