// Internal launch interface between the C ABI (spin.hip and the other host
// sources) and the gfx950 kernels (kernels.hip, corr.hip, cluster.hip; the
// batched kernel's interface is batch_kernels.hpp).  Not part of the public
// ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spin {

enum Model : int { kIsing = 0, kBlumeCapel = 1 };

// Acceptance groups: Ising uses 2 (dE = 4J, 8J); Blume-Capel uses 13 --
// nine for the pair {s -> 0, 0 -> s'} at y = -4..4 (exactly one of the two
// families can have dE > 0 for a given y) and four for s -> -s at y = 1..4.
constexpr int kIsingGroups = 2;
constexpr int kBcGroups = 13;
// Blume-Capel with Delta = 0: the positive energy changes are J {1,2,3,4,6,8},
// so the 13 groups merge into 6 (see bc_tile).
constexpr int kBcGroupsDelta0 = 6;
constexpr int kMaxGroups = 16;

struct GroupTable {
    uint32_t thr[kMaxGroups];   // integer threshold of the group
    uint32_t rng_bits;          // bit g: group g needs a random number
    uint32_t never_bits;        // bit g: group g is never accepted (T = 0)
    uint32_t sel_a_bits;        // Blume-Capel: bit v (y = v - 4): the group's
                                // positive family is s -> 0 (else 0 -> s')
    // Threshold bits of groups 0..7 plane by plane: byte q of word b has bit
    // g set when bit 31 - (4 b + q) of thr[g] is set (the groups whose
    // threshold bit is 1 in plane 4 b + q).  Used by the six-group test.
    uint32_t plane_groups[8];
};

struct Lattice {
    uint32_t *planes;  // colour plane 0, then colour plane 1
    uint32_t L;        // linear size
    uint32_t W;        // 32-bit words per plane row (L / 64)
    uint64_t plane_u32;// uint32 words per colour plane (L * W, doubled for BC)
    int model;
    uint32_t key0, key1;
    uint32_t bc_groups;  // Blume-Capel acceptance groups in use: 13, or 6 when Delta = 0
    int variant;         // sweep strategy, see variant_rows / variant_compact
};

// Sweep strategies: rows walked per thread (4 or 8) and whether words still
// undecided after eight planes go to the wavefront's LDS work list
// (ising_tile_compact, bc_tile_compact) or each thread finishes its word's
// lazy test itself (ising_tile_lazy, bc_tile).
//   0: 8 rows, per word   1: 4 rows, compacting   2: 8 rows, compacting   3: 4 rows, per word
//   4: 8 rows, compacting with a 16-slot list (most undecided words finish in
//      place; the same results, slower)
constexpr int kVariants = 5;
__host__ __device__ constexpr int variant_rows(int v) { return (v == 1 || v == 3) ? 4 : 8; }
__host__ __device__ constexpr bool variant_compact(int v) { return v == 1 || v == 2 || v == 4; }
__host__ __device__ constexpr int variant_list_cap(int v) { return v == 4 ? 16 : 128; }

// Counters of the energy/magnetisation reduction (both colours):
//   acc[0] = #(s != 0)  acc[1] = #(s < 0)
//   acc[2] = #bonds with both ends non-zero, acc[3] = #such bonds anti-aligned
// so sum s = acc0 - 2 acc1, sum s^2 = acc0, bond sum = acc2 - 2 acc3.
constexpr int kEmCounters = 4;

hipError_t launch_init(const Lattice &lat, hipStream_t st);
// Sweep work units (tiles of 256 word columns x rows) of one lattice for a
// rows-per-thread choice (4 or 8).
uint64_t sweep_tiles(const Lattice &lat, int rows);
hipError_t launch_half_sweep(const Lattice &lat, uint32_t colour, uint32_t t, const GroupTable &gt,
                             unsigned long long *em_acc, hipStream_t st);
hipError_t launch_measure_em(const Lattice &lat, unsigned long long *em_acc, hipStream_t st);
// Correlation counters for n_r (<= 8) separations: acc[2q] = #pairs with both
// ends non-zero, acc[2q + 1] = #such pairs anti-aligned; S(r) = a - 2 b.
constexpr int kCorrChunk = 8;
hipError_t launch_corr(const Lattice &lat, bool vertical, const uint32_t *r, int n_r,
                       unsigned long long *acc, hipStream_t st);
// Sparse separation set r in {1..16} u {round(16 * 2^(k/4)), k = 1..32}: the
// fast kernels take any prefix of it (counters laid out as launch_corr's).
bool sparse_prefix(const uint32_t *r, int n_r);
bool corr_sparse_x_ok(const Lattice &lat, const uint32_t *r, int n_r);
bool corr_sparse_y_ok(const Lattice &lat, const uint32_t *r, int n_r);
hipError_t launch_corr_sparse(const Lattice &lat, bool vertical, int n_r, unsigned long long *acc,
                              hipStream_t st);
hipError_t launch_fill_u64(unsigned long long *p, uint64_t n, unsigned long long v, hipStream_t st);

// Batched measurement: the E/M reduction and the sparse-set correlation
// kernels of many lattices of one model in one launch each.  Lattice k of a
// launch is items[ids[k]]; its counters start at items[.].acc and are laid
// out as for one lattice: kEmCounters E/M counters, then 2 n_r horizontal,
// then 2 n_r vertical.  Grid: x walks one lattice's units (blocks past a
// smaller lattice's units do nothing), y runs over the lattices.
struct MeasItem {
    Lattice lat;
    unsigned long long *acc;
};
// Blocks that the single-lattice launch would use for this lattice.
uint32_t measure_em_blocks(const Lattice &lat);
hipError_t launch_measure_em_batch(int model, const MeasItem *items, const uint32_t *ids, uint32_t n,
                                   uint32_t blocks, hipStream_t st);
// Kind of the sparse-set kernel for one axis of a lattice (lattices of one
// kind share a launch), and its blocks as in the single-lattice launch.
int corr_sparse_kind(const Lattice &lat, bool vertical);
uint32_t corr_sparse_blocks(const Lattice &lat, bool vertical);
hipError_t launch_corr_sparse_batch(int kind, bool vertical, const MeasItem *items, const uint32_t *ids, uint32_t n,
                                    uint32_t blocks, int n_r, hipStream_t st);
// Equilibrium study (paper App. B): one Swendsen-Wang step at sweep index t
// with the integer bond rule (thr, always), labels = L * L uint32 scratch;
// and the row / column sums of the spin field (row[L], col[L]; col zeroed by
// the caller).
hipError_t launch_sw_step(const Lattice &lat, uint32_t t, uint32_t thr, bool always, uint32_t *labels,
                          hipStream_t st);
hipError_t launch_line_sums(const Lattice &lat, long long *row, long long *col, hipStream_t st);
hipError_t launch_window(const Lattice &lat, uint32_t i0, uint32_t j0, uint32_t rows, uint32_t cols,
                         int8_t *out, hipStream_t st);

} // namespace spin
