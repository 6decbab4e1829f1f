// Internal launch interface of the batched half-sweep (batch_kernels.hip),
// used by the batch API (batch.hip).  Not part of the public ABI.
#pragma once

#include "kernels.hpp"

namespace spin {

// Strategies of the batched kernel: one sweep strategy for the Ising tiles
// and one for the Blume-Capel tiles of the same launch.  0..4 use strategy v
// for both models; 5..8 pair the compacting Ising tile with another
// Blume-Capel one: 5 = (2, 0), 6 = (2, 3), 7 = (1, 3), 8 = (2, 1) as
// (Ising strategy, Blume-Capel strategy).
constexpr int kBatchVariants = 9;
__host__ __device__ constexpr int batch_ising_variant(int bv) { return bv < 5 ? bv : (bv == 7 ? 1 : 2); }
__host__ __device__ constexpr int batch_bc_variant(int bv) { return bv < 5 ? bv : (bv == 5 ? 0 : bv == 8 ? 1 : 3); }

// One replica of a batch: its lattice, its schedule and its first tile in
// the batch's flat tile list.
struct BatchReplica {
    Lattice lat;
    uint32_t sched;
    uint32_t t0;    // sweep index of schedule step 0
    uint64_t tile0;
};

// Models present in a batch: bit 0 Ising, bit 1 Blume-Capel, bit 2
// Blume-Capel with Delta != 0 (13 acceptance groups; set only with bit 1).
// The batched kernel is specialised on it, so a batch without the 13-group
// replicas keeps their thresholds and masks out of its registers.
enum BatchModels : int { kBatchIsing = 1, kBatchBc = 2, kBatchBcGeneral = 4 };
// Batched half-sweep of colour c over a flat tile list of many lattices
// (tile_rep: replica of each tile, laid out by the rows per thread of the
// strategy pair).  The schedule step of a launch is *step_base + step
// (step_base: the batch's device step counter, which launch_advance_step
// moves on by n after a run).
hipError_t launch_batch_half_sweep(int variant, int models, const BatchReplica *reps, const uint32_t *tile_rep,
                                   uint64_t ntiles, const GroupTable *tables, uint32_t stride,
                                   const uint32_t *step_base, uint32_t step, uint32_t colour, hipStream_t st);
hipError_t launch_advance_step(uint32_t *step, uint32_t n, hipStream_t st);

} // namespace spin
