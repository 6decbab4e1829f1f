// gfx950 batched half-sweep: one launch advances one colour of every
// replica of a batch through the sweep tile functions of sweep_tiles.hpp,
// with one sweep strategy for the Ising tiles and one for the Blume-Capel
// tiles; and the device step counter that lets a captured run replay.
#include "batch_kernels.hpp"
#include "sweep_tiles.hpp"

namespace spin {

namespace {

// LDS of the batched kernel, per wavefront: only the lists of the models the
// batch holds and of the strategies it runs them with (an Ising-only batch
// keeps the Ising kernel's smaller LDS, so as many blocks fit on a CU as in
// the single-lattice launch; a per-word strategy needs no list).
template <int BV, int MODELS>
union BatchList {
    static constexpr int VI = batch_ising_variant(BV), VB = batch_bc_variant(BV);
    static constexpr bool kIsingList = (MODELS & kBatchIsing) != 0 && variant_compact(VI);
    static constexpr bool kBcList = (MODELS & kBatchBc) != 0 && variant_compact(VB);
    static constexpr bool kGenList = (MODELS & kBatchBcGeneral) != 0 && variant_compact(VB);
    std::conditional_t<kIsingList, WaveList<variant_list_cap(VI)>, char> ising;
    std::conditional_t<kBcList, BcList<kBcGroupsDelta0, bc_list_cap(VB), variant_rows(VB)>, char> d0;
    std::conditional_t<kGenList, BcList<kBcGroups, bc_list_cap(VB), variant_rows(VB)>, char> gen;
};

// Occupancy target: batches of one model (ensembles, protocol-2 batches)
// are compiled for eight wavefronts per SIMD, where it measured 4-6% faster
// with no register spills; the both-model kernel of the mix would spill at
// eight and takes seven (72 registers instead of 73, no spills, 1.3% faster
// on the 512-replica mix); batches with the 13-group Blume-Capel path keep
// the compiler's own target.
template <int MODELS>
constexpr int batch_waves()
{
    if constexpr (MODELS == kBatchIsing || MODELS == kBatchBc)
        return 8;
    else if constexpr (MODELS == (kBatchIsing | kBatchBc))
        return 7;
    else
        return 1;
}

// Batched half-sweep: one launch advances colour c of every replica.  The
// flat tile list maps each global tile to (replica, local tile); replica r's
// thresholds for this sweep are tables[sched(r) * stride + step] and its
// random stream runs at sweep index t0(r) + step.
template <int BV, int MODELS>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(batch_waves<MODELS>()))) void k_batch_half_sweep(
    const BatchReplica *__restrict__ reps, const uint32_t *__restrict__ tile_rep, uint64_t ntiles,
    const GroupTable *__restrict__ tables, uint32_t stride, const uint32_t *__restrict__ step_base, uint32_t step_off,
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
        const GroupTable *gtp = tables + (size_t)rep.sched * stride + step;
        const GroupTable gt = wave_uniform_copy(gtp);
        const uint32_t *pats = gtp->plane_groups;
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
                    else if (plain)
                        ising_tile_compact<false, RI, false, QL, true>(rep.lat, c, t, gt, local,
                                                                       Q[threadIdx.x >> 6].ising, e);
                    else
                        ising_tile_compact<false, RI, false>(rep.lat, c, t, gt, local, Q[threadIdx.x >> 6].ising, e);
                } else if (rep.lat.W % 64 == 0) {
                    ising_tile_lazy<false, RI, true>(rep.lat, c, t, gt, local, e);
                } else {
                    ising_tile_lazy<false, RI, false>(rep.lat, c, t, gt, local, e);
                }
            }
        } else if constexpr ((MODELS & kBatchBc) != 0) {
            const bool delta0 = (MODELS & kBatchBcGeneral) == 0 || rep.lat.bc_groups == kBcGroupsDelta0;
            if constexpr (variant_compact(VB)) {
                using QD = decltype(Q[0].d0);
                if (delta0 && bc_plain<kBcGroupsDelta0>(gt)) {
                    bc_tile_compact<false, RB, kBcGroupsDelta0, QD, true>(rep.lat, c, t, gt, pats, local,
                                                                          Q[threadIdx.x >> 6].d0, e);
                } else if (delta0) {
                    bc_tile_compact<false, RB, kBcGroupsDelta0>(rep.lat, c, t, gt, pats, local, Q[threadIdx.x >> 6].d0, e);
                } else if constexpr ((MODELS & kBatchBcGeneral) != 0) {
                    bc_tile_compact<false, RB, kBcGroups>(rep.lat, c, t, gt, pats, local, Q[threadIdx.x >> 6].gen, e);
                }
            } else if (delta0 && bc_plain<kBcGroupsDelta0>(gt)) {
                bc_tile<false, RB, kBcGroupsDelta0, true>(rep.lat, c, t, gt, pats, local, e);
            } else if (delta0) {
                bc_tile<false, RB, kBcGroupsDelta0>(rep.lat, c, t, gt, pats, local, e);
            } else if constexpr ((MODELS & kBatchBcGeneral) != 0) {
                bc_tile<false, RB, kBcGroups>(rep.lat, c, t, gt, pats, local, e);
            }
        }
    }
}

__global__ void k_advance_step(uint32_t *step, uint32_t n)
{
    if (blockIdx.x == 0 && threadIdx.x == 0)
        *step += n;
}

} // namespace

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
    constexpr int I = kBatchIsing, B = kBatchBc, G = kBatchBcGeneral;
    switch (models) {
    case I: return launch_batch_vm<V, I>(reps, tile_rep, ntiles, tables, stride, step_base, step, colour, st);
    case B: return launch_batch_vm<V, B>(reps, tile_rep, ntiles, tables, stride, step_base, step, colour, st);
    case I | B: return launch_batch_vm<V, I | B>(reps, tile_rep, ntiles, tables, stride, step_base, step, colour, st);
    case B | G: return launch_batch_vm<V, B | G>(reps, tile_rep, ntiles, tables, stride, step_base, step, colour, st);
    case I | B | G:
        return launch_batch_vm<V, I | B | G>(reps, tile_rep, ntiles, tables, stride, step_base, step, colour, st);
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
    case 8: return launch_batch_v<8>(models, reps, tile_rep, ntiles, tables, stride, step_base, step, colour, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_advance_step(uint32_t *step, uint32_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_advance_step, dim3(1), dim3(64), 0, st, step, n);
    return hipGetLastError();
}

} // namespace spin
