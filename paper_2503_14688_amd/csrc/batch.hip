// Batched replicas (C ABI spin_batch_*): many independent lattices of mixed
// size and model, each following its own bath-temperature schedule (paper,
// Thermal protocols), advanced together by one launch per half-sweep over a
// flat list of all replicas' tiles.  Runs of 2^k sweeps (k <= 8) are
// captured once each as HIP graphs of 2^(k+1) launches (plus one that
// advances the device step counter), and a run of any length replays them;
// the sweep strategy (rows per thread, per-word or compacting lazy test) is
// chosen by timing every strategy on scratch copies of the lattices.
#include "batch_kernels.hpp"
#include "host.hpp"

#include <algorithm>
#include <cerrno>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <tuple>
#include <vector>

using namespace spin_host;

// Tile layouts: rows per thread of the Ising tiles (4 or 8) x of the
// Blume-Capel tiles.
constexpr int kLayouts = 4;
// Runs are replayed from captured runs of 2^k sweeps, k <= kGraphLog: a run
// of n sweeps is n / 256 replays of the 256-sweep graph and one replay per
// set bit of n % 256.
constexpr int kGraphLog = 8;

struct spin_batch {
    std::vector<spin_handle *> reps;
    std::vector<uint32_t> table_of;     // replica -> threshold table id
    std::vector<uint64_t> t0;           // replica -> sweep index of schedule step 0
    std::vector<uint32_t> sched_of;     // replica -> schedule
    std::vector<double> T;              // the schedules (n_sched x n_steps), for the Swendsen-Wang rule
    uint32_t n_tables = 0, n_steps = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    uint64_t t = 0;                      // sweeps done (schedule step)
    int variant = -1;                    // batched strategy in use (-1: tune at first run)
    int models = 0;                      // spin::BatchModels bits of the replicas
    // per tile layout (rows per thread of the Ising and of the Blume-Capel tiles)
    spin::BatchReplica *d_reps[kLayouts] = {};
    uint32_t *d_tile_rep[kLayouts] = {};
    uint64_t ntiles[kLayouts] = {};
    GroupTable *d_tables = nullptr;
    unsigned long long *d_meas = nullptr;  // measurement counters of every replica
    size_t meas_cap = 0;                   // entries
    spin::MeasItem *d_items = nullptr;     // per replica: lattice and counter block
    uint32_t *d_ids = nullptr;             // replica lists of the batched measurement launches
    std::vector<spin::MeasItem> h_items;   // host sides of the two (kept until the copy is done)
    std::vector<uint32_t> h_ids;
    long long *d_fourier = nullptr;      // per replica: 4 E/M counters, L row sums, L column sums
    size_t fourier_len = 0;              // entries
    uint32_t *d_step = nullptr;          // schedule step on the device (= t between runs)
    // captured runs of 2^k sweeps, k = 0 .. kGraphLog, for strategy graph_variant
    hipGraph_t graph[kGraphLog + 1] = {};
    hipGraphExec_t exec[kGraphLog + 1] = {};
    int graph_variant = -1;
};

namespace {

// Tile layout of a batched strategy: bit 0 set when its Ising tiles walk 8
// rows per thread (else 4), bit 1 the same for its Blume-Capel tiles.
int layout_of(int bv)
{
    return (spin::variant_rows(spin::batch_ising_variant(bv)) == 8 ? 1 : 0) |
           (spin::variant_rows(spin::batch_bc_variant(bv)) == 8 ? 2 : 0);
}

void drop_graphs(spin_batch *b)
{
    for (int k = 0; k <= kGraphLog; ++k) {
        if (b->exec[k])
            (void)hipGraphExecDestroy(b->exec[k]);
        if (b->graph[k])
            (void)hipGraphDestroy(b->graph[k]);
        b->exec[k] = nullptr;
        b->graph[k] = nullptr;
    }
    b->graph_variant = -1;
}

void release(spin_batch *b)
{
    if (!b)
        return;
    if (b->stream)
        (void)hipStreamSynchronize(b->stream);
    drop_graphs(b);
    for (int k = 0; k < kLayouts; ++k) {
        if (b->d_reps[k])
            (void)hipFree(b->d_reps[k]);
        if (b->d_tile_rep[k])
            (void)hipFree(b->d_tile_rep[k]);
    }
    if (b->d_tables)
        (void)hipFree(b->d_tables);
    if (b->d_meas)
        (void)hipFree(b->d_meas);
    if (b->d_items)
        (void)hipFree(b->d_items);
    if (b->d_ids)
        (void)hipFree(b->d_ids);
    if (b->d_fourier)
        (void)hipFree(b->d_fourier);
    if (b->d_step)
        (void)hipFree(b->d_step);
    for (spin_handle *h : b->reps)
        spin_destroy(h);
    if (b->own_stream && b->stream)
        (void)hipStreamDestroy(b->stream);
    delete b;
}

// Tile list for one tile layout k (see layout_of): replicas with more tiles
// first (they bound the half-sweep's duration), each replica's tiles
// contiguous.
int build_tiles(spin_batch *b, int k)
{
    const size_t n = b->reps.size();
    std::vector<uint64_t> tiles(n);
    for (size_t r = 0; r < n; ++r) {
        const bool ising = b->reps[r]->lat.model == spin::kIsing;
        tiles[r] = spin::sweep_tiles(b->reps[r]->lat, (k & (ising ? 1 : 2)) ? 8 : 4);
    }
    std::vector<uint32_t> order(n);
    for (size_t r = 0; r < n; ++r)
        order[r] = (uint32_t)r;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t c) { return tiles[a] > tiles[c]; });
    std::vector<spin::BatchReplica> host(n);
    std::vector<uint32_t> tile_rep;
    uint64_t next = 0;
    for (uint32_t r : order) {
        host[r].lat = b->reps[r]->lat;
        host[r].sched = b->table_of[r];
        host[r].t0 = (uint32_t)b->t0[r];
        host[r].tile0 = next;
        for (uint64_t q = 0; q < tiles[r]; ++q)
            tile_rep.push_back(r);
        next += tiles[r];
    }
    b->ntiles[k] = next;
    HIP_TRY(hipMalloc(&b->d_reps[k], n * sizeof(spin::BatchReplica)), "hipMalloc");
    HIP_TRY(hipMalloc(&b->d_tile_rep[k], tile_rep.size() * sizeof(uint32_t)), "hipMalloc");
    HIP_TRY(hipMemcpy(b->d_reps[k], host.data(), n * sizeof(spin::BatchReplica), hipMemcpyHostToDevice),
            "hipMemcpy");
    HIP_TRY(hipMemcpy(b->d_tile_rep[k], tile_rep.data(), tile_rep.size() * sizeof(uint32_t),
                      hipMemcpyHostToDevice),
            "hipMemcpy");
    return 0;
}

// n sweeps at schedule steps *d_step + 0 .. n - 1; with advance, the device
// step counter moves on by n afterwards (a run), without it every sweep is
// repeated at the current step (tuning).
int launch_sweeps(spin_batch *b, int variant, uint32_t n, bool advance, hipStream_t st)
{
    const int k = layout_of(variant);
    for (uint32_t q = 0; q < n; ++q) {
        for (uint32_t c = 0; c < 2; ++c)
            HIP_TRY(spin::launch_batch_half_sweep(variant, b->models, b->d_reps[k], b->d_tile_rep[k], b->ntiles[k],
                                                  b->d_tables, b->n_steps, b->d_step, advance ? q : 0u, c, st),
                    "batched sweep launch");
    }
    if (advance)
        HIP_TRY(spin::launch_advance_step(b->d_step, n, st), "step counter launch");
    return 0;
}

// Choose the batched strategy on scratch copies of every lattice.  The cost
// of a sweep grows as a lattice relaxes from its T = infinity start, so the
// copies are first warmed up with eight sweeps at the current schedule step;
// then every strategy is timed (HIP events, two sweeps) in three interleaved
// rounds on the same evolving copies, and the best time of each counts.
// Strategies that run the batch's models exactly as an earlier one does (in
// a one-model batch, the other model's half of the pair) are skipped.
int autotune(spin_batch *b)
{
    auto padded = [](size_t bytes) { return (bytes + 255) / 256 * 256; };
    size_t total = 0;
    for (spin_handle *h : b->reps)
        total += padded(h->buf_bytes);
    char *scratch = nullptr;
    if (hipMalloc(&scratch, total) != hipSuccess) {
        (void)hipGetLastError();
        b->variant = 0;  // no room to tune: keep the default strategy
        return 0;
    }
    spin::BatchReplica *keep[kLayouts], *tmp[kLayouts] = {};
    for (int k = 0; k < kLayouts; ++k)
        keep[k] = b->d_reps[k];
    bool timed[spin::kBatchVariants] = {};
    for (int v = 0; v < spin::kBatchVariants; ++v) {
        timed[v] = true;
        for (int u = 0; u < v && timed[v]; ++u) {
            const bool same_i = !(b->models & spin::kBatchIsing) ||
                                spin::batch_ising_variant(u) == spin::batch_ising_variant(v);
            const bool same_b = !(b->models & spin::kBatchBc) || spin::batch_bc_variant(u) == spin::batch_bc_variant(v);
            if (same_i && same_b)
                timed[v] = false;
        }
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float best_ms[spin::kBatchVariants] = {};
    int rc = 0;
    hipError_t e = hipSuccess;
    do {
        size_t off = 0;
        for (spin_handle *h : b->reps) {
            if ((e = hipMemcpyAsync(scratch + off, h->buf, h->buf_bytes, hipMemcpyDeviceToDevice, b->stream)) !=
                hipSuccess)
                break;
            off += padded(h->buf_bytes);
        }
        // descriptor copies pointing at the scratch lattices, per tile shape
        const size_t n = b->reps.size();
        std::vector<spin::BatchReplica> host(n);
        for (int k = 0; k < kLayouts && e == hipSuccess; ++k) {
            if ((e = hipMemcpy(host.data(), keep[k], n * sizeof(spin::BatchReplica), hipMemcpyDeviceToHost)) !=
                hipSuccess)
                break;
            size_t o = 0;
            for (size_t r = 0; r < n; ++r) {
                host[r].lat.planes = (uint32_t *)(scratch + o);
                o += padded(b->reps[r]->buf_bytes);
            }
            if ((e = hipMalloc(&tmp[k], n * sizeof(spin::BatchReplica))) != hipSuccess)
                break;
            e = hipMemcpy(tmp[k], host.data(), n * sizeof(spin::BatchReplica), hipMemcpyHostToDevice);
        }
        if (e == hipSuccess && (e = hipEventCreate(&e0)) == hipSuccess)
            e = hipEventCreate(&e1);
        if (e != hipSuccess)
            break;
        for (int k = 0; k < kLayouts; ++k)
            b->d_reps[k] = tmp[k];
        // the current schedule step is the only one known to exist: every
        // tuning sweep uses it
        for (int w = 0; w < 8 && rc == 0; ++w)
            rc = launch_sweeps(b, 0, 1, false, b->stream);
        for (int round = 0; round < 3 && rc == 0 && e == hipSuccess; ++round) {
            for (int v = 0; v < spin::kBatchVariants && rc == 0 && e == hipSuccess; ++v) {
                if (!timed[v])
                    continue;
                if ((e = hipEventRecord(e0, b->stream)) != hipSuccess)
                    break;
                rc = launch_sweeps(b, v, 2, false, b->stream);
                if (rc)
                    break;
                float ms = 0.0f;
                if ((e = hipEventRecord(e1, b->stream)) == hipSuccess && (e = hipEventSynchronize(e1)) == hipSuccess)
                    e = hipEventElapsedTime(&ms, e0, e1);
                if (e == hipSuccess && (round == 0 || ms < best_ms[v]))
                    best_ms[v] = ms;
            }
        }
    } while (false);
    for (int k = 0; k < kLayouts; ++k)
        b->d_reps[k] = keep[k];
    if (rc == 0 && e != hipSuccess)
        rc = hip_fail(e, "batch strategy tuning");
    (void)hipStreamSynchronize(b->stream);
    for (int k = 0; k < kLayouts; ++k)
        if (tmp[k])
            (void)hipFree(tmp[k]);
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    (void)hipFree(scratch);
    if (rc)
        return rc;
    int best = 0;
    for (int v = 1; v < spin::kBatchVariants; ++v)
        if (timed[v] && best_ms[v] < best_ms[best])
            best = v;
    b->variant = best;
    return 0;
}

} // namespace

extern "C" {

int spin_batch_create(uint32_t n, const spin_replica_desc *descs, uint32_t n_sched, uint32_t n_steps,
                      const double *T, void *hip_stream, spin_batch **out)
{
    if (!out)
        return fail(-EINVAL, "NULL output pointer");
    *out = nullptr;
    if (n == 0 || !descs || n_sched == 0 || n_steps == 0 || !T)
        return fail(-EINVAL, "empty batch or schedule");
    if (n_steps > (1u << 31))
        return fail(-EINVAL, "schedule too long");
    for (uint64_t q = 0; q < (uint64_t)n_sched * n_steps; ++q)
        if (!(T[q] >= 0.0))
            return fail(-EINVAL, "schedule temperature %llu is negative or NaN", (unsigned long long)q);
    spin_batch *b = new (std::nothrow) spin_batch;
    if (!b)
        return fail(-ENOMEM, "out of host memory");
    b->n_steps = n_steps;
    b->T.assign(T, T + (size_t)n_sched * n_steps);
    if (hip_stream) {
        b->stream = (hipStream_t)hip_stream;
    } else {
        hipError_t e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete b;
            return hip_fail(e, "hipStreamCreateWithFlags");
        }
        b->own_stream = true;
    }
    // one threshold table per distinct (model, J, Delta, schedule)
    std::map<std::tuple<int, double, double, uint32_t>, uint32_t> ids;
    for (uint32_t r = 0; r < n; ++r) {
        const spin_replica_desc &d = descs[r];
        if (d.schedule >= n_sched) {
            release(b);
            return fail(-EINVAL, "replica %u: schedule %u out of range", r, d.schedule);
        }
        if (d.t0 + (uint64_t)n_steps > (1ull << 32)) {
            release(b);
            return fail(-EINVAL, "replica %u: sweep index t0 + steps passes 2^32", r);
        }
        spin_handle *h = nullptr;
        int rc = spin_create(d.model, d.L, d.seed, d.J, d.Delta, d.dev_buf, d.buf_bytes, b->stream, &h);
        if (rc) {
            std::string msg = spin_last_error();
            release(b);
            return fail(rc, "replica %u: %s", r, msg.c_str());
        }
        h->t = d.t0;
        h->batch_owned = true;
        b->models |= d.model == SPIN_ISING ? spin::kBatchIsing : spin::kBatchBc;
        if (d.model != SPIN_ISING && h->lat.bc_groups != spin::kBcGroupsDelta0)
            b->models |= spin::kBatchBcGeneral;
        b->reps.push_back(h);
        b->t0.push_back(d.t0);
        b->sched_of.push_back(d.schedule);
        auto key = std::make_tuple(d.model, d.J, d.Delta, d.schedule);
        auto it = ids.find(key);
        if (it == ids.end())
            it = ids.emplace(key, (uint32_t)ids.size()).first;
        b->table_of.push_back(it->second);
    }
    b->n_tables = (uint32_t)ids.size();
    std::vector<GroupTable> tables((size_t)b->n_tables * n_steps);
    std::vector<uint32_t> layout(ids.size());  // bc_groups of each table's replicas
    for (uint32_t r = 0; r < n; ++r)
        layout[b->table_of[r]] = b->reps[r]->lat.bc_groups;
    for (const auto &kv : ids) {
        const int model = std::get<0>(kv.first);
        const double J = std::get<1>(kv.first), Delta = std::get<2>(kv.first);
        const uint32_t s = std::get<3>(kv.first);
        const uint32_t bc_groups = layout[kv.second];
        for (uint32_t k = 0; k < n_steps; ++k) {
            const double Tk = T[(size_t)s * n_steps + k];
            if (k > 0 && Tk == T[(size_t)s * n_steps + k - 1])
                tables[(size_t)kv.second * n_steps + k] = tables[(size_t)kv.second * n_steps + k - 1];
            else
                tables[(size_t)kv.second * n_steps + k] = make_groups(model, bc_groups, J, Delta, Tk);
        }
    }
    hipError_t e = hipMalloc(&b->d_tables, tables.size() * sizeof(GroupTable));
    if (e == hipSuccess)
        e = hipMemcpy(b->d_tables, tables.data(), tables.size() * sizeof(GroupTable), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        release(b);
        return hip_fail(e, "threshold tables");
    }
    e = hipMalloc(&b->d_step, sizeof(uint32_t));
    if (e == hipSuccess) {
        const uint32_t zero = 0;
        e = hipMemcpy(b->d_step, &zero, sizeof zero, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        release(b);
        return hip_fail(e, "step counter");
    }
    for (int k = 0; k < kLayouts; ++k) {
        int rc = build_tiles(b, k);
        if (rc) {
            std::string msg = spin_last_error();
            release(b);
            return fail(rc, "%s", msg.c_str());
        }
    }
    *out = b;
    return 0;
}

int spin_batch_init_random(spin_batch *b)
{
    if (!b)
        return fail(-EINVAL, "NULL batch");
    for (spin_handle *h : b->reps)
        if (int rc = spin_init_random(h))
            return rc;
    return 0;
}

int spin_batch_run(spin_batch *b, uint32_t n, uint32_t flags)
{
    if (!b)
        return fail(-EINVAL, "NULL batch");
    const uint32_t forced = (flags >> 4) & 0xFu;
    if ((flags & ~(SPIN_BATCH_DIRECT | 0xF0u)) || forced > (uint32_t)spin::kBatchVariants)
        return fail(-EINVAL, "unknown flags 0x%x", flags);
    if (b->t + n > b->n_steps)
        return fail(-EINVAL, "schedule has %u steps, %llu done, %u asked", b->n_steps, (unsigned long long)b->t, n);
    if (n == 0)
        return 0;
    if (forced)
        b->variant = (int)forced - 1;
    else if (b->variant < 0) {
        if (int rc = autotune(b))
            return rc;
    }
    if (flags & SPIN_BATCH_DIRECT) {
        if (int rc = launch_sweeps(b, b->variant, n, true, b->stream))
            return rc;
    } else {
        if (b->graph_variant != b->variant) {
            HIP_TRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
            drop_graphs(b);
            b->graph_variant = b->variant;
        }
        // The captured launches read their schedule steps from the device
        // counter and advance it at the end, so the graphs of a run's pieces
        // replay one after another as they are.
        for (uint32_t left = n; left > 0;) {
            int k = kGraphLog;
            while ((1u << k) > left)
                --k;
            if (!b->exec[k]) {
                HIP_TRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
                HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
                int rc = launch_sweeps(b, b->variant, 1u << k, true, b->stream);
                hipGraph_t g = nullptr;
                hipError_t e = hipStreamEndCapture(b->stream, &g);
                if (rc) {
                    if (g)
                        (void)hipGraphDestroy(g);
                    return rc;
                }
                if (e != hipSuccess)
                    return hip_fail(e, "hipStreamEndCapture");
                b->graph[k] = g;
                e = hipGraphInstantiate(&b->exec[k], g, nullptr, nullptr, 0);
                if (e != hipSuccess) {
                    b->exec[k] = nullptr;
                    return hip_fail(e, "hipGraphInstantiate");
                }
            }
            HIP_TRY(hipGraphLaunch(b->exec[k], b->stream), "hipGraphLaunch");
            left -= 1u << k;
        }
    }
    b->t += n;
    for (size_t r = 0; r < b->reps.size(); ++r) {
        b->reps[r]->t = b->t0[r] + b->t;
        b->reps[r]->em_valid = false;
    }
    return 0;
}

int spin_batch_sw(spin_batch *b)
{
    if (!b)
        return fail(-EINVAL, "NULL batch");
    if (b->t + 1 > b->n_steps)
        return fail(-EINVAL, "schedule has %u steps, %llu done, 1 asked", b->n_steps, (unsigned long long)b->t);
    for (spin_handle *h : b->reps)
        if (h->L > kMaxSwL)
            return fail(-EINVAL, "Swendsen-Wang steps need L <= %u (got %u)", kMaxSwL, h->L);
    for (spin_handle *h : b->reps)
        if (!h->d_labels) {
            hipError_t e = hipMalloc(&h->d_labels, (size_t)h->L * h->L * sizeof(uint32_t));
            if (e != hipSuccess) {
                h->d_labels = nullptr;
                return fail(-ENOMEM, "cluster labels for L = %u: %s", h->L, hipGetErrorString(e));
            }
        }
    // each replica's step at its own schedule's temperature and sweep index,
    // as spin_sw on the replica alone; then the device step counter moves on
    // with the host's, so later runs read the next schedule step
    for (size_t r = 0; r < b->reps.size(); ++r) {
        spin_handle *h = b->reps[r];
        const double Tk = b->T[(size_t)b->sched_of[r] * b->n_steps + b->t];
        uint32_t thr;
        const bool always = sw_rule(h->J, Tk, &thr);
        HIP_TRY(spin::launch_sw_step(h->lat, (uint32_t)(b->t0[r] + b->t), thr, always, h->d_labels, b->stream),
                "Swendsen-Wang launch");
    }
    HIP_TRY(spin::launch_advance_step(b->d_step, 1, b->stream), "step counter launch");
    b->t += 1;
    for (size_t r = 0; r < b->reps.size(); ++r) {
        b->reps[r]->t = b->t0[r] + b->t;
        b->reps[r]->em_valid = false;
    }
    return 0;
}

int spin_batch_measure_fourier(spin_batch *b, spin_fourier *out)
{
    if (!b || !out)
        return fail(-EINVAL, "NULL batch or result pointer");
    const size_t n = b->reps.size();
    std::vector<size_t> off(n + 1, 0);
    for (size_t r = 0; r < n; ++r)
        off[r + 1] = off[r] + spin::kEmCounters + 2 * (size_t)b->reps[r]->L;
    const size_t total = off[n];
    if (total > b->fourier_len) {
        HIP_TRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
        if (b->d_fourier)
            (void)hipFree(b->d_fourier);
        b->fourier_len = 0;
        hipError_t e = hipMalloc(&b->d_fourier, total * sizeof(long long));
        if (e != hipSuccess) {
            b->d_fourier = nullptr;
            return fail(-ENOMEM, "row and column sums: %s", hipGetErrorString(e));
        }
        b->fourier_len = total;
    }
    // one fill, the E/M reduction and the line sums of every replica, one
    // copy, one synchronisation
    HIP_TRY(spin::launch_fill_u64((unsigned long long *)b->d_fourier, total, 0ull, b->stream), "fill kernel launch");
    for (size_t r = 0; r < n; ++r) {
        long long *base = b->d_fourier + off[r];
        const uint32_t L = b->reps[r]->L;
        HIP_TRY(spin::launch_measure_em(b->reps[r]->lat, (unsigned long long *)base, b->stream),
                "measure kernel launch");
        HIP_TRY(spin::launch_line_sums(b->reps[r]->lat, base + spin::kEmCounters, base + spin::kEmCounters + L,
                                       b->stream),
                "line-sum kernel launch");
    }
    std::vector<long long> host(total);
    HIP_TRY(hipMemcpyAsync(host.data(), b->d_fourier, total * sizeof(long long), hipMemcpyDeviceToHost, b->stream),
            "hipMemcpyAsync");
    HIP_TRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    for (size_t r = 0; r < n; ++r) {
        unsigned long long acc[spin::kEmCounters];
        for (int q = 0; q < spin::kEmCounters; ++q)
            acc[q] = (unsigned long long)host[off[r] + q];
        finish_fourier(b->reps[r], acc, host.data() + off[r] + spin::kEmCounters, out + r);
    }
    return 0;
}

int spin_batch_sync(spin_batch *b)
{
    if (!b)
        return fail(-EINVAL, "NULL batch");
    HIP_TRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    return 0;
}

int spin_batch_replica(spin_batch *b, uint32_t k, spin_handle **out)
{
    if (!b || !out || k >= b->reps.size())
        return fail(-EINVAL, "bad batch, output or replica index");
    *out = b->reps[k];
    return 0;
}

int spin_batch_measure(spin_batch *b, const uint32_t *r, uint32_t n_r, spin_meas *out, int64_t *Sx, int64_t *Sy)
{
    if (!b || !out || (n_r && (!r || !Sx || !Sy)))
        return fail(-EINVAL, "bad batch or NULL output");
    for (uint32_t q = 1; q < n_r; ++q)
        if (r[q] <= r[q - 1])
            return fail(-EINVAL, "separations must be strictly increasing");
    for (size_t k = 0; k < b->reps.size(); ++k) {
        const uint32_t L = b->reps[k]->L;
        for (uint32_t q = 0; q < n_r; ++q)
            if (r[q] == 0 || r[q] >= L)
                return fail(-EINVAL, "separation %u outside 0 < r < L = %u of replica %zu", r[q], L, k);
    }
    // every replica's counters in one buffer: one fill, then one launch per
    // kernel and model (or kernel kind) for all replicas at once, one copy,
    // one synchronisation
    const size_t per = measure_counters(n_r), total = per * b->reps.size();
    if (total > b->meas_cap) {
        HIP_TRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
        if (b->d_meas)
            (void)hipFree(b->d_meas);
        b->d_meas = nullptr;
        b->meas_cap = 0;
        hipError_t e = hipMalloc(&b->d_meas, total * sizeof(unsigned long long));
        if (e != hipSuccess) {
            b->d_meas = nullptr;
            return fail(-ENOMEM, "measurement counters (%zu): %s", total, hipGetErrorString(e));
        }
        b->meas_cap = total;
    }
    const size_t n = b->reps.size();
    if (n > 65535)
        return fail(-EINVAL, "%zu replicas: at most 65535 per batched measurement", n);
    if (!b->d_items) {
        hipError_t e = hipMalloc(&b->d_items, n * sizeof(spin::MeasItem));
        if (e == hipSuccess)
            e = hipMalloc(&b->d_ids, 3 * n * sizeof(uint32_t));
        if (e != hipSuccess) {
            if (b->d_items)
                (void)hipFree(b->d_items);
            b->d_items = nullptr;
            b->d_ids = nullptr;
            return fail(-ENOMEM, "measurement descriptors: %s", hipGetErrorString(e));
        }
    }
    // Launch lists: E/M by model (0, 1); horizontal correlations by kernel
    // kind (2..5) and vertical by kind (6, 7) when r is a prefix of the
    // sparse set; replicas whose vertical kind does not apply take the
    // general correlation kernels one by one.
    constexpr int kLists = 8;
    std::vector<uint32_t> list[kLists], single;
    uint32_t blocks[kLists] = {};
    const bool sparse = n_r > 0 && spin::sparse_prefix(r, (int)n_r);
    b->h_items.resize(n);
    for (size_t k = 0; k < n; ++k) {
        const spin::Lattice &lat = b->reps[k]->lat;
        b->h_items[k] = spin::MeasItem{lat, b->d_meas + k * per};
        auto add = [&](int l, uint32_t blk) {
            list[l].push_back((uint32_t)k);
            blocks[l] = std::max(blocks[l], blk);
        };
        add(lat.model == spin::kIsing ? 0 : 1, spin::measure_em_blocks(lat));
        if (n_r == 0)
            continue;
        const int ky = sparse ? spin::corr_sparse_kind(lat, true) : -1;
        if (ky < 0) {
            single.push_back((uint32_t)k);
            continue;
        }
        add(2 + spin::corr_sparse_kind(lat, false), spin::corr_sparse_blocks(lat, false));
        add(6 + ky, spin::corr_sparse_blocks(lat, true));
    }
    b->h_ids.clear();
    uint32_t first[kLists];
    for (int l = 0; l < kLists; ++l) {
        first[l] = (uint32_t)b->h_ids.size();
        b->h_ids.insert(b->h_ids.end(), list[l].begin(), list[l].end());
        // E/M and horizontal kernels: about 8192 blocks over all replicas
        // (32 per CU), each walking more units than in the single-lattice
        // grid (at most 16 times as many, which keeps the horizontal
        // kernel's 32-bit lane counters far from overflow); fewer blocks
        // also mean fewer counter atomics at the end of each block.
        if (l < 6 && !list[l].empty()) {
            const uint32_t cnt = (uint32_t)list[l].size();
            const uint32_t want = std::max((8192u + cnt - 1) / cnt, (blocks[l] + 15u) / 16u);
            blocks[l] = std::min(blocks[l], want);
        }
    }
    HIP_TRY(hipMemcpyAsync(b->d_items, b->h_items.data(), n * sizeof(spin::MeasItem), hipMemcpyHostToDevice,
                           b->stream),
            "hipMemcpyAsync");
    if (!b->h_ids.empty())
        HIP_TRY(hipMemcpyAsync(b->d_ids, b->h_ids.data(), b->h_ids.size() * sizeof(uint32_t),
                               hipMemcpyHostToDevice, b->stream),
                "hipMemcpyAsync");
    HIP_TRY(spin::launch_fill_u64(b->d_meas, total, 0ull, b->stream), "fill kernel launch");
    for (int l = 0; l < kLists; ++l) {
        const uint32_t cnt = (uint32_t)list[l].size();
        const uint32_t *ids = b->d_ids + first[l];
        if (l < 2)
            HIP_TRY(spin::launch_measure_em_batch(l, b->d_items, ids, cnt, blocks[l], b->stream),
                    "batched measure kernel launch");
        else if (l < 6)
            HIP_TRY(spin::launch_corr_sparse_batch(l - 2, false, b->d_items, ids, cnt, blocks[l], (int)n_r, b->stream),
                    "batched correlation kernel launch");
        else
            HIP_TRY(spin::launch_corr_sparse_batch(l - 6, true, b->d_items, ids, cnt, blocks[l], (int)n_r, b->stream),
                    "batched correlation kernel launch");
    }
    for (uint32_t k : single)
        if (int rc = queue_correlations(b->reps[k]->lat, r, n_r, b->d_meas + k * per, b->stream))
            return rc;
    std::vector<unsigned long long> acc(total);
    HIP_TRY(hipMemcpyAsync(acc.data(), b->d_meas, total * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                           b->stream),
            "hipMemcpyAsync");
    HIP_TRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    for (size_t k = 0; k < b->reps.size(); ++k)
        finish_measure(b->reps[k], acc.data() + k * per, r, n_r, out + k, n_r ? Sx + k * n_r : nullptr,
                       n_r ? Sy + k * n_r : nullptr, nullptr);
    return 0;
}

int spin_batch_info(const spin_batch *b, uint32_t *n_replicas, uint64_t *t, int *variant, uint64_t *tiles)
{
    if (!b)
        return fail(-EINVAL, "NULL batch");
    if (n_replicas)
        *n_replicas = (uint32_t)b->reps.size();
    if (t)
        *t = b->t;
    if (variant)
        *variant = b->variant;
    if (tiles)
        *tiles = b->variant >= 0 ? b->ntiles[layout_of(b->variant)] : 0;
    return 0;
}

int spin_batch_destroy(spin_batch *b)
{
    release(b);
    return 0;
}

} // extern "C"
