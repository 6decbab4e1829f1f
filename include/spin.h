/*
 * spin.h -- C ABI of the MI355X (gfx950) library for the checkerboard
 * Metropolis dynamics of the 2D spin-1/2 Ising and spin-1 Blume-Capel models
 * (Bisson, Vasilopoulos, Bernaschi, Fatica, Fytas, Gonzalez-Adalid Pemartin,
 * Martin-Mayor, "Universal exotic dynamics in critical mesoscopic systems",
 * arXiv:2503.14688).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Lattice: L x L square lattice with periodic boundaries, site (i, j),
 *   row i, column j (paper, Models: Eq. 1).  L must be a multiple of 64,
 *   64 <= L <= 2^22.
 * - Hamiltonian: H = -J sum_<x,y> s_x s_y + Delta sum_x s_x^2 (Eq. 1) with
 *   J > 0.  Ising: s in {-1, +1} and Delta must be 0.  Blume-Capel: s in
 *   {-1, 0, +1}, any finite Delta.
 * - Dynamics: single-spin-flip Metropolis with checkerboard decomposition
 *   and multispin coding (paper, Introduction).  Colour c = (i + j) & 1;
 *   one sweep updates colour 0, then colour 1.  Ising proposes s' = -s;
 *   Blume-Capel proposes one of the two other states with probability 1/2
 *   each.  Sweeps are counted by t = 0, 1, 2, ...
 * - Randomness (the paper only says its generator works on 32-bit integers,
 *   App. B): Philox4x32-10 with key (seed mod 2^32, seed >> 32) and counter
 *   (i, w, t, purpose << 16 | c << 8 | blk), w = m >> 5 with m = j >> 1.
 *   Lane b = m & 31 of plane k (k < 32) is bit b of output word k & 3 of the
 *   block blk = k >> 2; the site's 32-bit uniform u has plane 0 as its most
 *   significant bit.  purpose 0 = initial state (t = 0), 1 = acceptance,
 *   2 = Blume-Capel proposal (u >= 2^31 selects s' = -s for s != 0 and
 *   s' = -1 for s = 0; otherwise s' = 0, respectively +1).
 * - Acceptance: dE = -J * (double)((s' - s) * h) + Delta * (double)(s'^2 - s^2)
 *   with h the sum of the four neighbours, evaluated in IEEE double.  A move
 *   is accepted iff dE <= 0, or 2^32 exp(-dE / T) >= 2^32, or
 *   u < floor(2^32 exp(-dE / T)) (C library exp, no contraction).
 * - Initial state (protocol 1, T = infinity start): Ising s = +1 iff
 *   u < 2^31; Blume-Capel s = floor(3u / 2^32) - 1.
 *
 * Device layout (the caller's buffer, spin_lattice_bytes() long):
 *   Ising:        uint32 P[2][L][L/64]; bit b of P[c][i][w] is 1 iff the
 *                 spin at (i, j = 2(32w + b) + ((i + c) & 1)) is -1.
 *   Blume-Capel:  uint32 P[2][L][L/64][2]; word 0 (Z) bit = (s != 0),
 *                 word 1 (S) bit = (s < 0), S = 0 wherever Z = 0.
 *
 * Ownership and threading: the caller owns the device buffer (for instance a
 * torch uint8 tensor) and every host array; the library never frees them.
 * The library owns only its handle and small device scratch (reduction
 * counters, window staging), released by spin_destroy.  Device work is
 * queued on the handle's HIP stream (NULL = the default stream) and is
 * asynchronous unless a call says it synchronises.  Calls on one handle are
 * not reentrant; different handles may be used from different threads.
 *
 * Errors: every int-returning call returns 0 on success or a negative
 * errno-style code: -EINVAL (bad argument), -ENOMEM (host or scratch
 * allocation), -EIO (a HIP call failed).  spin_last_error() then describes
 * the failure (thread-local; HIP messages included).  No exception crosses
 * the ABI.
 */
#ifndef SPIN_H
#define SPIN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPIN_ISING 0
#define SPIN_BLUME_CAPEL 1

/* spin_sweep_ex flag: fuse the energy/magnetisation sums into the colour-1
 * pass of the last sweep, for the next spin_measure to reuse. */
#define SPIN_FUSE_MEASURE 1u

/* spin_schedule_fill kinds (paper, Thermal protocols; Table II). */
#define SPIN_SCHEDULE_CONSTANT 0    /* T(t) = p[0]                              */
#define SPIN_SCHEDULE_TWO_STEP 1    /* T(t) = p[0] for t < p[1], else p[2]      */
#define SPIN_SCHEDULE_EXPONENTIAL 2 /* T(t) = p[1] + (p[0] - p[1]) exp(-t/p[2]) */

typedef struct spin_handle spin_handle;

/* Result of spin_measure.  Integer sums are exact; the doubles are derived
 * from them in IEEE double. */
typedef struct spin_meas {
    uint64_t t;      /* sweeps completed when measured                          */
    int64_t sum_s;   /* sum_x s_x                                               */
    int64_t sum_s2;  /* sum_x s_x^2                                             */
    int64_t bond;    /* sum over nearest-neighbour pairs s_x s_y = Sx(1)+Sy(1)  */
    double e;        /* energy density (-J bond + Delta sum_s2) / L^2, which is
                        Eq. 3 read with the sign of H (Eq. 1)                   */
    double m;        /* magnetisation density sum_s / L^2                       */
    double xi;       /* coherence length I2 / I1 (App. C): trapezoid rule over
                        r = 0 and the requested r up to r_cut, the last r
                        before the first C-hat(r) <= 0; 0 if undefined          */
} spin_meas;

/* Bytes of device memory a lattice needs: L^2 / 8 (Ising, one bit per spin)
 * or L^2 / 4 (Blume-Capel, two bit planes); paper, Introduction (multispin
 * coding).  Returns -EINVAL for an unknown model or an unsupported L. */
int64_t spin_lattice_bytes(int model, uint32_t L);

/* Create a handle over a caller-owned device buffer of at least
 * spin_lattice_bytes(model, L) bytes, 256-byte aligned.  Does not touch the
 * buffer's contents; sets t = 0.  hip_stream is a hipStream_t (NULL allowed).
 * -EINVAL: bad model, L, J <= 0 or not finite, Delta not finite, Ising with
 * Delta != 0, NULL or short or misaligned buffer. */
int spin_create(int model, uint32_t L, uint64_t seed, double J, double Delta,
                void *dev_buf, size_t buf_bytes, void *hip_stream, spin_handle **out);

/* Fill the lattice with the T = infinity start of the thermal protocols
 * (paper, Thermal protocols).  Asynchronous. */
int spin_init_random(spin_handle *h);

/* n sweeps; sweep k uses bath temperature T[k] (host array of n doubles) and
 * stream sweep index t + k, then t += n (paper, Thermal protocols: protocol 1
 * is a constant T, protocol 2 a time-dependent one).  T[k] must be >= 0 and
 * not NaN; +inf accepts every move, 0 rejects every dE > 0.  Asynchronous.
 * sweep(a) followed by sweep(b) equals sweep(a + b) bit for bit.
 * -EINVAL also when t + n would exceed 2^32 (the counter word holding t). */
int spin_sweep(spin_handle *h, uint32_t n, const double *T);

/* spin_sweep with flags (SPIN_FUSE_MEASURE).  With n == 0 and the flag set,
 * only the fused sums of the current state are taken. */
int spin_sweep_ex(spin_handle *h, uint32_t n, const double *T, uint32_t flags);

/* Measure the current state (paper Eqs. 2-3 and App. C).  Synchronises the
 * handle's stream.  r: n_r strictly increasing separations, 0 < r < L (host
 * array).  Sx[q] = sum_{i,j} s(i,j) s(i, j + r_q), Sy[q] = sum_{i,j}
 * s(i,j) s(i + r_q, j) (periodic, unnormalised), C_hat[q] = (Sx[q] + Sy[q]) /
 * (2 L^2); each output pointer may be NULL when n_r == 0, C_hat may always be
 * NULL.  The energy/magnetisation sums come from the fused pass of the
 * previous spin_sweep_ex when it had SPIN_FUSE_MEASURE and nothing changed
 * since; otherwise a reduction kernel computes them (same integers). */
int spin_measure(spin_handle *h, const uint32_t *r, uint32_t n_r, spin_meas *out,
                 int64_t *Sx, int64_t *Sy, double *C_hat);

/* spin_measure for callers that cannot allocate device memory (code that
 * must not call hipMalloc: serving loops, harnesses that forbid it).  The
 * same kernels and the same results as spin_measure, bit for bit, but the
 * counters live in one fixed file-scope device array per GPU (about 48 KiB,
 * held until the process ends) instead of the handle's reduction buffer, and
 * the energy/magnetisation sums are always recomputed by the reduction kernel
 * (fused sums are ignored).  Allocates no device memory and calls no
 * allocating library routine.  n_r <= 1024, else -EINVAL.  Synchronises the
 * handle's stream.  All calls on one GPU share its array: calls are
 * serialised by a process-wide lock, the counters a call uses are cleared on
 * its stream at its start, and work that other code queues on the array
 * while a call runs would race with it. */
int spin_measure_noalloc(spin_handle *h, const uint32_t *r, uint32_t n_r, spin_meas *out,
                         int64_t *Sx, int64_t *Sy, double *C_hat);

/* Copy the whole lattice to host as int8 s[i * L + j].  Synchronises. */
int spin_get_spins(spin_handle *h, int8_t *host);

/* Copy rows i0 .. i0 + rows - 1 and columns j0 .. j0 + cols - 1 (periodic,
 * i0, j0 < L, rows, cols <= L) to host as int8 win[a * cols + b].
 * Synchronises.  Meant for sampled checks of lattices too large for host. */
int spin_get_window(spin_handle *h, uint32_t i0, uint32_t j0, uint32_t rows, uint32_t cols,
                    int8_t *host);

/* Overwrite the whole lattice from host int8 s[i * L + j]; -EINVAL if a
 * value is outside the model's alphabet.  Synchronises. */
int spin_set_spins(spin_handle *h, const int8_t *host);

/* Set / read the sweep counter t (checkpoint and resume). t < 2^32. */
int spin_set_t(spin_handle *h, uint64_t t);
int spin_get_t(const spin_handle *h, uint64_t *t);

/* The library's integer acceptance thresholds for bath temperature T (host
 * only, no device work).  For Ising, out[0] and out[1] are the thresholds of
 * dE = 4J and 8J; for Blume-Capel, out[q] for q = 9f + (y + 4) covers move
 * family f (0: s -> 0 with y = s h, 1: 0 -> s' with y = s' h, 2: s -> -s
 * with y = s h) and y in [-4, 4].  always[q] is 1 when the move needs no
 * random number (dE <= 0 or probability 1).  Returns the entry count. */
int spin_threshold_table(int model, double J, double Delta, double T, uint32_t *out,
                         uint8_t *always, int capacity);

/* Sweep strategy of a handle (results never depend on it; speed does):
 *   0: 8 rows per thread, each thread finishes its words' random planes
 *   1: 4 rows per thread; Ising words still undecided after 8 planes go
 *      to a per-wavefront work list that the wavefront drains together
 *   2: 8 rows per thread, work list        3: 4 rows per thread, per word
 *   4: as 2 with a 16-slot list (the other undecided words finish in place)
 * spin_set_variant sets one (-EINVAL outside 0..4); spin_tune times every
 * strategy on a scratch lattice of the handle's model and size (capped at
 * L = 32768; allocated and freed by the call) at bath temperature T, after
 * 16 warm-up sweeps from a T = infinity start, best of three interleaved
 * rounds, and keeps the fastest.  Synchronises the handle's stream; the
 * handle's own lattice and sweep index are untouched. */
int spin_set_variant(spin_handle *h, int variant);
int spin_get_variant(const spin_handle *h, int *variant);
int spin_tune(spin_handle *h, double T, int *chosen);

/* Fill out[k] = T(t0 + k), k < n, for a schedule kind (host FP64). */
int spin_schedule_fill(int kind, const double *params, uint64_t t0, uint32_t n, double *out);

/* Release the handle and the library's scratch; never the caller's buffer.
 * Synchronises the stream first. */
int spin_destroy(spin_handle *h);

/* Thread-local description of the last failure on this thread. */
const char *spin_last_error(void);

/* ------------------------------------------------------------------------
 * Equilibrium study of the Blume-Capel critical temperature (paper App. B):
 * Swendsen-Wang cluster updates restricted to the sites with s = +-1,
 * combined by the caller with Metropolis sweeps into the paper's elementary
 * Monte Carlo step (10 sweeps, then one Swendsen-Wang step), and the Fourier
 * moments of the spin field behind the Binder cumulant U4 and the
 * second-moment correlation length xi_2.
 * ------------------------------------------------------------------------ */

/* Fourier moments of one configuration, M(k) = sum_x exp(i k.x) s_x with
 * x = (i, j) (paper App. B, Eq. for M(k)).  Integer sums are exact; the
 * doubles are summed in IEEE double from the exact row and column sums. */
typedef struct spin_fourier {
    uint64_t t;      /* sweep index when measured                              */
    int64_t sum_s;   /* M(0)                                                    */
    int64_t sum_s2;  /* sum_x s_x^2                                             */
    int64_t bond;    /* nearest-neighbour bond sum, as in spin_meas             */
    double e;        /* energy density, as in spin_meas                         */
    double re_k1, im_k1;  /* M(2 pi / L, 0): phase 2 pi i / L (row index i)     */
    double re_k2, im_k2;  /* M(0, 2 pi / L): phase 2 pi j / L (column index j)  */
} spin_fourier;

/* n Swendsen-Wang steps restricted to the non-zero spins (paper App. B;
 * Swendsen and Wang 1987): step k at bath temperature T[k] uses sweep index
 * t + k, then t += n, like n sweeps.  Every bond between two equal non-zero
 * spins is active iff u < floor(2^32 (1 - exp(-2J / T))) (IEEE double, C
 * library exp; every such bond when 2^32 (1 - exp(-2J/T)) reaches 2^32, i.e.
 * T = 0; none at T = +inf), u = word 0 (bond to (i, j+1)) or word 1 (bond to
 * (i+1, j)) of Philox4x32-10 at counter (i, j, t, 3 << 16); the clusters
 * (connected components of active bonds, periodic) each flip iff word 0 of
 * Philox4x32-10 at counter (n, 0, t, 4 << 16) is >= 2^31, n = i L + j being
 * the cluster's smallest site index.  Vacancies never change.  Asynchronous.
 * The first call allocates the cluster forest (4 L^2 bytes, released by
 * spin_destroy).  -EINVAL for L > 32768, a negative or NaN T, or t + n
 * beyond 2^32; -ENOMEM if the forest cannot be allocated. */
int spin_sw(spin_handle *h, uint32_t n, const double *T);

/* Fourier moments of the current state (paper App. B), plus the row sums
 * row_sums[i] = sum_j s(i, j) and column sums col_sums[j] = sum_i s(i, j)
 * they come from (each may be NULL; otherwise L entries).  Synchronises the
 * handle's stream; the first call allocates 16 L bytes of device scratch. */
int spin_measure_fourier(spin_handle *h, spin_fourier *out, int64_t *row_sums, int64_t *col_sums);

/* ------------------------------------------------------------------------
 * Batched replicas: many independent lattices (any mix of model and L), each
 * with its own seed and bath-temperature schedule (paper, Thermal protocols:
 * the quench of protocol 1 and the time-dependent bath of protocol 2),
 * advanced together.  Every replica evolves exactly as it would alone
 * through spin_sweep with the same T array.  One launch per half-sweep
 * covers all replicas; runs of 2^k sweeps (k <= 8) are captured once as HIP
 * graphs, and a run of any length replays them.
 * ------------------------------------------------------------------------ */

typedef struct spin_batch spin_batch;

typedef struct spin_replica_desc {
    int model;          /* SPIN_ISING or SPIN_BLUME_CAPEL                      */
    uint32_t L;         /* as for spin_create                                  */
    uint64_t seed;
    double J, Delta;
    void *dev_buf;      /* caller-owned, spin_lattice_bytes(model, L) bytes    */
    size_t buf_bytes;
    uint32_t schedule;  /* row of the schedule table this replica follows      */
    uint64_t t0;        /* sweeps the replica has already done: its random
                           stream continues at sweep index t0 (0 for a fresh
                           lattice); schedule step k runs sweep t0 + k         */
} spin_replica_desc;

/* spin_batch_run flags: SPIN_BATCH_DIRECT launches directly instead of
 * capturing a graph; SPIN_BATCH_VARIANT(v) forces batched strategy v,
 * 0 <= v < SPIN_BATCH_VARIANTS, instead of the tuned one.  A batched strategy
 * is a pair of sweep strategies (see spin_set_variant), one for the Ising and
 * one for the Blume-Capel replicas: v = 0..4 runs strategy v for both; 5, 6,
 * 7 and 8 run (Ising, Blume-Capel) = (2, 0), (2, 3), (1, 3) and (2, 1).
 * Every strategy gives the same lattices. */
#define SPIN_BATCH_DIRECT 1u
#define SPIN_BATCH_VARIANT(v) ((uint32_t)((v) + 1) << 4)
#define SPIN_BATCH_VARIANTS 9

/* Create a batch of n replicas.  T holds n_sched schedules of
 * n_steps temperatures each: T[s * n_steps + k] is the bath temperature of
 * sweep k for schedule s (host array, copied into threshold tables).  The
 * batch owns one handle per replica (spin_batch_replica) and works on
 * hip_stream, or on a stream of its own when hip_stream is NULL (a graph
 * cannot be captured on the legacy default stream).  -EINVAL as for
 * spin_create (message names the replica), or a schedule index out of range,
 * or a negative / NaN temperature, or t0 + n_steps beyond 2^32. */
int spin_batch_create(uint32_t n, const spin_replica_desc *reps, uint32_t n_sched, uint32_t n_steps,
                      const double *T, void *hip_stream, spin_batch **out);

/* T = infinity start of every replica.  Asynchronous. */
int spin_batch_init_random(spin_batch *b);

/* Advance every replica by n sweeps (schedule steps t .. t + n - 1, replica
 * sweep indices t0 + t .. t0 + t + n - 1, t = sweeps this batch has run).  The
 * first run chooses the sweep strategy by timing each on scratch copies of
 * the lattices, unless SPIN_BATCH_VARIANT forces one.  Asynchronous; -EINVAL
 * past the end of the schedule. */
int spin_batch_run(spin_batch *b, uint32_t n, uint32_t flags);

/* Wait for the batch's queued work. */
int spin_batch_sync(spin_batch *b);

/* Borrow replica k's handle (measure, get/set spins); owned by the batch.
 * spin_sweep, spin_sweep_ex, spin_sw and spin_set_t on a borrowed handle
 * return -EINVAL: only spin_batch_run advances a replica, so no sweep index
 * (and no random number) is ever used twice. */
int spin_batch_replica(spin_batch *b, uint32_t k, spin_handle **out);

/* Measure every replica's current state, as spin_measure on each replica's
 * handle (paper Eqs. 2-3 and App. C): out[k] for replica k, Sx[k * n_r + q]
 * and Sy[k * n_r + q] for separation r[q] (caller-owned host arrays of n and
 * n * n_r entries; Sx, Sy may be NULL when n_r == 0).  Every r[q] must lie in
 * 0 < r < L of every replica, and a batch holds at most 65535 replicas for
 * this call (-EINVAL beyond).  Each reduction and correlation kernel runs
 * once for all replicas of a model (and kernel kind) when r is a prefix of
 * the sparse set; replicas whose rows the sparse vertical kernel cannot take,
 * and every replica for other r, get the general kernels one by one.  All
 * sums land in one counter buffer (allocated at the first call, kept by the
 * batch), copied back once; synchronises the batch's stream once. */
int spin_batch_measure(spin_batch *b, const uint32_t *r, uint32_t n_r, spin_meas *out, int64_t *Sx,
                       int64_t *Sy);

/* One Swendsen-Wang step on every replica (paper App. B; as spin_sw on each
 * replica alone): replica k's step runs at its schedule's temperature for
 * the batch's current step and at sweep index t0 + t, then the batch moves
 * on by one step, like a one-sweep spin_batch_run, so runs and steps can
 * alternate (the elementary Monte Carlo step of the equilibrium study: n
 * sweeps, then one cluster step).  Every replica must have L <= 32768
 * (-EINVAL otherwise); cluster labels (L * L uint32 per replica) are
 * allocated at the first call and kept by the replica's handle. */
int spin_batch_sw(spin_batch *b);

/* Fourier moments of every replica's current state, as spin_measure_fourier
 * on each replica alone (without the row and column sums): out[k] for
 * replica k (caller-owned host array of n entries).  One counter buffer for
 * all replicas (allocated at the first call, kept by the batch), one copy
 * back, one synchronisation of the batch's stream. */
int spin_batch_measure_fourier(spin_batch *b, spin_fourier *out);

/* Replica count, sweeps this batch has run, batched strategy in use (-1 before
 * the first run) and tiles per half-sweep; any output may be NULL. */
int spin_batch_info(const spin_batch *b, uint32_t *n_replicas, uint64_t *t, int *variant, uint64_t *tiles);

/* Release the batch, its handles and device tables (never the lattices). */
int spin_batch_destroy(spin_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* SPIN_H */
