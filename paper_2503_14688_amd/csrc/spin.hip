// Host implementation of the C ABI declared in include/spin.h: argument
// checks, the integer acceptance tables (host FP64 exp), launch sequencing
// on the handle's stream, and the FP64 observables derived from the exact
// integer sums.
#include "../../include/spin.h"
#include "host.hpp"
#include "kernels.hpp"

#include <cerrno>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

// IEEE double throughout, no fused multiply-add: the thresholds and the
// derived observables are defined by plain double arithmetic.
#pragma clang fp contract(off)

namespace spin_host {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(-EIO, "%s: %s", what, hipGetErrorString(e));
}

bool valid_L(uint32_t L) { return L >= 64 && L <= (1u << 22) && (L % 64) == 0; }

// Energy change of s -> sp with neighbour sum h (Hamiltonian, paper Eq. 1).
double delta_energy(double J, double Delta, int s, int sp, int h)
{
    const int dh = (sp - s) * h;
    const int q = sp * sp - s * s;
    return -J * (double)dh + Delta * (double)q;
}

enum Rule { kRng = 0, kAlways = 1, kNever = 2 };

// Metropolis in integers: accept iff dE <= 0, or 2^32 e^{-dE/T} >= 2^32,
// or u < floor(2^32 e^{-dE/T}); a zero threshold never accepts.
Rule metropolis_rule(double dE, double T, uint32_t *thr)
{
    *thr = 0;
    if (dE <= 0.0)
        return kAlways;
    const double p = std::exp(-dE / T);
    const double x = std::ldexp(p, 32);
    if (x >= 4294967296.0)
        return kAlways;
    *thr = (uint32_t)std::floor(x);
    return *thr == 0 ? kNever : kRng;
}

void set_group(GroupTable &gt, int g, Rule rule, uint32_t thr)
{
    gt.thr[g] = thr;
    if (rule == kRng)
        gt.rng_bits |= 1u << g;
    else if (rule == kNever)
        gt.never_bits |= 1u << g;
}

// Blume-Capel groups merged for Delta = 0 (kernels.hip, bc_tile): members
// (s, s', h) per group; every member must give the same threshold.
struct Member {
    int s, sp, h;
};
const Member kMerged[6][3] = {
    {{1, 0, 1}, {0, 1, -1}, {0, 1, -1}},   // dE = J
    {{1, 0, 2}, {0, 1, -2}, {1, -1, 1}},   // 2J
    {{1, 0, 3}, {0, 1, -3}, {0, 1, -3}},   // 3J
    {{1, 0, 4}, {0, 1, -4}, {1, -1, 2}},   // 4J
    {{1, -1, 3}, {1, -1, 3}, {1, -1, 3}},  // 6J
    {{1, -1, 4}, {1, -1, 4}, {1, -1, 4}},  // 8J
};

bool merged_groups(double J, double Delta, double T, GroupTable &gt)
{
    if (Delta != 0.0)
        return false;
    std::memset(&gt, 0, sizeof gt);
    for (int g = 0; g < 6; ++g) {
        uint32_t thr0 = 0;
        const Rule r0 = metropolis_rule(delta_energy(J, Delta, kMerged[g][0].s, kMerged[g][0].sp, kMerged[g][0].h),
                                        T, &thr0);
        for (int k = 1; k < 3; ++k) {
            uint32_t thr;
            const Rule r = metropolis_rule(
                delta_energy(J, Delta, kMerged[g][k].s, kMerged[g][k].sp, kMerged[g][k].h), T, &thr);
            if (r != r0 || thr != thr0)
                return false;
        }
        set_group(gt, g, r0, thr0);
    }
    return true;
}

// Group tables as the kernels consume them (see kernels.hpp): bc_groups is
// the lattice's Blume-Capel group layout (13 general, 6 for Delta = 0).
// Plane-by-plane threshold bits of groups 0..7 (GroupTable::plane_groups).
void fill_plane_groups(GroupTable &gt)
{
    for (uint32_t k = 0; k < 32; ++k) {
        uint32_t pat = 0;
        for (uint32_t g = 0; g < 8; ++g)
            pat |= ((gt.thr[g] >> (31u - k)) & 1u) << g;
        gt.plane_groups[k / 4] |= pat << (8u * (k % 4));
    }
}

GroupTable make_groups(int model, uint32_t bc_groups, double J, double Delta, double T)
{
    GroupTable gt;
    std::memset(&gt, 0, sizeof gt);
    uint32_t thr;
    if (model == SPIN_BLUME_CAPEL && bc_groups == spin::kBcGroupsDelta0) {
        merged_groups(J, Delta, T, gt);  // exactness checked when the layout was chosen
        fill_plane_groups(gt);
        return gt;
    }
    if (model == SPIN_ISING) {
        // three aligned neighbours (s h = 2) and four (s h = 4)
        Rule r = metropolis_rule(delta_energy(J, Delta, 1, -1, 2), T, &thr);
        set_group(gt, 0, r, thr);
        r = metropolis_rule(delta_energy(J, Delta, 1, -1, 4), T, &thr);
        set_group(gt, 1, r, thr);
        fill_plane_groups(gt);
        return gt;
    }
    for (int v = 0; v < 9; ++v) {
        const int y = v - 4;
        const double dA = delta_energy(J, Delta, 1, 0, y);  // s -> 0, y = s h
        const double dB = delta_energy(J, Delta, 0, 1, y);  // 0 -> s', y = s' h
        if (dA > 0.0) {
            gt.sel_a_bits |= 1u << v;
            set_group(gt, v, metropolis_rule(dA, T, &thr), thr);
        } else {
            set_group(gt, v, metropolis_rule(dB, T, &thr), thr);
        }
    }
    for (int y = 1; y <= 4; ++y) {
        const double dC = delta_energy(J, Delta, 1, -1, y);  // s -> -s, y = s h
        set_group(gt, 8 + y, metropolis_rule(dC, T, &thr), thr);
    }
    return gt;
}

int check_handle(const spin_handle *h)
{
    if (!h)
        return fail(-EINVAL, "NULL handle");
    return 0;
}

int ensure_acc(spin_handle *h, size_t entries)
{
    if (entries <= h->acc_cap)
        return 0;
    size_t cap = h->acc_cap ? h->acc_cap : 64;
    while (cap < entries)
        cap *= 2;
    HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    unsigned long long *p = nullptr;
    hipError_t e = hipMalloc(&p, cap * sizeof(unsigned long long));
    if (e != hipSuccess)
        return fail(-ENOMEM, "hipMalloc(%zu counters): %s", cap, hipGetErrorString(e));
    if (h->em_valid)  // keep fused sums across the move
        HIP_TRY(hipMemcpy(p, h->d_acc, spin::kEmCounters * sizeof(unsigned long long), hipMemcpyDeviceToDevice),
                "hipMemcpy");
    if (h->d_acc)
        (void)hipFree(h->d_acc);
    h->d_acc = p;
    h->acc_cap = cap;
    return 0;
}

double xi_from_sums(const uint32_t *r, const int64_t *Sx, const int64_t *Sy, uint32_t n_r, double N, double C0,
                    double *C_hat)
{
    // C-hat(r) = (Sx + Sy) / (2 L^2); trapezoid rule for I_n = int r^n C(r) dr
    // over (0, C0) and the sampled points up to the first non-positive C-hat
    // (paper App. C, Eq. for I_n)
    for (uint32_t q = 0; C_hat && q < n_r; ++q)
        C_hat[q] = (double)(Sx[q] + Sy[q]) / (2.0 * N);
    if (!(C0 > 0.0))
        return 0.0;
    double I1 = 0.0, I2 = 0.0;
    double ra = 0.0, ca = C0;
    uint32_t used = 0;
    for (uint32_t q = 0; q < n_r; ++q) {
        const double rb = (double)r[q], cb = (double)(Sx[q] + Sy[q]) / (2.0 * N);
        if (!(cb > 0.0))
            break;
        const double w = rb - ra;
        I1 += w * (ra * ca + rb * cb) / 2.0;
        I2 += w * (ra * ra * ca + rb * rb * cb) / 2.0;
        ra = rb;
        ca = cb;
        ++used;
    }
    if (used == 0 || !(I1 > 0.0))
        return 0.0;
    return I2 / I1;
}

size_t measure_counters(uint32_t n_r) { return spin::kEmCounters + 4 * (size_t)n_r; }

int queue_correlations(const spin::Lattice &lat, const uint32_t *r, uint32_t n_r, unsigned long long *acc,
                       hipStream_t st)
{
    const size_t base_x = spin::kEmCounters, base_y = base_x + 2 * (size_t)n_r;
    for (int axis = 0; axis < 2; ++axis) {
        const bool vertical = axis == 1;
        unsigned long long *dst = acc + (vertical ? base_y : base_x);
        const bool fast = vertical ? spin::corr_sparse_y_ok(lat, r, (int)n_r) : spin::corr_sparse_x_ok(lat, r, (int)n_r);
        if (fast) {
            HIP_TRY(spin::launch_corr_sparse(lat, vertical, (int)n_r, dst, st), "correlation kernel launch");
            continue;
        }
        for (uint32_t q0 = 0; q0 < n_r; q0 += spin::kCorrChunk) {
            const int cnt = (int)((n_r - q0) < (uint32_t)spin::kCorrChunk ? (n_r - q0) : spin::kCorrChunk);
            HIP_TRY(spin::launch_corr(lat, vertical, r + q0, cnt, dst + 2 * q0, st), "correlation kernel launch");
        }
    }
    return 0;
}

void finish_measure(const spin_handle *h, const unsigned long long *acc, const uint32_t *r, uint32_t n_r,
                    spin_meas *out, int64_t *Sx, int64_t *Sy, double *C_hat)
{
    const size_t base_x = spin::kEmCounters, base_y = base_x + 2 * (size_t)n_r;
    const double N = (double)h->L * (double)h->L;
    out->t = h->t;
    out->sum_s = (int64_t)acc[0] - 2 * (int64_t)acc[1];
    out->sum_s2 = (int64_t)acc[0];
    out->bond = (int64_t)acc[2] - 2 * (int64_t)acc[3];
    out->e = (-h->J * (double)out->bond + h->Delta * (double)out->sum_s2) / N;
    out->m = (double)out->sum_s / N;
    // pairs with both ends non-zero: every pair for Ising (L^2 per axis and r)
    const int64_t all_pairs = (int64_t)h->L * (int64_t)h->L;
    for (uint32_t q = 0; q < n_r; ++q) {
        const int64_t ax = h->model == SPIN_ISING ? all_pairs : (int64_t)acc[base_x + 2 * q];
        const int64_t ay = h->model == SPIN_ISING ? all_pairs : (int64_t)acc[base_y + 2 * q];
        Sx[q] = ax - 2 * (int64_t)acc[base_x + 2 * q + 1];
        Sy[q] = ay - 2 * (int64_t)acc[base_y + 2 * q + 1];
    }
    out->xi = xi_from_sums(r, Sx, Sy, n_r, N, (double)out->sum_s2 / N, C_hat);
}

} // namespace spin_host

using namespace spin_host;

extern "C" {

int64_t spin_lattice_bytes(int model, uint32_t L)
{
    if ((model != SPIN_ISING && model != SPIN_BLUME_CAPEL) || !valid_L(L))
        return fail(-EINVAL, "unsupported model %d or L %u (need 64 <= L <= 2^22, L %% 64 == 0)", model, L);
    const int64_t spins = (int64_t)L * (int64_t)L;
    return model == SPIN_ISING ? spins / 8 : spins / 4;
}

int spin_create(int model, uint32_t L, uint64_t seed, double J, double Delta, void *dev_buf, size_t buf_bytes,
                void *hip_stream, spin_handle **out)
{
    if (!out)
        return fail(-EINVAL, "NULL output handle pointer");
    *out = nullptr;
    const int64_t need = spin_lattice_bytes(model, L);
    if (need < 0)
        return (int)need;
    if (!(J > 0.0) || !std::isfinite(J))
        return fail(-EINVAL, "J must be finite and > 0 (got %g)", J);
    if (!std::isfinite(Delta))
        return fail(-EINVAL, "Delta must be finite");
    if (model == SPIN_ISING && Delta != 0.0)
        return fail(-EINVAL, "Delta must be 0 for the Ising model");
    if (!dev_buf || buf_bytes < (size_t)need)
        return fail(-EINVAL, "device buffer of %zu bytes is smaller than the %lld needed", buf_bytes,
                    (long long)need);
    if (((uintptr_t)dev_buf & 255u) != 0)
        return fail(-EINVAL, "device buffer must be 256-byte aligned");
    hipPointerAttribute_t attr;
    std::memset(&attr, 0, sizeof attr);
    hipError_t e = hipPointerGetAttributes(&attr, dev_buf);
    if (e != hipSuccess || attr.type != hipMemoryTypeDevice) {
        (void)hipGetLastError();
        return fail(-EINVAL, "buffer is not device memory allocated through HIP");
    }
    spin_handle *h = new (std::nothrow) spin_handle;
    if (!h)
        return fail(-ENOMEM, "out of host memory");
    std::memset(h, 0, sizeof *h);
    h->model = model;
    h->L = L;
    h->seed = seed;
    h->J = J;
    h->Delta = Delta;
    h->buf = dev_buf;
    h->buf_bytes = buf_bytes;
    h->stream = (hipStream_t)hip_stream;
    h->device = attr.device;
    h->lat.planes = (uint32_t *)dev_buf;
    h->lat.L = L;
    h->lat.W = L / 64;
    h->lat.plane_u32 = (uint64_t)L * (L / 64) * (model == SPIN_ISING ? 1 : 2);
    h->lat.model = model;
    h->lat.key0 = (uint32_t)seed;
    h->lat.key1 = (uint32_t)(seed >> 32);
    h->lat.variant = 0;
    h->lat.bc_groups = spin::kBcGroups;
    {
        // merged groups need every member to give the same dE; that does not
        // depend on T, so one check decides for all temperatures
        GroupTable probe;
        if (model == SPIN_BLUME_CAPEL && merged_groups(J, Delta, 1.0, probe))
            h->lat.bc_groups = spin::kBcGroupsDelta0;
    }
    *out = h;  // reduction scratch is allocated at the first measurement
    return 0;
}

int spin_init_random(spin_handle *h)
{
    if (int rc = check_handle(h))
        return rc;
    HIP_TRY(spin::launch_init(h->lat, h->stream), "init kernel launch");
    h->em_valid = false;
    return 0;
}

int spin_sweep_ex(spin_handle *h, uint32_t n, const double *T, uint32_t flags)
{
    if (int rc = check_handle(h))
        return rc;
    if (flags & ~SPIN_FUSE_MEASURE)
        return fail(-EINVAL, "unknown flags 0x%x", flags);
    if (h->batch_owned)
        return fail(-EINVAL, "the handle belongs to a batch: advance it with spin_batch_run");
    if (n > 0 && !T)
        return fail(-EINVAL, "NULL temperature array");
    if (h->t + n > (1ull << 32))
        return fail(-EINVAL, "sweep index would pass 2^32");
    for (uint32_t k = 0; k < n; ++k) {
        if (!(T[k] >= 0.0))
            return fail(-EINVAL, "T[%u] = %g is negative or NaN", k, T[k]);
    }
    const bool fuse = (flags & SPIN_FUSE_MEASURE) != 0;
    if (fuse)
        if (int rc = ensure_acc(h, 64))
            return rc;
    if (fuse)
        HIP_TRY(spin::launch_fill_u64(h->d_acc, spin::kEmCounters, 0ull, h->stream), "fill kernel launch");
    if (n == 0) {
        if (fuse) {
            HIP_TRY(spin::launch_measure_em(h->lat, h->d_acc, h->stream), "measure kernel launch");
            h->em_valid = true;
        }
        return 0;
    }
    h->em_valid = false;
    GroupTable gt;
    double last_T = std::nan("");
    for (uint32_t k = 0; k < n; ++k) {
        if (!(T[k] == last_T)) {
            gt = make_groups(h->model, h->lat.bc_groups, h->J, h->Delta, T[k]);
            last_T = T[k];
        }
        const uint32_t t = (uint32_t)(h->t + k);
        for (uint32_t c = 0; c < 2; ++c) {
            unsigned long long *acc = (fuse && k + 1 == n && c == 1) ? h->d_acc : nullptr;
            HIP_TRY(spin::launch_half_sweep(h->lat, c, t, gt, acc, h->stream), "sweep kernel launch");
        }
    }
    h->t += n;
    h->em_valid = fuse;
    return 0;
}

int spin_sweep(spin_handle *h, uint32_t n, const double *T) { return spin_sweep_ex(h, n, T, 0u); }

int spin_measure(spin_handle *h, const uint32_t *r, uint32_t n_r, spin_meas *out, int64_t *Sx, int64_t *Sy,
                 double *C_hat)
{
    if (int rc = check_handle(h))
        return rc;
    if (!out)
        return fail(-EINVAL, "NULL result pointer");
    if (n_r > 0 && (!r || !Sx || !Sy))
        return fail(-EINVAL, "NULL separation or output array");
    for (uint32_t q = 0; q < n_r; ++q) {
        if (r[q] == 0 || r[q] >= h->L || (q > 0 && r[q] <= r[q - 1]))
            return fail(-EINVAL, "separations must be strictly increasing in (0, L)");
    }
    const size_t entries = measure_counters(n_r);
    if (int rc = ensure_acc(h, entries))
        return rc;
    if (!h->em_valid) {
        HIP_TRY(spin::launch_fill_u64(h->d_acc, spin::kEmCounters, 0ull, h->stream), "fill kernel launch");
        HIP_TRY(spin::launch_measure_em(h->lat, h->d_acc, h->stream), "measure kernel launch");
        h->em_valid = true;
    }
    if (n_r > 0) {
        HIP_TRY(spin::launch_fill_u64(h->d_acc + spin::kEmCounters, 4 * (uint64_t)n_r, 0ull, h->stream),
                "fill kernel launch");
        if (int rc = queue_correlations(h->lat, r, n_r, h->d_acc, h->stream))
            return rc;
    }
    std::vector<unsigned long long> acc(entries);
    HIP_TRY(hipMemcpyAsync(acc.data(), h->d_acc, acc.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                           h->stream),
            "hipMemcpyAsync");
    HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    finish_measure(h, acc.data(), r, n_r, out, Sx, Sy, C_hat);
    return 0;
}

int spin_get_spins(spin_handle *h, int8_t *host)
{
    if (int rc = check_handle(h))
        return rc;
    if (!host)
        return fail(-EINVAL, "NULL host array");
    const uint32_t L = h->L, W = h->lat.W;
    std::vector<uint32_t> packed;
    try {
        packed.resize(2 * h->lat.plane_u32);
    } catch (...) {
        return fail(-ENOMEM, "host staging for %llu words", (unsigned long long)(2 * h->lat.plane_u32));
    }
    HIP_TRY(hipMemcpyAsync(packed.data(), h->buf, packed.size() * 4, hipMemcpyDeviceToHost, h->stream),
            "hipMemcpyAsync");
    HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    for (uint32_t i = 0; i < L; ++i) {
        for (uint32_t j = 0; j < L; ++j) {
            const uint32_t c = (i + j) & 1u, m = j >> 1;
            const size_t word = (size_t)i * W + (m >> 5);
            const uint32_t bit = m & 31u;
            int8_t v;
            if (h->model == SPIN_ISING) {
                v = ((packed[c * h->lat.plane_u32 + word] >> bit) & 1u) ? -1 : 1;
            } else {
                const uint32_t z = packed[c * h->lat.plane_u32 + 2 * word];
                const uint32_t s = packed[c * h->lat.plane_u32 + 2 * word + 1];
                v = ((z >> bit) & 1u) ? (((s >> bit) & 1u) ? -1 : 1) : 0;
            }
            host[(size_t)i * L + j] = v;
        }
    }
    return 0;
}

int spin_set_spins(spin_handle *h, const int8_t *host)
{
    if (int rc = check_handle(h))
        return rc;
    if (!host)
        return fail(-EINVAL, "NULL host array");
    const uint32_t L = h->L, W = h->lat.W;
    std::vector<uint32_t> packed;
    try {
        packed.assign(2 * h->lat.plane_u32, 0u);
    } catch (...) {
        return fail(-ENOMEM, "host staging for %llu words", (unsigned long long)(2 * h->lat.plane_u32));
    }
    for (uint32_t i = 0; i < L; ++i) {
        for (uint32_t j = 0; j < L; ++j) {
            const int v = host[(size_t)i * L + j];
            const bool ok = h->model == SPIN_ISING ? (v == 1 || v == -1) : (v >= -1 && v <= 1);
            if (!ok)
                return fail(-EINVAL, "spin %d at (%u, %u) is outside the model's alphabet", v, i, j);
            const uint32_t c = (i + j) & 1u, m = j >> 1;
            const size_t word = (size_t)i * W + (m >> 5);
            const uint32_t bit = 1u << (m & 31u);
            if (h->model == SPIN_ISING) {
                if (v < 0)
                    packed[c * h->lat.plane_u32 + word] |= bit;
            } else {
                if (v != 0)
                    packed[c * h->lat.plane_u32 + 2 * word] |= bit;
                if (v < 0)
                    packed[c * h->lat.plane_u32 + 2 * word + 1] |= bit;
            }
        }
    }
    HIP_TRY(hipMemcpyAsync(h->buf, packed.data(), packed.size() * 4, hipMemcpyHostToDevice, h->stream),
            "hipMemcpyAsync");
    HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    h->em_valid = false;
    return 0;
}

int spin_get_window(spin_handle *h, uint32_t i0, uint32_t j0, uint32_t rows, uint32_t cols, int8_t *host)
{
    if (int rc = check_handle(h))
        return rc;
    if (!host || i0 >= h->L || j0 >= h->L || rows == 0 || cols == 0 || rows > h->L || cols > h->L)
        return fail(-EINVAL, "bad window (%u, %u) %u x %u for L = %u", i0, j0, rows, cols, h->L);
    const size_t bytes = (size_t)rows * cols;
    if (bytes > h->win_cap) {
        HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
        if (h->d_win)
            (void)hipFree(h->d_win);
        h->d_win = nullptr;
        h->win_cap = 0;
        hipError_t e = hipMalloc(&h->d_win, bytes);
        if (e != hipSuccess)
            return fail(-ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
        h->win_cap = bytes;
    }
    HIP_TRY(spin::launch_window(h->lat, i0, j0, rows, cols, h->d_win, h->stream), "window kernel launch");
    HIP_TRY(hipMemcpyAsync(host, h->d_win, bytes, hipMemcpyDeviceToHost, h->stream), "hipMemcpyAsync");
    HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    return 0;
}

int spin_set_t(spin_handle *h, uint64_t t)
{
    if (int rc = check_handle(h))
        return rc;
    if (t >= (1ull << 32))
        return fail(-EINVAL, "t must be below 2^32");
    if (h->batch_owned)
        return fail(-EINVAL, "the handle belongs to a batch, which keeps its sweep index");
    h->t = t;
    return 0;
}

int spin_get_t(const spin_handle *h, uint64_t *t)
{
    if (int rc = check_handle(h))
        return rc;
    if (!t)
        return fail(-EINVAL, "NULL output");
    *t = h->t;
    return 0;
}

int spin_set_variant(spin_handle *h, int variant)
{
    if (int rc = check_handle(h))
        return rc;
    if (variant < 0 || variant >= spin::kVariants)
        return fail(-EINVAL, "variant %d outside 0..%d", variant, spin::kVariants - 1);
    h->lat.variant = variant;
    return 0;
}

int spin_get_variant(const spin_handle *h, int *variant)
{
    if (int rc = check_handle(h))
        return rc;
    if (!variant)
        return fail(-EINVAL, "NULL output");
    *variant = h->lat.variant;
    return 0;
}

int spin_tune(spin_handle *h, double T, int *chosen)
{
    if (int rc = check_handle(h))
        return rc;
    if (!(T >= 0.0))
        return fail(-EINVAL, "T must be >= 0");
    const uint32_t Ls = h->L < 32768u ? h->L : 32768u;
    const int64_t bytes = spin_lattice_bytes(h->model, Ls);
    void *scratch = nullptr;
    hipError_t e = hipMalloc(&scratch, (size_t)bytes);
    if (e != hipSuccess)
        return fail(-ENOMEM, "tuning scratch of %lld bytes: %s", (long long)bytes, hipGetErrorString(e));
    spin::Lattice lat = h->lat;
    lat.planes = (uint32_t *)scratch;
    lat.L = Ls;
    lat.W = Ls / 64;
    lat.plane_u32 = (uint64_t)Ls * lat.W * (h->model == SPIN_ISING ? 1 : 2);
    const GroupTable gt = make_groups(h->model, lat.bc_groups, h->J, h->Delta, T);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = 0;
    float best_ms[spin::kVariants];
    int best = h->lat.variant;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        rc = fail(-EIO, "hipEventCreate failed");
    // The cost of a sweep depends on how many sites need random planes, which
    // grows as the lattice relaxes from its T = infinity start: warm the
    // scratch lattice up first, then time the strategies in interleaved
    // rounds (best of three, two sweeps each) on the same evolving state.
    constexpr uint32_t kWarm = 16, kRounds = 3, kTimed = 2;
    uint32_t t = 0;
    hipError_t err = rc ? hipSuccess : spin::launch_init(lat, h->stream);
    lat.variant = 0;
    for (; t < kWarm && err == hipSuccess && rc == 0; ++t)
        for (uint32_t c = 0; c < 2 && err == hipSuccess; ++c)
            err = spin::launch_half_sweep(lat, c, t, gt, nullptr, h->stream);
    for (uint32_t round = 0; round < kRounds && rc == 0 && err == hipSuccess; ++round) {
        for (int v = 0; v < spin::kVariants && err == hipSuccess; ++v) {
            lat.variant = v;
            err = hipEventRecord(e0, h->stream);
            for (uint32_t k = 0; k < 2 * kTimed && err == hipSuccess; ++k)
                err = spin::launch_half_sweep(lat, k & 1u, t + (k >> 1), gt, nullptr, h->stream);
            t += kTimed;
            if (err == hipSuccess)
                err = hipEventRecord(e1, h->stream);
            if (err == hipSuccess)
                err = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (err == hipSuccess)
                err = hipEventElapsedTime(&ms, e0, e1);
            if (err == hipSuccess && (round == 0 || ms < best_ms[v]))
                best_ms[v] = ms;
        }
    }
    if (rc == 0 && err != hipSuccess)
        rc = hip_fail(err, "tuning sweep");
    if (rc == 0) {
        best = 0;
        for (int v = 1; v < spin::kVariants; ++v)
            if (best_ms[v] < best_ms[best])
                best = v;
    }
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    (void)hipFree(scratch);
    if (rc)
        return rc;
    h->lat.variant = best;
    if (chosen)
        *chosen = best;
    return 0;
}

int spin_threshold_table(int model, double J, double Delta, double T, uint32_t *out, uint8_t *always, int capacity)
{
    if (model != SPIN_ISING && model != SPIN_BLUME_CAPEL)
        return fail(-EINVAL, "unknown model %d", model);
    if (!(T >= 0.0))
        return fail(-EINVAL, "T must be >= 0");
    const int n = model == SPIN_ISING ? 2 : 27;
    if (!out || !always || capacity < n)
        return fail(-EINVAL, "need room for %d entries", n);
    uint32_t thr;
    if (model == SPIN_ISING) {
        for (int q = 0; q < 2; ++q) {
            const Rule r = metropolis_rule(delta_energy(J, Delta, 1, -1, 2 + 2 * q), T, &thr);
            out[q] = thr;
            always[q] = r == kAlways;
        }
        return n;
    }
    for (int f = 0; f < 3; ++f) {
        for (int v = 0; v < 9; ++v) {
            const int y = v - 4;
            double dE;
            if (f == 0)
                dE = delta_energy(J, Delta, 1, 0, y);
            else if (f == 1)
                dE = delta_energy(J, Delta, 0, 1, y);
            else
                dE = delta_energy(J, Delta, 1, -1, y);
            const Rule r = metropolis_rule(dE, T, &thr);
            out[9 * f + v] = thr;
            always[9 * f + v] = r == kAlways;
        }
    }
    return n;
}

int spin_schedule_fill(int kind, const double *p, uint64_t t0, uint32_t n, double *out)
{
    if (n > 0 && (!p || !out))
        return fail(-EINVAL, "NULL parameter or output array");
    for (uint32_t k = 0; k < n; ++k) {
        const double t = (double)(t0 + k);
        switch (kind) {
        case SPIN_SCHEDULE_CONSTANT: out[k] = p[0]; break;
        case SPIN_SCHEDULE_TWO_STEP: out[k] = t < p[1] ? p[0] : p[2]; break;
        case SPIN_SCHEDULE_EXPONENTIAL: out[k] = p[1] + (p[0] - p[1]) * std::exp(-t / p[2]); break;
        default: return fail(-EINVAL, "unknown schedule kind %d", kind);
        }
    }
    return 0;
}

int spin_destroy(spin_handle *h)
{
    if (!h)
        return 0;
    int rc = 0;
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess)
        rc = hip_fail(e, "hipStreamSynchronize");
    if (h->d_acc)
        (void)hipFree(h->d_acc);
    if (h->d_win)
        (void)hipFree(h->d_win);
    if (h->d_labels)
        (void)hipFree(h->d_labels);
    if (h->d_lines)
        (void)hipFree(h->d_lines);
    delete h;
    return rc;
}

const char *spin_last_error(void) { return g_err.c_str(); }

} // extern "C"
