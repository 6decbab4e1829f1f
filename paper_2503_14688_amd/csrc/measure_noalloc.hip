// spin_measure_noalloc: the measurement of spin_measure (paper Eqs. 2-3 and
// App. C) for callers that must not allocate device memory.  Its counters
// live in one file-scope device array per GPU instead of the handle's lazily
// allocated reduction buffer; the kernels are the ones spin_measure launches.
#include "host.hpp"

#include <cerrno>
#include <mutex>

#pragma clang fp contract(off)

namespace {

// Largest separation count one call accepts.
constexpr uint32_t kMaxR = 1024;
// Layout (64-bit words): the reduction counters as spin_measure lays them
// out (4 energy/magnetisation counters, then 2 per separation and axis), then
// the finished sums: sum_s, sum_s2, bond, Sx[n_r], Sy[n_r].
constexpr size_t kCounters = spin::kEmCounters + 4 * (size_t)kMaxR;
constexpr size_t kResults = 3 + 2 * (size_t)kMaxR;
constexpr size_t kScratchWords = kCounters + kResults;  // 49,208 bytes

static __device__ __align__(256) unsigned long long scratch[kScratchWords];

constexpr int kMaxDevices = 64;
std::mutex g_lock;                        // one call at a time per process
unsigned long long *g_ptr[kMaxDevices];   // device address of scratch, per GPU

// Turn the counters into the signed sums (the arithmetic spin_measure does on
// the host): S(r) = (#pairs with both ends non-zero) - 2 (#such pairs
// anti-aligned), and every pair counts for Ising.
__global__ void k_finish_sums(const unsigned long long *acc, long long *res, int model, uint32_t L, uint32_t n_r)
{
    const long long all_pairs = (long long)L * (long long)L;
    const size_t bx = spin::kEmCounters, by = bx + 2 * (size_t)n_r;
    for (uint32_t q = threadIdx.x; q < 3 + 2 * n_r; q += blockDim.x) {
        long long v;
        if (q == 0) {
            v = (long long)acc[0] - 2 * (long long)acc[1];
        } else if (q == 1) {
            v = (long long)acc[0];
        } else if (q == 2) {
            v = (long long)acc[2] - 2 * (long long)acc[3];
        } else {
            const uint32_t k = q - 3;
            const size_t base = k < n_r ? bx + 2 * (size_t)k : by + 2 * (size_t)(k - n_r);
            const long long pairs = model == SPIN_ISING ? all_pairs : (long long)acc[base];
            v = pairs - 2 * (long long)acc[base + 1];
        }
        res[q] = v;
    }
}

// Device address of this GPU's scratch array, looked up once per device with
// that device current.  Called with g_lock held.
int scratch_on(int device, unsigned long long **out)
{
    if (device < 0 || device >= kMaxDevices)
        return spin_host::fail(-EINVAL, "device %d outside 0..%d", device, kMaxDevices - 1);
    if (!g_ptr[device]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        g_ptr[device] = (unsigned long long *)p;
    }
    *out = g_ptr[device];
    return 0;
}

int measure(spin_handle *h, const uint32_t *r, uint32_t n_r, spin_meas *out, int64_t *Sx, int64_t *Sy,
            double *C_hat)
{
    unsigned long long *acc = nullptr;
    if (int rc = scratch_on(h->device, &acc))
        return rc;
    long long *res = (long long *)(acc + kCounters);
    const size_t base_x = spin::kEmCounters, base_y = base_x + 2 * (size_t)n_r;
    // every counter this call uses starts at zero (the array keeps the last
    // call's contents)
    HIP_TRY(spin::launch_fill_u64(acc, base_y + 2 * (size_t)n_r, 0ull, h->stream), "fill kernel launch");
    HIP_TRY(spin::launch_measure_em(h->lat, acc, h->stream), "measure kernel launch");
    for (int axis = 0; axis < 2 && n_r > 0; ++axis) {
        const bool vertical = axis == 1;
        unsigned long long *dst = acc + (vertical ? base_y : base_x);
        const bool fast = vertical ? spin::corr_sparse_y_ok(h->lat, r, (int)n_r)
                                   : spin::corr_sparse_x_ok(h->lat, r, (int)n_r);
        if (fast) {
            HIP_TRY(spin::launch_corr_sparse(h->lat, vertical, (int)n_r, dst, h->stream), "correlation kernel launch");
            continue;
        }
        for (uint32_t q0 = 0; q0 < n_r; q0 += spin::kCorrChunk) {
            const int cnt = (int)((n_r - q0) < (uint32_t)spin::kCorrChunk ? (n_r - q0) : spin::kCorrChunk);
            HIP_TRY(spin::launch_corr(h->lat, vertical, r + q0, cnt, dst + 2 * q0, h->stream),
                    "correlation kernel launch");
        }
    }
    hipLaunchKernelGGL(k_finish_sums, dim3(1), dim3(256), 0, h->stream, acc, res, h->model, h->L, n_r);
    HIP_TRY(hipGetLastError(), "finishing kernel launch");
    long long em[3];
    HIP_TRY(hipMemcpyAsync(em, res, sizeof em, hipMemcpyDeviceToHost, h->stream), "hipMemcpyAsync");
    if (n_r > 0) {
        HIP_TRY(hipMemcpyAsync(Sx, res + 3, n_r * sizeof(int64_t), hipMemcpyDeviceToHost, h->stream),
                "hipMemcpyAsync");
        HIP_TRY(hipMemcpyAsync(Sy, res + 3 + n_r, n_r * sizeof(int64_t), hipMemcpyDeviceToHost, h->stream),
                "hipMemcpyAsync");
    }
    HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    const double N = (double)h->L * (double)h->L;
    out->t = h->t;
    out->sum_s = em[0];
    out->sum_s2 = em[1];
    out->bond = em[2];
    out->e = (-h->J * (double)out->bond + h->Delta * (double)out->sum_s2) / N;
    out->m = (double)out->sum_s / N;
    out->xi = spin_host::xi_from_sums(r, Sx, Sy, n_r, N, (double)out->sum_s2 / N, C_hat);
    return 0;
}

} // namespace

extern "C" int spin_measure_noalloc(spin_handle *h, const uint32_t *r, uint32_t n_r, spin_meas *out, int64_t *Sx,
                                    int64_t *Sy, double *C_hat)
{
    if (!h)
        return spin_host::fail(-EINVAL, "NULL handle");
    if (!out)
        return spin_host::fail(-EINVAL, "NULL result pointer");
    if (n_r > kMaxR)
        return spin_host::fail(-EINVAL, "%u separations requested, at most %u without allocation", n_r, kMaxR);
    if (n_r > 0 && (!r || !Sx || !Sy))
        return spin_host::fail(-EINVAL, "NULL separation or output array");
    for (uint32_t q = 0; q < n_r; ++q) {
        if (r[q] == 0 || r[q] >= h->L || (q > 0 && r[q] <= r[q - 1]))
            return spin_host::fail(-EINVAL, "separations must be strictly increasing in (0, L)");
    }
    std::lock_guard<std::mutex> hold(g_lock);
    int current = 0;
    HIP_TRY(hipGetDevice(&current), "hipGetDevice");
    if (current != h->device)
        HIP_TRY(hipSetDevice(h->device), "hipSetDevice");
    const int rc = measure(h, r, n_r, out, Sx, Sy, C_hat);
    if (current != h->device)
        (void)hipSetDevice(current);
    return rc;
}
