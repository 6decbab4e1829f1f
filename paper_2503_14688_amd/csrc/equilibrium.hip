// C ABI of the equilibrium study of the Blume-Capel critical temperature
// (paper App. B): the Swendsen-Wang step restricted to s = +-1 and the
// Fourier moments M(0), M(k_min) behind the Binder cumulant and the
// second-moment correlation length.  Host side: argument checks, the integer
// bond rule in host FP64, launch sequencing, and the FP64 Fourier sums from
// the exact row and column sums.
#include "host.hpp"

#include <cerrno>
#include <cmath>
#include <vector>

#pragma clang fp contract(off)

using namespace spin_host;

namespace spin_host {

// Bond rule of the Swendsen-Wang step: a bond between equal non-zero spins is
// active with probability p = 1 - exp(-2J/T); in integers, u < floor(2^32 p),
// or always when 2^32 p reaches 2^32.
bool sw_rule(double J, double T, uint32_t *thr)
{
    const double p = 1.0 - std::exp(-2.0 * J / T);
    const double x = std::ldexp(p, 32);
    *thr = 0;
    if (x >= 4294967296.0)
        return true;
    *thr = (uint32_t)std::floor(x);
    return false;
}

void finish_fourier(const spin_handle *h, const unsigned long long *acc, const long long *lines, spin_fourier *out)
{
    const uint32_t L = h->L;
    const double N = (double)L * (double)L;
    out->t = h->t;
    out->sum_s = (int64_t)acc[0] - 2 * (int64_t)acc[1];
    out->sum_s2 = (int64_t)acc[0];
    out->bond = (int64_t)acc[2] - 2 * (int64_t)acc[3];
    out->e = (-h->J * (double)out->bond + h->Delta * (double)out->sum_s2) / N;
    // M(k) = sum_x exp(i k.x) s_x for k = (2 pi / L, 0) and (0, 2 pi / L):
    // the phase depends on one coordinate only, so M(k) is the discrete
    // Fourier sum of the row (resp. column) sums
    const double two_pi = 2.0 * std::acos(-1.0);
    double re1 = 0.0, im1 = 0.0, re2 = 0.0, im2 = 0.0;
    for (uint32_t q = 0; q < L; ++q) {
        const double a = two_pi * (double)q / (double)L;
        const double ca = std::cos(a), sa = std::sin(a);
        re1 += (double)lines[q] * ca;
        im1 += (double)lines[q] * sa;
        re2 += (double)lines[L + q] * ca;
        im2 += (double)lines[L + q] * sa;
    }
    out->re_k1 = re1;
    out->im_k1 = im1;
    out->re_k2 = re2;
    out->im_k2 = im2;
}

} // namespace spin_host

extern "C" {

int spin_sw(spin_handle *h, uint32_t n, const double *T)
{
    if (!h)
        return fail(-EINVAL, "NULL handle");
    if (n > 0 && !T)
        return fail(-EINVAL, "NULL temperature array");
    if (h->batch_owned)
        return fail(-EINVAL, "the handle belongs to a batch: advance it with spin_batch_run");
    if (h->L > kMaxSwL)
        return fail(-EINVAL, "Swendsen-Wang steps need L <= %u (got %u)", kMaxSwL, h->L);
    if (h->t + n > (1ull << 32))
        return fail(-EINVAL, "sweep index would pass 2^32");
    for (uint32_t k = 0; k < n; ++k)
        if (!(T[k] >= 0.0))
            return fail(-EINVAL, "T[%u] = %g is negative or NaN", k, T[k]);
    if (n == 0)
        return 0;
    if (!h->d_labels) {
        hipError_t e = hipMalloc(&h->d_labels, (size_t)h->L * h->L * sizeof(uint32_t));
        if (e != hipSuccess) {
            h->d_labels = nullptr;
            return fail(-ENOMEM, "cluster labels for L = %u: %s", h->L, hipGetErrorString(e));
        }
    }
    for (uint32_t k = 0; k < n; ++k) {
        uint32_t thr;
        const bool always = sw_rule(h->J, T[k], &thr);
        HIP_TRY(spin::launch_sw_step(h->lat, (uint32_t)(h->t + k), thr, always, h->d_labels, h->stream),
                "Swendsen-Wang launch");
    }
    h->t += n;
    h->em_valid = false;
    return 0;
}

int spin_measure_fourier(spin_handle *h, spin_fourier *out, int64_t *row_sums, int64_t *col_sums)
{
    if (!h)
        return fail(-EINVAL, "NULL handle");
    if (!out)
        return fail(-EINVAL, "NULL result pointer");
    const uint32_t L = h->L;
    if (!h->d_lines) {
        hipError_t e = hipMalloc(&h->d_lines, 2 * (size_t)L * sizeof(long long));
        if (e != hipSuccess) {
            h->d_lines = nullptr;
            return fail(-ENOMEM, "row and column sums: %s", hipGetErrorString(e));
        }
    }
    if (int rc = ensure_acc(h, spin::kEmCounters))
        return rc;
    if (!h->em_valid) {
        HIP_TRY(spin::launch_fill_u64(h->d_acc, spin::kEmCounters, 0ull, h->stream), "fill kernel launch");
        HIP_TRY(spin::launch_measure_em(h->lat, h->d_acc, h->stream), "measure kernel launch");
        h->em_valid = true;
    }
    long long *row = h->d_lines, *col = h->d_lines + L;
    HIP_TRY(spin::launch_fill_u64((unsigned long long *)col, L, 0ull, h->stream), "fill kernel launch");
    HIP_TRY(spin::launch_line_sums(h->lat, row, col, h->stream), "line-sum kernel launch");
    std::vector<long long> lines(2 * (size_t)L);
    unsigned long long acc[spin::kEmCounters];
    HIP_TRY(hipMemcpyAsync(lines.data(), h->d_lines, lines.size() * sizeof(long long), hipMemcpyDeviceToHost,
                           h->stream),
            "hipMemcpyAsync");
    HIP_TRY(hipMemcpyAsync(acc, h->d_acc, sizeof acc, hipMemcpyDeviceToHost, h->stream), "hipMemcpyAsync");
    HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    finish_fourier(h, acc, lines.data(), out);
    for (uint32_t q = 0; row_sums && q < L; ++q)
        row_sums[q] = lines[q];
    for (uint32_t q = 0; col_sums && q < L; ++q)
        col_sums[q] = lines[L + q];
    return 0;
}

} // extern "C"
