// Host-side internals shared by the C ABI translation units (not public).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/spin.h"
#include "kernels.hpp"

using spin::GroupTable;

struct spin_handle {
    spin::Lattice lat;
    int model;
    uint32_t L;
    uint64_t seed;
    double J, Delta;
    void *buf;
    size_t buf_bytes;
    hipStream_t stream;
    uint64_t t;
    unsigned long long *d_acc;  // [4 EM counters | corr counters]
    size_t acc_cap;             // entries
    int8_t *d_win;
    size_t win_cap;             // bytes
    bool em_valid;              // d_acc[0..3] describe the current state
    int device;                 // HIP device holding the lattice buffer
    uint32_t *d_labels;         // Swendsen-Wang cluster forest, L * L entries once used
    long long *d_lines;         // row and column sums, 2 L entries once used
    bool batch_owned;           // advanced only through its batch (spin_batch_run)
};

namespace spin_host {

// Record a failure for spin_last_error() and return code.
int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
// Acceptance-group table of a model at bath temperature T (host FP64 exp),
// for the lattice's Blume-Capel group layout bc_groups.
GroupTable make_groups(int model, uint32_t bc_groups, double J, double Delta, double T);
int ensure_acc(spin_handle *h, size_t entries);
// Measurement in two halves: queue the correlation kernels of n_r
// separations into acc (laid out as spin_measure's counters: 4 energy /
// magnetisation counters, then 2 per separation for x, then for y), and
// turn copied-back counters into the results.
size_t measure_counters(uint32_t n_r);
int queue_correlations(const spin::Lattice &lat, const uint32_t *r, uint32_t n_r, unsigned long long *acc,
                       hipStream_t st);
void finish_measure(const spin_handle *h, const unsigned long long *acc, const uint32_t *r, uint32_t n_r,
                    spin_meas *out, int64_t *Sx, int64_t *Sy, double *C_hat);
// Swendsen-Wang steps (paper App. B): largest L of the cluster forest (labels
// are 32-bit site indices), the integer bond rule at bath temperature T
// (returns true when every bond between equal non-zero spins is active,
// else sets *thr), and the Fourier moments from copied-back E/M counters and
// row / column sums (lines[0..L) rows, lines[L..2L) columns).
constexpr uint32_t kMaxSwL = 32768;
bool sw_rule(double J, double T, uint32_t *thr);
void finish_fourier(const spin_handle *h, const unsigned long long *acc, const long long *lines, spin_fourier *out);
// Coherence length I2 / I1 (trapezoid rule up to the first non-positive
// C-hat) from the correlation sums; writes C-hat(r_q) when C_hat is not NULL.
double xi_from_sums(const uint32_t *r, const int64_t *Sx, const int64_t *Sy, uint32_t n_r, double N, double C0,
                    double *C_hat);

} // namespace spin_host

#define HIP_TRY(expr, what)                                                                                  \
    do {                                                                                                     \
        hipError_t e_ = (expr);                                                                              \
        if (e_ != hipSuccess)                                                                                \
            return spin_host::hip_fail(e_, what);                                                            \
    } while (0)
