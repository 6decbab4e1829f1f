/*
 * CPU oracle for the equilibrium Blume-Capel machinery of the paper's App. B
 * (critical temperature of the Blume-Capel model at Delta = 0): the
 * Swendsen-Wang cluster update restricted to the sites with s = +-1, and the
 * Fourier moments of the spin field behind the Binder cumulant and the
 * second-moment correlation length.
 *
 * TEST INFRASTRUCTURE ONLY, like spin_oracle.c: only the tests, the smoke
 * check and the CPU-baseline leg of the benchmark use it, and it shares no
 * code with the HIP library.
 *
 * Swendsen-Wang (Swendsen and Wang, PRL 58, 86 (1987)) on H = -J sum s_x s_y
 * + Delta sum s_x^2: with s^2 held fixed the signs of the non-zero spins are
 * an Ising model on the graph of bonds between two non-zero sites, so every
 * such bond whose two spins agree is activated with probability
 * p = 1 - exp(-2J / T); the connected components of the active bonds
 * (clusters) are flipped, each with probability 1/2.  Vacancies (s = 0) keep
 * their value.  For the Ising model every site is non-zero and this is the
 * plain Swendsen-Wang algorithm.
 *
 * Random stream of one Swendsen-Wang step at sweep index t (the step takes
 * one sweep index, like a Metropolis sweep; key = (seed mod 2^32, seed >> 32)):
 *   bonds: Philox4x32-10 at counter (i, j, t, 3 << 16) gives four words; word
 *          0 is the uniform u of the bond from (i, j) to (i, j + 1), word 1
 *          that of the bond from (i, j) to (i + 1, j) (periodic).  A bond is
 *          active iff both spins are non-zero and equal and u < thr, with
 *          thr = floor(2^32 p) in IEEE double and C library exp, and every
 *          agreeing bond active when 2^32 p reaches 2^32 (T = 0).
 *   flips: a cluster is named by the smallest linear index n = i L + j of its
 *          sites; it flips iff word 0 of Philox4x32-10 at counter
 *          (n mod 2^32, n >> 32, t, 4 << 16) is >= 2^31.
 *
 * Clusters are found by the textbook method: visit the sites in raster order
 * and grow the cluster of every site not yet labelled by a depth-first walk
 * over its active bonds.  The first site of a cluster met in raster order is
 * its smallest index, which is the cluster's name.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

#define ORC_PURPOSE_SW_BOND 3u
#define ORC_PURPOSE_SW_FLIP 4u

/* Integer bond rule: returns 1 when every agreeing bond is active, else 0
 * with *thr = floor(2^32 p). */
int orc_sw_threshold(double J, double T, uint32_t *thr)
{
    double p = 1.0 - exp(-2.0 * J / T);
    double x = ldexp(p, 32);
    *thr = 0;
    if (x >= 4294967296.0)
        return 1;
    *thr = (uint32_t)floor(x);
    return 0;
}

static void bond_words(uint64_t seed, uint32_t t, uint32_t i, uint32_t j, uint32_t out[4])
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {i, j, t, ORC_PURPOSE_SW_BOND << 16};
    orc_philox4x32_10(ctr, key, out);
}

static int cluster_flips(uint64_t seed, uint32_t t, uint64_t n)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {(uint32_t)n, (uint32_t)(n >> 32), t, ORC_PURPOSE_SW_FLIP << 16};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return out[0] >= 0x80000000u;
}

/* Active bonds of the configuration: right[x] (x to its right neighbour) and
 * down[x] (x to the site below), 1 if active. */
static void active_bonds(int L, uint64_t seed, double J, double T, uint32_t t, const int8_t *s, uint8_t *right,
                         uint8_t *down)
{
    uint32_t thr;
    const int always = orc_sw_threshold(J, T, &thr);
    for (int i = 0; i < L; ++i) {
        for (int j = 0; j < L; ++j) {
            const size_t x = (size_t)i * L + j;
            const int8_t v = s[x];
            const int8_t vr = s[(size_t)i * L + (j + 1) % L];
            const int8_t vd = s[(size_t)((i + 1) % L) * L + j];
            uint32_t u[4];
            bond_words(seed, t, (uint32_t)i, (uint32_t)j, u);
            right[x] = v != 0 && v == vr && (always || u[0] < thr);
            down[x] = v != 0 && v == vd && (always || u[1] < thr);
        }
    }
}

/* Cluster names: label[x] = smallest linear index of x's cluster (raster-order
 * depth-first labelling with an explicit stack). */
static int label_clusters(int L, const uint8_t *right, const uint8_t *down, uint64_t *label)
{
    const size_t N = (size_t)L * L;
    size_t *stack = (size_t *)malloc(N * sizeof(size_t));
    if (!stack)
        return -12;
    for (size_t x = 0; x < N; ++x)
        label[x] = UINT64_MAX;
    for (size_t root = 0; root < N; ++root) {
        if (label[root] != UINT64_MAX)
            continue;
        size_t top = 0;
        stack[top++] = root;
        label[root] = root;
        while (top > 0) {
            const size_t x = stack[--top];
            const int i = (int)(x / L), j = (int)(x % L);
            /* the four bonds of x: its own right/down, and the left/up
             * neighbours' right/down */
            const size_t nb[4] = {(size_t)i * L + (j + 1) % L, (size_t)((i + 1) % L) * L + j,
                                  (size_t)i * L + (j + L - 1) % L, (size_t)((i + L - 1) % L) * L + j};
            const int on[4] = {right[x], down[x], right[nb[2]], down[nb[3]]};
            for (int q = 0; q < 4; ++q) {
                if (on[q] && label[nb[q]] == UINT64_MAX) {
                    label[nb[q]] = root;
                    stack[top++] = nb[q];
                }
            }
        }
    }
    free(stack);
    return 0;
}

/* n Swendsen-Wang steps at bath temperatures T[k] and sweep indices t0 + k.
 * labels (may be NULL) receives the cluster names of the last step. */
int orc_sw(int model, int L, uint64_t seed, double J, int8_t *s, uint32_t t0, uint32_t n, const double *T,
           uint64_t *labels)
{
    if ((model != 0 && model != 1) || L < 2 || !(J > 0.0))
        return -22;
    for (uint32_t k = 0; k < n; ++k)
        if (!(T[k] >= 0.0))
            return -22;
    const size_t N = (size_t)L * L;
    uint8_t *right = (uint8_t *)malloc(N), *down = (uint8_t *)malloc(N);
    uint64_t *label = labels ? labels : (uint64_t *)malloc(N * sizeof(uint64_t));
    int rc = (!right || !down || !label) ? -12 : 0;
    for (uint32_t k = 0; k < n && rc == 0; ++k) {
        const uint32_t t = t0 + k;
        active_bonds(L, seed, J, T[k], t, s, right, down);
        rc = label_clusters(L, right, down, label);
        if (rc)
            break;
        for (size_t x = 0; x < N; ++x)
            if (s[x] != 0 && cluster_flips(seed, t, label[x]))
                s[x] = (int8_t)-s[x];
    }
    free(right);
    free(down);
    if (!labels)
        free(label);
    return rc;
}

/* Fourier moments of the spin field (App. B): M(k) = sum_x exp(i k.x) s_x with
 * x = (i, j).  out[0] = M(0); out[1], out[2] = real and imaginary parts of
 * M(2 pi / L, 0) (phase 2 pi i / L, along the rows' index i); out[3], out[4]
 * those of M(0, 2 pi / L) (phase 2 pi j / L).  Straight double sum. */
int orc_fourier(int L, const int8_t *s, double out[5])
{
    if (L < 2)
        return -22;
    const double two_pi = 2.0 * acos(-1.0);
    double m0 = 0.0, re1 = 0.0, im1 = 0.0, re2 = 0.0, im2 = 0.0;
    for (int i = 0; i < L; ++i) {
        for (int j = 0; j < L; ++j) {
            const double v = (double)s[(size_t)i * L + j];
            const double a = two_pi * (double)i / (double)L, b = two_pi * (double)j / (double)L;
            m0 += v;
            re1 += v * cos(a);
            im1 += v * sin(a);
            re2 += v * cos(b);
            im2 += v * sin(b);
        }
    }
    out[0] = m0;
    out[1] = re1;
    out[2] = im1;
    out[3] = re2;
    out[4] = im2;
    return 0;
}
