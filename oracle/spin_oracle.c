/*
 * CPU oracle for the checkerboard Metropolis dynamics of the 2D Ising and
 * spin-1 Blume-Capel models (Bisson et al., "Universal exotic dynamics in
 * critical mesoscopic systems", arXiv:2503.14688).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may load this file:
 * only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark use it.  It shares no code, header, table or helper with the HIP
 * library; the two meet only through the published definitions restated here.
 *
 * Plain and slow on purpose: int8 spins, one site at a time, the energy change
 * taken straight from the Hamiltonian, a fresh exp() per attempted move, and
 * correlation sums by the brute-force double loop.  OpenMP splits the rows of
 * one colour, which never changes a result (sites of one colour are never
 * neighbours when L is even).
 *
 * Definitions followed:
 *   Hamiltonian      H = -J sum_<x,y> s_x s_y + Delta sum_x s_x^2, periodic
 *                    L x L square lattice (paper Eq. 1); Ising is s = +-1.
 *   Dynamics         single-spin-flip Metropolis with the checkerboard split
 *                    (paper, Introduction: multispin coding, checkerboard and
 *                    domain decomposition).  Colour c = (i + j) & 1; colour 0
 *                    is updated first, then colour 1; one sweep = both.
 *   Randomness       the paper says only that its generator works on 32-bit
 *                    integers (App. B).  Here it is Philox4x32-10
 *                    (Salmon, Moraes, Dror, Shaw, SC'11) and the bit-plane
 *                    uniform below.
 *   Observables      C(r;t) as the normalised sum over pairs at separation r
 *                    (paper Eq. 2); the energy from r = (1,0) and (0,1)
 *                    (paper Eq. 3, read with the minus sign of H).
 *
 * Random stream (one definition for all three purposes):
 *   key      = (seed mod 2^32, seed >> 32)
 *   counter  = (i, w, t, purpose << 16 | c << 8 | blk),   blk in [0, 8)
 *   site (i, j) of colour c has m = j >> 1, w = m >> 5, b = m & 31
 *   plane k (k in [0, 32)) = output word (k & 3) of the call with blk = k >> 2
 *   u(site) = sum_k bit_b(plane k) << (31 - k)        (plane 0 is the MSB)
 *   purpose 0 = initial state (t = 0), 1 = acceptance, 2 = proposal (BC).
 *
 * Acceptance threshold: thr(dE, T) = floor(2^32 exp(-dE / T)) in IEEE double
 * with the C library exp; a move is accepted iff dE <= 0, or 2^32 exp(-dE/T)
 * reaches 2^32 (T = +inf), or u < thr.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_ISING 0
#define ORC_BC 1

#define ORC_PURPOSE_INIT 0u
#define ORC_PURPOSE_ACCEPT 1u
#define ORC_PURPOSE_PROPOSE 2u

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (SC'11, "Parallel random numbers: as easy as 1, 2, 3").    */
/* Round: two 32x32->64 products of counter words 0 and 2 with the          */
/* multipliers, the high halves xored with the other counter words and the  */
/* round key, words permuted; the key grows by the Weyl constants between   */
/* rounds.                                                                  */
/* ------------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* The 32 bit planes of word w of row i, colour c, sweep t, for a purpose. */
static void word_planes(uint64_t seed, uint32_t purpose, uint32_t t, uint32_t c,
                        uint32_t i, uint32_t w, uint32_t planes[32])
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (uint32_t blk = 0; blk < 8; ++blk) {
        uint32_t ctr[4] = {i, w, t, (purpose << 16) | (c << 8) | blk};
        uint32_t out[4];
        orc_philox4x32_10(ctr, key, out);
        for (int q = 0; q < 4; ++q)
            planes[4 * blk + q] = out[q];
    }
}

/* Lane b's 32-bit uniform, plane 0 as the most significant bit. */
static uint32_t assemble(const uint32_t planes[32], uint32_t b)
{
    uint32_t u = 0;
    for (int k = 0; k < 32; ++k)
        u |= ((planes[k] >> b) & 1u) << (31 - k);
    return u;
}

uint32_t orc_uniform(uint64_t seed, uint32_t purpose, uint32_t t, uint32_t c,
                     uint32_t i, uint32_t m)
{
    uint32_t planes[32];
    word_planes(seed, purpose, t, c, i, m >> 5, planes);
    return assemble(planes, m & 31u);
}

/* ------------------------------------------------------------------------ */
/* Metropolis acceptance in integers.                                        */
/* Returns 1 when the move is accepted without a random number, 0 when      */
/* u < *thr decides (thr = 0 rejects every u).                              */
/* ------------------------------------------------------------------------ */
int orc_threshold(double dE, double T, uint32_t *thr)
{
    *thr = 0;
    if (dE <= 0.0)
        return 1;
    double p = exp(-dE / T);
    double x = ldexp(p, 32);
    if (x >= 4294967296.0)
        return 1;
    *thr = (uint32_t)floor(x);
    return 0;
}

/* Energy change of s -> sp with neighbour sum h, straight from Eq. 1. */
static double delta_energy(double J, double Delta, int s, int sp, int h)
{
    int dh = (sp - s) * h;
    int q = sp * sp - s * s;
    return -J * (double)dh + Delta * (double)q;
}

static int valid_model(int model) { return model == ORC_ISING || model == ORC_BC; }

/* ------------------------------------------------------------------------ */
/* Initial state: T = infinity (paper, thermal protocols).                  */
/* ------------------------------------------------------------------------ */
static int8_t initial_spin(int model, uint32_t u)
{
    if (model == ORC_ISING)
        return (int8_t)(u < 0x80000000u ? 1 : -1);
    /* uniform over {-1, 0, +1}: floor(3u / 2^32) - 1 */
    return (int8_t)((int)((3ull * (uint64_t)u) >> 32) - 1);
}

int orc_init(int model, int L, uint64_t seed, int8_t *s)
{
    if (!valid_model(model) || L < 4 || (L & 1))
        return -22;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < L; ++i) {
        for (int j = 0; j < L; ++j) {
            uint32_t c = (uint32_t)((i + j) & 1);
            uint32_t u = orc_uniform(seed, ORC_PURPOSE_INIT, 0, c, (uint32_t)i, (uint32_t)(j >> 1));
            s[(size_t)i * L + j] = initial_spin(model, u);
        }
    }
    return 0;
}

/* Initial state of a window of the L x L lattice, rows i0.., columns j0..
 * (periodic), as orc_init would produce there. */
int orc_init_window(int model, int L, uint64_t seed, int i0, int j0, int H, int W, int8_t *win)
{
    if (!valid_model(model) || L < 4 || (L & 1) || H <= 0 || W <= 0)
        return -22;
    for (int a = 0; a < H; ++a) {
        int i = (int)(((int64_t)i0 + a) % L);
        for (int b = 0; b < W; ++b) {
            int j = (int)(((int64_t)j0 + b) % L);
            uint32_t c = (uint32_t)((i + j) & 1);
            uint32_t u = orc_uniform(seed, ORC_PURPOSE_INIT, 0, c, (uint32_t)i, (uint32_t)(j >> 1));
            win[(size_t)a * W + b] = initial_spin(model, u);
        }
    }
    return 0;
}

/* One attempted move at (i, j); nb = sum of the four neighbours.
 * Returns the new spin, adds the accepted energy change to *dE_acc. */
static int8_t attempt(int model, double J, double Delta, double T, int s, int h,
                      uint32_t u_acc, uint32_t u_prop, double *dE_acc)
{
    int sp;
    if (model == ORC_ISING) {
        sp = -s;
    } else {
        int x = u_prop >= 0x80000000u;
        if (s != 0)
            sp = x ? -s : 0;
        else
            sp = x ? -1 : 1;
    }
    double dE = delta_energy(J, Delta, s, sp, h);
    uint32_t thr;
    int accept = orc_threshold(dE, T, &thr) || u_acc < thr;
    if (accept) {
        *dE_acc += dE;
        return (int8_t)sp;
    }
    return (int8_t)s;
}

/* n sweeps on the full lattice; sweep k uses bath temperature T[k] and
 * stream sweep index t0 + k.  If dE_out is not NULL, dE_out[2k + c] receives
 * the summed energy change of the moves accepted in half-sweep c of sweep k. */
int orc_sweep(int model, int L, uint64_t seed, double J, double Delta, int8_t *s,
              uint32_t t0, uint32_t n, const double *T, double *dE_out)
{
    if (!valid_model(model) || L < 4 || (L & 1))
        return -22;
    if (model == ORC_ISING && Delta != 0.0)
        return -22;
    for (uint32_t k = 0; k < n; ++k) {
        if (!(T[k] >= 0.0))
            return -22;
    }
    const int half = L / 2;
    const int words = (half + 31) / 32;
    for (uint32_t k = 0; k < n; ++k) {
        uint32_t t = t0 + k;
        for (uint32_t c = 0; c < 2; ++c) {
            double acc_total = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : acc_total)
            for (int i = 0; i < L; ++i) {
                uint32_t pa[32], pp[32];
                double acc_row = 0.0;
                for (int w = 0; w < words; ++w) {
                    word_planes(seed, ORC_PURPOSE_ACCEPT, t, c, (uint32_t)i, (uint32_t)w, pa);
                    if (model == ORC_BC)
                        word_planes(seed, ORC_PURPOSE_PROPOSE, t, c, (uint32_t)i, (uint32_t)w, pp);
                    for (int b = 0; b < 32; ++b) {
                        int m = 32 * w + b;
                        if (m >= half)
                            break;
                        int j = 2 * m + ((i + (int)c) & 1);
                        int up = (i + L - 1) % L, dn = (i + 1) % L;
                        int lf = (j + L - 1) % L, rt = (j + 1) % L;
                        int h = s[(size_t)up * L + j] + s[(size_t)dn * L + j] +
                                s[(size_t)i * L + lf] + s[(size_t)i * L + rt];
                        uint32_t ua = assemble(pa, (uint32_t)b);
                        uint32_t up_ = model == ORC_BC ? assemble(pp, (uint32_t)b) : 0u;
                        int8_t *site = &s[(size_t)i * L + j];
                        *site = attempt(model, J, Delta, T[k], *site, h, ua, up_, &acc_row);
                    }
                }
                acc_total += acc_row;
            }
            if (dE_out)
                dE_out[2 * k + c] = acc_total;
        }
    }
    return 0;
}

/* Light-cone evolution of a window.  win holds the sites (i0 + a, j0 + b)
 * (periodic in the L x L lattice) for a < H, b < W.  Each half-sweep updates
 * only the sites whose four neighbours are still exact; the exact region
 * shrinks by one site per half-sweep, so after n sweeps the sites with
 * 2n <= a < H - 2n and 2n <= b < W - 2n equal those of the full run. */
int orc_window_sweep(int model, int L, uint64_t seed, double J, double Delta, int8_t *win,
                     int i0, int j0, int H, int W, uint32_t t0, uint32_t n, const double *T)
{
    if (!valid_model(model) || L < 4 || (L & 1) || H <= 0 || W <= 0)
        return -22;
    if (model == ORC_ISING && Delta != 0.0)
        return -22;
    int lo_a = 0, hi_a = H, lo_b = 0, hi_b = W;
    for (uint32_t k = 0; k < n; ++k) {
        if (!(T[k] >= 0.0))
            return -22;
        uint32_t t = t0 + k;
        for (uint32_t c = 0; c < 2; ++c) {
            double dummy = 0.0;
            for (int a = lo_a + 1; a < hi_a - 1; ++a) {
                int i = (int)(((int64_t)i0 + a) % L);
                for (int b = lo_b + 1; b < hi_b - 1; ++b) {
                    int j = (int)(((int64_t)j0 + b) % L);
                    if ((uint32_t)((i + j) & 1) != c)
                        continue;
                    int m = j >> 1;
                    uint32_t ua = orc_uniform(seed, ORC_PURPOSE_ACCEPT, t, c, (uint32_t)i, (uint32_t)m);
                    uint32_t up_ = model == ORC_BC
                                       ? orc_uniform(seed, ORC_PURPOSE_PROPOSE, t, c, (uint32_t)i, (uint32_t)m)
                                       : 0u;
                    int h = win[(size_t)(a - 1) * W + b] + win[(size_t)(a + 1) * W + b] +
                            win[(size_t)a * W + b - 1] + win[(size_t)a * W + b + 1];
                    int8_t *site = &win[(size_t)a * W + b];
                    *site = attempt(model, J, Delta, T[k], *site, h, ua, up_, &dummy);
                }
            }
            lo_a++; hi_a--; lo_b++; hi_b--;
            if (lo_a >= hi_a || lo_b >= hi_b)
                return -33; /* window too small for n sweeps */
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Measurements by the brute-force definition of Eq. 2 (unnormalised sums).  */
/*   sums[0] = sum s, sums[1] = sum s^2,                                     */
/*   sums[2] = bond sum over nearest-neighbour pairs = Sx(1) + Sy(1)         */
/*   Sx[q] = sum_{i,j} s(i,j) s(i, j + r_q),  Sy[q] = sum s(i,j) s(i + r_q, j) */
/* ------------------------------------------------------------------------ */
int orc_measure(int L, const int8_t *s, const uint32_t *r, int nr, int64_t sums[3],
                int64_t *Sx, int64_t *Sy)
{
    if (L < 2 || nr < 0)
        return -22;
    int64_t s1 = 0, s2 = 0, bond = 0;
#pragma omp parallel for schedule(static) reduction(+ : s1, s2, bond)
    for (int i = 0; i < L; ++i) {
        for (int j = 0; j < L; ++j) {
            int v = s[(size_t)i * L + j];
            s1 += v;
            s2 += v * v;
            bond += v * s[(size_t)i * L + (j + 1) % L];
            bond += v * s[(size_t)((i + 1) % L) * L + j];
        }
    }
    sums[0] = s1;
    sums[1] = s2;
    sums[2] = bond;
    for (int q = 0; q < nr; ++q) {
        int rr = (int)(r[q] % (uint32_t)L);
        int64_t sx = 0, sy = 0;
#pragma omp parallel for schedule(static) reduction(+ : sx, sy)
        for (int i = 0; i < L; ++i) {
            for (int j = 0; j < L; ++j) {
                int v = s[(size_t)i * L + j];
                sx += v * s[(size_t)i * L + (j + rr) % L];
                sy += v * s[(size_t)((i + rr) % L) * L + j];
            }
        }
        Sx[q] = sx;
        Sy[q] = sy;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Bath-temperature schedules T(t), t = 0-based sweep index (host FP64).     */
/*   kind 0: constant      T(t) = p0                      (protocol 1)       */
/*   kind 1: two-step      T(t) = p0 for t < p1, else p2  (protocol 2)       */
/*   kind 2: exponential   T(t) = p1 + (p0 - p1) exp(-t / p2)                */
/* ------------------------------------------------------------------------ */
int orc_schedule(int kind, const double *p, uint32_t t0, uint32_t n, double *out)
{
    for (uint32_t k = 0; k < n; ++k) {
        double t = (double)(t0 + k);
        switch (kind) {
        case 0: out[k] = p[0]; break;
        case 1: out[k] = t < p[1] ? p[0] : p[2]; break;
        case 2: out[k] = p[1] + (p[0] - p[1]) * exp(-t / p[2]); break;
        default: return -22;
        }
    }
    return 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}
