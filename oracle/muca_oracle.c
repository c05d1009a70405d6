/*
 * muca_oracle.c -- plain CPU oracle for the parallel multicanonical method.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * statement of what the GPU path computes.  It shares no code, header,
 * table or constant generator with the product library; only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark load it.
 *
 * Method (Gross, Zierenberg, Weigel, Janke, "Massively parallel
 * multicanonical simulations"):
 *   - 2D Ising model on a periodic L x L lattice, J = 1 (Sec. 3, Eq. 5).
 *     Energies E = -2N + 4k, k = 0..N, N = L*L; the bins k = 1 and
 *     k = N-1 (E = -(2N-4) and E = 2N-4) are forbidden (Sec. 3).
 *   - Multicanonical weights W(E) = exp(omega(E)) replace the Boltzmann
 *     factor (Sec. 2.1, Eqs. 1-3); the update of a single spin is accepted
 *     with probability min(1, exp[omega(E') - omega(E)]) (Sec. 2.3).
 *   - p walkers share one weight table and add their histograms
 *     H = sum_i H_i (Sec. 2.2, Fig. 1); the weights are then updated by
 *     W <- W / H, i.e. omega <- omega - ln H (Sec. 2.1, Eq. 4).
 *   - Random numbers come from the counter-based generator Philox4x32-10
 *     (Sec. 2.3; Salmon et al. 2011), labelled by walker and site.
 *   - A production run uses the same sweeps with frozen weights and gives
 *     ln Omega(E) = ln H(E) - omega(E) + const (Sec. 2.1, Sec. 3.3).
 *
 * Readings where the paper leaves details open (all listed in the design
 * notes of the repository):
 *   - typewriter site order i = y*L + x for every walker;
 *   - draw for (walker w, sweep t, site i) = word (i & 3) of
 *     Philox4x32-10(key = (seed, w), counter = (i >> 2, t mod 2^32, t >> 32, 0));
 *     the initial spins use counter word 3 = 1 and t = 0, spin = +1 iff the
 *     top bit of the draw is set;
 *   - acceptance is the integer comparison r < T[k][d] with
 *     T = floor(min(1, exp(omega[k'] - omega[k])) * 2^32) computed once per
 *     call from the double-precision log weights (T lies in [0, 2^32]);
 *   - the energy after every recorded attempt goes into the histogram;
 *   - empty bins keep their weight (H is read as max(H, 1));
 *   - flatness = min over reachable bins of H divided by their mean.
 *
 * No fused multiply-add or fast-math: build with plain -O2.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------------- */
/* Philox4x32-10, written out from its published definition:               */
/* ten rounds of two 32x32->64 multiplications, with the key bumped by the  */
/* Weyl constants before every round but the first.                         */
/* ---------------------------------------------------------------------- */
#define PHILOX_MUL_A 0xD2511F53u
#define PHILOX_MUL_B 0xCD9E8D57u
#define PHILOX_WEYL_A 0x9E3779B9u
#define PHILOX_WEYL_B 0xBB67AE85u

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_WEYL_A;
            k1 += PHILOX_WEYL_B;
        }
        uint64_t prod_a = (uint64_t)PHILOX_MUL_A * (uint64_t)c0;
        uint64_t prod_b = (uint64_t)PHILOX_MUL_B * (uint64_t)c2;
        uint32_t hi_a = (uint32_t)(prod_a >> 32), lo_a = (uint32_t)prod_a;
        uint32_t hi_b = (uint32_t)(prod_b >> 32), lo_b = (uint32_t)prod_b;
        uint32_t n0 = hi_b ^ c1 ^ k0;
        uint32_t n1 = lo_b;
        uint32_t n2 = hi_a ^ c3 ^ k1;
        uint32_t n3 = lo_a;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* One 32-bit draw for (walker, sweep, site) in the given domain
 * (0 = Metropolis acceptance, 1 = initial spins). */
uint32_t oracle_draw(uint32_t seed, uint32_t walker, uint64_t sweep, uint32_t site,
                     uint32_t domain)
{
    uint32_t ctr[4] = {site >> 2, (uint32_t)(sweep & 0xffffffffu), (uint32_t)(sweep >> 32),
                       domain};
    uint32_t key[2] = {seed, walker};
    uint32_t out[4];
    oracle_philox4x32_10(ctr, key, out);
    return out[site & 3];
}

/* ---------------------------------------------------------------------- */
/* Ising model on the periodic L x L lattice (Sec. 3, Eq. 5).              */
/* spins: int8 +1/-1, walker-major, site i = y*L + x.                       */
/* ---------------------------------------------------------------------- */
static int site_index(int L, int x, int y)
{
    x = ((x % L) + L) % L;
    y = ((y % L) + L) % L;
    return y * L + x;
}

/* E = -J sum over nearest-neighbour pairs s_i s_j, each bond once. */
int32_t oracle_energy(int L, const int8_t *spins)
{
    int32_t e = 0;
    for (int y = 0; y < L; ++y) {
        for (int x = 0; x < L; ++x) {
            int s = spins[site_index(L, x, y)];
            int right = spins[site_index(L, x + 1, y)];
            int down = spins[site_index(L, x, y + 1)];
            e -= s * (right + down);
        }
    }
    return e;
}

/* Initial spins and energies of n walkers; walker j carries the global index
 * ids[j] (ids == NULL: index j), which is the second word of its key. */
void oracle_init_ids(int L, int n, const uint32_t *ids, uint32_t seed, int8_t *spins,
                     int32_t *energies)
{
    int N = L * L;
    for (int j = 0; j < n; ++j) {
        uint32_t w = ids ? ids[j] : (uint32_t)j;
        int8_t *s = spins + (size_t)j * N;
        for (int i = 0; i < N; ++i) {
            uint32_t u = oracle_draw(seed, w, 0, (uint32_t)i, 1);
            s[i] = (u >> 31) ? 1 : -1;
        }
        energies[j] = oracle_energy(L, s);
    }
}

void oracle_init(int L, int W, uint32_t seed, int8_t *spins, int32_t *energies)
{
    oracle_init_ids(L, W, NULL, seed, spins, energies);
}

/* ---------------------------------------------------------------------- */
/* Acceptance thresholds: T[k*5 + d], d = 0..4 <-> Delta E = 4d - 8.        */
/* T = 0 when the target bin lies outside [0, N]; 2^32 when                 */
/* omega[k'] >= omega[k]; else floor(exp(omega[k'] - omega[k]) * 2^32).     */
/* ---------------------------------------------------------------------- */
void oracle_thresholds(int N, const double *omega, uint64_t *table)
{
    for (int k = 0; k <= N; ++k) {
        for (int d = 0; d < 5; ++d) {
            int kp = k + d - 2;
            uint64_t t;
            if (kp < 0 || kp > N) {
                t = 0;
            } else if (omega[kp] >= omega[k]) {
                t = (uint64_t)1 << 32;
            } else {
                double ratio = exp(omega[kp] - omega[k]);
                double scaled = ldexp(ratio, 32);
                t = (uint64_t)floor(scaled);
            }
            table[k * 5 + d] = t;
        }
    }
}

/* ---------------------------------------------------------------------- */
/* The chain (Sec. 2.3).  Attempts are numbered per walker from 0: attempt  */
/* p is made at site i = p mod N of sweep p div N (typewriter order), with  */
/* the draw of (sweep, site).  A call runs attempts pos0 .. pos0+count-1,   */
/* so it may start and stop inside a sweep; with record != 0 the energy bin */
/* after every attempt is counted.  hist (N+1 entries) is ADDED to.         */
/* ---------------------------------------------------------------------- */
static void walker_attempts(int L, uint32_t seed, uint32_t walker, int8_t *s, int32_t *energy,
                            const uint64_t *table, uint64_t pos0, uint64_t count, int record,
                            uint64_t *hist)
{
    int N = L * L;
    int32_t e = *energy;
    for (uint64_t p = pos0; p < pos0 + count; ++p) {
        uint64_t sweep = p / (uint64_t)N;
        int i = (int)(p % (uint64_t)N);
        uint32_t r = oracle_draw(seed, walker, sweep, (uint32_t)i, 0);
        int x = i % L, y = i / L;
        int nb = s[site_index(L, x - 1, y)] + s[site_index(L, x + 1, y)] +
                 s[site_index(L, x, y - 1)] + s[site_index(L, x, y + 1)];
        int de = 2 * s[i] * nb;
        int d = de / 4 + 2;
        int k = (e + 2 * N) / 4;
        if ((uint64_t)r < table[k * 5 + d]) {
            s[i] = (int8_t)(-s[i]);
            e += de;
        }
        if (record)
            hist[(e + 2 * N) / 4] += 1;
    }
    *energy = e;
}

void oracle_attempts_ids(int L, int n, const uint32_t *ids, uint32_t seed, int8_t *spins,
                         int32_t *energies, const uint64_t *table, uint64_t pos0, uint64_t count,
                         int record, uint64_t *hist, int nthreads)
{
    int N = L * L;
    int nt = 1;
#ifdef _OPENMP
    nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
#endif
    uint64_t *partial = (uint64_t *)calloc((size_t)nt * (N + 1), sizeof(uint64_t));
#pragma omp parallel for schedule(static) num_threads(nt)
    for (int j = 0; j < n; ++j) {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        uint32_t w = ids ? ids[j] : (uint32_t)j;
        walker_attempts(L, seed, w, spins + (size_t)j * N, energies + j, table, pos0, count,
                        record, partial + (size_t)tid * (N + 1));
    }
    for (int t = 0; t < nt; ++t)
        for (int k = 0; k <= N; ++k)
            hist[k] += partial[(size_t)t * (N + 1) + k];
    free(partial);
}

/* Whole sweeps sweep0 .. sweep0+nsweeps-1. */
void oracle_sweeps_ids(int L, int n, const uint32_t *ids, uint32_t seed, int8_t *spins,
                       int32_t *energies, const uint64_t *table, uint64_t sweep0,
                       uint32_t nsweeps, int record, uint64_t *hist, int nthreads)
{
    uint64_t N = (uint64_t)L * L;
    oracle_attempts_ids(L, n, ids, seed, spins, energies, table, sweep0 * N, nsweeps * N, record,
                        hist, nthreads);
}

void oracle_sweeps(int L, int W, uint32_t seed, int8_t *spins, int32_t *energies,
                   const uint64_t *table, uint64_t sweep0, uint32_t nsweeps, int record,
                   uint64_t *hist, int nthreads)
{
    oracle_sweeps_ids(L, W, NULL, seed, spins, energies, table, sweep0, nsweeps, record, hist,
                      nthreads);
}

/* ---------------------------------------------------------------------- */
/* Weight update (Sec. 2.1, Eq. 4): omega <- omega - ln H for H > 0.        */
/* ---------------------------------------------------------------------- */
void oracle_reweight(int N, double *omega, const uint64_t *hist)
{
    for (int k = 0; k <= N; ++k)
        if (hist[k] > 0)
            omega[k] -= log((double)hist[k]);
}

static int reachable(int N, int k) { return k != 1 && k != N - 1; }

/* min H / mean H over the N - 1 reachable bins. */
double oracle_flatness(int N, const uint64_t *hist)
{
    uint64_t sum = 0, mn = UINT64_MAX;
    for (int k = 0; k <= N; ++k) {
        if (!reachable(N, k))
            continue;
        sum += hist[k];
        if (hist[k] < mn)
            mn = hist[k];
    }
    if (sum == 0)
        return 0.0;
    double mean = (double)sum / (double)(N - 1);
    return (double)mn / mean;
}

/* Chebyshev distance (App. A, Eq. A.1): max |H/m - 1| over reachable bins,
 * m = (sum H) / (N - 1). */
double oracle_chebyshev(int N, const uint64_t *hist)
{
    uint64_t sum = 0;
    for (int k = 0; k <= N; ++k)
        if (reachable(N, k))
            sum += hist[k];
    if (sum == 0)
        return 0.0;
    double m = (double)sum / (double)(N - 1);
    double best = 0.0;
    for (int k = 0; k <= N; ++k) {
        if (!reachable(N, k))
            continue;
        double dev = fabs((double)hist[k] / m - 1.0);
        if (dev > best)
            best = dev;
    }
    return best;
}

/* Kullback-Leibler divergence (Sec. 3, Eq. 6) of P = H / sum H from the
 * flat Q = 1/w, w = max(w_prev, 10), with w_prev the number of reachable bins
 * inside the energy range the previous histogram covered (0 at first).  The
 * paper counts L^2 - 1 accessible energies; Q over reachable bins makes a
 * flat histogram on the full range give d_k = 0.  Empty bins contribute
 * nothing. */
double oracle_kl_divergence(int N, const uint64_t *hist, int w_prev)
{
    uint64_t sum = 0;
    for (int k = 0; k <= N; ++k)
        sum += hist[k];
    if (sum == 0)
        return 0.0;
    double w = (double)(w_prev > 10 ? w_prev : 10);
    double dk = 0.0;
    for (int k = 0; k <= N; ++k) {
        if (hist[k] == 0)
            continue;
        double p = (double)hist[k] / (double)sum;
        dk += p * log(p * w);
    }
    return dk;
}

/* Width, in bins, of the energy range a histogram covers (lowest to highest
 * visited bin, inclusive; the full range is N + 1). */
int oracle_width(int N, const uint64_t *hist)
{
    int lo = -1, hi = -1;
    for (int k = 0; k <= N; ++k) {
        if (hist[k] > 0) {
            if (lo < 0)
                lo = k;
            hi = k;
        }
    }
    return lo < 0 ? 0 : hi - lo + 1;
}

/* Reachable bins inside that range (the forbidden bins 1 and N-1 left out). */
int oracle_reachable_width(int N, const uint64_t *hist)
{
    int lo = -1, hi = -1;
    for (int k = 0; k <= N; ++k) {
        if (hist[k] > 0) {
            if (lo < 0)
                lo = k;
            hi = k;
        }
    }
    if (lo < 0)
        return 0;
    int n = 0;
    for (int k = lo; k <= hi; ++k)
        n += reachable(N, k);
    return n;
}

/* ---------------------------------------------------------------------- */
/* Density of states from a production histogram (Sec. 2.1, Sec. 3.3):      */
/* ln g[k] = ln H[k] - omega[k] + C on reachable bins with H > 0, -inf      */
/* elsewhere.  norm 0: ln g[0] = ln 2 (two ground states); norm 1:          */
/* sum_k exp(ln g[k]) = 2^N.  Returns 0, or -1 if the chosen anchor is      */
/* missing (H[0] = 0 for norm 0, empty histogram for norm 1).               */
/* ---------------------------------------------------------------------- */
int oracle_log_dos(int N, const uint64_t *hist, const double *omega, int norm, double *out)
{
    double mx = -INFINITY;
    for (int k = 0; k <= N; ++k) {
        if (reachable(N, k) && hist[k] > 0) {
            out[k] = log((double)hist[k]) - omega[k];
            if (out[k] > mx)
                mx = out[k];
        } else {
            out[k] = -INFINITY;
        }
    }
    double c;
    if (norm == 0) {
        if (hist[0] == 0)
            return -1;
        c = log(2.0) - out[0];
    } else {
        if (mx == -INFINITY)
            return -1;
        double s = 0.0;
        for (int k = 0; k <= N; ++k)
            if (out[k] != -INFINITY)
                s += exp(out[k] - mx);
        c = (double)N * log(2.0) - (mx + log(s));
    }
    for (int k = 0; k <= N; ++k)
        if (out[k] != -INFINITY)
            out[k] += c;
    return 0;
}
