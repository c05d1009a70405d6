/*
 * muca.h -- C ABI of the MI355X parallel multicanonical library (libmuca).
 *
 * The library determines multicanonical weights W(E) = exp(omega(E)) for the
 * 2D Ising model on a periodic L x L lattice (J = 1) that make the energy
 * histogram flat, and estimates the density of states with a final
 * production run at fixed weights ("Nature of problem" in the program
 * summary; Sec. 2.1, Eqs. 1-4; Sec. 3.3).  Many independent walkers share
 * one weight table and add their histograms (Sec. 2.2, Fig. 1); every
 * walker runs single-spin-flip Metropolis sweeps on its own lattice
 * (Sec. 2.3).
 *
 * Conventions used by every entry point
 *   N = L*L spins.  Energy bins k = 0..N hold E = -2N + 4k (Sec. 3: states are
 *   spaced by 4; k = 1 and k = N-1 are forbidden, the other N-1 bins are
 *   reachable).  Site i = y*L + x; a sweep visits i = 0..N-1 in that order.
 *   Walker w uses the Philox4x32-10 stream with key (seed, w); the draw for
 *   site i in the instance's sweep number t is word (i & 3) of the block
 *   with counter (i >> 2, t mod 2^32, t >> 32, 0) (Sec. 2.3: sub-streams
 *   labelled by site and walker).  Initial spins use counter word 3 = 1 and
 *   t = 0; spin = +1 iff the top bit of the draw is set.
 *   An attempt at a site with energy change dE (d = dE/4 + 2 in 0..4) is
 *   accepted iff r < T[k][d], r the 32-bit draw, with the threshold
 *   T[k][d] = floor(min(1, exp(omega[k'] - omega[k])) * 2^32), k' = k + d - 2,
 *   computed on the host in IEEE double once per call (T = 0 where k' is
 *   outside 0..N).  T lies in [0, 2^32], so it is stored as uint64.
 *   After every recorded attempt the current energy bin is counted.
 *   Every sweep (thermalisation or recorded) advances the instance's sweep
 *   counter by one; it is never reset.
 *
 * Ownership: the library owns the instance and, unless the caller passes a
 * device workspace, all device memory.  Host arrays passed in are read or
 * written during the call only and never retained.  A caller-provided HIP
 * stream stays owned by the caller; all device work of an instance is
 * ordered on it, and every call returns only after that work is complete.
 *
 * Errors: every function returns a muca_status.  Nothing throws across the
 * ABI.  After MUCA_ERR_DEVICE the instance is poisoned: later calls return
 * MUCA_ERR_STATE, except muca_destroy and muca_last_error.
 *
 * Threads: one instance must not be used by two threads at once; distinct
 * instances are independent.
 */
#ifndef MUCA_H
#define MUCA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct muca_instance muca_instance;

typedef enum muca_status {
    MUCA_OK = 0,
    MUCA_ERR_INVALID_ARG = 1,   /* NULL pointer, L odd or < 4 or > MUCA_MAX_L,
                                   walkers == 0, a size argument that does not
                                   match, non-finite log weights             */
    MUCA_ERR_OUT_OF_MEMORY = 2, /* a device or pinned-host allocation failed,
                                   or a caller workspace is too small        */
    MUCA_ERR_DEVICE = 3,        /* a HIP call failed; the instance is poisoned */
    MUCA_ERR_OVERFLOW = 4,      /* a merged histogram bin would pass 2^64     */
    MUCA_ERR_NOT_CONVERGED = 5, /* ln g requested but the lowest bin is empty */
    MUCA_ERR_STATE = 6          /* the instance was poisoned earlier         */
} muca_status;

#define MUCA_MAX_L 128u

/* flags of muca_params: choices of the launch shape that never change a
 * result bit.  Bits 0-15: the most sweeps one kernel launch may run (0: the
 * largest count whose 32-bit on-chip histogram counters cannot overflow).   */
#define MUCA_FLAG_DEFAULT 0u
#define MUCA_FLAG_SWEEPS_PER_LAUNCH_MASK 0xffffu
/* Sweep kernel choice (same results, bit for bit).  By default, for L <= 64
 * and when no reachable threshold is 0, the split kernel runs: 32-bit
 * thresholds and the histogram interleaved in LDS, random numbers from a
 * second wave, the next attempt's thresholds fetched ahead.  With more than
 * two of its workgroups (64 walkers each) per compute unit, or with FAST, the
 * one-wave form of it runs instead; GENERIC always runs the kernel with
 * 64-bit thresholds read from LDS (L <= 66) or L2.                           */
#define MUCA_FLAG_GENERIC_KERNEL 0x10000u
#define MUCA_FLAG_FAST_KERNEL 0x20000u

typedef struct muca_params {
    uint32_t L;       /* even, 4 <= L <= MUCA_MAX_L                          */
    uint32_t walkers; /* number of independent walkers, >= 1 (Sec. 2.2)      */
    uint32_t seed;    /* first word of every walker's Philox key             */
    uint32_t flags;   /* MUCA_FLAG_*                                         */
} muca_params;

typedef struct muca_info {
    uint64_t attempts;      /* spin-flip attempts of the call, all sweeps    */
    uint64_t hist_sum;      /* sum of the histogram = walkers * sweeps * N   */
    uint64_t sweep_counter; /* instance sweep counter after the call         */
    uint32_t iteration;     /* weight updates applied so far                 */
    uint32_t visited_bins;  /* bins with H > 0                               */
    double flatness;        /* min H / mean H over the N-1 reachable bins    */
    double kl_divergence;   /* Eq. 6 with P = H / sum H, Q = 1/max(w', 10),
                               w' the width in bins of the range covered by
                               the previous recorded call (0 at first)       */
    double chebyshev;       /* Eq. A.1: max |H/m - 1|, m = sum H / (N-1)     */
    double kernel_ms;       /* device time of the sweep launches (HIP events) */
    uint32_t kernel_launches; /* sweep kernel launches of the call           */
    uint32_t kernel_variant;  /* 0: generic, 1: fast, 2: split sweep kernel  */
} muca_info;

/* Device bytes an instance with these parameters holds (lattices, energies,
 * histogram, threshold table), for admission by memory footprint.
 * Returns 0 for invalid parameters.                                         */
size_t muca_state_bytes(const muca_params* p);

/* Create an instance: allocate (or carve from device_workspace, which must
 * hold muca_state_bytes(p) bytes, be 256-byte aligned and stay alive until
 * muca_destroy) and draw the initial random +-1 spins of every walker on the
 * device, with their energies.  omega starts at 0 in every bin and the sweep
 * counter at 0.  hip_stream: a hipStream_t, or NULL for a stream of the
 * instance's own.  On failure *out is NULL and muca_last_error(NULL) tells
 * why.                                                                      */
int muca_create(const muca_params* p, void* hip_stream, void* device_workspace,
                size_t workspace_bytes, muca_instance** out);

/* Release everything the instance owns.  NULL is accepted.                  */
int muca_destroy(muca_instance* h);

/* One weight iteration (Sec. 2.2, Fig. 1): compute the thresholds from the
 * current omega, run therm_sweeps unrecorded and then sweeps recorded sweeps
 * of every walker, sum all walker histograms into H, and apply Eq. 4 in
 * logarithmic form, omega[k] -= ln H[k] for every bin with H[k] > 0 (empty
 * bins keep their weight).  info (may be NULL) describes H before the
 * update.                                                                   */
int muca_iterate(muca_instance* h, uint32_t therm_sweeps, uint32_t sweeps, muca_info* info);

/* Production run (Sec. 2.1, Sec. 3.3): the same sweeps with omega frozen.
 * Each call replaces the stored histogram, so a caller can split a run into
 * blocks (the paper uses 100 calls for its jackknife errors).               */
int muca_production(muca_instance* h, uint32_t therm_sweeps, uint32_t sweeps, muca_info* info);

/* Histogram H[k], k = 0..N, of the most recent recorded call.  n_bins must
 * equal N+1.                                                                */
int muca_histogram(const muca_instance* h, uint64_t* out, size_t n_bins);

/* Current log weights omega[k] (n_bins == N+1).                             */
int muca_log_weights(const muca_instance* h, double* out, size_t n_bins);

/* Replace omega (n_bins == N+1, every value finite).                        */
int muca_set_log_weights(muca_instance* h, const double* in, size_t n_bins);

/* Threshold table T[k*5 + d] (n == 5*(N+1)) used by the most recent sweep
 * call, or computed from the current omega if there was none.               */
int muca_thresholds(const muca_instance* h, uint64_t* out, size_t n);

/* Current energy of every walker (n == walkers).                            */
int muca_energies(const muca_instance* h, int32_t* out, size_t walkers);

/* Current spins, walker-major, +1/-1: out[w*N + i] (n == walkers*N).        */
int muca_spins(const muca_instance* h, int8_t* out, size_t n);

/* ln g[k] estimated from the stored histogram and omega (Sec. 3.3):
 * ln g = ln H - omega + C on reachable bins with H > 0, -inf elsewhere.
 * normalization 0: C makes ln g[0] = ln 2 (the two ground states);
 * normalization 1: C makes sum_k exp(ln g[k]) = 2^N (the paper's choice).
 * MUCA_ERR_NOT_CONVERGED if the anchor bin is empty.  n == N+1.             */
int muca_log_dos(const muca_instance* h, int normalization, double* out, size_t n);

/* Diagnostics of the most recent sweep call (zeros before the first).       */
int muca_last_info(const muca_instance* h, muca_info* out);

/* Message for the last failure on h (NULL: the last failed muca_create of
 * this thread).  Valid until the next call on h.                            */
const char* muca_last_error(const muca_instance* h);

#ifdef __cplusplus
}
#endif

#endif /* MUCA_H */
