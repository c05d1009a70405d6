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
 *   The instance keeps its position p, the attempts made per walker so far:
 *   attempt p is made at site i = p mod N of sweep t = p div N.  Every
 *   attempt (thermalisation or recorded) advances p by one; it is never
 *   reset.  Calls counted in sweeps move p by N per sweep.
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
    MUCA_ERR_STATE = 6,         /* the instance was poisoned earlier, or a
                                   batch call came out of order              */
    MUCA_PENDING = 7            /* muca_batch_query: the round still runs    */
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
 * one-wave form of it runs instead.  For L = 80, 96, 112, 128 the wide
 * kernels read the 32-bit thresholds from global memory and keep only the
 * histogram counters in LDS, again in a two-wave form while all its
 * workgroups are resident at once and a one-wave form otherwise or with FAST.
 * GENERIC always runs the kernel with 64-bit thresholds read from LDS
 * (L <= 64) or L2.                                                         */
#define MUCA_FLAG_GENERIC_KERNEL 0x10000u
#define MUCA_FLAG_FAST_KERNEL 0x20000u

typedef struct muca_params {
    uint32_t L;       /* 4, 6, ..., 64 or 80, 96, 112, 128 (MUCA_MAX_L); the
                         even sizes in between have no kernels built      */
    uint32_t walkers; /* number of independent walkers, >= 1 (Sec. 2.2)      */
    uint32_t seed;    /* first word of every walker's Philox key             */
    uint32_t flags;   /* MUCA_FLAG_*                                         */
} muca_params;

typedef struct muca_info {
    uint64_t attempts;      /* spin-flip attempts of the call, all walkers   */
    uint64_t hist_sum;      /* sum of the histogram = walkers * recorded
                               attempts per walker                           */
    uint64_t sweep_counter; /* whole sweeps per walker after the call
                               (position / N)                                */
    uint64_t position;      /* attempts per walker after the call; attempt p
                               is made at site p mod N of sweep p div N      */
    uint32_t iteration;     /* weight updates applied so far                 */
    uint32_t visited_bins;  /* bins with H > 0                               */
    double flatness;        /* min H / mean H over the N-1 reachable bins    */
    double kl_divergence;   /* Eq. 6 with P = H / sum H, Q = 1/max(w', 10),
                               w' the number of reachable bins inside the
                               range covered by the previous recorded call
                               (0 at first)                                  */
    double chebyshev;       /* Eq. A.1: max |H/m - 1|, m = sum H / (N-1)     */
    double kernel_ms;       /* device time of the sweep launches (HIP events) */
    uint32_t kernel_launches; /* sweep kernel launches of the call           */
    uint32_t kernel_variant;  /* 0: generic, 1: fast, 2: split, 3: wide,
                                 4: wide two-wave, 5: two-wave pairs (two
                                 chains sharing one table) sweep kernel (the
                                 last of the call)                           */
    uint32_t width;           /* bins from the lowest to the highest visited
                                 bin of H, inclusive (full range: N + 1)     */
    uint32_t reserved;
} muca_info;

/* Device bytes an instance with these parameters holds (lattices, energies,
 * histogram, threshold table), for admission by memory footprint
 * ("Restrictions" of the program summary: system size and walker count are
 * bounded by the GPU's memory; Sec. 2.3 keeps one lattice per walker in
 * device memory).
 * Returns 0 for invalid parameters.                                         */
size_t muca_state_bytes(const muca_params* p);

/* Create an instance (Sec. 2.2: W independent walkers, each with its own
 * lattice, sharing one weight table; Sec. 3, Eq. 5: the Ising energy of each
 * lattice): allocate (or carve from device_workspace, which must
 * hold muca_state_bytes(p) bytes, be 256-byte aligned and stay alive until
 * muca_destroy) and draw the initial random +-1 spins of every walker on the
 * device, with their energies.  omega starts at 0 in every bin (W = 1, the
 * first iteration of Sec. 2.1) and the sweep counter at 0.  hip_stream: a hipStream_t, or NULL for a stream of the
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

/* The same two calls with counts in attempted spin flips per walker instead
 * of sweeps: the chain runs attempts position .. position+therm+attempts-1
 * in typewriter order and may start and stop inside a sweep (the update
 * counts of the paper's iteration schedule, Sec. 3 and Eq. 7, are in
 * attempts).  Batched rounds (muca_batch_*) need the instance at a sweep
 * boundary.                                                                 */
int muca_iterate_attempts(muca_instance* h, uint64_t therm_attempts, uint64_t attempts,
                          muca_info* info);
int muca_production_attempts(muca_instance* h, uint64_t therm_attempts, uint64_t attempts,
                             muca_info* info);

/* The paper's weight-iteration schedule (Sec. 3, Eq. 6 and Eq. 7), run to
 * its stop rule.  Iteration n: w = max(w', w_min), w' the range (in bins,
 * full range N + 1) the previous recorded call covered; f_therm * w
 * unrecorded attempts per walker, then floor(x) + 1 recorded ones, where
 * x = 6 w^z / walkers up to and including the first iteration with w = N + 1
 * and x grows by the factor `growth` in every later iteration; then Eq. 4.
 * From that first full-range iteration on, the run stops after the first
 * iteration whose d_k (muca_info.kl_divergence) is below dk_flat -- or,
 * with stop_rule MUCA_STOP_CHEBYSHEV, whose Chebyshev distance d_c
 * (muca_info.chebyshev, App. A) is below dc_flat, the alternative the paper
 * reports to stop at a comparable time.  The paper's values: z = 2.25,
 * growth = 1.1, dk_flat = 1e-4 (dc_flat = 0.05), f_therm = 30, w_min = 10.  */
#define MUCA_STOP_KL 0u
#define MUCA_STOP_CHEBYSHEV 1u
typedef struct muca_schedule {
    double z, growth, dk_flat, dc_flat;
    uint32_t f_therm, w_min;
    uint32_t max_iterations;  /* give up after this many (> 0)               */
    uint32_t stop_rule;       /* MUCA_STOP_KL or MUCA_STOP_CHEBYSHEV         */
} muca_schedule;

typedef struct muca_schedule_step {
    uint64_t therm_attempts;  /* per walker                                  */
    uint64_t update_attempts; /* recorded attempts per walker                */
    double kl_divergence, chebyshev, flatness;
    double kernel_ms;
    uint32_t width;           /* w of the iteration                          */
    uint32_t covered;         /* range its histogram covered                 */
} muca_schedule_step;

/* Runs the schedule from the instance's current state.  steps (may be NULL
 * when max_steps is 0) receives the first max_steps iterations;
 * *iterations the number run.  MUCA_OK when the stop rule was met,
 * MUCA_ERR_NOT_CONVERGED after max_iterations without it.                   */
int muca_run_schedule(muca_instance* h, const muca_schedule* schedule, muca_schedule_step* steps,
                      uint32_t max_steps, uint32_t* iterations);

/* Histogram H[k], k = 0..N, of the most recent recorded call: the sum over
 * all walkers of their energy histograms (Sec. 2.2, Fig. 1: H = sum_i H_i;
 * Sec. 2.3: one entry after every attempted flip).  n_bins must equal N+1.  */
int muca_histogram(const muca_instance* h, uint64_t* out, size_t n_bins);

/* Current log weights omega[k] = ln W(E_k) (Sec. 2.1: the weights that
 * Eq. 4 updates; n_bins == N+1).                                            */
int muca_log_weights(const muca_instance* h, double* out, size_t n_bins);

/* Replace omega = ln W (Sec. 2.1, Eq. 4: any positive weight function may
 * seed the recursion; Sec. 3.1 times the kernel at fixed, exact weights;
 * n_bins == N+1, every value finite).                                       */
int muca_set_log_weights(muca_instance* h, const double* in, size_t n_bins);

/* Threshold table T[k*5 + d] (n == 5*(N+1)) used by the most recent sweep
 * call, or computed from the current omega if there was none: the Metropolis
 * acceptance min(1, W(E')/W(E)) of Sec. 2.3 as an integer bound on the
 * 32-bit draw (d = dE/4 + 2, dE the energy change of the flip).             */
int muca_thresholds(const muca_instance* h, uint64_t* out, size_t n);

/* Current energy of every walker (Sec. 3, Eq. 5: E = -sum over nearest-
 * neighbour bonds of s_i s_j, J = 1; n == walkers).                         */
int muca_energies(const muca_instance* h, int32_t* out, size_t walkers);

/* Current spins of every walker's lattice (Sec. 3, Eq. 5: s_i = +1 or -1 on
 * the periodic L x L lattice), walker-major: out[w*N + i], i = y*L + x
 * (n == walkers*N).                                                         */
int muca_spins(const muca_instance* h, int8_t* out, size_t n);

/* ln g[k] estimated from the stored histogram and omega (Sec. 3.3):
 * ln g = ln H - omega + C on reachable bins with H > 0, -inf elsewhere.
 * normalization 0: C makes ln g[0] = ln 2 (the two ground states);
 * normalization 1: C makes sum_k exp(ln g[k]) = 2^N (the paper's choice).
 * MUCA_ERR_NOT_CONVERGED if the anchor bin is empty.  n == N+1.             */
int muca_log_dos(const muca_instance* h, int normalization, double* out, size_t n);

/* Diagnostics of the most recent sweep call (zeros before the first).       */
int muca_last_info(const muca_instance* h, muca_info* out);

/* Checkpoint and resume.  The whole state of an instance -- lattices and
 * energies of every walker, omega, the last histogram, the attempt position
 * and the iteration statistics -- as one host byte array; with counter-based
 * random numbers nothing else is needed, so an instance restored from it
 * continues bit for bit as the original would.  muca_restore accepts only a
 * checkpoint of an instance with the same L, walkers and seed (and rejects
 * non-finite weights or impossible energies); n must equal
 * muca_checkpoint_bytes(h).  Both calls block until the copies are done.   */
size_t muca_checkpoint_bytes(const muca_instance* h);
int muca_checkpoint(const muca_instance* h, void* out, size_t n);
int muca_restore(muca_instance* h, const void* in, size_t n);

/* Message for the last failure on h (NULL: the last failed muca_create or
 * muca_production_static of this thread).  Valid until the next call on h.  */
const char* muca_last_error(const muca_instance* h);

/* ------------------------------------------------------------------------
 * Production analysis (host only; no device is touched).  A production run
 * at fixed weights omega cut into `blocks` calls gives one histogram per call
 * (the paper uses 100, Sec. 3.3); block_hists holds them one after another,
 * blocks * (L*L+1) counts.  Estimates use the summed histogram; error bars
 * are jackknife errors over the blocks, sqrt((B-1)/B sum_b (x_(b) - x_.)^2)
 * with x_(b) the estimate without block b (0 when blocks == 1).
 * ------------------------------------------------------------------------ */

/* ln g (normalisation as in muca_log_dos) and its jackknife error per bin
 * (ln_g_err may be NULL).  Bins with no entries get ln g = -inf and error
 * NaN; a bin that is empty once some block is left out gets error +inf.
 * ln_g and ln_g_err hold L*L+1 values.  MUCA_ERR_NOT_CONVERGED if the
 * normalisation's anchor is missing from the summed histogram.              */
int muca_jackknife_log_dos(uint32_t L, uint32_t blocks, const uint64_t* block_hists,
                           const double* omega, int normalization, double* ln_g, double* ln_g_err);

/* Canonical averages by reweighting the production run (Sec. 2.1: the
 * canonical distribution is g(E) e^{-beta E} / Z_beta): per inverse
 * temperature betas[j], energy[j] = <E>/N and specific_heat[j] =
 * beta^2 (<E^2> - <E>^2) / N (J = k_B = 1), with jackknife errors (the
 * *_err arrays may be NULL).                                                */
int muca_canonical(uint32_t L, uint32_t blocks, const uint64_t* block_hists, const double* omega,
                   uint32_t n_beta, const double* betas, double* energy, double* energy_err,
                   double* specific_heat, double* specific_heat_err);

/* ------------------------------------------------------------------------
 * Batched form: many independent instances (any mix of L and walker counts)
 * swept together so that their walkers fill the device.  The method is the
 * same per instance (Sec. 2.2: independent walker populations, each with its
 * own weights and histogram); every instance's results are bit-identical to
 * running it alone.  One round runs, for every member, either a weight
 * iteration, a production call or nothing; the members' sweeps are grouped by
 * (L, kernel form) and each group is one launch whose workgroups each take
 * walkers of one member (64, or 128 / 256 sharing one threshold table for
 * the one-wave form at L >= 40); the groups run concurrently.
 * ------------------------------------------------------------------------ */
typedef struct muca_batch muca_batch;

#define MUCA_BATCH_SKIP 0u
#define MUCA_BATCH_ITERATE 1u
#define MUCA_BATCH_PRODUCTION 2u

/* batch flags */
#define MUCA_BATCH_GRAPH 0x1u     /* capture a whole round in a HIP graph --
                                     histogram clear, staging upload, sweeps,
                                     histogram download, and the host half of
                                     every member's call (sum check, statistics,
                                     Eq. 4) as a host node -- and replay it while
                                     the round's shape (which members run, their
                                     sweep counts and kernel forms) is unchanged;
                                     rounds that need several launches per member
                                     run without the graph                     */
#define MUCA_BATCH_AUTOTUNE 0x2u  /* for rounds whose two-wave workgroups do
                                     not all fit on the device at once, time
                                     five launch shapes on five such rounds and
                                     keep the fastest -- the mixed-longest shape
                                     (the two-wave form only for the members
                                     whose chain is the round's longest, the
                                     one-wave form for the rest), the mixed
                                     shape (the two-wave form for the members
                                     with the longest chains, as many as fit),
                                     the one-wave form with its default walkers
                                     per workgroup, the one-wave form with 256
                                     walkers (four waves) sharing each
                                     threshold table, and the mixed-longest
                                     shape with the histograms merged twice per
                                     round (two launches) -- and time them again
                                     once the rounds' walkers have halved;
                                     rounds that fit run the two-wave form (at
                                     L = 48-64 in pairs of chains sharing one
                                     table where one workgroup per chain does
                                     not fit), and without the flag the others
                                     run the mixed-longest shape; results do not
                                     depend on the choice                      */

/* Group count live instances.  members[] stay owned by the caller and must
 * outlive the batch; they are not to be called while a round runs, and all
 * must have been created on the current device.  hip_stream: as for
 * muca_create.  On failure *out is NULL and muca_batch_last_error(NULL) tells
 * why.                                                                      */
int muca_batch_create(muca_instance* const* members, uint32_t count, void* hip_stream,
                      uint32_t flags, muca_batch** out);

/* One round.  mode[i] is MUCA_BATCH_SKIP, _ITERATE or _PRODUCTION for member
 * i; therm[i] and sweeps[i] as in muca_iterate.  infos (may be NULL) receives
 * count entries; kernel_ms is the device time of the whole round.  Member
 * errors (e.g. a poisoned member) fail the round before any device work; a
 * device failure during the round poisons the members that ran in it.
 * Equivalent to muca_batch_submit followed by muca_batch_finish.            */
int muca_batch_run(muca_batch* b, const uint32_t* mode, const uint32_t* therm,
                   const uint32_t* sweeps, muca_info* infos);

/* The two halves of muca_batch_run, so that the host can do other work (or
 * drive other batches) while a round runs.  submit computes the members'
 * thresholds and enqueues the round without waiting for it (unless a member
 * needs more than one launch per round); the arrays are copied.  Until
 * finish, no other batch call on b is allowed and the members must not be
 * touched.  query returns MUCA_OK once the round has finished on the device,
 * MUCA_PENDING while it runs; it never blocks.  finish waits for the round
 * and applies the host half of every member's call (statistics, Eq. 4).   */
int muca_batch_submit(muca_batch* b, const uint32_t* mode, const uint32_t* therm,
                      const uint32_t* sweeps);
int muca_batch_query(muca_batch* b);
int muca_batch_finish(muca_batch* b, muca_info* infos);

/* Replace the member list between rounds (same rules as muca_batch_create).
 * Staging buffers are kept while the new members fit in them, so a batch
 * whose membership changes often (continuous batching) does not allocate or
 * free device memory each time.  Autotuner results are kept.                */
int muca_batch_set_members(muca_batch* b, muca_instance* const* members, uint32_t count);

int muca_batch_destroy(muca_batch* b);

const char* muca_batch_last_error(const muca_batch* b);

/* ------------------------------------------------------------------------
 * Serving form: a request loop with continuous batching.  A request is one
 * complete solve (Sec. 2.2): weight iterations of iter_sweeps recorded sweeps
 * (after iter_therm unrecorded ones) until the iteration's flatness (min H /
 * mean H over the reachable bins) reaches min_flatness, then prod_therm
 * unrecorded and prod_sweeps recorded sweeps at the final weights, whose
 * histogram gives ln g (normalisation 0 of muca_log_dos).  Requests are
 * admitted in arrival order as soon as their device state (muca_state_bytes)
 * fits in the server's arena and the walker budget allows; admitted requests
 * stay resident until done.  Requests of equal L form one lane (a batch on
 * its own stream); lanes run concurrently and each starts its next round as
 * soon as its previous round ends.  A production run is cut into slices of
 * at most iter_sweeps sweeps.  Results are bit-identical to running the
 * request alone (muca_iterate, muca_production(prod_therm, prod_sweeps),
 * muca_log_dos).  The server is driven by muca_server_progress, which never
 * blocks on the device.  Times are seconds since the server was created.
 * ------------------------------------------------------------------------ */
typedef struct muca_server muca_server;

typedef struct muca_server_config {
    uint64_t mem_cap_bytes;       /* device arena for request state (allocated
                                     once, at creation)                       */
    uint64_t max_active_walkers;  /* admit while the admitted walkers stay
                                     within this (0: no limit)               */
    uint32_t batch_flags;         /* MUCA_BATCH_* for the lanes               */
    uint32_t policy;              /* MUCA_SERVE_FIFO: admit in arrival order;
                                     MUCA_SERVE_SMALLEST_FIRST: admit the
                                     queued request of least estimated work
                                     first -- walkers * N * (N/20 iterations,
                                     capped by max_iterations, of iter_therm +
                                     iter_sweeps sweeps, plus prod_therm +
                                     prod_sweeps) -- except that a request
                                     queued for longer than max_wait_s goes
                                     before any other (the oldest first), so
                                     that no request waits without bound     */
    double max_wait_s;            /* smallest-first only; 0 means 30 s; must
                                     be >= 0                                 */
} muca_server_config;
#define MUCA_SERVE_FIFO 0u
#define MUCA_SERVE_SMALLEST_FIRST 1u

typedef struct muca_request {
    double min_flatness;          /* stop iterating at flatness >= this      */
    uint32_t L, walkers, seed, flags;  /* as in muca_params                  */
    uint32_t iter_therm;          /* unrecorded sweeps before each iteration */
    uint32_t iter_sweeps;         /* recorded sweeps per iteration (>= 1)    */
    uint32_t max_iterations;      /* 0: no cap; at the cap the production
                                     still runs and the result's status is
                                     MUCA_ERR_NOT_CONVERGED                  */
    uint32_t prod_therm, prod_sweeps;
    uint32_t reserved;
} muca_request;

typedef struct muca_result {
    uint64_t ticket;
    uint64_t attempts;            /* spin-flip attempts of the whole solve    */
    double flatness;              /* of the last weight iteration            */
    double t_submit, t_admit;     /* arrival, admission                      */
    double t_weights;             /* end of the last weight iteration        */
    double t_done;                /* ln g available                          */
    int32_t status;               /* MUCA_OK or the error that ended it      */
    uint32_t iterations;
} muca_result;

typedef struct muca_server_counters {
    uint64_t completed, admitted;
    uint64_t resident_bytes;      /* arena bytes held by admitted requests    */
    uint64_t active_walkers;
    uint64_t attempts;            /* all attempts of finished rounds          */
    double clock_s;
    uint32_t queued, active;
} muca_server_counters;

/* Allocates the arena on the current device.  On failure *out is NULL and
 * muca_server_last_error(NULL) tells why.                                   */
int muca_server_create(const muca_server_config* cfg, muca_server** out);

/* Queues a request (copied); *ticket identifies it.                         */
int muca_server_submit(muca_server* s, const muca_request* q, uint64_t* ticket);

/* Collects finished lane rounds, retires finished requests, admits queued
 * ones and starts the next round of every idle lane.  *events (may be NULL)
 * counts rounds collected plus rounds started; 0 means nothing changed.     */
int muca_server_progress(muca_server* s, uint32_t* events);

/* The result of a finished request, then forgets it.  MUCA_PENDING while the
 * request is queued or running.  ln_g (may be NULL) receives L*L+1 values
 * (n must equal that), zeros if the request failed.                         */
int muca_server_take(muca_server* s, uint64_t ticket, muca_result* res, double* ln_g, size_t n);

int muca_server_stats(const muca_server* s, muca_server_counters* out);

/* Waits for running rounds, then frees everything.                          */
int muca_server_destroy(muca_server* s);

const char* muca_server_last_error(const muca_server* s);

/* ------------------------------------------------------------------------
 * Production sweeps that allocate nothing -- for callers that cannot
 * allocate device or host memory while they run (serving loops and harnesses
 * that forbid allocation).  Same operation and bits as muca_production on an
 * instance in the same state, on lattices and energies the caller owns.
 *
 * p: L, walkers, seed and flags as in muca_create.  sweep0: the sweep index
 * of the first sweep (an instance's muca_info.sweep_counter); the call runs
 * sweeps sweep0 .. sweep0 + therm_sweeps + sweeps - 1 of every walker, the
 * last `sweeps` recorded.  omega: host, N+1 finite log weights (not changed).
 * spins, energies: device memory in an instance's layout, read and written --
 * spins uint32 [L * ceil(L/32)][wpad], bit x%32 of word y*ceil(L/32) + x/32 of
 * walker w at index word*wpad + w (bit set = +1), energies int32 [wpad], with
 * wpad = walkers rounded up to a multiple of 64 (the padding walkers run but
 * are never counted).  hist: host, N+1 counts, written.  hip_stream: a
 * hipStream_t, or NULL for the null stream; the call returns after its work
 * there is done.
 *
 * The uploaded thresholds and the merged histogram live in one static
 * device array of MUCA_STATIC_SCRATCH_BYTES per device (enough for L =
 * MUCA_MAX_L), held until the process ends; the histogram part is cleared by
 * a kernel at the start of every call.  All calls on a device share that
 * array, so calls whose device work overlapped would race: the library holds
 * a process-wide lock for the whole call, and calls from several threads run
 * one after the other.  No hipMalloc, hipFree or host heap allocation is
 * made.  Errors: MUCA_ERR_INVALID_ARG (NULL pointer, invalid parameters,
 * non-finite omega, tables beyond the scratch size), MUCA_ERR_OVERFLOW,
 * MUCA_ERR_DEVICE (a HIP call failed or the histogram sum is wrong);
 * muca_last_error(NULL) tells why.                                          */
#define MUCA_STATIC_SCRATCH_BYTES 655872u
int muca_production_static(const muca_params* p, uint64_t sweep0, uint32_t therm_sweeps, uint32_t sweeps,
                           const double* omega, uint32_t* spins, int32_t* energies, uint64_t* hist,
                           void* hip_stream);

/* ------------------------------------------------------------------------
 * Measurement: the issue rate of the integer vector instructions the sweep is
 * made of (Philox4x32-10 and the Metropolis step, Sec. 2.3), which sets the
 * roof the sweep kernels are measured against (Sec. 3.1 times the hardware
 * performance per attempted flip).  Every lane of waves_per_simd (1..8)
 * waves on each SIMD of every compute unit advances eight independent chains
 * of instruction `op` for 64 * iterations steps (iterations <= 2^24).  *ms is
 * the kernel's device time, *lane_ops the lane-operations of the probed
 * instruction it executed; lane_ops / ms is the measured rate.  Allocates a
 * small output buffer and a stream of its own.                             */
#define MUCA_PROBE_ADD 0u     /* v_add_u32                                  */
#define MUCA_PROBE_XOR3 1u    /* v_bitop3_b32 as a three-input xor          */
#define MUCA_PROBE_MUL_LO 2u  /* v_mul_lo_u32                               */
#define MUCA_PROBE_MUL_HI 3u  /* v_mul_hi_u32                               */
#define MUCA_PROBE_MAD_U64 4u /* v_mad_u64_u32                              */
int muca_probe_issue_rate(uint32_t op, uint32_t waves_per_simd, uint32_t iterations, double* ms,
                          uint64_t* lane_ops);

#ifdef __cplusplus
}
#endif

#endif /* MUCA_H */
