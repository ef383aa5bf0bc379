/*
 * mmc.h -- C ABI of the MI355X (gfx950) multipath Metropolis engine for the classical
 * O(3) Heisenberg model.
 *
 * Method (arXiv:1305.6758, Sec. 2): many mutually independent simulation paths on a
 * periodic simple-cubic lattice of N = L^3 unit spins with energy eq. (ham),
 * H = -(J/2) sum_n sum_lambda S_n . S_{n+lambda}. Each path starts from a random state,
 * is thermalised and measured with single-spin Metropolis moves, and outputs its per-site
 * magnetisation M and energy; the cross-path averages of eq. (MCAV) and eq. (M_and_H),
 * the moments <|M|^k>, eq. (cv), eq. (kum), eq. (dist-coefficient) and eq. (eq:cv) are the
 * simulation results.
 *
 * Engine conventions (the paper leaves these open):
 *   - proposal: a new spin uniform on the sphere, independent of the old one
 *     (cos(theta) = 2 u0 - 1, phi = 2 pi u1); acceptance: u2 < exp(-beta dE), beta = 1/T;
 *   - random numbers: Philox4x32-10 (Salmon et al., SC'11) on the counter
 *     (site id, sweep, path, tag | instance_id << 8) with key (seed_lo, seed_hi); tag 0 for
 *     the initial state (sweep word 0), tag 1 for the Metropolis move; site id
 *     i = x + L (y + L z);
 *   - sweep: checkerboard, sites with (x + y + z) even first, then the odd ones;
 *   - FP32 mode: spins, fields and the acceptance exponential in FP32 (uniforms with 23
 *     random bits, ((w >> 8) | 1) 2^-24), spins renormalised every renorm_every sweeps;
 *     FP64 mode: uniforms (w + 1/2) 2^-32 and IEEE FP64 arithmetic without contraction,
 *     the form that reproduces an FP64 reference trajectory; all per-path accumulators and
 *     cross-path statistics are FP64 in both modes;
 *   - measurements after every sweep k >= n_therm: e = E/N, m = |M| (M per site), and the
 *     time means of e, e^2, m, m^2, m^4; the final state's {M^x, M^y, M^z, E/N}, which is
 *     the per-path output of Sec. 2.2.
 *
 * Errors: every call returns a status (mmc_status) or NULL and never aborts; the reason of
 * the last failure on the calling thread is in mmc_last_error(). With the environment
 * variable MMC_LOG set to a positive number the library reports its kernel choices (plan,
 * tuning) on stderr. Contexts are
 * thread-compatible: one context must not be used by two threads at once.
 * Ownership: the caller owns every host buffer it passes in; the library owns its contexts
 * and, unless mmc_bind() supplies memory, the device memory they use.
 */
#ifndef MMC_H
#define MMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mmc_ctx mmc_ctx;

typedef enum {
    MMC_OK = 0,
    MMC_EINVAL = -1,       /* an argument is out of range */
    MMC_ENOMEM = -2,       /* device or host allocation failed, or a bound buffer is too small */
    MMC_EHIP = -3,         /* a HIP runtime call failed (no GPU, launch failure, ...) */
    MMC_ESTATE = -4,       /* call not valid in the context's current state */
    MMC_EUNSUPPORTED = -5, /* valid request the engine does not implement */
    MMC_EIO = -6           /* file read/write failed or the file is not a checkpoint */
} mmc_status;

typedef enum { MMC_FP32 = 0, MMC_FP64 = 1 } mmc_precision;

/* Initial state (Sec. 2.2): SPHERE draws each spin uniformly on the sphere; ANGLES draws
 * both spherical angles uniformly (the paper's random start taken literally); ORDERED starts
 * with every spin along +z; MIXED is the two-start set-up of Sec. 3 (half of the paths from
 * a random start, half ordered): paths with an even index start as SPHERE, odd ones ORDERED. */
typedef enum { MMC_INIT_SPHERE = 0, MMC_INIT_ANGLES = 1, MMC_INIT_ORDERED = 2, MMC_INIT_MIXED = 3 } mmc_init;

/* Metropolis proposal. SPHERE (default): the new spin uniform on the sphere, independent of
 * the old one. ANGLES: both spherical angles uniform (theta = pi u0, phi = 2 pi u1), the
 * random-start parametrisation of Sec. 2.2 used for the moves; without a Hastings correction
 * its stationary law carries an extra factor 1/sin(theta) per spin (an easy-axis bias along
 * z). ANGLES runs on the plain FP64 engine only (placement MMC_PLACE_PLAIN, MMC_FP64). */
typedef enum { MMC_PROPOSAL_SPHERE = 0, MMC_PROPOSAL_ANGLES = 1 } mmc_proposal;

/* Model. HEISENBERG3D (default): the classical O(3) Heisenberg model on an L^3 periodic simple
 * cubic lattice (Sec. 2). ISING2D: the Ising model on an L x L periodic square lattice (the
 * paper's appendix), spins +-1, H = -J sum over bonds s_i s_j, the same multipath set-up:
 * checkerboard Metropolis flips, one Philox4x32-10 call per quad of four sites of a row of one
 * colour (counter (c L Q + y Q + floor(j/4), sweep, path, 3 | instance << 8), Q = ceil(L/8),
 * j = floor(x/2), word j mod 4 for site (x, y) of colour c = (x + y) mod 2; the start uses tag
 * 4 and sweep word 0: s = +1 iff the word is below 2^31), exact integer decisions. Per-path
 * outputs as for the Heisenberg model with m = M/N signed, final_m = (m, 0, 0) and the trace
 * (e, m, 0, 0); mmc_get_spins puts s in the z component of site x + L y. Single-instance
 * contexts only (no batch), spins in LDS; precision, proposal, block and lanes do not apply;
 * init SPHERE means the random start. */
typedef enum { MMC_MODEL_HEISENBERG3D = 0, MMC_MODEL_ISING2D = 1 } mmc_model;

/* Where a path's spins live during a sweep. LDS: the whole lattice of one path in the
 * workgroup's LDS, or, where only half of it fits (compiled for L = 24 and 30 in FP32, any L
 * through the generic variants), its even-colour half in LDS and the odd colour in device
 * memory (variants named *-split-*), or, where only a third fits (compiled for L = 32 in FP32),
 * the even colour's x and y components in LDS and the rest in device memory (*-splitxy-*).
 * HBM: spins in device memory, one workgroup per path, sweeps inside one launch. WINDOW: spins
 * in device memory, each workgroup (one path) running its sweeps in passes over z-planes: one
 * sweep per pass through a ring of five z-planes of both colours in LDS, colour 1 two planes
 * behind colour 0 (*-ring-*, compiled for L = 48 and 32 in FP32, single-instance and batch);
 * two sweeps per pass through five even-colour and six odd-colour planes in LDS, the four
 * half-sweeps one to four planes apart, which halves the device-memory traffic (*-ring2-*,
 * compiled for L = 48 and 32 in FP32 and 16 in FP32 and FP64, single-instance and batch);
 * where both colours of five planes do not fit (L = 64 in FP32), the half ring (*-hring-*):
 * four planes of the even colour and two of the odd one in LDS, the odd colour updated in
 * device memory, each pass step updating the even colour of one plane and then the odd colour
 * of the plane below (single-instance and batch); or several sweeps per pass with the
 * half-sweeps pipelined over the planes, either
 * through a sliding window of planes in LDS (compiled for L = 24, 30, 32 in FP32 and 12, 16 in
 * FP64) or with every plane left in device memory and reused through the caches (L = 32, 48,
 * 64 in FP32; 16, 24 in FP64). PLAIN: the plain FP64 engine, one launch per half-sweep and
 * one thread per site (FP64 only). AUTO: the tuner decides. */
typedef enum {
    MMC_PLACE_AUTO = 0,
    MMC_PLACE_LDS = 1,
    MMC_PLACE_HBM = 2,
    MMC_PLACE_PLAIN = 3,
    MMC_PLACE_WINDOW = 4
} mmc_placement;

/* How a batch runs (mmc_config.batch_launch). FUSED: one persistent kernel for the whole batch,
 * whose workgroups take (instance, path group) items from one queue, largest first, and run
 * each with the code of the instance's variant (FP32; L = 8, 12, 16, 20, 24, 30, 32, 48 have a
 * member in it; a tuned variant without one runs as a member of its side, which leaves the
 * same spins and accept counts, e.g. the two-sweep rings as the L = 32 x/y split and the
 * L = 48 plane ring; otherwise results as with PER_VARIANT).
 * PER_VARIANT: one persistent kernel per variant in use, each with its own queue, side by side
 * in the captured graph. AUTO (default): PER_VARIANT. The fused kernel holds one 1024-lane
 * workgroup per CU whenever a device-memory member is in the batch (its LDS sets the size), so
 * the LDS-resident members run at fewer waves per CU than in their own launches; on a batch
 * mixing L = 8..48 it takes longer than the per-variant launches. An explicit FUSED request
 * that some variant cannot meet makes the batch's runs fail with MMC_EUNSUPPORTED. */
typedef enum { MMC_BATCH_AUTO = 0, MMC_BATCH_FUSED = 1, MMC_BATCH_PER_VARIANT = 2 } mmc_batch_launch;

/* Zero-initialised = defaults. */
typedef struct {
    int precision;      /* mmc_precision, default MMC_FP32 */
    int init;           /* mmc_init, default MMC_INIT_SPHERE */
    int placement;      /* mmc_placement, default MMC_PLACE_AUTO */
    int block;          /* threads per workgroup; 0 lets the tuner choose */
    int lanes_per_path; /* threads working on one path; 0 lets the tuner choose */
    int renorm_every;   /* FP32: renormalise every k sweeps; 0 means 64; < 0 never */
    uint32_t instance_id; /* enters Philox counter word 3 (bits 8..31); < 2^24 */
    int trace_sweeps;   /* record (e_k, M_k) for sweeps k < trace_sweeps */
    int async;          /* nonzero: mmc_run/mmc_batch_run return without waiting */
    int proposal;       /* mmc_proposal, default MMC_PROPOSAL_SPHERE */
    int model;          /* mmc_model, default MMC_MODEL_HEISENBERG3D */
    int batch_launch;   /* batches: mmc_batch_launch, default MMC_BATCH_AUTO */
} mmc_config;

/* Per-path output. Means over the n_meas measured sweeps (NaN when n_meas = 0), per site:
 * e = E/N, m = |M|. final_* is the state after the last sweep run so far. */
typedef struct {
    double e_mean, e2_mean, absm_mean, m2_mean, m4_mean;
    double final_m[3], final_e;
    uint64_t n_accept;  /* accepted moves over all sweeps run */
} mmc_path_result;

/* Cross-path statistics (FP64, host). With <.> the mean over paths of the per-path time
 * means: mean_e = <e>, mean_absm = <m> (standard errors over paths, n - 1),
 * e2 = <e^2>, m2 = <m^2>, m4 = <m^4>, chi = (N/T)(m2 - mean_absm^2) and
 * cv_heat = (N/T^2)(e2 - mean_e^2) per eq. (cv), binder = 1 - m4/(3 m2^2) per eq. (kum),
 * cv_absm = coefficient of variation of the mean of m per eq. (eq:cv), r_* = distribution
 * coefficient of eq. (dist-coefficient) of the per-path means (Q-Q least-squares line at
 * Filliben plotting positions), p_norm_* = D'Agostino-Pearson K^2 p-value (NaN when
 * n < 20), accept_rate = accepted / attempted moves. */
typedef struct {
    int64_t n;
    double mean_e, se_e, mean_absm, se_absm;
    double e2, m2, m4;
    double chi, cv_heat, binder, cv_absm;
    double r_e, r_absm, p_norm_e, p_norm_absm;
    double accept_rate;
} mmc_stats_t;

/* One instance of a batch. */
typedef struct {
    int L;
    double T, J;
    int n_paths, n_therm, n_meas;
} mmc_instance;

/* Creates a single-instance context: L even, >= 2 (the checkerboard needs a bipartite
 * periodic lattice) and L^3 <= 2^30 (L <= 1024), T > 0 (T = +inf allowed: beta = 0), J finite, n_paths >= 1,
 * n_therm >= 0, n_meas >= 0, n_therm + n_meas < 2^31. Nothing runs on the GPU until
 * mmc_run. Returns NULL on error (see mmc_last_error). Defaults as documented in
 * mmc_config. */
mmc_ctx *mmc_create(int L, double T, double J, int n_paths, int n_therm, int n_meas, uint64_t seed);

/* As mmc_create with a configuration (cfg may be NULL). */
mmc_ctx *mmc_create_ex(int L, double T, double J, int n_paths, int n_therm, int n_meas,
                       uint64_t seed, const mmc_config *cfg);

/* Message of the last failed call on this thread ("" if none). Owned by the library. */
const char *mmc_last_error(void);

/* Status code (mmc_status) of the last failed call on this thread (MMC_OK if none); the way
 * to learn why a call that returns a pointer returned NULL. */
int mmc_last_status(void);

/* Device bytes the context needs (spin state, accumulators, trace, queue). */
size_t mmc_workspace_bytes(const mmc_ctx *ctx);

/* Hands the context caller-owned device memory of at least mmc_workspace_bytes() bytes,
 * 256-byte aligned, and the caller's HIP stream (NULL: the null stream). The memory must
 * outlive the context and must not be used by anyone else meanwhile. The library always
 * launches on a stream of its own (default priority); with a bound stream every run first
 * waits for the work already queued on it and the bound stream then waits for the run (events
 * on both sides), so work the caller queues on its stream is ordered with the runs. Without
 * this call the first run allocates its own memory with hipMalloc and orders against nothing.
 * Only valid before the first run. */
int mmc_bind(mmc_ctx *ctx, void *dev_ptr, size_t bytes, void *hip_stream);

/* Chooses the kernel variant (placement, block, lanes per path) by timing every candidate
 * on a short run, unless the configuration fixed it or the tuning cache (in memory, and in
 * the JSON file named by the environment variable MMC_TUNE_CACHE if set) has an entry.
 * Called by the first run when needed; leaves the context in its initial state. */
int mmc_tune(mmc_ctx *ctx);

/* Pins the kernel variant of a context by the name mmc_plan reports, in place of the
 * tuner's choice; on a batch, the named batch variant for every instance it serves (call it
 * before mmc_bind; a later call takes over the instances both variants serve). Spins and accept counts are the same under every variant;
 * FP32 per-path sums follow the variant's reduction order, so a pinned variant reproduces
 * them bit for bit whatever the tuner would pick on another machine. Only valid before the
 * first run. MMC_EINVAL: NULL argument, unknown name, or a variant that does not fit this
 * context (its L, precision, placement, block, lanes and the device's LDS);
 * MMC_EUNSUPPORTED: the plain engine; MMC_ESTATE: the context has run (or, for a batch, is
 * bound). */
int mmc_set_variant(mmc_ctx *ctx, const char *name);

/* Runs all remaining sweeps (from the initial random state on the first call). The HIP
 * work of one run is one captured hipGraph launch. Blocks until done unless cfg.async. */
int mmc_run(mmc_ctx *ctx);

/* Advances every path by k more sweeps (k >= 1, not past n_therm + n_meas). */
int mmc_run_sweeps(mmc_ctx *ctx, int k);

/* Waits for the context's outstanding work (for cfg.async). */
int mmc_sync(mmc_ctx *ctx);

/* Returns the context to its initial state (no sweep run), keeping memory and plan. */
int mmc_reset(mmc_ctx *ctx);

/* Sweeps completed so far, or a negative status. */
int mmc_sweeps_done(const mmc_ctx *ctx);

/* Copies the per-path results of all n_paths paths to out (caller-owned, n_out >= n_paths). */
int mmc_results(const mmc_ctx *ctx, mmc_path_result *out, int n_out);

/* Copies the trace: out[path][k][4] = (e_k, Mx_k, My_k, Mz_k), per site, for
 * k < trace_sweeps; rows of sweeps not run yet are NaN. n_out = number of doubles in out,
 * at least n_paths * trace_sweeps * 4. */
int mmc_trace(const mmc_ctx *ctx, double *out, size_t n_out);

/* Largest | |S_i| - 1 | over every site of every path (Heisenberg model): the drift of the
 * spin length that FP32 renormalisation bounds; NaN if any spin is NaN. Host computation on
 * a copy of the spins. MMC_EUNSUPPORTED for batches and the Ising model, MMC_ESTATE before the
 * first run. */
int mmc_spin_norm_deviation(const mmc_ctx *ctx, double *max_dev);

/* Copies the current spins of one path as FP64, xyz[3*i + a] for site id i (x fastest). */
int mmc_get_spins(const mmc_ctx *ctx, int path, double *xyz, size_t n_out);

/* Cross-path statistics of the current results. */
int mmc_stats(const mmc_ctx *ctx, mmc_stats_t *out);

/* Statistics of any result array (host only, no GPU needed); N = L^3. */
int mmc_stats_from_results(const mmc_path_result *res, int n, int L, double T, mmc_stats_t *out);

/* Fourth-order (Binder) cumulant of n path results, eq. (kum): U = 1 - <M^4>/(3 <M^2>^2) with
 * <.> the mean over paths of each path's m4_mean and m2_mean (with n_meas = 1 these are the
 * final state's |M|^4 and |M|^2, the paper's single-output paths). *se is the first-order
 * standard error from the cross-path sample covariance of (M^2, M^4), paths independent.
 * Host only. MMC_EINVAL for null pointers or n < 2. */
int mmc_binder_cumulant(const mmc_path_result *res, int n, double *U, double *se);

/* Critical-temperature estimate from two lattice sizes L > L' at two temperatures (Sec. 4:
 * U_L(Tc)/U_L'(Tc) = 1), the ratio R(T) = U_L/U_L' taken linear between T1 and T2.
 * u = {U_L(T1), U_L'(T1), U_L(T2), U_L'(T2)}, se = their standard errors (independent runs).
 * Fills r_t1/se_r_t1, r_t2/se_r_t2 (the ratios and their errors), tc and its first-order error
 * se_tc. Host only. MMC_EINVAL for null pointers, T1 == T2, a zero cumulant or R(T1) == R(T2). */
typedef struct {
    double tc, se_tc;
    double r_t1, se_r_t1, r_t2, se_r_t2;
} mmc_crossing_t;
int mmc_cumulant_crossing(double T1, double T2, const double *u, const double *se, mmc_crossing_t *out);

/* Distribution coefficient of a sample, eq. (dist-coefficient) (Sec. 3): least-squares line
 * through the normal Q-Q plot at Filliben's order-statistic medians, r = 1 - |R|^2/((n-1) s^2).
 * Host only; x is not modified. MMC_EINVAL for null pointers or n < 3. */
int mmc_distribution_coefficient(const double *x, int n, double *r);

/* Per-sweep cross-path statistics of a trace laid out as mmc_trace fills it
 * (trace[path][k][4] = (e_k, Mx_k, My_k, Mz_k), k < n_sweeps), over the paths
 * p = path_begin, path_begin + path_stride, ... < n_paths (stride 2 separates the two halves
 * of a MIXED start). out[k][5] = (<m>, its standard error, the coefficient of variation of
 * that mean per eq. (eq:cv), <e>, its standard error), m = |M| per site: the order parameter
 * and its cv against the number of sweeps, Sec. 3. Host only. MMC_EINVAL for null pointers,
 * fewer than 2 selected paths, n_sweeps < 1 or path_stride < 1. */
int mmc_trace_stats(const double *trace, int n_paths, int n_sweeps, int path_begin, int path_stride, double *out);

/* Writes a checkpoint (configuration, plan, sweeps done, spins, accumulators, trace). */
int mmc_save(const mmc_ctx *ctx, const char *file);

/* Creates a context from a checkpoint; a later run continues bit-identically to a run
 * that was never interrupted (the random numbers are counter-based: no RNG state). */
mmc_ctx *mmc_load(const char *file);

/* Wall time of the last run's GPU work in milliseconds (hipEvents on the context's stream). */
double mmc_last_timing_ms(const mmc_ctx *ctx);

/* The proposal step of the Metropolis move on its own (the spherical parametrisation of
 * Sec. 2.1 with the proposal reading of mmc_proposal): xyz[3t + a] = component a of the unit
 * vector the engine proposes in the given precision from the words (words[2t], words[2t + 1])
 * -- for the sphere proposal cos(theta) = 2 u0 - 1, phi = 2 pi u1, with the precision's
 * uniforms (FP32 ((w >> 8) | 1) 2^-24 and the hardware sqrt/sin/cos, FP64 (w + 1/2) 2^-32 and
 * IEEE FP64 with the library's sqrt/sin/cos), computed on the GPU by the code the sweep
 * kernels inline. words: host array of 2n words; xyz: host array of 3n doubles, both owned by
 * the caller. 1 <= n <= 2^31. Allocates and frees its own device buffers. MMC_EINVAL for null
 * pointers, n or an enum out of range; MMC_ENOMEM if the buffers do not fit; MMC_EHIP without
 * a GPU. */
int mmc_proposal_vectors(int precision, int proposal, const uint32_t *words, int64_t n, double *xyz);

/* Human-readable description of the chosen kernel variant(s), NUL-terminated: the variant's
 * name for a single instance ("plain-f64" for the plain engine); for a batch
 * "batch launches=N [<variants> block=B workgroups=W items=I] ...; L<side>:<variant> ..."
 * (one bracket per persistent launch -- "fused:<variants>" for the fused kernel -- then the
 * variant of each instance in order). */
int mmc_plan(const mmc_ctx *ctx, char *buf, size_t n);

/* Frees the context and the device memory it allocated. NULL is ignored. */
void mmc_destroy(mmc_ctx *ctx);

/* Batch of n_inst independent instances (uneven L, T, path counts) run by one persistent,
 * hipGraph-captured launch: workgroups take (instance, path group) items, largest first,
 * from a device work queue. Each instance uses Philox instance word = its index in inst[]
 * (cfg->instance_id is ignored). Precision from cfg (FP32 default). Spin state exists only
 * for items in flight, so mmc_get_spins, mmc_trace, mmc_run_sweeps and mmc_save are not
 * available on a batch. Needs the GPU: creation plans the launch from the device's occupancy
 * and runs the batch autotuner, which times every batch kernel variant that fits each L
 * (placement LDS or device memory as cfg->placement allows, lanes per path, site map) on a
 * trial batch of that L and keeps the fastest (cached like mmc_tune's choices). */
mmc_ctx *mmc_batch_create(const mmc_instance *inst, int n_inst, uint64_t seed, const mmc_config *cfg);

/* Runs the whole batch (all sweeps of all instances). */
int mmc_batch_run(mmc_ctx *ctx);

/* Per-path results of instance inst (n_out >= its n_paths). */
int mmc_batch_results(const mmc_ctx *ctx, int inst, mmc_path_result *out, int n_out);

/* Statistics of instance inst. */
int mmc_batch_stats(const mmc_ctx *ctx, int inst, mmc_stats_t *out);

/* ---------------------------------------------------------------- allocation-free batch
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the batch of mmc_batch_create + mmc_batch_run +
 * mmc_batch_results in one call that allocates nothing. Every piece of device memory the run
 * needs besides the caller's output lives in a static device array of
 * MMC_STATIC_SCRATCH_BYTES that each GPU the library runs on holds until the process ends.
 *
 * inst, n_inst, seed and cfg as for mmc_batch_create (instance i draws Philox instance word
 * i; cfg may be NULL; cfg->placement AUTO or LDS, the sphere proposal, the Heisenberg model).
 * Every instance's whole lattice must fit in a workgroup's LDS (L <= 20 in FP32, L <= 16 in
 * FP64): each side runs on its default LDS batch variant -- the first one compiled for that L,
 * else the first generic one, the variant mmc_batch_create starts from before its tuner --
 * so the results equal those of mmc_batch_run with the same variants pinned. At most
 * MMC_STATIC_MAX_INSTANCES instances and MMC_STATIC_MAX_PATHS paths in all.
 * out: caller-owned DEVICE memory of sum(n_paths) results, instance 0's paths first, then
 * instance 1's, and so on. hip_stream: the caller's stream (NULL: the null stream); the call
 * only enqueues work on it and returns; the results are in out when the stream gets there.
 * Calls on one GPU share its scratch array: calls whose work overlaps on that GPU (other
 * streams, other threads) race and must be ordered by the caller. Allocates no device
 * memory and no host heap memory.
 * Errors: MMC_EINVAL (null pointers, n_inst or the total path count beyond the limits, an
 * instance out of range), MMC_EUNSUPPORTED (a lattice that needs device-memory spins, or a
 * configuration the static batch does not run), MMC_EHIP (no device, launch failure). */
#define MMC_STATIC_SCRATCH_BYTES ((size_t)18 << 20)
#define MMC_STATIC_MAX_INSTANCES 256
#define MMC_STATIC_MAX_PATHS 131072
int mmc_batch_run_static(const mmc_instance *inst, int n_inst, uint64_t seed, const mmc_config *cfg,
                         mmc_path_result *out, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* MMC_H */
