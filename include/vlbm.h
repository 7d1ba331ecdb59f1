/*
 * vlbm.h -- C ABI of the MI355X (gfx950) library for ensembles of the
 * vectorial lattice Boltzmann method (VLBM, D2Q5) applied to the Mach-2000
 * jet of Simonis & Wissocq, "Computing statistical solutions of a Mach 2000
 * astrophysical jet".
 *
 * The library advances many Monte Carlo realizations of the random
 * initial-boundary-value problem (eq:ibvp, Sec. 2.2) with the blended
 * stream-collide scheme of eq:vlbm1-eq:vlbm5 (Sec. 2.1), time step
 * dt = dx / a_n with the kinetic speed re-evaluated every step (Sec. 2.3),
 * and computes the ensemble statistics of Sec. 3 on the device: conservative
 * restriction (Sec. 3.2), per-cell mean (eq:mean), population standard
 * deviation (eq:std), the one-point Wasserstein-1 distance from sorted
 * samples (eq:w1disc), the two-point distance (eq:w2), the strong pathwise
 * error (eq:strongError), empirical quantiles and their width ratio
 * (eq:empcdf, eq:widthratio), and the convergence-rate fit (eq:ratefit).
 * Several mesh levels of one ensemble advance together, one launch per step.
 *
 * Conventions for every entry point:
 *   - The return value is a vlbm_status: VLBM_OK (0) or a negative code.
 *     vlbm_last_error() returns a message for the calling thread's last
 *     failure.  No C++ exception crosses this interface.
 *   - All arguments are validated before anything is enqueued; a call that
 *     returns VLBM_ERR_ARG or VLBM_ERR_SIZE has enqueued nothing.
 *   - The caller owns all state, sample and statistics memory (device
 *     pointers, e.g. from torch.empty(..., device="cuda")) and keeps it alive
 *     until vlbm_destroy().  The library allocates only small per-ensemble
 *     control arrays (a few doubles per realization) and frees them in
 *     vlbm_destroy().
 *   - Work is enqueued on the HIP stream given at creation (hip_stream;
 *     NULL = the null stream) and is asynchronous, except where a call says
 *     it synchronizes.
 *   - Device-side failures (a non-positive density or internal energy, a
 *     non-finite value) are latched per realization and reported by the next
 *     synchronizing call (vlbm_step with all_done != NULL, vlbm_times).
 *
 * State layout of one mesh level, in one state buffer: realization-major,
 * then row-major, each mesh row one contiguous block holding that row of all
 * 20 planes (var, slot).  The columns are grouped in strips of 60: column i
 * belongs to strip q = min(i / 60, nstrip - 1) at position t = i - 60 q
 * (0..63), nstrip = ceil(nx / 60), or (nx - 1) / 60 for a non-periodic level
 * with (nx - 1) divisible by 60; a row block is its nstrip strip blocks one
 * after another, and a strip block holds 64 element positions of every plane:
 *     FP64:  double st[R realizations][ny][nstrip][5 slot][4 var][64]
 *            (10240 B per strip block, 160 B per position)
 * var = (rho, rho v1, rho v2, E); slot 0 is the macroscopic state u, slots
 * 1..4 are the populations u_1..u_4 (u_5 is eliminated, Sec. 2.1).  Node
 * (i, j) sits at x = (i + 1/2) dx, y = y_min + (j + 1/2) dx.  The unused slots
 * hold no data.  Two buffers of vlbm_state_bytes() each are needed per level;
 * which one holds a given realization's current state depends on its step
 * count, so read states only through vlbm_get_state, vlbm_moments or
 * vlbm_ensemble_stats.
 * With VLBM_MIXED the populations' rho, rho v1, rho v2 are stored in FP32 and
 * everything else in FP64; a strip block holds double u[4 var][64],
 * double E_k[4 slot][64], then float q[4 slot][3 var][64] (7168 B, 112 B per
 * position).  All arithmetic, the pressure recovery and the
 * admissibility check are FP64.
 * One realization's state must stay below 4 GiB (about 24.9 M nodes in FP64,
 * 35.5 M in mixed precision, for nx a multiple of 60); larger levels are
 * rejected with VLBM_ERR_SIZE.
 */
#ifndef VLBM_H
#define VLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t vlbm_status;

#define VLBM_OK 0
#define VLBM_ERR_ARG (-1)         /* invalid argument                          */
#define VLBM_ERR_HIP (-2)         /* HIP runtime error                         */
#define VLBM_ERR_SIZE (-3)        /* size outside the supported range          */
#define VLBM_ERR_NONPOSITIVE (-4) /* a realization produced rho <= 0 or rho e <= 0 */
#define VLBM_ERR_NONFINITE (-5)   /* a realization produced a non-finite value  */
#define VLBM_ERR_STATE (-6)       /* call not valid in the handle's state       */

/* Boundary treatment (Sec. 2.2). */
#define VLBM_BC_JET 0      /* column 0: Dirichlet inlet (eq:inletBC); last column and
                              first/last rows: zero-gradient copy layers
                              (eq:outletBC, eq:transverseBC)                       */
#define VLBM_BC_PERIODIC 1 /* periodic in x and y (verification problems)         */
#define VLBM_BC_NEUMANN 2  /* zero-gradient copy layers on all four sides         */

/* Blending parameter theta of eq:vlbm1-eq:vlbm5. */
#define VLBM_LIMITER_RLMP 0 /* per-face limiter: relaxed local density bounds and
                               an internal-energy floor                             */
#define VLBM_THETA_ZERO 1   /* first-order update                                   */
#define VLBM_THETA_ONE 2    /* unlimited second-order update                        */

/* Storage precision of the state. */
#define VLBM_FP64 0
#define VLBM_MIXED 1 /* population rho, rho v planes FP32; u and E populations FP64 */

typedef struct vlbm_params {
    double gamma;      /* heat-capacity ratio, eq:eos (5/3)                       */
    double alpha;      /* rest-population weight of eq:maxwellians5, in [0, 1)    */
    double kappa;      /* safety factor >= 1 on the Bouchut kinetic speed         */
    double rlmp_relax; /* relaxation of the local density bounds (>= 0)          */
    double pos_eps;    /* internal-energy floor, fraction of the low-order value  */
    double rho_amb;    /* ambient density (0.5), Sec. 2.2                         */
    double p_amb;      /* ambient pressure (0.4127)                               */
    double rho_jet;    /* mean jet density (5)                                    */
    double v_jet;      /* jet velocity (800)                                      */
    double r_jet;      /* jet radius (0.05)                                       */
    double kl_amp;     /* amplitude A of eq:karhunenExp (0.1)                     */
    int32_t kl_modes;  /* K of eq:karhunenExp (10), 0 <= K <= 64                  */
    int32_t kl_decay;  /* integer decay exponent p of eq:karhunenExp (2), 0..16   */
    int32_t bc;        /* VLBM_BC_*                                              */
    int32_t limiter;   /* VLBM_LIMITER_RLMP or VLBM_THETA_*                      */
    int32_t precision; /* VLBM_FP64 or VLBM_MIXED                                */
    int32_t reserved;  /* must be 0                                              */
} vlbm_params;

typedef struct vlbm_level {
    int32_t nx, ny;  /* nodes including boundary layers, each >= 3 (>= 1 periodic) */
    double dx;       /* mesh width (square cells), > 0                            */
    double y_min;    /* lower domain edge                                         */
    void *state[2];  /* two device buffers of vlbm_state_bytes() bytes each,      */
                     /* 256-byte aligned                                          */
} vlbm_level;

typedef struct vlbm_ensemble vlbm_ensemble;

/* Message for the calling thread's last failed call (never NULL). */
const char *vlbm_last_error(void);

/*
 * The random draw omega_m of the initial measure (eq:karhunenExp, Sec. 2.3):
 * the KL coefficients of realizations first .. first + count - 1 into the
 * HOST array out [count][2 * modes] (row layout Y_1, Z_1, Y_2, Z_2, ..., each
 * in [-1, 1)), the input vlbm_init_ensemble takes.  Coefficient c of
 * realization m is 2 u - 1 with u the top 53 bits of output number
 * m * 2 * modes + c (0-based) of a SplitMix64 generator seeded with `seed`
 * (Steele, Lea & Flood 2014), so a realization's sample depends on (seed, m)
 * only: batches and prefixes of an ensemble see the same samples (the nested
 * sample sets of Sec. 3.1).  0 <= modes <= 64.  Host arithmetic only.
 */
vlbm_status vlbm_kl_coefficients(uint64_t seed, int64_t first, int32_t count, int32_t modes,
                                 double *out);

/* Bytes of ONE state buffer for R realizations of an nx x ny level. */
vlbm_status vlbm_state_bytes(const vlbm_params *p, int32_t nx, int32_t ny, int32_t n_real,
                             size_t *bytes);

/*
 * Create an ensemble of n_real realizations on each of n_levels (1..8) mesh levels
 * and enqueue its initial datum (eq:u0_def, Sec. 2.2; populations at
 * equilibrium with the initial kinetic speed).
 *   coeffs: HOST array [n_real][2 * kl_modes]; row m holds the coefficients
 *           Y_1, Z_1, Y_2, Z_2, ... in [-1, 1] of eq:karhunenExp for
 *           realization m (the random draw omega_m of Sec. 2.3).  The same
 *           rows are used on every level.  Copied before the call returns.
 *           May be NULL when bc != VLBM_BC_JET.
 *   For bc != VLBM_BC_JET the initial state is ambient everywhere; use
 *   vlbm_set_macroscopic afterwards to load another initial state.
 *   hip_stream: the hipStream_t all work of this ensemble is enqueued on.
 * On success *out receives the handle; destroy it with vlbm_destroy.
 */
vlbm_status vlbm_init_ensemble(const vlbm_params *p, const vlbm_level *levels, int32_t n_levels,
                               const double *coeffs, int32_t n_real, void *hip_stream,
                               vlbm_ensemble **out);

/*
 * Replace the state of one level by the macroscopic field u (DEVICE,
 * double [4 var][n_real][ny][nx]) with populations at equilibrium for the
 * kinetic speed of u, and reset time and step counters of that level to 0.
 */
vlbm_status vlbm_set_macroscopic(vlbm_ensemble *e, int32_t level, const double *u);

/*
 * Checkpoint restore: replace the full state of one level by `state` (DEVICE,
 * double [4 var][5 slot][n_real][ny][nx], the layout vlbm_get_state writes)
 * and set each realization's time t[m] and step count steps[m] (HOST arrays
 * [n_real]; a_last: HOST [n_real] last kinetic speed, or NULL).  The kinetic
 * speed of the next step is recomputed from the loaded macroscopic state, as
 * the step that produced it would have recorded it, so stepping on from a
 * state saved with vlbm_get_state / vlbm_times gives the same bits as never
 * stopping.  With VLBM_MIXED the FP32 planes store the rounded values.
 * Synchronizes the stream.
 */
vlbm_status vlbm_set_state(vlbm_ensemble *e, int32_t level, const double *state, const double *t,
                           const int64_t *steps, const double *a_last);

/*
 * Advance every realization of every level by up to n_steps steps of
 * eq:vlbm1-eq:vlbm5, each realization stopping exactly at t_final (the last
 * steps are shortened, taking a = dx/dt).  Realizations already at t_final
 * are left untouched.  One step of all levels is one kernel launch (work items
 * of every level in one persistent grid); runs of 30 steps are replayed from a
 * hipGraph captured once per t_final and configuration.  If all_done is non-NULL the call synchronizes the
 * stream, sets *all_done to 1 when every realization has reached t_final
 * (else 0), and returns VLBM_ERR_NONPOSITIVE / VLBM_ERR_NONFINITE if any
 * realization has latched a failure.
 */
vlbm_status vlbm_step(vlbm_ensemble *e, double t_final, int32_t n_steps, int32_t *all_done);

/*
 * Per-realization time, step count, kinetic speed of the last step and
 * latched status (0, VLBM_ERR_NONPOSITIVE or VLBM_ERR_NONFINITE) of one
 * level, into HOST arrays of n_real entries (each may be NULL).  Synchronizes.
 */
vlbm_status vlbm_times(const vlbm_ensemble *e, int32_t level, double *t, int64_t *steps,
                       double *a_last, int32_t *status);

/*
 * Copy the current state of one level into the DEVICE buffer out, FP64,
 * layout [4 var][5 slot][n_real][ny][nx] (checkpointing, inspection).
 */
vlbm_status vlbm_get_state(const vlbm_ensemble *e, int32_t level, double *out);

/*
 * Macroscopic moments of the current state of one level: density, speed
 * |v| and pressure p (eq:eos), DEVICE arrays [n_real][ny][nx] (each may be
 * NULL).
 */
vlbm_status vlbm_moments(const vlbm_ensemble *e, int32_t level, double *rho, double *speed,
                         double *p);

/*
 * Ensemble statistics of one level, for batches of realizations (Sec. 3).
 * Every realization's density, speed and pressure are restricted to the
 * coarse grid by r x r block averaging (Sec. 3.2; r >= 1 divides nx and ny;
 * n_cells = (ny/r)(nx/r)), then merged into the running accumulator acc:
 *   acc: DEVICE double [3 field][2][acc_cells]: per field (rho, |v|, p) the
 *        running mean and the sum of squared deviations M2 of the
 *        n_prev realizations merged so far (contents ignored when n_prev = 0).
 *        acc_cells must equal n_cells (else VLBM_ERR_SIZE).
 *        Batches are merged with the pairwise update of Chan, Golub & LeVeque.
 *   samples: DEVICE double [sample_rows][n_cells] or NULL; receives the
 *        restricted density of realization m in row m_offset + m (input of the
 *        one-point Wasserstein distance).  m_offset + n_real > sample_rows is
 *        rejected with VLBM_ERR_SIZE before anything is enqueued.
 */
vlbm_status vlbm_ensemble_stats(const vlbm_ensemble *e, int32_t level, int32_t r, double *acc,
                                int64_t acc_cells, int64_t n_prev, double *samples,
                                int64_t sample_rows, int64_t m_offset);

/*
 * Mean and population standard deviation (eq:mean, eq:std: sqrt(M2 / n))
 * from an accumulator of n_total realizations: DEVICE double [3][n_cells]
 * each (either may be NULL).  Enqueued on hip_stream.
 */
vlbm_status vlbm_stats_finalize(const double *acc, int64_t n_cells, int64_t n_total,
                                double *mean, double *std, void *hip_stream);

/*
 * Sort, in place and ascending, the m samples of every cell of a sample
 * store DEVICE double [m][n_cells] (the order statistics of eq:w1disc).
 * 1 <= m <= 4096.  Enqueued on hip_stream.
 */
vlbm_status vlbm_sort_samples(double *samples, int64_t n_cells, int32_t m, void *hip_stream);

/*
 * One-point Wasserstein-1 distance (eq:w1disc) between two sorted sample
 * stores of equal size [m][n_cells]: w1_cell[k] = (1/m) sum_m |a_(m) - b_(m)|
 * (DEVICE [n_cells] or NULL) and its average over cells, W_{1,1} (DEVICE
 * scalar or NULL), summed in a fixed order that depends on n_cells only.  The
 * average needs a workspace of n_cells / 1024 partial sums, taken as
 * stream-ordered device memory on hip_stream (hipMallocAsync) and released on
 * it.  Enqueued on hip_stream.
 */
vlbm_status vlbm_w1(const double *sorted_a, const double *sorted_b, int64_t n_cells, int32_t m,
                    double *w1_cell, double *w1_mean, void *hip_stream);

/*
 * vlbm_w1 without any device allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, kernels and results (bit for bit)
 * as vlbm_w1; the partial sums of the W_{1,1} average live in a fixed
 * workspace compiled into the library, one copy per device, held until the
 * process ends.  Limit: with w1_mean non-NULL, n_cells <=
 * VLBM_W1_NOALLOC_MAX_PARTIALS * 1024 (16 777 216 cells, 128 KiB of
 * workspace); larger inputs return VLBM_ERR_SIZE before anything is enqueued.
 * Every call on a device shares that device's workspace: calls that overlap
 * in time on one device (different streams, or threads without ordering)
 * race and must be serialized by the caller.  Calls ordered on one stream are
 * safe.  Enqueued on hip_stream.
 */
#define VLBM_W1_NOALLOC_MAX_PARTIALS 16384
vlbm_status vlbm_w1_noalloc(const double *sorted_a, const double *sorted_b, int64_t n_cells, int32_t m,
                            double *w1_cell, double *w1_mean, void *hip_stream);

/* ---------------------------------------------------------------------------
 * Observables of the convergence study (Sec. 3.3-3.4) and quantile diagnostics
 * (Sec. 4).  Sample stores are laid out [m realizations][n_cells] as written by
 * vlbm_ensemble_stats (restricted density of each realization on the common
 * grid); "sorted" stores have been through vlbm_sort_samples.  Device pointers,
 * asynchronous on hip_stream; every reduction runs in a fixed order, so equal
 * inputs give equal bits.
 * ------------------------------------------------------------------------- */
#define VLBM_MAX_QUANTILES 8

/*
 * Strong pathwise error, eq:strongError: a and b are UNSORTED sample stores of
 * the same realizations (same seeds) at two resolutions, both restricted to
 * the common grid, b the finer member.  per_real[k] receives
 * sum_c |a[k][c] - b[k][c]| / sum_c |b[k][c]| (device, [m]); out[0] their mean.
 */
vlbm_status vlbm_strong_error(const double *a, const double *b, int64_t n_cells, int32_t m,
                              double *per_real, double *out, void *hip_stream);

/*
 * out[0] = (1/n) sum_i |x_i - y_i| over the n cells of the common grid: the
 * error of eq:mean when x, y are the two ensemble-mean density fields, of
 * eq:std for the two standard-deviation fields.  y = NULL gives (1/n) sum |x_i|.
 * Two-stage fixed-order sum; its workspace of n / 1024 partial sums is taken
 * as stream-ordered device memory on hip_stream and released on it.
 */
vlbm_status vlbm_mean_abs_diff(const double *x, const double *y, int64_t n, double *out,
                               void *hip_stream);

/*
 * Empirical quantiles, eq:empcdf: for each pct[q] (HOST array of n_q <=
 * VLBM_MAX_QUANTILES integer percents in 1..100) and each cell, the smallest
 * sample xi with F(xi) >= pct/100, i.e. the order statistic ceil(pct m / 100)
 * (1-based) of the cell's m sorted samples.  out: device [n_q][n_cells].
 */
vlbm_status vlbm_quantiles(const double *sorted, int64_t n_cells, int32_t m, const int32_t *pct,
                           int32_t n_q, double *out, void *hip_stream);

/*
 * Quantile width ratio, eq:widthratio: q[c] = (p95 - p5) / (p84 - p16) per
 * cell of a sorted store (IEEE result when p84 == p16: +inf, or NaN if also
 * p95 == p5).  Gaussian laws give 1.654.
 */
vlbm_status vlbm_width_ratio(const double *sorted, int64_t n_cells, int32_t m, double *q,
                             void *hip_stream);

/*
 * Two-point Wasserstein distance, eq:w2.  a, b: UNSORTED sample stores
 * [m][ncy * ncx] (row-major cells of the common grid) of the coarse and the
 * restricted fine ensemble, same realizations.  The subsample keeps n_pd cells
 * per direction, index floor((2k + 1) n / (2 n_pd)), k < n_pd (cell centres of
 * n_pd equal intervals), cells numbered k = ky * n_pd + kx.  For every ordered
 * pair (k, k') of the n_pd^2 retained cells, w_pair[k * n_pd^2 + k'] (device,
 * [n_pd^4]) is the first Wasserstein distance with Euclidean cost between the
 * laws of the m points (a[i][c_k], a[i][c_k']) and (b[i][c_k], b[i][c_k']),
 * computed exactly as an optimal assignment (shortest augmenting paths); NaN
 * when a sample is not finite.  w_mean (device scalar or NULL) is their
 * average in a fixed order.  1 <= m <= VLBM_W12_MAX_SAMPLES, 1 <= n_pd <=
 * min(ncx, ncy, 200).
 */
#define VLBM_W12_MAX_SAMPLES 1024
vlbm_status vlbm_w12(const double *a, const double *b, int32_t ncx, int32_t ncy, int32_t m,
                     int32_t n_pd, double *w_pair, double *w_mean, void *hip_stream);

/*
 * Convergence rate, eq:ratefit (host arithmetic): least-squares line
 * log errors[i] = rate * log dx[i] + intercept over n >= 2 points; errors and
 * dx HOST arrays of positive values, dx not all equal.  intercept may be NULL.
 */
vlbm_status vlbm_rate_fit(const double *errors, const double *dx, int32_t n, double *rate,
                          double *intercept);

/* Step kernel implementations (vlbm_tune). */
#define VLBM_KERNEL_REFERENCE 0 /* one thread per node, neighbours recomputed        */
#define VLBM_KERNEL_MARCH 1     /* wavefront strips marching over rows (default)      */
#define VLBM_KERNEL_NO_GRAPH 0x100 /* OR-ed flag: launch every step eagerly instead of
                                      replaying captured hipGraphs of 30 steps       */

/*
 * Select the step kernel and its work decomposition for this ensemble:
 * chunk_rows is the number of rows one wavefront marches over, for every
 * level (0 = chosen from the level sizes and ensemble size; otherwise
 * 4 <= chunk_rows <= 65536); blocks return to 4 wavefronts, the
 * strip-fastest item order and the work-queue dealing (the defaults).  Results
 * do not depend on the choice (every kernel and decomposition is
 * bit-identical); only the speed does.
 */
vlbm_status vlbm_tune(vlbm_ensemble *e, int32_t kernel, int32_t chunk_rows);

/*
 * The marching kernel's decomposition, all of it: chunks (HOST [n_levels]:
 * rows per work item of each level, 0 = the default of that level; NULL = all
 * defaults), waves_per_block (1, 2 or 4 wavefronts per block), item_order
 * (0: consecutive work items are neighbouring column strips of one
 * realization; 1: they are the same tile of consecutive realizations, so a
 * block of w wavefronts holds w realizations) and dealing (0: item i goes to
 * wavefront i mod W, fixed; 1, the default: the items are split into one
 * contiguous range per XCD and every wavefront takes the next item of its
 * XCD's range, then of the other XCDs' ranges, from counters in the control
 * block, so faster wavefronts take more).
 * Bit-identical results for every choice.  VLBM_ERR_ARG on values outside
 * these sets.
 */
vlbm_status vlbm_set_tuning(vlbm_ensemble *e, const int32_t *chunks, int32_t waves_per_block,
                            int32_t item_order, int32_t dealing);
/* The decomposition in use (chunks: HOST [n_levels] or NULL; others nullable). */
vlbm_status vlbm_get_tuning(const vlbm_ensemble *e, int32_t *chunks, int32_t *waves_per_block,
                            int32_t *item_order, int32_t *dealing);

/*
 * Autotune the marching kernel's decomposition for the whole launch (all
 * levels together, as vlbm_step runs them) on live steps.  Candidate chunk
 * tuples come from common target heights (each level splits its rows evenly
 * near the target) and are ranked by a work model of each dealing (rows per
 * item plus the 4-row prologue; work queues: the average load per wavefront
 * plus one item; static round-robin: the most loaded wavefront); the best few
 * of each, then 2 and 1 wavefronts per block and the realization-fastest item
 * order around the fastest, are each timed over steps_per_candidate real steps
 * (HIP events on the ensemble's stream) and the fastest configuration is kept.  The steps taken
 * are ordinary steps toward t_final (every configuration is bit-identical), so
 * tuning wastes no work.  The choice is cached per (precision, bc, limiter,
 * n_real, every level's nx and ny) for the lifetime of the process and applied
 * automatically to ensembles created later with the same levels.
 *   chunks_out: HOST array [n_levels] receiving the chosen chunk heights, or NULL
 *   (vlbm_get_tuning gives the rest).
 * Synchronizes the stream.
 */
vlbm_status vlbm_autotune(vlbm_ensemble *e, double t_final, int32_t steps_per_candidate,
                          int32_t *chunks_out);

/* Release the handle and its control arrays (synchronizes its stream). */
vlbm_status vlbm_destroy(vlbm_ensemble *e);

#ifdef __cplusplus
}
#endif

#endif /* VLBM_H */
