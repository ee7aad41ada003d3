/*
 * agg.h - C ABI of libagg: the right-hand side of the multi-particle
 * aggregation (Smoluchowski-type) system with kernels in canonical polyadic
 * (CP) form, and its explicit second-order Runge-Kutta (Heun) integration, on
 * one AMD Instinct MI355X (gfx950).
 *
 * The system (Sec. 1 of Stefonishin, Matveev, Zheltkov, "Tensors in modelling
 * multi-particle interactions"), truncated to sizes k = 1..N:
 *
 *   dn_k/dt = sum_{d=2..D} ( p_k^(d) + q_k^(d) )
 *   p_k^(d) =  1/d!      * sum_{i in [1,N]^d, i_1+..+i_d = k} C^(d)_i n_{i_1}..n_{i_d}
 *   q_k^(d) = -n_k/(d-1)! * sum_{i in [1,N]^(d-1)} C^(d)_{i,k} n_{i_1}..n_{i_{d-1}}
 *
 * with every kernel tensor given by CP factors (Sec. 1, CP remark):
 *   C^(d)_{i_1..i_d} = sum_{r=1..R_d} prod_{m=1..d} U^(d)_m(i_m, r).
 * The size index k of the loss term sits in the LAST mode (m = d).  Mass that
 * would grow past size N is dropped (no sink class).
 *
 * Conventions shared by every entry point:
 *   - A state vector is binary64, n[k-1] = n_k; a batch is B such vectors back to
 *     back (B*N doubles).  State pointers are DEVICE pointers.
 *   - Calls that take a plan are stream-ordered and asynchronous on the plan's
 *     HIP stream, like HIP API calls: the caller synchronises that stream before
 *     reading results on the host.  A plan is not thread-safe.
 *   - The spectral path (FFT convolutions) runs in the plan's precision; the state,
 *     the loss-term dot products, the Heun update and all moments are binary64.
 *   - No exception crosses the ABI; every call returns an agg_status and, on
 *     error, sets a thread-local message readable with agg_last_error().
 */
#ifndef AGG_H
#define AGG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AGG_MAX_D 8

typedef int32_t agg_status;
enum {
  AGG_OK = 0,
  AGG_PENDING = 1,        /* agg_poll: the request has not finished yet          */
  AGG_EINVAL = -1,        /* an argument is out of its documented range         */
  AGG_ENOMEM = -2,        /* device/host allocation failed or budget exceeded   */
  AGG_EHIP = -3,          /* a HIP runtime call failed                          */
  AGG_ENONFINITE = -4,    /* non-finite factor, initial value or final state    */
  AGG_ENOTFOUND = -5,     /* unknown ticket                                     */
  AGG_ECANCELLED = -6,    /* request cancelled (engine destroyed)               */
  AGG_EUNSUPPORTED = -7   /* valid but beyond the library's limits (size, u)   */
};

/* Arithmetic of the spectral path.  AGG_FP32C carries float-float (hi+lo)
 * pairs through every FFT pass, twiddle and product (error-free transforms).
 * Entry points take the precision as an int32_t holding an agg_precision
 * value (so that an option bit keeps the argument a valid value).
 * AGG_PLAIN may be OR-ed into the precision of agg_plan_create: the plan then
 * evaluates the right-hand side term by term, one rank-one term (d, r) at a
 * time with its own d transforms (no column shared, not even equal ones),
 * accumulating f, with separate forward, row, inverse and Heun launches per
 * stage: the unshared, unfused reference evaluation.
 * AGG_MIXED_RADIX may be OR-ed into the precision of agg_plan_create,
 * agg_plan_create_tt, agg_plan_tables, agg_plan_tables_tt and agg_submit: the
 * transform length may then be 3 2^a or
 * 5 2^a (radix-3 or radix-5 first stage in the column transforms) when that is
 * shorter than the power of two, e.g. 5 2^20 instead of 2^23 for D = 5,
 * N = 2^20 (37.5% fewer spectral bytes): the smallest 3 2^a or 5 2^a (a >= 4)
 * at least D_e N - 1, kept when its two-pass split has a column length in
 * {96, 192, 384, 768, 1536} or {160, 320, 640, 1280}, else the power of two.
 * It is not combined with AGG_PLAIN. */
typedef enum { AGG_FP64 = 0, AGG_FP32 = 1, AGG_FP32C = 2 } agg_precision;
#define AGG_PLAIN 0x100
#define AGG_MIXED_RADIX 0x200

/* One collision order d: C^(d) = sum_r weight[r] prod_m U_m(i_m, r).
 * U[m-1] is a HOST pointer to N*rank doubles, column-major by rank:
 * U[m-1][r*N + (i-1)] = U^(d)_m(i, r), for m = 1..d.  Mode m = d is the k-mode.
 * weight is a HOST pointer to rank doubles, or NULL for all ones: the CP form
 * of Sec. 1 has no weights, and a weight is only a scalar factor of rank-one
 * term r, carried into that term's coefficient, so that factor columns equal
 * up to a scale can be given (and shared) as one column.
 * rank = 0 means the order is absent.  Entries U[d..AGG_MAX_D-1] are ignored. */
typedef struct {
  int32_t d;
  int32_t rank;
  const double* U[AGG_MAX_D];
  const double* weight;
} agg_term;

typedef struct agg_plan agg_plan;

/* Build a plan for `batch` independent states that share one kernel set given
 * by its CP factors (Sec. 1, CP remark: the right-hand side then costs
 * O(N D R log N) through FFT convolutions).
 * Results are deterministic for a plan; plans of different batch sizes may
 * group the binary64 loss-term dot sums differently (a plan whose launches
 * would leave CUs idle narrows its column groups), so they agree to rounding.
 * Terms: 2 <= d <= D, each d at most once, any order; orders not listed are
 * absent.  The factors are copied (deduplicated by bitwise column equality)
 * into plan-owned device memory: the caller may free them on return.
 * hip_stream: a hipStream_t (NULL = the null stream) on which every later call
 * of this plan is enqueued.
 * prec may carry the AGG_PLAIN option bit.
 * Errors: AGG_EINVAL (D outside [2, AGG_MAX_D], N < 1, bad/duplicate d, rank < 0,
 * NULL factor with rank > 0, batch < 1, unknown precision, out == NULL),
 * AGG_ENONFINITE (a non-finite factor), AGG_EUNSUPPORTED (transform length
 * above 2^23, a gain term with more distinct columns than a row-pass chunk
 * holds, or row-pass tables beyond a workgroup's LDS),
 * AGG_ENOMEM, AGG_EHIP. */
agg_status agg_plan_create(int32_t D, int64_t N, const agg_term* terms, int32_t nterms,
                           int32_t prec, int32_t batch, void* hip_stream,
                           agg_plan** out);
agg_status agg_plan_destroy(agg_plan* plan);

/* One collision order d with its kernel in tensor-train form (Sec. 2, the TT
 * decomposition of the kernel tensor):
 *   C^(d)_{i_1..i_d} = sum_{r_1..r_{d-1}} H^(1)_{1,i_1,r_1} H^(2)_{r_1,i_2,r_2} ... H^(d)_{r_{d-1},i_d,1}.
 * ranks: r_0..r_d (r_0 = r_d = 1, the others in [1, 8]); H[m-1] is a HOST
 * pointer to core m as r_{m-1} x r_m columns of N doubles:
 *   H[m-1][(a*r_m + b)*N + (i-1)] = H^(m)_{a, i, b}   (m = 1..d; mode d is the k-mode).
 * Entries past d are ignored. */
typedef struct {
  int32_t d;
  int32_t ranks[AGG_MAX_D + 1];
  const double* H[AGG_MAX_D];
} agg_tt_term;

/* agg_plan_create for kernels in tensor-train form: the method of Sec. 1 at its
 * O(N D R^2 log N) cost.  Every distinct non-zero core column is weighted by
 * the state and transformed once; per frequency bin the gain of order d is the
 * product of the d cores' r_{m-1} x r_m matrices of spectra (times 1/d!), and
 * the loss weights of order d come from the product of the first d-1 cores'
 * matrices of dot products U_c . n (times 1/(d-1)!), applied to core d's
 * columns.  Same state layout, calls (agg_rhs, agg_rk2_step, agg_solve,
 * agg_rhs_noalloc), precisions and AGG_MIXED_RADIX option as a CP plan; no
 * AGG_PLAIN option.
 * Errors: as agg_plan_create, and AGG_EINVAL for ranks outside [1, 8] or
 * r_0, r_d != 1; AGG_EUNSUPPORTED when the transform's rows exceed 512 values
 * (N D above 2^20) or one core has more distinct columns than a row-pass chunk
 * holds. */
agg_status agg_plan_create_tt(int32_t D, int64_t N, const agg_tt_term* terms, int32_t nterms,
                              int32_t prec, int32_t batch, void* hip_stream, agg_plan** out);

/* Exponential tilting of a binary32 plan's gain transforms (a numerical device,
 * not in the paper).  The gain term of Sec. 1 is a sum of d-fold convolutions,
 * and the convolution of inputs scaled by exp(theta s) is the convolution scaled
 * by exp(theta k): the weighted inputs enter the transforms as
 * U_c(s) n_s exp(theta s) and the gain leaves them multiplied by exp(-theta k).
 * For states decaying like exp(-theta k) this flattens the spectra's dynamic
 * range, so small tail values keep their relative accuracy in binary32 (the
 * loss term and the state are binary64 either way).  theta = 0 turns it off.
 * It applies to agg_rhs only: in a time loop the rounding noise that binary32
 * spectra leave in a state's far tail is lifted by exp(theta s) at every
 * evaluation and grows (measured: non-finite within 40 Heun steps of the D=3,
 * N=4096 exp(-k/8) state at theta = 1/12), so agg_rk2_step and agg_solve run
 * untilted.  The caller keeps the tilted values in range: n_s exp(theta s) for
 * s <= N and the tilted gain sums up to D N must stay finite in binary32; a
 * theta below the state's decay rate (e.g. (1 - 1/D) times it) keeps the
 * tilted D-fold gain bounded.
 * Errors: AGG_EINVAL (NULL, theta < 0 or non-finite, a plan of another
 * precision). */
agg_status agg_plan_set_tilt(agg_plan* plan, double theta);

/* dndt = f(n) for each of the batch states (Sec. 1, the full right-hand side).
 * n, dndt: device, batch*N doubles each, must not overlap.  Asynchronous. */
agg_status agg_rhs(agg_plan* plan, const double* n, double* dndt);

/* agg_rhs without plan-owned workspace, for callers that cannot allocate
 * device memory when they evaluate (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): the same launches and results as
 * agg_rhs (bit for bit when batch equals the plan's batch), with the per-state
 * workspace taken from a static device array of the library of
 * AGG_NOALLOC_SCRATCH_BYTES bytes on each device the library runs on, held
 * until the process ends.  Nothing is allocated or freed by the call.
 *   plan   a shared-column plan (not AGG_PLAIN) created beforehand; its factor
 *          copies, tables and twiddles are read, its own workspace is not used
 *   n      device, batch*N doubles (first `batch` states of the plan's layout)
 *   dndt   device, batch*N doubles, must not overlap n
 *   batch  1 <= batch <= the plan's batch
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents (no part of it needs to start at zero): calls that overlap on one
 * GPU (different streams, threads or plans) race and must be ordered by the
 * caller.  Stream-ordered and asynchronous on the plan's stream.
 * Errors: AGG_EINVAL (NULL argument, AGG_PLAIN plan, batch out of range),
 * AGG_EUNSUPPORTED (batch times the per-state workspace, u*M + M stored complex
 * values plus u*(M2+1) doubles, exceeds the array), AGG_EHIP. */
#define AGG_NOALLOC_SCRATCH_BYTES (64ull << 20)
agg_status agg_rhs_noalloc(agg_plan* plan, const double* n, double* dndt, int32_t batch);

/* One Heun step in place (Sec. 3: explicit second-order Runge-Kutta, two
 * right-hand-side evaluations): k1 = f(n), n~ = n + dt k1, k2 = f(n~),
 * n <- n + dt/2 (k1 + k2).  n: device, batch*N.  dt > 0 and finite.  Async. */
agg_status agg_rk2_step(agg_plan* plan, double* n, double dt);

typedef struct {
  int64_t steps;        /* Heun steps taken                                     */
  int64_t rhs_evals;    /* right-hand-side evaluations (2 per step, per state)  */
  double t_final;       /* time reached                                         */
  double m0_initial, m1_initial;   /* sum n_k and sum k n_k over the batch, t=0 */
  double m0_final, m1_final;       /* the same at t_final                       */
  int64_t nonfinite;    /* count of non-finite entries of the final state       */
} agg_solve_stats;

/* Integrate n from t = 0 to t_end with step dt in place by repeated Heun steps
 * (Sec. 3, as agg_rk2_step; full steps are replayed from captured HIP graphs of
 * 16 steps, and a solve of at most 64 steps that repeats the previous call's
 * state pointer, dt and t_end from one captured graph of the whole solve; both
 * compute exactly what eager steps compute).  Time grid: the step
 * count is round(t_end/dt) when t_end/dt is within 1e-9 (relative) of an
 * integer, else ceil(t_end/dt) with the last step shortened to reach t_end;
 * t_end = 0 takes no step.  With st == NULL the call is asynchronous.  With st
 * non-NULL it synchronises the stream, fills st (binary64 moments) and returns
 * AGG_ENONFINITE if the final state holds a non-finite value (state still
 * written).  Errors: AGG_EINVAL for dt <= 0, t_end < 0, or non-finite. */
agg_status agg_solve(agg_plan* plan, double* n, double dt, double t_end, agg_solve_stats* st);

/* ---- timing aid ------------------------------------------------------------
 * Runs one pass of the evaluation pipeline `reps` times back to back on the
 * plan's stream for the batch state n (device, batch*N; not modified) and
 * writes the mean device time per launch in microseconds, measured with HIP
 * events on that stream.  A full right-hand side is evaluated first so every
 * intermediate buffer is valid.  pass: 0 forward column pass (weighting,
 * column transforms, dot products), 1 row pass (row transforms, spectral
 * combine, inverse row transforms), 2 inverse column pass with the f epilogue,
 * 3 fused column pass of a time step (inverse + epilogue + Heun stage-1 update
 * + forward pass of the updated state).  Synchronises the stream.
 * Errors: AGG_EINVAL (NULL, pass outside [0,3], reps < 1), AGG_EHIP. */
agg_status agg_profile_pass(agg_plan* plan, const double* n, int32_t pass, int32_t reps,
                            double* us_per_launch);

/* ---- introspection (host only: no device is touched) ----------------------
 * agg_plan_tables writes the plan's integer tables as int64 (layout:
 * [L, M1, M2, g, u, Tp, Tq, De, column id per (d, m, r) in scan order d, m, r,
 *  per gain term: d, multiplicity, ids[d],
 *  per loss term: d, multiplicity, k-mode id, ids[d-1],
 *  number of row-pass chunks H (0 when every column fits the row pass at once),
 *  per chunk: ncols, nterms, column ids[ncols], gain-term indices[nterms]])
 * into out[0..cap) and its full length into *len.  AGG_EINVAL if cap is short
 * (len still set).  agg_twiddles writes exp(-2 pi i e / P) for e = 0..P-1 as
 * interleaved binary64 (re, im) pairs into out[0..2P): P a power of two, or
 * 3 2^k or 5 2^k with k >= 3 (the mixed-radix lengths); AGG_EINVAL otherwise. */
agg_status agg_plan_tables(int32_t D, int64_t N, const agg_term* terms, int32_t nterms,
                           int32_t prec, int64_t* out, int64_t cap, int64_t* len);
agg_status agg_twiddles(int64_t P, double* out);
/* agg_plan_tables for a tensor-train kernel set:
 * [L, M1, M2, g, u, number of terms T, number of cores K, effective order,
 *  per term: d,
 *  per core (terms by ascending d, cores m = 1..d): term index, m, r_{m-1}, r_m,
 *    column ids of its r_{m-1} x r_m columns (row-major, -1 for an all-zero column),
 *  number of row-pass chunks H, per chunk: ncols, ncores, column ids, core indices] */
agg_status agg_plan_tables_tt(int32_t D, int64_t N, const agg_tt_term* terms, int32_t nterms,
                              int32_t prec, int64_t* out, int64_t cap, int64_t* len);

/* ---- host kernel compression (no device is touched) ------------------------
 * For kernels that depend on the total size only, C^(d)_{i_1..i_d} =
 * f(i_1 + ... + i_d), the paper knows no robust CP construction in general
 * (Sec. 1, remark on CP decompositions); this class has one through a 1-D
 * exponential sum, because exp(-a (i_1+..+i_d)) = prod_m exp(-a i_m):
 *     f(s) ~ w[0] + sum_{r=1..R} w[r] exp(-alpha[r-1] s),
 * and order d then has CP rank R+1: term r has weight w[r] and the column
 * exp(-alpha[r-1] i) in every mode (term 0: ones), so that the R+1 columns are
 * shared by every mode and order.  One fit over
 * [2, D N] serves every order d <= D; the kernel error of order d is the fit
 * error over [d, d N].
 *   f       host, f[s - smin] = f(s) for every integer s in [smin, smax]
 *   R       number of exponentials, 0..64
 *   relative 0: minimise the absolute error; else the error relative to |f(s)|
 *           (every f(s) must then be non-zero)
 *   alpha   host out, R exponents (> 0, ascending)
 *   w       host out, R+1 weights (w[0] the constant)
 *   max_err host out, max over every integer s in [smin, smax] of |fit(s) - f(s)|,
 *           divided by |f(s)| for a relative fit
 * Exponents lie on a geometric grid whose ends are picked among a few
 * multiples of 1/smax and 1/smin; weights come from least squares on a sample
 * of the range (its first 1024 integers and 8192 geometric points), refined
 * toward the smallest maximum error by iterative reweighting.  Weights of
 * alternating sign and magnitudes above max|f| are normal: their cancellation
 * costs accuracy in the lower precisions.
 * Errors: AGG_EINVAL (NULL pointer, smin < 1, smax < smin, R outside [0, 64],
 * fewer than R+1 sizes in the range, a zero f(s) in a relative fit), AGG_ENONFINITE (a non-finite f value),
 * AGG_EUNSUPPORTED (no fit found), AGG_ENOMEM. */
agg_status agg_expsum_fit(const double* f, int64_t smin, int64_t smax, int32_t R, int32_t relative,
                          double* alpha, double* w, double* max_err);

/* Host: a kernel of order d given in tensor-train form (Sec. 2),
 *   C^(d)_{i_1..i_d} = H^(1)_{i_1} H^(2)_{i_2} ... H^(d)_{i_d},
 * H^(m)_{i} an r_{m-1} x r_m matrix (r_0 = r_d = 1), written as CP factors: one
 * rank-one term per rank path (r_1, .., r_{d-1}) whose core columns are all
 * non-zero, with the column H^(m)_{r_{m-1}, :, r_m} in mode m.  Exact (no
 * rounding: columns are copied).  Paths are listed in lexicographic order.
 *   ranks  host, d+1 values r_0..r_d (r_0 = r_d = 1, others in [1, 4096])
 *   H      host, H[m-1] holds core m as r_{m-1} x r_m columns of N doubles:
 *          H[m-1][(a*r_m + b)*N + (i-1)] = H^(m)_{a, i, b}
 *   cap    capacity of U in paths (0: only count)
 *   U      host out, d*npaths*N doubles, mode-major: mode m's factor array
 *          (the agg_term U[m-1] of rank npaths) starts at U + (m-1)*npaths*N
 *   npaths host out, the number of non-zero paths
 * The planner merges the resulting terms whose column sets agree (for the
 * generalised Brownian cores of Sec. 2 all d! paths become one term).
 * Errors: AGG_EINVAL (bad sizes, NULL pointers, cap > 0 but short: npaths is
 * set), AGG_ENONFINITE (non-finite core entry), AGG_EUNSUPPORTED (more than
 * 2^20 non-zero paths), AGG_ENOMEM. */
agg_status agg_tt_expand(int32_t d, int64_t N, const int32_t* ranks, const double* const* H, int64_t cap,
                         double* U, int64_t* npaths);

/* Host: a kernel tensor of order d given by a function of the index tuple,
 * approximated in tensor-train form by cross approximation (TT-cross: the
 * method the paper builds its TT kernels with, Sec. 1, references on TT and
 * TT-cross) - for kernels with no known CP or TT construction (general
 * non-separable kernels, e.g. the ballistic kernel of binary aggregation).
 *   f       callback: for count index tuples idx[t*d + m] (sizes, 1-based, mode
 *           m+1) writes C at each into out[t]; called with up to 2^20 tuples
 *           at a time; must be deterministic
 *   tol     stop when the estimated error (below) is at most tol
 *   rmax    largest TT rank, 1..8 (the ranks agg_plan_create_tt accepts)
 *   max_sweeps  pairs of sweeps, >= 1; the ranks grow by one per pair while
 *           the estimate exceeds tol
 *   seed    of the random initial index sets and of the error sample
 *   ranks   out, d+1 ranks (r_0 = r_d = 1)
 *   cores   out, the cores in the agg_tt_term layout, core m (r_{m-1} x r_m
 *           columns of N) starting after cores 1..m-1; capacity cap doubles
 *   len     out, doubles written (or needed)
 *   err_est out, max over 4096 random index tuples of |C_tt - C| / max |C|
 * The train interpolates C exactly at the cross points (the index sets), and is
 * then rounded (truncated SVDs along the train), so that the ranks returned are
 * those the kernel numerically has up to rmax.
 * Errors: AGG_EINVAL (bad sizes or pointers, rmax outside [1, 8], cap short:
 * len, ranks and err_est are set), AGG_ENONFINITE (a non-finite value of f),
 * AGG_EUNSUPPORTED (a singular cross), AGG_ENOMEM. */
typedef void (*agg_kernel_fn)(const int64_t* idx, int64_t count, int32_t d, double* out, void* ctx);
agg_status agg_tt_cross(int32_t d, int64_t N, agg_kernel_fn f, void* ctx, double tol, int32_t rmax,
                        int32_t max_sweeps, uint64_t seed, int32_t* ranks, double* cores, int64_t cap,
                        int64_t* len, double* err_est);

/* ---- serving: continuous batching of whole solves ------------------------- */
typedef struct {
  int32_t device;          /* HIP device ordinal                                 */
  int64_t mem_budget;      /* device bytes reserved at creation, from which every
                              admitted request gets one block (0 = 8 GiB); a
                              pinned host region of a quarter of it (64 MiB to
                              2 GiB) is reserved for staging too                */
  int32_t max_slots;       /* concurrent solves on the device (0 = 256)          */
} agg_engine_config;

typedef struct {
  double t_submit, t_admit, t_finish;  /* seconds on the engine's steady clock  */
  int64_t steps;
  int32_t status;                      /* final agg_status of the solve          */
} agg_request_stats;

typedef struct agg_engine agg_engine;

/* cfg may be NULL (all defaults).  Errors: AGG_EINVAL (negative budget or slot
 * count, no such device, out == NULL), AGG_ENOMEM (the reservations failed),
 * AGG_EHIP. */
agg_status agg_engine_create(const agg_engine_config* cfg, agg_engine** out);
/* Stops the scheduler after the work already on the device; queued and running
 * requests are dropped with the engine, and no ticket may be polled after this
 * call.  NULL is a no-op. */
agg_status agg_engine_destroy(agg_engine* e);

/* Queue one solve n(0) = n0 -> n(t_end) (same time grid as agg_solve).  Host
 * pointers; the calling thread builds the request's tables and stages them with
 * n0 in the engine's pinned region (or in pageable memory while that region is
 * full), so factors and n0 may be reused on return.  Never blocks on the GPU.
 * Requests are admitted in submission order as device memory frees up.  A
 * result equals, bit for bit, the same request served alone by an engine.
 * Thread-safe with agg_poll and other agg_submit calls.
 * Errors as agg_plan_create/agg_solve, plus AGG_ENOMEM when the request's
 * footprint alone exceeds the device budget or the pinned region, and
 * AGG_EINVAL when every order has rank 0. */
agg_status agg_submit(agg_engine* e, int32_t D, int64_t N, const agg_term* terms,
                      int32_t nterms, const double* n0, double dt, double t_end,
                      int32_t prec, uint64_t* ticket);

/* agg_submit for a kernel set in tensor-train form (the cores as
 * agg_plan_create_tt takes them; Sec. 2, the O(N D R^2 log N) evaluation of
 * Sec. 1): the same queue, admission, time grid, results and errors, plus the
 * errors of agg_plan_create_tt.  The cores may be reused on return.  A request
 * runs in the bucket of its launch geometry (its chunked row pass) beside CP
 * requests of other geometries. */
agg_status agg_submit_tt(agg_engine* e, int32_t D, int64_t N, const agg_tt_term* terms,
                         int32_t nterms, const double* n0, double dt, double t_end,
                         int32_t prec, uint64_t* ticket);

/* Non-blocking.  AGG_PENDING until done; then writes n_out (host, N doubles)
 * and st (nullable), forgets the ticket, and returns the solve's status
 * (AGG_OK, AGG_ENONFINITE, ...).  AGG_ENOTFOUND for an unknown ticket. */
agg_status agg_poll(agg_engine* e, uint64_t ticket, double* n_out, agg_request_stats* st);

/* Engine-wide counters: completed solves, in-flight slots, queued requests,
 * device bytes in use. */
agg_status agg_engine_counters(agg_engine* e, int64_t* completed, int64_t* running,
                               int64_t* queued, int64_t* bytes_in_use);

const char* agg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* AGG_H */
