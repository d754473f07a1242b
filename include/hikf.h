/*
 * hikf.h -- C ABI of the MI355X (gfx950) HiKF hot path.
 *
 * HiKF (Li, Ambikasaran, Darve, Kitanidis) is the Kalman filter for the
 * random-walk state-space model x_t = x_{t-1} + w_t, z_t = H x_t + v_t,
 * w ~ N(0, Q), v ~ N(0, R) (Sec. 2.1, eqs. equation_state_evolution,
 * equation_measurement, equation_random_walk), where Q_ij = K(|x_i - x_j|)
 * is a kernel matrix on a uniform grid (Sec. 3.1 end; Sec. 4.2 eq.
 * equation_Q).  The filter carries only the cross-covariance C = P H^T
 * (m x p), the state x_hat and the variances diag P (Algorithm
 * Algorithm_HiKF, Sec. 3.1).  The one O(m^2) product C_Q = Q H^T is formed
 * once, at init, with a Chebyshev-interpolated H^2 / fast multipole method
 * (Sec. 3.2).
 *
 * Notation: m = number of grid cells (unknowns), p = number of measurements
 * (the paper's n), r = n_c^dim Chebyshev nodes per box.
 *
 * Memory model.  The library never allocates device memory (its one fixed
 * array, the workspace of hikf_cov_apply_noalloc, is part of its device code
 * and is loaded with it).  The caller
 * obtains the two sizes from hikf_plan, allocates a RESIDENT region (kept
 * for the filter's lifetime) and a SCRATCH region (needed only until the
 * work queued by hikf_init has finished on its stream) and passes both to
 * hikf_init.  Every pointer argument named *_dev is a device pointer; all
 * other pointers are host pointers.  All device work is queued on the
 * caller's stream (a hipStream_t passed as void*, NULL = legacy default
 * stream) and is asynchronous; host-side argument errors are returned
 * immediately, errors found in device data are reported by hikf_query.
 *
 * Threading.  A filter is not re-entrant; distinct filters may be used
 * concurrently on distinct streams.  No function aborts or throws across
 * this boundary.
 */
#ifndef HIKF_H
#define HIKF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum hikf_status {
    HIKF_OK = 0,
    HIKF_E_INVALID = 1,     /* bad shape/parameter, NaN/Inf input, bad H  */
    HIKF_E_UNSUPPORTED = 2, /* valid but outside what the library supports */
    HIKF_E_NOMEM = 3,       /* workspace smaller than hikf_plan asked for   */
    HIKF_E_NOT_SPD = 4,     /* Cholesky of H C + R failed; step not applied */
    HIKF_E_DEVICE = 5       /* a HIP runtime call failed                    */
} hikf_status;

/* Kernel families, K(r) on the Euclidean distance r between cell centres. */
enum {
    /* K(r) = theta * exp(-(r/ell)^gamma), 0 < gamma <= 2: Sec. 4.2 eq.
     * equation_Q (gamma = 1 exponential, gamma = 2 Gaussian, Sec. 3.3). */
    HIKF_KERNEL_POWEXP = 0,
    /* K(r) = theta * r^2: test-only kernel, a polynomial of degree 2 per
     * coordinate that Chebyshev interpolation with n_c >= 3 reproduces
     * exactly.  Not a covariance; steps with it are meaningless. */
    HIKF_KERNEL_TEST_R2 = 1
};

/* Initial covariance P_0 (Sec. 3.1 end; Sec. 4.2 end). */
enum {
    HIKF_PRIOR_ZERO = 0,     /* P_0 = 0            -> C_0 = 0,        var_0 = 0     */
    HIKF_PRIOR_SCALED_I = 1, /* P_0 = alpha I      -> C_0 = alpha H^T, var_0 = alpha */
    HIKF_PRIOR_KERNEL = 2    /* P_0 = Q            -> C_0 = C_Q,      var_0 = K(0)  */
};

/* Arithmetic of the H^2 product (the per-step update is always FP64). */
enum {
    HIKF_FMM_F32 = 0,        /* FP32 operands and accumulation, C_Q kept in FP32 */
    HIKF_FMM_F64 = 1,        /* FP64 throughout, C_Q kept in FP64                */
    HIKF_FMM_BF16X3 = 2,     /* as F32, but the M2L and P2P products run on BF16
                                MFMA with every FP32 operand split into
                                a = hi + lo (hi = bf16(a), lo = bf16(a - hi)) and
                                A B ~ A_hi B_hi + A_hi B_lo + A_lo B_hi with FP32
                                accumulation (relative error ~1e-5)          */
    HIKF_FMM_BF16 = 3        /* the same products from A_hi B_hi alone (no
                                refinement; relative error ~1e-3), kept to
                                show what the refinement terms contribute    */
};

/*
 * The assimilation problem (Sec. 2.1-2.2 with Sec. 3.1).
 * Grid: the N^dim cell centres ((i+1/2)/N, ...) of the unit square/cube,
 * grid order = lexicographic with the first coordinate fastest.  Every
 * m-vector and every row of an m x p matrix at this ABI is in grid order.
 * H (p x m) is CSR with 0-based column indices; R = diag(r_diag).
 * Device arrays are read during hikf_init only (copied into the resident
 * region); they may be freed once hikf_init's work has completed.
 */
typedef struct hikf_problem {
    int32_t dim;             /* 2 or 3                                        */
    int32_t n;               /* cells per axis, N; m = N^dim                  */
    int32_t kernel_family;   /* HIKF_KERNEL_*                                 */
    int32_t prior_kind;      /* HIKF_PRIOR_*                                  */
    double theta, ell, gamma;/* kernel parameters (theta > 0, ell > 0)        */
    double alpha;            /* P_0 = alpha I for HIKF_PRIOR_SCALED_I         */
    int32_t p;               /* number of measurements (rows of H)            */
    int32_t reserved0;
    int64_t nnz;             /* nonzeros of H                                 */
    const int64_t *h_rowptr_dev; /* [p+1], rowptr[0] = 0, rowptr[p] = nnz     */
    const int32_t *h_col_dev;    /* [nnz], in [0, m)                          */
    const double  *h_val_dev;    /* [nnz], finite                             */
    const double  *r_diag_dev;   /* [p], finite and > 0                       */
    const double  *x0_dev;       /* [m] prior mean, or NULL for zero          */
} hikf_problem;

typedef struct hikf_options {
    int32_t n_c;             /* Chebyshev nodes per axis, 1..8 (r = n_c^dim) */
    int32_t fmm_precision;   /* HIKF_FMM_*                                   */
    int32_t direct;          /* 1: exact near-field sum over all leaves, no
                                far field (C_Q exact up to rounding; O(m^2),
                                for small grids and tests)                   */
    int32_t timing;          /* 1: bracket every phase with HIP events on the
                                launch stream; hikf_query reports the sums    */
    int32_t riccati;         /* 0: form G = H C_prior and h = H x_hat from the
                                rows of C every step (a gather over the
                                nonzeros of H).  N >= 1: do that every N-th
                                step only and carry G, h in between with the
                                exact p-space recursion
                                  G <- G S^{-1} R + H C_Q,  h <- h + G S^{-1} nu
                                (from C_post = K R; O(p^3) instead of a read
                                of nnz(H) rows of C).  Import_state forces the
                                next step to gather.  Every periodic gather
                                also measures the drift of the carried values
                                (hikf_stats.riccati_drift_g / _h).            */
    int32_t history;         /* steps of history kept for hikf_cov_apply (the
                                prior cross-covariance and S^{-1} of every
                                applied step: history * (m p + p^2) doubles
                                of RESIDENT); 0 = none                        */
    int32_t graph;           /* 1: capture the step's kernels once, at init,
                                into a HIP graph and replay it per step (y is
                                first copied into the resident region).
                                Ignored when timing = 1.  Results are bitwise
                                those of the launched kernels.                */
    int32_t sparse;          /* 1: P2M and the near field read only the
                                nonzeros of W = H^T, bucketed by leaf at init
                                (no dense m x p W is formed; the scratch
                                shrinks by m p words).  Same H^2 product up to
                                the order of rounding; the near field is then
                                summed in FP32 (FP64 in HIKF_FMM_F64) in every
                                precision mode.  Ignored when direct = 1.     */
    int32_t rowpass_variant; /* launch form of the fused row pass (the step's
                                dominant kernel).  0: automatic, i.e. the
                                entry of tune_cache for this p and C_Q type
                                (nearest m) when tune_cache names a readable
                                cache, else the built-in default.  1 + v
                                forces variant v = 0..7: v & 1 persistent
                                workgroups (one per compute unit, looping over
                                row tiles; in the 8-wave forms p / 16 must be
                                even, else ignored), v & 2 32-row tiles with
                                the columns in four parts instead of 64-row
                                tiles in two halves (always the case for
                                p > 256), v & 4 the dual form: 4-wave
                                workgroups, one wave per SIMD holding two row
                                groups (built for p = 64, 128, 256; ignored
                                otherwise).  Results do not depend on the
                                variant beyond the order in which x_hat and
                                the variance add their column parts.          */
    int32_t reserved1;
    const char *tune_cache;  /* path of a JSON tuning cache written by the
                                package's tuner (python -m
                                paper_1404_3816_amd.tune), or NULL; read by
                                hikf_init only                                */
    int32_t psd_guard;       /* 1: keep the measurement-space prior positive
                                semidefinite.  The H^2 approximation of a
                                smooth kernel makes H Q H^T indefinite by
                                about its error; every step adds it, and
                                S = H P H^T + R then fails its Cholesky after
                                a number of steps set by the most negative
                                eigenvalue (for Gaussian kernels within tens
                                of steps even at n_c = 8).  With the guard,
                                hikf_init replaces H C_Q by its PSD part (the
                                nearest PSD matrix; never farther from the
                                exact H Q H^T) and G = H C_prior, h = H x_hat
                                are carried by the exact p-space recursion
                                (see riccati) from H C_0 + that part (2 x it
                                for P_0 = Q) and H x_0.  riccati = N >= 1
                                then only checks the carried values against a
                                gather every N-th step (riccati_drift_*).
                                0: off (the literal algorithm).               */
    int32_t reserved4;
    double m2l_eps;          /* > 0: low-rank M2L (the SVD compression of the
                                black-box FMM).  Per level the translations
                                share a basis U of rank k: the left singular
                                vectors of all of the level's M2L operators
                                with singular values at least m2l_eps times
                                the largest (Sec. 3.2 cites theorems that fix
                                the rank for an accuracy).  Multipoles are
                                compressed by U^T, translated by U^T T U
                                (k x k) and expanded by U, so a list entry
                                costs 2 k^2 p instead of 2 r^2 p.  The ranks
                                are in hikf_stats.m2l_ranks.  hikf_init then
                                synchronises its stream once (the bases are
                                computed on the host).  0: dense r x r M2L.   */
} hikf_options;

/* Phases timed when hikf_options.timing = 1 (indices of hikf_stats.time_ms). */
enum {
    HIKF_PHASE_OPERATORS = 0, /* Chebyshev and M2L operator construction      */
    HIKF_PHASE_P2M = 1,
    HIKF_PHASE_M2M = 2,       /* all levels together                          */
    HIKF_PHASE_M2L = 3,       /* all levels together                          */
    HIKF_PHASE_L2L = 4,       /* all levels together                          */
    HIKF_PHASE_P2P = 5,       /* fused L2P + P2P                              */
    HIKF_PHASE_INIT = 6,      /* copies, checks, W = H^T, initial state       */
    HIKF_PHASE_GATHER = 7,    /* G = H C_prior, h = H x_hat partial sums       */
    HIKF_PHASE_REDUCE = 8,
    HIKF_PHASE_PSPACE = 9,    /* S, Cholesky, L^{-1}, S^{-1}, innovation      */
    HIKF_PHASE_ROWPASS = 10,  /* gain, state, variance, cross-covariance      */
    HIKF_PHASE_OUTPUT = 11,   /* copies to the caller's x / var buffers       */
    HIKF_NUM_PHASES = 12
};

typedef struct hikf_plan_info {
    size_t resident_bytes;   /* size of the RESIDENT region                  */
    size_t scratch_bytes;    /* size of the SCRATCH region                   */
    int64_t m;               /* N^dim                                        */
    int32_t depth;           /* tree depth D (leaves are 8x8 / 4x4x4 cells)  */
    int32_t r;               /* Chebyshev nodes per box                      */
    int64_t near_pairs;      /* (target leaf, source leaf) pairs in P2P       */
    int64_t far_pairs;       /* interaction-list pairs over all M2L levels    */
    size_t query_bytes;      /* scratch needed by hikf_cov_apply              */
    int32_t rowpass_variant; /* the row-pass variant hikf_init will use (0..7):
                                forced by the options, else from tune_cache,
                                else the built-in default                     */
    int32_t reserved3;
} hikf_plan_info;

typedef struct hikf_stats {
    int64_t steps_applied;   /* assimilation steps applied since init         */
    int32_t last_status;     /* hikf_status of the most recent step           */
    int32_t init_status;     /* hikf_status of the device-side init checks    */
    double min_pivot;        /* smallest Cholesky diagonal of the last step   */
    int64_t negative_variances; /* variance entries that came out negative, summed
                                over all steps since init (no clamping)       */
    double time_ms[HIKF_NUM_PHASES];     /* summed event time per phase       */
    int64_t time_count[HIKF_NUM_PHASES]; /* timed executions per phase        */
    int32_t rowpass_variant; /* row-pass variant in use (0..7, see options)    */
    int32_t reserved2;
    /* Drift of the p-space recursion (options.riccati >= 1): at every
     * periodic gather the carried G = H C_prior and h = H x_hat are compared
     * with the gathered ones; the largest max-norm difference relative to
     * the max-norm of the gathered value seen since init, for G and for h,
     * and the number of such checks.  Zero without the recursion.           */
    double riccati_drift_g;
    double riccati_drift_h;
    int64_t riccati_checks;
    int32_t m2l_ranks[20];   /* rank of the low-rank M2L at each tree level
                                (0 where unused: levels 0-1, dense M2L)       */
} hikf_stats;

typedef struct hikf_filter hikf_filter;

/*
 * Validate a problem and report the workspace it needs.  Host only; reads
 * no device memory and allocates nothing.
 * Errors: HIKF_E_INVALID (dim not 2/3, N < 1, p < 1, nnz < 0, theta/ell not
 * positive, gamma outside (0, 2], n_c outside 1..8, rowpass_variant outside
 * 0..8, psd_guard not 0 or 1, m2l_eps outside [0, 1), NULL arrays),
 * HIKF_E_UNSUPPORTED (p not a multiple of 16 or above 512, n_c^dim above
 * 64, a tree of 2^31 cells or more).  Any N >= 1 is accepted: the tree
 * covers Npad = leaf * 2^D >= N cells per axis (leaf 8 in 2-D, 4 in 3-D) of
 * the same size 1/N, the cells beyond N carry no weight, and out.depth is D.
 */
hikf_status hikf_plan(const hikf_problem *prob, const hikf_options *opt,
                      hikf_plan_info *out);

/*
 * Build the filter: copy H, R and x_0 into RESIDENT, form W = H^T, compute
 * C_Q = Q H^T with the H^2 / FMM passes (Sec. 3.2: P2M, M2M, M2L, L2L, L2P,
 * P2P), then set C_0, var_0, x_0 from the prior (Sec. 3.1 end).
 * resident_dev / scratch_dev: caller-owned device regions of at least the
 * planned sizes, 256-byte aligned.  RESIDENT must outlive the filter;
 * SCRATCH may be reused once this call's work has completed on `stream`.
 * *out receives a host-side handle (free it with hikf_destroy).
 * Errors: as hikf_plan, HIKF_E_NOMEM (a region too small or misaligned),
 * HIKF_E_DEVICE (a launch failed).  Bad device data (column out of range,
 * non-finite values, R not positive) poisons the filter: hikf_query then
 * reports init_status = HIKF_E_INVALID and every step is a no-op.
 */
hikf_status hikf_init(const hikf_problem *prob, const hikf_options *opt,
                      void *resident_dev, size_t resident_bytes,
                      void *scratch_dev, size_t scratch_bytes,
                      void *stream, hikf_filter **out);

/*
 * One assimilation step with measurement y_k (p doubles, y_dev), i.e. the
 * prediction and correction of Algorithm Algorithm_HiKF:
 *   C <- C + C_Q, var <- var + K(0); G = H C; S = (G + G^T)/2 + R = L L^T;
 *   K = C S^{-1}; x_hat += K (y - H x_hat); var_i -= sum_j K_ij C_ij;
 *   C <- K R   (equal to C - K G, the posterior cross-covariance).
 * x_out_dev / var_out_dev (m doubles each, grid order) receive x_hat_{k|k}
 * and diag P_{k|k}; either may be NULL to skip the copy.
 * Transactional: if S is not positive definite or y holds a NaN/Inf the
 * state is left unchanged and hikf_query reports the status.
 * Errors (immediate): HIKF_E_INVALID (NULL filter or y), HIKF_E_DEVICE.
 */
hikf_status hikf_step(hikf_filter *f, const double *y_dev, double *x_out_dev,
                      double *var_out_dev, void *stream);

/*
 * Grouped step for a serving loop: hikf_step(filters[i], y_dev[i], x_out[i],
 * var_out[i]) for i = 0 .. count-1.  The steps run concurrently on a few
 * internal streams of the device (created on first use, kept for the life
 * of the process), ordered after the work already queued on `stream`, and
 * `stream` waits for all of them before anything queued on it later.
 * x_out_dev / var_out_dev may be NULL (no copies for any filter) or hold
 * NULL entries.  Each filter's result is exactly its solo hikf_step result;
 * the filters must be distinct.
 * Errors: HIKF_E_INVALID (count < 0, NULL arrays, a NULL filter or y, a
 * filter listed twice: then no filter is stepped), otherwise the first
 * immediate error of a step
 * (the filters before it have been stepped, the ones after it have not).
 */
hikf_status hikf_step_batch(hikf_filter *const *filters, const double *const *y_dev,
                            double *const *x_out_dev, double *const *var_out_dev,
                            int32_t count, void *stream);

/*
 * Posterior covariance times a vector: out = P_{t|t} v for the current step
 * t (Sec. 3.1 keeps P only implicitly; Sec. 4 uses variances and
 * cross-covariances for risk analysis).  With P_{s|s} = P_{s|s-1} -
 * C_s S_s^{-1} C_s^T and P_{s|s-1} = P_{s-1|s-1} + Q,
 *   P_t v = P_0 v + t Q v - sum_{s=1..t} C_s (S_s^{-1} (C_s^T v)),
 * where C_s is the prior cross-covariance and S_s the innovation covariance
 * of step s, kept in the history (hikf_options.history >= t).  Q v is one
 * FMM product with the filter's tree and n_c (FP32 for the BF16 modes).
 * v_dev, out_dev: m doubles in grid order.  scratch: at least
 * hikf_plan_info.query_bytes, 256-byte aligned.  Synchronises the stream.
 * Errors: HIKF_E_INVALID (NULL arguments), HIKF_E_UNSUPPORTED (no history,
 * or more steps applied than it holds), HIKF_E_NOMEM, HIKF_E_DEVICE.
 */
hikf_status hikf_cov_apply(hikf_filter *f, const double *v_dev, double *out_dev,
                           void *scratch, size_t scratch_bytes, void *stream);

/*
 * hikf_cov_apply without a workspace argument, for callers that cannot
 * allocate device memory (code under stream capture, tight serving loops,
 * harnesses that forbid allocation).  The workspace is a fixed array of
 * HIKF_NOALLOC_SCRATCH_BYTES inside the library's device code, one per
 * device, held until the process ends; the call allocates nothing and
 * frees nothing.  Every call on a device shares that device's array, so
 * calls that overlap on one device (on different streams or host threads)
 * race: serialise them.  Results equal hikf_cov_apply's.  Synchronises the
 * stream.
 * Errors: as hikf_cov_apply; HIKF_E_NOMEM when the query needs more than
 * HIKF_NOALLOC_SCRATCH_BYTES (hikf_plan_info.query_bytes; about 11 MB for a
 * 256 x 256 grid, p = 64, eight steps of history), with the sizes in
 * hikf_last_error.
 */
#define HIKF_NOALLOC_SCRATCH_BYTES (32u << 20)
hikf_status hikf_cov_apply_noalloc(hikf_filter *f, const double *v_dev, double *out_dev,
                                   void *stream);

/*
 * Synchronise the filter's last stream and read its device status and, if
 * timing is on, the phase times accumulated since init.
 * Errors: HIKF_E_INVALID (NULL), HIKF_E_DEVICE.
 */
hikf_status hikf_query(hikf_filter *f, hikf_stats *out);

/*
 * Copy the state into caller device buffers (any may be NULL):
 * x_dev [m], var_dev [m], c_dev [m*p] (row i = grid cell i, p contiguous).
 */
hikf_status hikf_export_state(hikf_filter *f, double *x_dev, double *var_dev,
                              double *c_dev, void *stream);

/* Overwrite the state from caller device buffers (same layouts; NULL keeps
 * that part).  The next step gathers G and h from the imported rows (with
 * the PSD guard, which has no gather, use hikf_import_checkpoint).  For a
 * checkpoint that carries its step count and problem identity, use
 * hikf_export_checkpoint / hikf_import_checkpoint. */
hikf_status hikf_import_state(hikf_filter *f, const double *x_dev,
                              const double *var_dev, const double *c_dev,
                              void *stream);

/* Identity and position of a checkpoint (filled by hikf_export_checkpoint). */
typedef struct hikf_checkpoint_info {
    uint64_t problem_hash;   /* digest of H, R, x_0, grid, kernel, prior and
                                the options that shape the state (n_c, FMM
                                arithmetic, direct, sparse, psd_guard)        */
    int64_t steps_applied;   /* steps applied when the checkpoint was taken   */
    int64_t steps_issued;    /* steps issued (the recursion's gather period)  */
    int32_t p;               /* measurements; pspace_dev holds p*p + p values */
    int32_t carried;         /* 1: G and h were carried (recursion or guard) */
} hikf_checkpoint_info;

/*
 * Checkpoint: x_hat (m), diag P (m), C (m*p), and the p-space state
 * pspace_dev = [G (p*p, row-major) | h (p)] that the recursion or the PSD
 * guard carries (any pointer may be NULL to skip that part), plus *info.
 * Synchronises the stream (the step count is read from the device).
 * Errors: HIKF_E_INVALID (NULL filter or info), HIKF_E_DEVICE.
 */
hikf_status hikf_export_checkpoint(hikf_filter *f, double *x_dev, double *var_dev,
                                   double *c_dev, double *pspace_dev,
                                   hikf_checkpoint_info *info, void *stream);

/*
 * Resume from a checkpoint of a filter built from the same problem and
 * options: the parts given are copied in, the step count is restored, and
 * with pspace_dev (and info->carried) the carried G, h are restored so the
 * next step continues exactly as the exported filter's would have.
 * Errors (nothing is copied): HIKF_E_INVALID (NULL filter or info, a
 * problem hash or p that differs from this filter's, or the PSD guard
 * without pspace_dev), HIKF_E_DEVICE.
 */
hikf_status hikf_import_checkpoint(hikf_filter *f, const double *x_dev, const double *var_dev,
                                   const double *c_dev, const double *pspace_dev,
                                   const hikf_checkpoint_info *info, void *stream);

/*
 * Copy C_Q = Q H^T (m x p, grid order, p contiguous) widened to FP64 into
 * cq_dev.  This is the H^2 product of Sec. 3.2 as the filter uses it.
 */
hikf_status hikf_export_cq(hikf_filter *f, double *cq_dev, void *stream);

/* Release the host-side handle (device regions belong to the caller). */
void hikf_destroy(hikf_filter *f);

/* Static text for a status code. */
const char *hikf_status_string(hikf_status s);

/* Text of the last error seen on this filter (empty if none). */
const char *hikf_last_error(const hikf_filter *f);

#ifdef __cplusplus
}
#endif

#endif /* HIKF_H */
