/*
 * hikf_enkf.h -- C ABI of the ensemble Kalman filter on the MI355X (gfx950).
 *
 * The perturbed-observation EnKF of Sec. 2.3 (eqs. equation_samplemean,
 * equation_samplecov1, equation_samplegain_enkf), the method the paper
 * compares HiKF with, on the same random-walk model (Sec. 2.1, eq.
 * equation_random_walk) and the same sparse H and diagonal R.  One step,
 * for the ensemble X = [x^1 ... x^N] (m x N):
 *
 *   forecast  x^j <- x^j + w^j                      (w^j from N(0, Q), given)
 *   mean      x~ = X 1 / N;  A = (X - x~ 1^T) / sqrt(N - 1);  Sigma~ = A A^T
 *   gain      K~ = A (H A)^T S^{-1},  S = (H A)(H A)^T + R
 *   analysis  x^j <- x^j + K~ (y + v^j - H x^j)      (v^j from N(0, R), given)
 *
 * Sigma~ is never formed.  The library applies the analysis to the whole
 * ensemble as one product X <- X W with the N x N matrix
 *   W = I + (I - 1 1^T / N) T / sqrt(N - 1),  T = (H A)^T S^{-1} D,
 * D = y 1^T + V - H X (column j: the innovation of member j); this equals
 * x^j + K~ (d^j - H x^j) for every member.  Every random draw is an input:
 * the library draws nothing.
 *
 * Memory model, pointers, streams, errors: as in hikf.h (the caller owns a
 * RESIDENT region sized by hikf_enkf_plan; *_dev pointers are device
 * pointers; work is queued on the caller's stream; device-side failures are
 * reported by hikf_enkf_query).  Ensemble layout: row i = grid cell i (the
 * grid order of hikf.h), members contiguous; the library stores X with a
 * row pitch of hikf_enkf_plan_info.ld >= N doubles.
 */
#ifndef HIKF_ENKF_H
#define HIKF_ENKF_H

#include <stddef.h>
#include <stdint.h>

#include "hikf.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hikf_enkf_problem {
    int64_t m;                   /* state size (grid cells), >= 1             */
    int32_t p;                   /* measurements (rows of H), 1..512          */
    int32_t n_ens;               /* ensemble members N, 2..512                 */
    int64_t nnz;                 /* nonzeros of H                              */
    const int64_t *h_rowptr_dev; /* [p+1], rowptr[0] = 0, rowptr[p] = nnz     */
    const int32_t *h_col_dev;    /* [nnz], in [0, m)                           */
    const double  *h_val_dev;    /* [nnz], finite                              */
    const double  *r_diag_dev;   /* [p], finite and > 0                        */
    int32_t timing;              /* 1: HIP events around the step's phases     */
    int32_t tile_rows;           /* rows per workgroup of the ensemble
                                    transform: 32, 64, 128 (N <= 256 only), or
                                    0 = automatic (128 for N <= 256, else 64) */
} hikf_enkf_problem;

typedef struct hikf_enkf_plan_info {
    size_t resident_bytes;       /* RESIDENT region for hikf_enkf_init         */
    int32_t ld;                  /* row pitch (doubles) of the stored ensemble
                                    and of the model-error draws E: N rounded
                                    up to the width of a transform tile        */
    int32_t gather_chunks;       /* workgroups of the H X gather (0 before init:
                                    it depends on the device row pointer)      */
} hikf_enkf_plan_info;

/* Phases timed with HIP events (hikf_enkf_stats.time_ms). */
enum {
    HIKF_ENKF_PHASE_GATHER = 0,    /* H (X + E): the ray rows of the forecast  */
    HIKF_ENKF_PHASE_NSPACE = 1,    /* H A, D, S, S^{-1}, T, W (p- and N-space) */
    HIKF_ENKF_PHASE_TRANSFORM = 2, /* X <- (X + E) W, mean and variance rows   */
    HIKF_ENKF_NUM_PHASES = 4
};

typedef struct hikf_enkf_stats {
    int64_t steps_applied;       /* steps whose analysis was applied           */
    int32_t last_status;         /* hikf_status of the last step               */
    int32_t init_status;         /* device-side checks of H and R at init      */
    double min_pivot;            /* smallest Cholesky diagonal of S, last step */
    double time_ms[HIKF_ENKF_NUM_PHASES];   /* sums since init (timing = 1)   */
    int64_t time_count[HIKF_ENKF_NUM_PHASES];
} hikf_enkf_stats;

typedef struct hikf_enkf hikf_enkf;

/*
 * Validate a problem and report the workspace (host only, reads no device
 * memory).  Errors: HIKF_E_INVALID (m < 1, p < 1, N < 2, nnz < 0, NULL
 * arrays, tile_rows not 0, 32, 64 or 128), HIKF_E_UNSUPPORTED (p > 512 or
 * N > 512: the transform keeps a member row in the registers of a wave and
 * the sweep inverse handles p <= 512; tile_rows 128 with N > 256).
 */
hikf_status hikf_enkf_plan(const hikf_enkf_problem *prob, hikf_enkf_plan_info *out);

/*
 * Build the filter: copy H and R into RESIDENT (checked on the device: a
 * column out of range, a non-finite value or R <= 0 poisons the filter and
 * every step is then a no-op reported by hikf_enkf_query), and the initial
 * ensemble x0_dev (m x N, row i = cell i, members contiguous, pitch N) into
 * the stored ensemble.  Reads the row pointer of H back to the host to cut
 * the gather into chunks (synchronises `stream`).
 * Errors: as hikf_enkf_plan, HIKF_E_NOMEM (RESIDENT too small or not
 * 256-byte aligned), HIKF_E_DEVICE.
 */
hikf_status hikf_enkf_init(const hikf_enkf_problem *prob, const double *x0_dev,
                           void *resident_dev, size_t resident_bytes, void *stream,
                           hikf_enkf **out);

/*
 * One forecast + analysis step.
 *   e_dev   model-error draws w^j: m rows of plan ld doubles (member j in
 *           column j; the columns N..ld-1 are ignored), or NULL for none;
 *   y_dev   the data y (p doubles);
 *   v_dev   observation perturbations v^j: p x N, pitch N (row = ray);
 *   mean_out_dev, var_out_dev   m doubles each (either may be NULL): the
 *           analysis sample mean x~ and the diagonal of Sigma~ (eq.
 *           equation_samplecov1, 1/(N-1) normalisation).
 * Transactional: if S is not positive definite or y, V or the innovations
 * hold a NaN/Inf, the ensemble is left unchanged (the forecast is not
 * applied either) and hikf_enkf_query reports the status.
 * Errors (immediate): HIKF_E_INVALID (NULL filter, y or v), HIKF_E_DEVICE.
 */
hikf_status hikf_enkf_step(hikf_enkf *f, const double *e_dev, const double *y_dev,
                           const double *v_dev, double *mean_out_dev, double *var_out_dev,
                           void *stream);

/* Synchronise the last stream and read the status, counters and phase
 * times.  Errors: HIKF_E_INVALID (NULL), HIKF_E_DEVICE. */
hikf_status hikf_enkf_query(hikf_enkf *f, hikf_enkf_stats *out);

/* Copy the ensemble out to x_dev (m x N, pitch N) / in from x_dev (same
 * layout; the step count is kept).  Errors: HIKF_E_INVALID, HIKF_E_DEVICE. */
hikf_status hikf_enkf_export(hikf_enkf *f, double *x_dev, void *stream);
hikf_status hikf_enkf_import(hikf_enkf *f, const double *x_dev, void *stream);

/* Release the host-side handle (the device region belongs to the caller). */
void hikf_enkf_destroy(hikf_enkf *f);

/* Text of the last error seen on this filter (empty if none). */
const char *hikf_enkf_last_error(const hikf_enkf *f);

#ifdef __cplusplus
}
#endif

#endif /* HIKF_ENKF_H */
