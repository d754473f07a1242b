// Internal declarations of the ensemble Kalman filter sources (enkf.hip and
// the enkf_transform_*.hip units); not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hikf {

// Widths of a transform tile: the stored ensemble has ld = 16 * NT columns
// with NT the smallest of these at or above N / 16 (N <= 512).
constexpr int kEnTileCounts[] = {1, 2, 3, 4, 5, 6, 8, 10, 12, 16, 20, 24, 25, 28, 32};
constexpr int kEnMaxMembers = 512;

inline int enkf_ld(int n_ens) {
    for (int nt : kEnTileCounts)
        if (16 * nt >= n_ens) return 16 * nt;
    return 0;
}

// X <- (X + E) W on the m rows of the ensemble (pitch ld), with the row
// means and variances over the first n_ens columns in xmean / xvar; E may be
// null.  tile_rows: rows per workgroup, 32 or 64 (0 = by ld).  Does nothing
// when status[kStStep] is not HIKF_OK; otherwise adds one to applied[0].
hipError_t launch_enkf_transform(int tile_rows, int64_t m, int n_ens, int ld, double *X,
                                 const double *E, const double *W, double *xmean, double *xvar,
                                 const int *status, long long *applied, hipStream_t s);

// the transform for ld = 16 NT (defined in enkf_transform.h, instantiated
// by one of the enkf_transform_*.hip units)
template <int NT>
hipError_t enkf_transform_nt(int tile_rows, int64_t m, int n_ens, double *X, const double *E,
                             const double *W, double *xmean, double *xvar, const int *status,
                             long long *applied, hipStream_t s);

}  // namespace hikf
