// The blocked symmetric sweep inverse of the p-space pass (pspace.hip),
// exported for the other p x p users of the library.
#pragma once

#include <hip/hip_runtime.h>

namespace hikf {

// S = (G + G^T)/2 + diag(rdiag) (p x p, row-major G), padded to pp = 32
// ceil(p / 32) with an identity block, inverted by pp / 32 launches on
// `s`.  Launch 0 clears status[kStStep] (INVALID if status[kStInit] is set
// or y holds a NaN / Inf, OK otherwise) and writes nu = y - hvec; a
// non-positive pivot sets HIKF_E_NOT_SPD and leaves Sinv unwritten.  On
// success Sinv (p x p) holds S^{-1}, minpiv[0] the smallest Cholesky
// diagonal and steps[0] is incremented.  A and X: two pp x pp work buffers;
// pivs: pp / 32 doubles.
struct SweepArgs {
    int p, pp;
    const double *G, *rdiag, *y, *hvec;
    double *A, *X, *Sinv, *nu, *pivs, *minpiv;
    int *status;
    long long *steps;
};

hipError_t launch_sweep_inverse(const SweepArgs &a, hipStream_t s);

}  // namespace hikf
