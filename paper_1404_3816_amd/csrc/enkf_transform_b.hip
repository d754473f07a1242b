// Ensemble transform kernels for the tile widths ld = 16 NT, NT in {10, 12, 16, 20}.
#include "enkf_transform.h"

namespace hikf {

template hipError_t enkf_transform_nt<10>(int, int64_t, int, double *, const double *,
                                         const double *, double *, double *, const int *,
                                         long long *, hipStream_t);
template hipError_t enkf_transform_nt<12>(int, int64_t, int, double *, const double *,
                                         const double *, double *, double *, const int *,
                                         long long *, hipStream_t);
template hipError_t enkf_transform_nt<16>(int, int64_t, int, double *, const double *,
                                         const double *, double *, double *, const int *,
                                         long long *, hipStream_t);
template hipError_t enkf_transform_nt<20>(int, int64_t, int, double *, const double *,
                                         const double *, double *, double *, const int *,
                                         long long *, hipStream_t);

}  // namespace hikf
