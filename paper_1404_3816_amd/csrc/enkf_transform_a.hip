// Ensemble transform kernels for the tile widths ld = 16 NT, NT in {1, 2, 3, 4, 5, 6, 8}.
#include "enkf_transform.h"

namespace hikf {

template hipError_t enkf_transform_nt<1>(int, int64_t, int, double *, const double *,
                                         const double *, double *, double *, const int *,
                                         long long *, hipStream_t);
template hipError_t enkf_transform_nt<2>(int, int64_t, int, double *, const double *,
                                         const double *, double *, double *, const int *,
                                         long long *, hipStream_t);
template hipError_t enkf_transform_nt<3>(int, int64_t, int, double *, const double *,
                                         const double *, double *, double *, const int *,
                                         long long *, hipStream_t);
template hipError_t enkf_transform_nt<4>(int, int64_t, int, double *, const double *,
                                         const double *, double *, double *, const int *,
                                         long long *, hipStream_t);
template hipError_t enkf_transform_nt<5>(int, int64_t, int, double *, const double *,
                                         const double *, double *, double *, const int *,
                                         long long *, hipStream_t);
template hipError_t enkf_transform_nt<6>(int, int64_t, int, double *, const double *,
                                         const double *, double *, double *, const int *,
                                         long long *, hipStream_t);
template hipError_t enkf_transform_nt<8>(int, int64_t, int, double *, const double *,
                                         const double *, double *, double *, const int *,
                                         long long *, hipStream_t);

}  // namespace hikf
