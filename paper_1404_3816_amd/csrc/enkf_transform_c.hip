// Ensemble transform kernels for the tile widths ld = 16 NT, NT in {24, 25}.
#include "enkf_transform.h"

namespace hikf {

template hipError_t enkf_transform_nt<24>(int, int64_t, int, double *, const double *,
                                         const double *, double *, double *, const int *,
                                         long long *, hipStream_t);
template hipError_t enkf_transform_nt<25>(int, int64_t, int, double *, const double *,
                                         const double *, double *, double *, const int *,
                                         long long *, hipStream_t);

}  // namespace hikf
