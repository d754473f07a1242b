// Ensemble transform kernels for the tile width ld = 16 NT, NT = 32.
#include "enkf_transform.h"

namespace hikf {

template hipError_t enkf_transform_nt<32>(int, int64_t, int, double *, const double *,
                                         const double *, double *, double *, const int *,
                                         long long *, hipStream_t);

}  // namespace hikf
