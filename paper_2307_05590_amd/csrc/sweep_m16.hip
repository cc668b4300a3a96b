// Instantiations of the sweep kernels for the M <= 16 bucket.
#include "sweep_impl.h"

namespace mpt {
template hipError_t launch_plain<16, false>(const mpt_rom&, const double*, int64_t, double*,
    double*, int32_t*, const double*, double*, int, const MatSens&, hipStream_t);
template hipError_t launch_persistent<16, false>(const mpt_rom*, const int4*, int,
    unsigned int*, const double*, double*, int32_t*, const double*, double*, int, int, hipStream_t);
template hipError_t launch_plain<16, true>(const mpt_rom&, const double*, int64_t, double*,
    double*, int32_t*, const double*, double*, int, const MatSens&, hipStream_t);
template hipError_t launch_persistent<16, true>(const mpt_rom*, const int4*, int,
    unsigned int*, const double*, double*, int32_t*, const double*, double*, int, int, hipStream_t);
}  // namespace mpt
