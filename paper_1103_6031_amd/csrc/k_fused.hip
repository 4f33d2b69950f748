// Fused red+black sweep for large periodic levels (placeholder: not yet enabled).
#include "mg_internal.h"

namespace mgic {

template <class T>
bool fused_sweep_supported(Dims) {
    return false;
}

template <class T>
void launch_rbgs_fused(const T*, T*, const T*, Dims, double, hipStream_t) {}

template bool fused_sweep_supported<double>(Dims);
template bool fused_sweep_supported<float>(Dims);
template void launch_rbgs_fused<double>(const double*, double*, const double*, Dims, double, hipStream_t);
template void launch_rbgs_fused<float>(const float*, float*, const float*, Dims, double, hipStream_t);

}  // namespace mgic
