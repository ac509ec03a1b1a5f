// 3D kernels (D3Q15 / D3Q19): not built yet.
#include "lks_device.hpp"

namespace lks {

template <typename T>
hipError_t launch_fwd3d(const FwdArgs<T> &, int, hipStream_t) { return hipErrorNotSupported; }
template <typename T>
hipError_t launch_adj3d(const AdjArgs<T> &, int, hipStream_t) { return hipErrorNotSupported; }

template hipError_t launch_fwd3d<float>(const FwdArgs<float> &, int, hipStream_t);
template hipError_t launch_fwd3d<double>(const FwdArgs<double> &, int, hipStream_t);
template hipError_t launch_adj3d<float>(const AdjArgs<float> &, int, hipStream_t);
template hipError_t launch_adj3d<double>(const AdjArgs<double> &, int, hipStream_t);

}  // namespace lks
