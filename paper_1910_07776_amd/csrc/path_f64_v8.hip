// Fused scoring kernel variants for double counters, 8 columns per lane.
#include "path_impl.hpp"

namespace sugg {
template hipError_t launch_path_vpl<double, 8>(const PathArgs<double>&, int, int, int, const PathLaunch&, hipStream_t);
}  // namespace sugg
