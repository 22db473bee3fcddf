// Fused scoring kernel variants for double counters, 4 columns per lane.
#include "path_impl.hpp"

namespace sugg {
template hipError_t launch_path_vpl<double, 4>(const PathArgs<double>&, int, int, int, const PathLaunch&, hipStream_t);
}  // namespace sugg
