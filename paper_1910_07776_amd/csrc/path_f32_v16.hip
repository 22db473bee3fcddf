// Fused scoring kernel variants for float counters, 16 columns per lane.
#include "path_impl.hpp"

namespace sugg {
template hipError_t launch_path_vpl<float, 16>(const PathArgs<float>&, int, int, int, const PathLaunch&, hipStream_t);
}  // namespace sugg
