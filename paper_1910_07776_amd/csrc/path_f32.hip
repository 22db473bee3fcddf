// Instantiation of the fused scoring kernel for float counters.
#include "path_impl.hpp"

namespace sugg {

template <>
hipError_t launch_path<float>(const PathArgs<float>& a, int max_item_rows, int max_item_kernels, int max_B,
                            const PathLaunch& cfg, hipStream_t s) {
  return launch_path_impl<float>(a, max_item_rows, max_item_kernels, max_B, cfg, s);
}

}  // namespace sugg
