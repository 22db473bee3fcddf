// Chooses the fused scoring kernel's column-per-lane variant from E.
#include "kernels.hpp"

namespace sugg {

template <typename T>
hipError_t launch_path(const PathArgs<T>& a, int max_item_rows, int max_item_kernels, int max_B,
                       const PathLaunch& cfg, hipStream_t s) {
  if (a.E <= 16 * 4) return launch_path_vpl<T, 4>(a, max_item_rows, max_item_kernels, max_B, cfg, s);
  if (a.E <= 16 * 8) return launch_path_vpl<T, 8>(a, max_item_rows, max_item_kernels, max_B, cfg, s);
  return launch_path_vpl<T, 16>(a, max_item_rows, max_item_kernels, max_B, cfg, s);
}

template hipError_t launch_path<float>(const PathArgs<float>&, int, int, int, const PathLaunch&, hipStream_t);
template hipError_t launch_path<double>(const PathArgs<double>&, int, int, int, const PathLaunch&, hipStream_t);

}  // namespace sugg
