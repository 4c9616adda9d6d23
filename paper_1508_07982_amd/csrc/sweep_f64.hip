// Instantiation of the fused sweep for double storage.
#include "sweep.hpp"

namespace lbm {

hipError_t launch_sweep_f64(int n, const SweepArgs& a, int grid, int split, hipStream_t stream) {
  return dev::launch_sweep_t<double>(n, a, grid, split, stream);
}

int sweep_split_f64(int n, int requested) { return dev::sweep_split_t<double>(n, requested); }

}  // namespace lbm
