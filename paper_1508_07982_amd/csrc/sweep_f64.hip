// Instantiation of the fused sweep for double storage.
#include "sweep.hpp"

namespace lbm {

hipError_t launch_sweep_f64(int n, const SweepArgs& a, int grid, hipStream_t stream) {
  return dev::launch_sweep_t<double>(n, a, grid, stream);
}

}  // namespace lbm
