// Instantiation of the fused sweep for float storage.
#include "sweep.hpp"

namespace lbm {

hipError_t launch_sweep_f32(int n, const SweepArgs& a, int grid, hipStream_t stream) {
  return dev::launch_sweep_t<float>(n, a, grid, stream);
}

}  // namespace lbm
