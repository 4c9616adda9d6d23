// Instantiation of the fused sweep for float storage.
#include "sweep.hpp"

namespace lbm {

hipError_t launch_sweep_f32(int n, const SweepArgs& a, int grid, int split, hipStream_t stream) {
  return dev::launch_sweep_t<float>(n, a, grid, split, stream);
}

int sweep_split_f32(int n, int requested) { return dev::sweep_split_t<float>(n, requested); }

}  // namespace lbm
