// Instantiation of the fused sweep for __half storage.
#include "sweep.hpp"

namespace lbm {

hipError_t launch_sweep_f16(int n, const SweepArgs& a, int grid, int split, hipStream_t stream) {
  return dev::launch_sweep_t<__half>(n, a, grid, split, stream);
}

int sweep_split_f16(int n, int requested) { return dev::sweep_split_t<__half>(n, requested); }

}  // namespace lbm
