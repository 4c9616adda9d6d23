// Instantiation of the fused sweep for __half storage.
#include "sweep.hpp"

namespace lbm {

hipError_t launch_sweep_f16(int n, const SweepArgs& a, int grid, hipStream_t stream) {
  return dev::launch_sweep_t<__half>(n, a, grid, stream);
}

}  // namespace lbm
