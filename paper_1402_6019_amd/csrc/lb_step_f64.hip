// Step and batch launchers of the F64 storage mode: the instantiations of the fused
// step kernels for this mode (one translation unit per mode, compiled in parallel).

#include "lb_step.hpp"

namespace lb355 {

hipError_t launch_step_f64(int ns, int walls, int what, int tx, int nb, const StepArgs &a, hipStream_t st) {
  return launch_step_m<MODE_F64>(ns, walls, what, tx, nb, a, st);
}

hipError_t launch_batch_f64(int ns, int walls, int what, int tx, int grid, const BatchArgs &b, hipStream_t st) {
  return launch_batch_m<MODE_F64>(ns, walls, what, tx, grid, b, st);
}

int blocks_per_cu_f64(int ns, int walls, int tx) { return blocks_per_cu_m<MODE_F64>(ns, walls, tx); }

}  // namespace lb355
