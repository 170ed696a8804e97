// Step and batch launchers of the F64 storage mode: the instantiations of the fused
// step kernels for this mode (one translation unit per mode, compiled in parallel).

#include "lb_step.hpp"
#include "lb_step2.hpp"

namespace lb355 {

hipError_t launch_step_f64(int ns, int walls, int what, int tx, int nb, const StepArgs &a, hipStream_t st) {
  return launch_step_m<MODE_F64>(ns, walls, what, tx, nb, a, st);
}

hipError_t launch_batch_f64(int ns, int walls, int what, int tx, int grid, const BatchArgs &b, hipStream_t st) {
  return launch_batch_m<MODE_F64>(ns, walls, what, tx, grid, b, st);
}

int blocks_per_cu_f64(int ns, int walls, int tx) { return blocks_per_cu_m<MODE_F64>(ns, walls, tx); }

template <int NS, bool WALLS>
static hipError_t launch2_t(int streaming, int nb, const StepArgs &a, hipStream_t st) {
  const size_t lds = step2_lds_bytes(MODE_F64, NS);
  if (streaming) hipLaunchKernelGGL((step2_kernel<MODE_F64, NS, WALLS, kStoreStreaming>), dim3(nb), dim3(64), lds, st, a);
  else hipLaunchKernelGGL((step2_kernel<MODE_F64, NS, WALLS, kStoreWriteThrough>), dim3(nb), dim3(64), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_step2_f64(int ns, int walls, int nb, const StepArgs &a, hipStream_t st) {
  if (ns == 1) return walls ? launch2_t<1, true>(a.stream_stores, nb, a, st) : launch2_t<1, false>(a.stream_stores, nb, a, st);
  return walls ? launch2_t<2, true>(a.stream_stores, nb, a, st) : launch2_t<2, false>(a.stream_stores, nb, a, st);
}

int blocks2_per_cu_f64(int ns, int walls) {
  int n = 0;
  hipError_t e;
  if (ns == 1) e = walls ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step2_kernel<MODE_F64, 1, true, kStoreWriteThrough>, 64, step2_lds_bytes(MODE_F64, 1))
                        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step2_kernel<MODE_F64, 1, false, kStoreWriteThrough>, 64, step2_lds_bytes(MODE_F64, 1));
  else e = walls ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step2_kernel<MODE_F64, 2, true, kStoreWriteThrough>, 64, step2_lds_bytes(MODE_F64, 2))
                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step2_kernel<MODE_F64, 2, false, kStoreWriteThrough>, 64, step2_lds_bytes(MODE_F64, 2));
  return e == hipSuccess && n > 0 ? n : 1;
}

}  // namespace lb355
