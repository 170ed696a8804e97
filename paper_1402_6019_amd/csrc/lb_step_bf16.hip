// Step and batch launchers of the BF16-deviation storage mode, rounding to nearest or
// stochastically: the instantiations of the fused step kernels for this mode (one translation
// unit per mode, compiled in parallel).  The stochastically rounding variant exists for the
// passes that store populations (and the observation pass of a reducing step); every other
// pass reads BF16 like the nearest-rounding variant.

#include "lb_step.hpp"
#include "lb_step2.hpp"

namespace lb355 {

hipError_t launch_step_bf16(bool stochastic, int ns, int walls, int what, int tx, int nb, const StepArgs &a,
                            hipStream_t st) {
  if (!stochastic || (what != WHAT_STEP && what != WHAT_STEP_ACCUM && what != WHAT_OBSERVE))
    return launch_step_m<MODE_BF16>(ns, walls, what, tx, nb, a, st);
  if (ns == 1) return walls ? launch_step_sr_t<1, true>(what, tx, nb, a, st) : launch_step_sr_t<1, false>(what, tx, nb, a, st);
  return walls ? launch_step_sr_t<2, true>(what, tx, nb, a, st) : launch_step_sr_t<2, false>(what, tx, nb, a, st);
}

hipError_t launch_batch_bf16(bool stochastic, int ns, int walls, int what, int tx, int grid, const BatchArgs &b,
                             hipStream_t st) {
  if (!stochastic || (what != WHAT_STEP && what != WHAT_STEP_ACCUM))
    return launch_batch_m<MODE_BF16>(ns, walls, what, tx, grid, b, st);
  if (ns == 1) return walls ? launch_batch_sr_t<1, true>(what, tx, grid, b, st) : launch_batch_sr_t<1, false>(what, tx, grid, b, st);
  return walls ? launch_batch_sr_t<2, true>(what, tx, grid, b, st) : launch_batch_sr_t<2, false>(what, tx, grid, b, st);
}

int blocks_per_cu_bf16(int ns, int walls, int tx) { return blocks_per_cu_m<MODE_BF16>(ns, walls, tx); }

template <int MODE, int NS, bool WALLS>
static hipError_t launch2_t(int streaming, int nb, const StepArgs &a, hipStream_t st) {
  const size_t lds = step2_lds_bytes(MODE, NS);
  if (streaming) hipLaunchKernelGGL((step2_kernel<MODE, NS, WALLS, kStoreStreaming>), dim3(nb), dim3(64), lds, st, a);
  else hipLaunchKernelGGL((step2_kernel<MODE, NS, WALLS, kStoreWriteThrough>), dim3(nb), dim3(64), lds, st, a);
  return hipGetLastError();
}

template <int MODE>
static hipError_t launch2_m(int ns, int walls, int nb, const StepArgs &a, hipStream_t st) {
  if (ns == 1) return walls ? launch2_t<MODE, 1, true>(a.stream_stores, nb, a, st) : launch2_t<MODE, 1, false>(a.stream_stores, nb, a, st);
  return walls ? launch2_t<MODE, 2, true>(a.stream_stores, nb, a, st) : launch2_t<MODE, 2, false>(a.stream_stores, nb, a, st);
}

hipError_t launch_step2_bf16(bool stochastic, int ns, int walls, int nb, const StepArgs &a, hipStream_t st) {
  return stochastic ? launch2_m<MODE_BF16SR>(ns, walls, nb, a, st) : launch2_m<MODE_BF16>(ns, walls, nb, a, st);
}

}  // namespace lb355
