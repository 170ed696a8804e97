// Internal declarations of the 3-D step (lb3_kernels.hip, lb3_api.cpp).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lb_internal.hpp"

namespace lb355 {

// Per-workgroup partial sums of the 3-D observation pass.
enum Red3Slot { RED3_MASS0 = 0, RED3_MASS1, RED3_PX, RED3_PY, RED3_PZ, RED3_FLOW, RED3_BAD, RED3_N };

// Kernel arguments of the 3-D fused step.
struct Lb3Args {
  const void *src;    // post-collision populations of the previous step (pull source)
  void *dst;          // post-collision populations of this step
  double *partials;   // WHAT_OBSERVE: [gridDim.x][RED3_N]
  void *out_rho;      // WHAT_MOMENTS: [ns][lz][ly][lx]
  void *out_u;        // WHAT_MOMENTS: [3][lz][ly][lx]
  int lx, ly, lz, pitch;       // lattice; row pitch in sites
  int sz, nstrip, nband, nseg; // z-planes per workgroup; grid = nstrip (64 columns) x nband (ty rows) x nseg
  int out_f32, cross_psi;
  double K[2][7];     // folded shell couplings G_ss,1 w(q) + G_ss,2 p(q), q = 1, 2, 3, 4, 5, 6, 8
  double T[2];        // G_AB t(1), G_AB t(2)
  double body[3];
  double tau[2], omega[2];
  double psi0, irho0;
  double rho_w[2], psi_w[2];
  double rho_ref[2];
};

// Arguments of the 3-D layout kernels.
struct Lb3Layout {
  const void *in;
  void *out;
  int lx, ly, lz, pitch, ns;
  double rho_ref[2];
};

hipError_t launch_step3(int mode, int ns, int walls, int what, int ty, int nblocks, const Lb3Args &a,
                        hipStream_t st);
hipError_t launch_reduce3(const double *partials, int nblocks, double *totals, hipStream_t st);
// kind: 0 init (in: rho [ns][lz][ly][lx]), 1 restore (in: canonical f), 2 checkpoint (out: canonical f)
hipError_t launch_layout3(int kind, int mode, int walls, const Lb3Layout &a, hipStream_t st);
size_t step3_lds_bytes(int mode, int ns, int ty);
int step3_blocks_per_cu(int mode, int ns, int walls, int ty);

}  // namespace lb355
