// Host-side helpers shared by the single-lattice runtime (lb_api.cpp) and the batch
// runtime (lb_batch.cpp): validation, argument folding, grid sizing, timing and graph
// capture.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <string>

#include "../../include/lb.h"
#include "lb_internal.hpp"

namespace lb355 {
namespace host {

constexpr int kPitchAlign = 256;  // elements: a multiple of the widest strip (see the step kernel's stores)
constexpr int kMaxBlocks = 1 << 20;
constexpr size_t kInfinityCacheBytes = (size_t)256 << 20;  // MI355X last-level (Infinity) cache

// Non-temporal population stores when the two population buffers cannot stay resident in
// the Infinity Cache together (see the store policy in the step kernel).
inline int streaming_stores(size_t one_buffer_bytes) { return 2 * one_buffer_bytes > kInfinityCacheBytes ? 1 : 0; }

inline size_t elem_size(int storage) { return storage == LB_F64 ? 8 : (storage == LB_F32 ? 4 : 2); }
inline int row_pitch(int lx) { return (lx + kPitchAlign - 1) / kPitchAlign * kPitchAlign; }

inline int validate(const lb_lattice *lat, const lb_couplings *cpl, const double tau[2], const lb_psi_params *psi,
             std::string &msg) {
  if (!lat || !cpl || !tau || !psi) { msg = "null argument"; return LB_EINVAL; }
  if (lat->lx < 5 || lat->ly < 5) { msg = "lx and ly must be >= 5"; return LB_EINVAL; }
  if (lat->ly > 65535 || (long long)lat->lx * lat->ly > (1LL << 31) / 16) {
    msg = "lattice too large (ly <= 65535, lx * ly <= 2^27)";
    return LB_EINVAL;
  }
  if (lat->n_species != 1 && lat->n_species != 2) { msg = "n_species must be 1 or 2"; return LB_EINVAL; }
  if (lat->walls != 0 && lat->walls != 1) { msg = "walls must be 0 or 1"; return LB_EINVAL; }
  if (lat->storage < LB_F64 || lat->storage > LB_BF16DEV) { msg = "unknown storage"; return LB_EINVAL; }
  for (int s = 0; s < lat->n_species; ++s) {
    if (!(tau[s] > 0.5) || !std::isfinite(tau[s])) { msg = "tau must be finite and > 1/2"; return LB_EINVAL; }
    if (!std::isfinite(cpl->g1[s]) || !std::isfinite(cpl->g2[s]) || !std::isfinite(cpl->rho_wall[s]) ||
        !std::isfinite(psi->rho_ref[s])) {
      msg = "non-finite coupling";
      return LB_EINVAL;
    }
    if (lat->walls && !(cpl->rho_wall[s] >= 0.0)) { msg = "rho_wall must be >= 0"; return LB_EINVAL; }
  }
  if (!std::isfinite(cpl->g_ab) || !std::isfinite(cpl->body_force[0]) || !std::isfinite(cpl->body_force[1])) {
    msg = "non-finite coupling";
    return LB_EINVAL;
  }
  for (int q = 0; q < 5; ++q)
    if (!std::isfinite(cpl->w[q]) || !std::isfinite(cpl->p[q])) { msg = "non-finite weight"; return LB_EINVAL; }
  if (!std::isfinite(cpl->t[0]) || !std::isfinite(cpl->t[1])) { msg = "non-finite weight"; return LB_EINVAL; }
  if (!(psi->psi0 > 0.0) || !(psi->rho0 > 0.0) || !std::isfinite(psi->psi0) || !std::isfinite(psi->rho0)) {
    msg = "psi0 and rho0 must be finite and > 0";
    return LB_EINVAL;
  }
  if (cpl->cross_uses_psi != 0 && cpl->cross_uses_psi != 1) { msg = "cross_uses_psi must be 0 or 1"; return LB_EINVAL; }
  if (!std::isfinite(cpl->wall_velocity[0]) || !std::isfinite(cpl->wall_velocity[1])) {
    msg = "non-finite wall velocity";
    return LB_EINVAL;
  }
  if (!lat->walls && (cpl->wall_velocity[0] != 0.0 || cpl->wall_velocity[1] != 0.0)) {
    msg = "wall_velocity needs a channel lattice (walls = 1)";
    return LB_EINVAL;
  }
  return LB_OK;
}

// Parameters as the kernels use them: FP64 stores plain populations (checkpoint / restore
// stay bit-exact), and a single component has no cross term and no second species.
inline void normalise(const lb_lattice &lat, lb_couplings &cpl, lb_psi_params &psi, double tau[2]) {
  if (lat.storage == LB_F64) psi.rho_ref[0] = psi.rho_ref[1] = 0.0;
  if (lat.n_species == 1) {
    cpl.g_ab = 0.0;
    cpl.g1[1] = cpl.g2[1] = 0.0;
    cpl.rho_wall[1] = 0.0;
    psi.rho_ref[1] = 0.0;
    tau[1] = tau[0];
  }
}

// Kernel arguments of one lattice: shell couplings folded as K(q) = G_1 w(q) + G_2 p(q), the
// A-B couplings G_AB t(q), and the wall ghosts' psi.
inline StepArgs make_step_args(const lb_lattice &lat, const lb_couplings &cpl, const lb_psi_params &psi,
                               const double tau[2], int pitch, long long plane, int sy) {
  StepArgs a;
  std::memset(&a, 0, sizeof(a));
  a.plane = plane;
  a.lx = lat.lx;
  a.ly = lat.ly;
  a.pitch = pitch;
  a.sy = sy;
  a.cross_psi = cpl.cross_uses_psi;
  for (int s = 0; s < 2; ++s) {
    for (int q = 0; q < 5; ++q) a.K[s][q] = cpl.g1[s] * cpl.w[q] + cpl.g2[s] * cpl.p[q];
    a.tau[s] = tau[s];
    a.omega[s] = 1.0 / tau[s];
    a.rho_w[s] = cpl.rho_wall[s];
    a.psi_w[s] = psi.psi0 * (1.0 - std::exp(-cpl.rho_wall[s] / psi.rho0));
    a.rho_ref[s] = psi.rho_ref[s];
  }
  a.T[0] = cpl.g_ab * cpl.t[0];
  a.T[1] = cpl.g_ab * cpl.t[1];
  a.body[0] = cpl.body_force[0];
  a.body[1] = cpl.body_force[1];
  a.psi0 = psi.psi0;
  a.irho0 = 1.0 / psi.rho0;
  // moving walls: a reflected population gains 6 W_l rho_w,s (c_l . U) = +-rho_w,s U / 6
  for (int w = 0; w < 2; ++w)
    for (int s = 0; s < 2; ++s) a.wall_mom[w][s] = lat.walls ? cpl.rho_wall[s] * cpl.wall_velocity[w] / 6.0 : 0.0;
  a.moving = lat.walls && (cpl.wall_velocity[0] != 0.0 || cpl.wall_velocity[1] != 0.0);
  return a;
}

inline int device_cu_count() {
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
    return ncu;
  return 256;
}

// Average milliseconds of one call of `launch` over `reps` calls (after `warm` untimed
// ones), timed with events on stream st.  Returns a negative value on error.
inline double time_launches(hipStream_t st, int warm, int reps, const std::function<hipError_t()> &launch) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  double ms = -1.0;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) goto done;
  for (int k = 0; k < warm; ++k)
    if (launch() != hipSuccess) goto done;
  if (hipEventRecord(e0, st) != hipSuccess) goto done;
  for (int k = 0; k < reps; ++k)
    if (launch() != hipSuccess) goto done;
  if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) goto done;
  {
    float f = 0.f;
    if (hipEventElapsedTime(&f, e0, e1) == hipSuccess) ms = (double)f / reps;
  }
done:
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return ms;
}

// Executable graphs of `steps` consecutive step launches, one per ping-pong parity (the
// launches read and write fixed buffers).  Captured on a private stream (the legacy default
// stream cannot capture) and replayed on the caller's stream.
struct GraphCache {
  hipGraphExec_t exec[2]{nullptr, nullptr};
  hipStream_t cap = nullptr;
  int steps = 0;

  void clear() {
    for (auto &e : exec)
      if (e) {
        (void)hipGraphExecDestroy(e);
        e = nullptr;
      }
  }
  void destroy() {
    clear();
    if (cap) (void)hipStreamDestroy(cap);
    cap = nullptr;
  }
  // launch(k, stream) enqueues step k of the sequence (k = 0 reads the parity's buffer).
  hipError_t get(int parity, const std::function<hipError_t(int, hipStream_t)> &launch, hipGraphExec_t *out) {
    if (exec[parity]) {
      *out = exec[parity];
      return hipSuccess;
    }
    hipError_t e = hipSuccess;
    if (!cap && (e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking)) != hipSuccess) return e;
    if ((e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal)) != hipSuccess) return e;
    hipError_t le = hipSuccess;
    for (int k = 0; k < steps && le == hipSuccess; ++k) le = launch(k, cap);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cap, &g);
    if (le != hipSuccess) e = le;
    if (e == hipSuccess) e = hipGraphInstantiate(&exec[parity], g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      exec[parity] = nullptr;
      return e;
    }
    *out = exec[parity];
    return hipSuccess;
  }
};

}  // namespace host
}  // namespace lb355
