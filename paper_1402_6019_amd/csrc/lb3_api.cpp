// Host runtime of the 3-D C ABI (include/lb3.h): validation, coefficient folding, ping-pong of
// the caller's population buffers, launches of the 3-D fused step on the caller's stream, FP64
// totals and the layout conversions.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>

#include "../../include/lb3.h"
#include "lb3_internal.hpp"

using namespace lb355;

namespace {

thread_local std::string g_init_error3;

constexpr int kPitch3 = 64;  // sites: a multiple of the 64-column strip (ragged strips store into the padding)

// D3Q19 weights by shell (sixth- and eighth-order isotropic sets on the 5x5x5 cube, E2 = 1/3):
// attractive belt |c|^2 = 1, 2, 3, 4 and repulsive belt |c|^2 = 1, 2, 3, 4, 5, 6, 8.
constexpr double kW3[7] = {2.0 / 45, 1.0 / 45, 1.0 / 180, 1.0 / 360, 0.0, 0.0, 0.0};
constexpr double kP3[7] = {4.0 / 135, 1.0 / 63, 2.0 / 315, 5.0 / 1512, 1.0 / 945, 1.0 / 1890, 1.0 / 15120};
constexpr double kT3[2] = {1.0 / 18, 1.0 / 36};

int pitch3(int lx) { return (lx + kPitch3 - 1) / kPitch3 * kPitch3; }
size_t elem3(int storage) { return storage == LB_F64 ? 8 : 4; }

int validate3(const lb3_lattice *lat, const lb3_couplings *cpl, const double tau[2], const lb_psi_params *psi,
              std::string &msg) {
  if (!lat || !cpl || !tau || !psi) { msg = "null argument"; return LB_EINVAL; }
  if (lat->lx < 5 || lat->ly < 5 || lat->lz < 5) { msg = "lx, ly and lz must be >= 5"; return LB_EINVAL; }
  if ((long long)lat->lx * lat->ly * lat->lz > (1LL << 30)) { msg = "lattice too large (lx ly lz <= 2^30)"; return LB_EINVAL; }
  if (lat->n_species != 1 && lat->n_species != 2) { msg = "n_species must be 1 or 2"; return LB_EINVAL; }
  if (lat->walls != 0 && lat->walls != 1) { msg = "walls must be 0 or 1"; return LB_EINVAL; }
  if (lat->storage != LB_F64 && lat->storage != LB_F32) { msg = "3-D storage must be LB_F64 or LB_F32"; return LB_EINVAL; }
  const size_t zplane = (size_t)lat->ly * 19 * pitch3(lat->lx) * lat->n_species * elem3(lat->storage);
  if (zplane >= ((size_t)1 << 32)) { msg = "one z-plane of a population buffer must stay below 4 GiB"; return LB_EINVAL; }
  for (int s = 0; s < lat->n_species; ++s) {
    if (!(tau[s] > 0.5) || !std::isfinite(tau[s])) { msg = "tau must be finite and > 1/2"; return LB_EINVAL; }
    if (!std::isfinite(cpl->g1[s]) || !std::isfinite(cpl->g2[s]) || !std::isfinite(cpl->rho_wall[s]) ||
        !std::isfinite(psi->rho_ref[s])) {
      msg = "non-finite coupling";
      return LB_EINVAL;
    }
    if (lat->walls && !(cpl->rho_wall[s] >= 0.0)) { msg = "rho_wall must be >= 0"; return LB_EINVAL; }
  }
  for (int d = 0; d < 3; ++d)
    if (!std::isfinite(cpl->body_force[d])) { msg = "non-finite body force"; return LB_EINVAL; }
  if (!std::isfinite(cpl->g_ab)) { msg = "non-finite coupling"; return LB_EINVAL; }
  for (int q = 0; q < 7; ++q)
    if (!std::isfinite(cpl->w[q]) || !std::isfinite(cpl->p[q])) { msg = "non-finite weight"; return LB_EINVAL; }
  if (!std::isfinite(cpl->t[0]) || !std::isfinite(cpl->t[1])) { msg = "non-finite weight"; return LB_EINVAL; }
  if (!(psi->psi0 > 0.0) || !(psi->rho0 > 0.0) || !std::isfinite(psi->psi0) || !std::isfinite(psi->rho0)) {
    msg = "psi0 and rho0 must be finite and > 0";
    return LB_EINVAL;
  }
  return LB_OK;
}

}  // namespace

struct lb3_ctx {
  lb3_lattice lat{};
  lb3_couplings cpl{};
  lb_psi_params psi{};
  double tau[2]{1.0, 1.0};
  void *pop[2]{nullptr, nullptr};
  int cur = 0;
  hipStream_t stream = nullptr;
  int pitch = 0;
  int ty = 4, sz = 16;
  int n_cu = 256;
  int64_t t = 0;
  double *d_partials = nullptr;
  int partial_cap = 0;
  double *d_totals = nullptr;
  std::string err;
};

namespace {

int fail3(lb3_ctx *c, int code, const std::string &msg) {
  if (c) c->err = msg;
  else g_init_error3 = msg;
  return code;
}

int hip_fail3(lb3_ctx *c, hipError_t e, const char *what) {
  return fail3(c, LB_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

void grid3(const lb3_ctx *c, int ty, int sz, int *nstrip, int *nband, int *nseg) {
  *nstrip = (c->lat.lx + 63) / 64;
  *nband = (c->lat.ly + ty - 1) / ty;
  *nseg = (c->lat.lz + sz - 1) / sz;
}

// Default shape: eight rows per workgroup in FP32 (the halo is pulled in one round, together
// with the workgroup's own sites: measured 6% faster than four rows at 256^3) and four in FP64
// (its registers allow no more), fewer when the lattice is narrower, and z-segments long enough
// that the whole grid is resident at once (one pass over the lattice; a second partial round
// costs nearly a full one).
void default_tile3(lb3_ctx *c) {
  c->ty = c->lat.storage == LB_F64 || c->lat.ly < 8 ? 4 : 8;
  int nstrip, nband, nseg;
  grid3(c, c->ty, c->lat.lz, &nstrip, &nband, &nseg);
  const int resident = std::max(1, step3_blocks_per_cu(c->lat.storage == LB_F64 ? MODE_F64 : MODE_F32,
                                                       c->lat.n_species, c->lat.walls, c->ty)) * c->n_cu;
  const int tiles = nstrip * nband;
  int segs = std::max(1, resident / std::max(1, tiles));
  c->sz = std::max(1, (c->lat.lz + segs - 1) / segs);
}

Lb3Args args3(const lb3_ctx *c) {
  Lb3Args a{};
  a.lx = c->lat.lx;
  a.ly = c->lat.ly;
  a.lz = c->lat.lz;
  a.pitch = c->pitch;
  a.cross_psi = c->cpl.cross_uses_psi ? 1 : 0;
  for (int s = 0; s < 2; ++s) {
    const int sp = c->lat.n_species == 2 ? s : 0;
    for (int q = 0; q < 7; ++q) a.K[s][q] = c->cpl.g1[sp] * c->cpl.w[q] + c->cpl.g2[sp] * c->cpl.p[q];
    a.tau[s] = c->tau[sp];
    a.omega[s] = 1.0 / c->tau[sp];
    a.rho_w[s] = c->cpl.rho_wall[sp];
    a.psi_w[s] = c->psi.psi0 * (1.0 - std::exp(-c->cpl.rho_wall[sp] / c->psi.rho0));
    a.rho_ref[s] = c->lat.storage == LB_F64 ? 0.0 : c->psi.rho_ref[sp];
  }
  a.T[0] = c->cpl.g_ab * c->cpl.t[0];
  a.T[1] = c->cpl.g_ab * c->cpl.t[1];
  for (int d = 0; d < 3; ++d) a.body[d] = c->cpl.body_force[d];
  a.psi0 = c->psi.psi0;
  a.irho0 = 1.0 / c->psi.rho0;
  a.sz = c->sz;
  grid3(c, c->ty, c->sz, &a.nstrip, &a.nband, &a.nseg);
  return a;
}

int mode3(const lb3_ctx *c) { return c->lat.storage == LB_F64 ? MODE_F64 : MODE_F32; }

int launch_what(lb3_ctx *c, int what, void *rho, void *u, int out_f32) {
  Lb3Args a = args3(c);
  const int nb = a.nstrip * a.nband * a.nseg;
  a.src = c->pop[c->cur];
  a.dst = c->pop[c->cur ^ 1];
  a.out_rho = rho;
  a.out_u = u;
  a.out_f32 = out_f32;
  if (what == WHAT_OBSERVE) {
    if (nb > c->partial_cap) {
      if (c->d_partials) (void)hipFree(c->d_partials);
      c->d_partials = nullptr;
      c->partial_cap = 0;
      hipError_t e = hipMalloc(&c->d_partials, (size_t)nb * RED3_N * sizeof(double));
      if (e != hipSuccess) return fail3(c, LB_ENOMEM, std::string("partials: ") + hipGetErrorString(e));
      c->partial_cap = nb;
    }
    a.partials = c->d_partials;
  }
  hipError_t e = launch_step3(mode3(c), c->lat.n_species, c->lat.walls, what, c->ty, nb, a, c->stream);
  if (e != hipSuccess) return hip_fail3(c, e, "3-D step launch");
  if (what == WHAT_OBSERVE) {
    e = launch_reduce3(c->d_partials, nb, c->d_totals, c->stream);
    if (e != hipSuccess) return hip_fail3(c, e, "3-D reduction launch");
  }
  return LB_OK;
}

Lb3Layout layout3(const lb3_ctx *c) {
  Lb3Layout la{};
  la.lx = c->lat.lx;
  la.ly = c->lat.ly;
  la.lz = c->lat.lz;
  la.pitch = c->pitch;
  la.ns = c->lat.n_species;
  for (int s = 0; s < 2; ++s) la.rho_ref[s] = c->lat.storage == LB_F64 ? 0.0 : c->psi.rho_ref[c->lat.n_species == 2 ? s : 0];
  return la;
}

}  // namespace

extern "C" {

int lb3_default_couplings(lb3_couplings *c) {
  if (!c) return LB_EINVAL;
  *c = lb3_couplings{};
  for (int q = 0; q < 7; ++q) {
    c->w[q] = kW3[q];
    c->p[q] = kP3[q];
  }
  c->t[0] = kT3[0];
  c->t[1] = kT3[1];
  return LB_OK;
}

size_t lb3_pop_bytes(const lb3_lattice *lat) {
  if (!lat || lat->lx < 5 || lat->ly < 5 || lat->lz < 5 || (lat->n_species != 1 && lat->n_species != 2) ||
      (lat->storage != LB_F64 && lat->storage != LB_F32))
    return 0;
  return (size_t)lat->lz * lat->ly * 19 * pitch3(lat->lx) * lat->n_species * elem3(lat->storage);
}

int lb3_init(lb3_ctx **out, const lb3_lattice *lat, const lb3_couplings *cpl, const double tau[2],
             const lb_psi_params *psi, const double *rho_init, void *pop_a, void *pop_b, size_t pop_bytes,
             void *hip_stream) {
  if (!out) return fail3(nullptr, LB_EINVAL, "null output");
  *out = nullptr;
  std::string msg;
  int rc = validate3(lat, cpl, tau, psi, msg);
  if (rc) return fail3(nullptr, rc, msg);
  if (!rho_init || !pop_a || !pop_b) return fail3(nullptr, LB_EINVAL, "null buffer");
  if (pop_bytes < lb3_pop_bytes(lat)) return fail3(nullptr, LB_ENOMEM, "population buffers smaller than lb3_pop_bytes()");
  const size_t nsite = (size_t)lat->lx * lat->ly * lat->lz;
  for (size_t i = 0; i < (size_t)lat->n_species * nsite; ++i)
    if (!(rho_init[i] > 0.0) || !std::isfinite(rho_init[i]))
      return fail3(nullptr, LB_EINVAL, "rho_init must be finite and > 0 everywhere");
  lb3_ctx *c = new (std::nothrow) lb3_ctx();
  if (!c) return fail3(nullptr, LB_ENOMEM, "context allocation");
  c->lat = *lat;
  c->cpl = *cpl;
  c->psi = *psi;
  c->tau[0] = tau[0];
  c->tau[1] = lat->n_species == 2 ? tau[1] : tau[0];
  c->pop[0] = pop_a;
  c->pop[1] = pop_b;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->pitch = pitch3(lat->lx);
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
      ncu > 0)
    c->n_cu = ncu;
  default_tile3(c);
  hipError_t e;
  void *d_rho = nullptr;
  const size_t rho_bytes = (size_t)lat->n_species * nsite * sizeof(double);
  if ((e = hipMalloc(&c->d_totals, RED3_N * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(&d_rho, rho_bytes)) != hipSuccess ||
      (e = hipMemcpyAsync(d_rho, rho_init, rho_bytes, hipMemcpyHostToDevice, c->stream)) != hipSuccess) {
    g_init_error3 = std::string("allocation / copy: ") + hipGetErrorString(e);
    if (d_rho) (void)hipFree(d_rho);
    lb3_destroy(c);
    return LB_EDEVICE;
  }
  Lb3Layout la = layout3(c);
  la.in = d_rho;
  la.out = c->pop[0];
  e = launch_layout3(0, mode3(c), lat->walls, la, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  (void)hipFree(d_rho);
  if (e != hipSuccess) {
    g_init_error3 = std::string("init kernel: ") + hipGetErrorString(e);
    lb3_destroy(c);
    return LB_EDEVICE;
  }
  *out = c;
  return LB_OK;
}

int lb3_step(lb3_ctx *c, int64_t n) {
  if (!c) return fail3(nullptr, LB_EINVAL, "null context");
  if (n < 0) return fail3(c, LB_EINVAL, "n must be >= 0");
  for (int64_t k = 0; k < n; ++k) {
    int rc = launch_what(c, WHAT_STEP, nullptr, nullptr, 0);
    if (rc) return rc;
    c->cur ^= 1;
    ++c->t;
  }
  return LB_OK;
}

int lb3_moments(lb3_ctx *c, void *rho, void *u, int32_t dtype) {
  if (!c) return fail3(nullptr, LB_EINVAL, "null context");
  if (dtype != LB_OUT_F64 && dtype != LB_OUT_F32) return fail3(c, LB_EINVAL, "unknown dtype");
  if (!rho && !u) return LB_OK;
  return launch_what(c, WHAT_MOMENTS, rho, u, dtype == LB_OUT_F32 ? 1 : 0);
}

int lb3_totals(lb3_ctx *c, double mass[2], double momentum[3], double *flow) {
  if (!c) return fail3(nullptr, LB_EINVAL, "null context");
  int rc = launch_what(c, WHAT_OBSERVE, nullptr, nullptr, 0);
  if (rc) return rc;
  double t[RED3_N];
  hipError_t e = hipMemcpyAsync(t, c->d_totals, sizeof(t), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail3(c, e, "3-D totals");
  if (mass) {
    mass[0] = t[RED3_MASS0];
    mass[1] = t[RED3_MASS1];
  }
  if (momentum) {
    momentum[0] = t[RED3_PX];
    momentum[1] = t[RED3_PY];
    momentum[2] = t[RED3_PZ];
  }
  if (flow) *flow = t[RED3_FLOW] / ((double)c->lat.lx * c->lat.lz);
  if (t[RED3_BAD] > 0.0) return fail3(c, LB_EUNSTABLE, "non-finite or non-positive density");
  return LB_OK;
}

int lb3_checkpoint(lb3_ctx *c, void *dst) {
  if (!c) return fail3(nullptr, LB_EINVAL, "null context");
  if (!dst) return fail3(c, LB_EINVAL, "null destination");
  Lb3Layout la = layout3(c);
  la.in = c->pop[c->cur];
  la.out = dst;
  hipError_t e = launch_layout3(2, mode3(c), c->lat.walls, la, c->stream);
  if (e != hipSuccess) return hip_fail3(c, e, "3-D checkpoint");
  return LB_OK;
}

int lb3_restore(lb3_ctx *c, const void *src) {
  if (!c) return fail3(nullptr, LB_EINVAL, "null context");
  if (!src) return fail3(c, LB_EINVAL, "null source");
  Lb3Layout la = layout3(c);
  la.in = src;
  la.out = c->pop[c->cur];
  hipError_t e = launch_layout3(1, mode3(c), c->lat.walls, la, c->stream);
  if (e != hipSuccess) return hip_fail3(c, e, "3-D restore");
  return LB_OK;
}

int lb3_set_tile(lb3_ctx *c, int32_t ty, int32_t sz) {
  if (!c) return fail3(nullptr, LB_EINVAL, "null context");
  const bool ty_ok = ty == 1 || ty == 2 || ty == 4 || (ty == 8 && c->lat.storage != LB_F64);
  if (!ty_ok || sz < 1) return fail3(c, LB_EINVAL, "ty must be 1, 2, 4 (or 8 with FP32 storage) and sz >= 1");
  c->ty = ty;
  c->sz = std::min(sz, c->lat.lz);
  return LB_OK;
}

int lb3_get_tile(const lb3_ctx *c, int32_t *ty, int32_t *sz) {
  if (!c) return LB_EINVAL;
  if (ty) *ty = c->ty;
  if (sz) *sz = c->sz;
  return LB_OK;
}

int64_t lb3_time(const lb3_ctx *c) { return c ? c->t : -1; }

const char *lb3_last_error(const lb3_ctx *c) { return c ? c->err.c_str() : g_init_error3.c_str(); }

void lb3_destroy(lb3_ctx *c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  if (c->d_partials) (void)hipFree(c->d_partials);
  if (c->d_totals) (void)hipFree(c->d_totals);
  delete c;
}

}  // extern "C"
