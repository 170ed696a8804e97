// Host runtime of the C ABI declared in include/lb.h: validation, coefficient folding,
// ping-pong of the caller's population buffers, launches on the caller's HIP stream,
// FP64 reductions and the latched health check.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "../../include/lb.h"
#include "lb_host.hpp"
#include "lb_internal.hpp"
#include "lb_tables.hpp"

using namespace lb355;
using namespace lb355::host;

namespace {

thread_local std::string g_init_error;


}  // namespace

struct lb_ctx {
  lb_lattice lat{};
  lb_couplings cpl{};
  lb_psi_params psi{};
  double tau[2]{1.0, 1.0};
  void *pop[2]{nullptr, nullptr};
  int cur = 0;
  size_t pop_bytes = 0;
  hipStream_t stream = nullptr;
  int pitch = 0;
  long long plane = 0;
  int tx = 256, sy = 16;
  int n_cu = 256;  // compute units of the device the context runs on
  int device = 0;  // device current at lb_init
  int reduce_every = 0;
  int store_policy = LB_STORES_AUTO;
  int two_step = LB_TWO_STEP_AUTO;  // plain steps in pairs, two time steps per launch
  int sy2 = 0;       // rows per segment of the two-step kernel (0: the resident-grid default)
  int rounding = LB_ROUND_NEAREST;  // BF16 stores: nearest or stochastic
  double *d_tbase = nullptr;        // step at which a graph replay starts (stochastic rounding)
  int64_t t = 0;
  double *d_partials = nullptr;  // [partial_cap][RED_N], grown to the largest launch
  int partial_cap = 0;
  double *d_totals = nullptr;    // [RED_N]
  double *d_acc = nullptr;       // [4]: wall stress sums (bot, top), count, bad
  double *d_accrows = nullptr;   // [accrow_cap][ACC_N]: per-workgroup running sums of reducing steps
  int accrow_cap = 0;
  int acc_nb = 0;                // workgroups of the reducing launches since the last flush
  int64_t acc_pending = 0;       // reducing launches since the last flush
  double *h_acc = nullptr;       // pinned copy of d_acc for the asynchronous health check
  hipEvent_t ev = nullptr;
  bool check_pending = false;
  bool unstable = false;
  GraphCache graph;  // graph.steps > 0: plain steps are replayed from captured graphs
  double *d_prof = nullptr;      // profile pass: [ncb][ly][PROF_N] block sums, then [ly][PROF_N] row sums
  size_t prof_cap = 0;           // doubles
  std::string err;
};

namespace {

int fail(lb_ctx *c, int code, const std::string &msg) {
  if (c) c->err = msg;
  else g_init_error = msg;
  return code;
}

int hip_fail(lb_ctx *c, hipError_t e, const char *what) {
  return fail(c, LB_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

int grid_blocks(const lb_ctx *c, int tx, int sy, int *nseg) {
  const int nstrip = (c->lat.lx + tx - 1) / tx;
  const int ns = (c->lat.ly + sy - 1) / sy;
  if (nseg) *nseg = ns;
  return nstrip * ns;
}

int ensure_partials(lb_ctx *c, int nb) {
  if (nb <= c->partial_cap) return LB_OK;
  if (c->d_partials) (void)hipFree(c->d_partials);
  c->d_partials = nullptr;
  c->partial_cap = 0;
  hipError_t e = hipMalloc(&c->d_partials, (size_t)nb * RED_N * sizeof(double));
  if (e != hipSuccess) return fail(c, LB_ENOMEM, std::string("partials: ") + hipGetErrorString(e));
  c->partial_cap = nb;
  return LB_OK;
}

void fill_step_args(const lb_ctx *c, StepArgs &a) {
  a = make_step_args(c->lat, c->cpl, c->psi, c->tau, c->pitch, c->plane, c->sy);
  a.stream_stores = c->store_policy == LB_STORES_AUTO ? streaming_stores(lb_pop_bytes(&c->lat))
                                                       : (c->store_policy == LB_STORES_STREAMING ? 1 : 0);
}

// Kernel variant of the passes that store populations.
static int step_mode(const lb_ctx *c) {
  return c->lat.storage == LB_BF16DEV && c->rounding == LB_ROUND_STOCHASTIC ? MODE_BF16SR : c->lat.storage;
}

// One plain step launch (no reductions) from buffer `from` to the other one, on stream st,
// as time step t_step (+ *t_base if t_base is set: a graph replay's first step).
hipError_t launch_plain_step(const lb_ctx *c, int from, hipStream_t st, uint32_t t_step, const double *t_base) {
  int nseg = 0;
  const int nb = grid_blocks(c, c->tx, c->sy, &nseg);
  StepArgs a;
  fill_step_args(c, a);
  a.nseg = nseg;
  a.src = c->pop[from];
  a.dst = c->pop[from ^ 1];
  a.t_step = t_step;
  a.t_base = t_base;
  return launch_step(step_mode(c), c->lat.n_species, c->lat.walls, WHAT_STEP, c->tx, nb, a, st);
}

// One plain step from buffer `from` that also writes what the adjoint's reverse step reads of
// that state (as launch_checkpoint_fields_from does): fields (FP64 if fp64) and the FP64
// populations of the rows next to the walls into dst.  Bitwise the same step and the same
// fields as the two separate launches, with one pass over the state.  sy > 0 overrides the
// context's segment height (any height gives bitwise the same step).
hipError_t launch_plain_step_fields(const lb_ctx *c, int from, void *dst, void *fields, int fp64, hipStream_t st,
                                    int sy = 0) {
  if (sy <= 0) sy = c->sy;
  int nseg = 0;
  const int nb = grid_blocks(c, c->tx, sy, &nseg);
  StepArgs a;
  fill_step_args(c, a);
  a.sy = sy;
  a.nseg = nseg;
  a.src = c->pop[from];
  a.dst = c->pop[from ^ 1];
  a.out_rho = fields;
  a.out_u = dst;
  return launch_step(step_mode(c), c->lat.n_species, c->lat.walls, fp64 ? WHAT_STEP_FIELDS : WHAT_STEP_FIELDS32, c->tx,
                     nb, a, st);
}

// Segments of the two-step kernel: rows per segment (the context's choice, or the default that
// makes the whole grid resident at once) and the grid size.
int grid2(const lb_ctx *c, int *sy_out, int *nseg_out) {
  const int nstrip = (c->lat.lx + 53) / 54;
  int sy = c->sy2;
  if (sy <= 0) {
    const int per_cu = c->lat.storage == LB_F64 ? blocks2_per_cu_f64(c->lat.n_species, c->lat.walls)
                                                : blocks2_per_cu_f32(c->lat.n_species, c->lat.walls);
    const int resident = std::max(1, per_cu) * c->n_cu;
    const int nseg = std::max(1, resident / nstrip);
    sy = std::max(1, (c->lat.ly + nseg - 1) / nseg);
  }
  sy = std::min(sy, c->lat.ly);
  const int nseg = (c->lat.ly + sy - 1) / sy;
  if (sy_out) *sy_out = sy;
  if (nseg_out) *nseg_out = nseg;
  return nstrip * nseg;
}

// Whether plain steps go in pairs: forced on or off, or (auto) where the pairs' halved HBM
// traffic measured worth more than their recomputed overlaps, for lattices whose two population
// buffers exceed the Infinity Cache: walled FP32 (10% faster on the 4096 x 512, 4096 x 1024 and
// 2048^2 channels; its periodic instantiation spills registers and is slower) and periodic
// FP64 (9-14% faster at 1024^2, 2048 x 1024, 4096 x 512 and 2048^2; walled FP64 gained nothing).
// Never for BF16, nor for a cache-resident FP32 lattice.
bool pairs_on(const lb_ctx *c) {
  if (c->two_step == LB_TWO_STEP_AUTO) {
    if (!streaming_stores(lb_pop_bytes(&c->lat))) return false;
    return (c->lat.storage == LB_F32 && c->lat.walls) || (c->lat.storage == LB_F64 && !c->lat.walls);
  }
  return c->two_step == LB_TWO_STEP_ON;
}

// Two plain steps in one launch (time steps t_step and t_step + 1) from buffer `from` to the
// other one.  Stores write through unless streaming is forced: with the traffic halved, the
// write-through variant measured faster at every footprint.
hipError_t launch_two_steps(const lb_ctx *c, int from, hipStream_t st, uint32_t t_step, const double *t_base) {
  int sy = 0, nseg = 0;
  const int nb = grid2(c, &sy, &nseg);
  StepArgs a;
  fill_step_args(c, a);
  a.stream_stores = c->store_policy == LB_STORES_STREAMING ? 1 : 0;
  a.sy = sy;
  a.nseg = nseg;
  a.src = c->pop[from];
  a.dst = c->pop[from ^ 1];
  a.t_step = t_step;
  a.t_base = t_base;
  return launch_step2(step_mode(c), c->lat.n_species, c->lat.walls, nb, a, st);
}

// What the adjoint's reverse step reads of the state in buffer `from`: the canonical FP64
// pre-collision populations of the rows next to the walls into dst ([s][l][2][lx]), and the
// fields rho, psi, j per species (FP64 if fp64) into fields, on stream st.
hipError_t launch_checkpoint_fields_from(const lb_ctx *c, int from, void *dst, void *fields, int fp64, hipStream_t st) {
  LayoutArgs la{};
  la.in = c->pop[from];
  la.out = dst;
  la.plane = c->plane;
  la.lx = c->lat.lx;
  la.ly = c->lat.ly;
  la.pitch = c->pitch;
  la.ns = c->lat.n_species;
  la.rho_ref[0] = c->psi.rho_ref[0];
  la.rho_ref[1] = c->psi.rho_ref[1];
  la.fields = fields;
  la.psi0 = c->psi.psi0;
  la.irho0 = 1.0 / c->psi.rho0;
  return launch_checkpoint_fields(c->lat.storage, c->lat.walls, fp64, la, st);
}

// Fold the running sums of the reducing steps since the last flush into d_acc.
int flush_acc(lb_ctx *c) {
  if (c->acc_pending == 0) return LB_OK;
  hipError_t e = launch_flush(c->d_accrows, c->acc_nb, c->d_acc, (double)c->acc_pending, 1.0 / c->lat.lx, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "reduction flush");
  c->acc_pending = 0;
  return LB_OK;
}

// Rows of running sums for nb workgroups, zeroed (flushing what they hold first).
int ensure_accrows(lb_ctx *c, int nb) {
  if (c->acc_pending > 0 && c->acc_nb != nb) {
    int rc = flush_acc(c);
    if (rc) return rc;
  }
  if (nb <= c->accrow_cap) return LB_OK;
  int rc = flush_acc(c);
  if (rc) return rc;
  if (c->d_accrows) {
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(c->d_accrows);
  }
  c->d_accrows = nullptr;
  c->accrow_cap = 0;
  hipError_t e = hipMalloc(&c->d_accrows, (size_t)nb * ACC_N * sizeof(double));
  if (e != hipSuccess) return fail(c, LB_ENOMEM, std::string("reduction rows: ") + hipGetErrorString(e));
  if ((e = launch_fill(c->d_accrows, 0.0, nb * ACC_N, c->stream)) != hipSuccess) return hip_fail(c, e, "reduction rows");
  c->accrow_cap = nb;
  return LB_OK;
}

// One launch of the fused kernel on the current buffer.
int run_step_kernel(lb_ctx *c, int what, void *out_rho, void *out_u, int out_f32) {
  int nseg = 0;
  const int nb = grid_blocks(c, c->tx, c->sy, &nseg);
  const bool reduce = what == WHAT_OBSERVE;
  if (reduce) {
    int rc = ensure_partials(c, nb);
    if (rc) return rc;
  }
  if (what == WHAT_STEP_ACCUM) {
    int rc = ensure_accrows(c, nb);
    if (rc) return rc;
  }
  StepArgs a;
  fill_step_args(c, a);
  a.nseg = nseg;
  a.src = c->pop[c->cur];
  a.dst = c->pop[c->cur ^ 1];
  a.partials = c->d_partials;
  a.accrows = c->d_accrows;
  a.out_rho = out_rho;
  a.out_u = out_u;
  a.out_f32 = out_f32;
  a.t_step = (uint32_t)c->t;
  hipError_t e = launch_step(step_mode(c), c->lat.n_species, c->lat.walls, what, c->tx, nb, a, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "step kernel launch");
  if (reduce) {
    e = launch_reduce(c->d_partials, nb, c->d_totals, c->d_acc, 0, 1.0 / c->lat.lx, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "reduce kernel launch");
  }
  if (what == WHAT_STEP_ACCUM) {
    c->acc_nb = nb;
    ++c->acc_pending;
  }
  return LB_OK;
}

// Latched health check: look at the last asynchronously copied accumulator if it is ready.
int poll_health(lb_ctx *c, bool wait) {
  if (c->check_pending) {
    hipError_t e = wait ? hipEventSynchronize(c->ev) : hipEventQuery(c->ev);
    if (e == hipSuccess) {
      c->check_pending = false;
      if (c->h_acc[3] > 0.0) c->unstable = true;
    } else if (e != hipErrorNotReady) {
      return hip_fail(c, e, "health check");
    }
  }
  if (c->unstable) return fail(c, LB_EUNSTABLE, "non-finite or non-positive density detected by the reductions");
  return LB_OK;
}


// Default launch shape: the widest strip the lattice fills, and segments sized so that the
// whole grid is resident at once (workgroups = resident workgroups per CU x CUs, at most):
// the step is one pass over the lattice, and a second, partial wave of workgroups would
// cost nearly as much as the first.
void default_tile(lb_ctx *c) {
  const int lx = c->lat.lx, ly = c->lat.ly;
  c->tx = lx >= 256 ? 256 : (lx >= 128 ? 128 : 64);
  const int nstrip = (lx + c->tx - 1) / c->tx;
  const int cap = step_blocks_per_cu(c->lat.storage, c->lat.n_species, c->lat.walls, c->tx) * c->n_cu;
  const int nseg = std::max(1, cap / nstrip);
  c->sy = std::min(ly, std::max(1, (ly + nseg - 1) / nseg));
}

}  // namespace

extern "C" {

int lb_stream_copy(void *dst, const void *src, size_t bytes, int32_t nontemporal, void *hip_stream) {
  if (!dst || !src) return fail(nullptr, LB_EINVAL, "null buffer");
  if (bytes % 16 || (reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) % 16)
    return fail(nullptr, LB_EINVAL, "copy size and addresses must be multiples of 16 bytes");
  const hipError_t e = launch_stream_copy(dst, src, bytes / 16, nontemporal ? 1 : 0, 4 * device_cu_count(),
                                          static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return fail(nullptr, LB_EDEVICE, std::string("copy launch: ") + hipGetErrorString(e));
  return LB_OK;
}

int lb_default_couplings(lb_couplings *c) {
  if (!c) return fail(nullptr, LB_EINVAL, "null argument");
  std::memset(c, 0, sizeof(*c));
  for (int q = 0; q < NSHELL; ++q) {
    c->w[q] = W_ATTR[q];
    c->p[q] = P_REP[q];
  }
  c->t[0] = T_CROSS[0];
  c->t[1] = T_CROSS[1];
  return LB_OK;
}

size_t lb_pop_bytes(const lb_lattice *lat) {
  if (!lat || lat->lx < 5 || lat->ly < 5 || (lat->n_species != 1 && lat->n_species != 2) ||
      lat->storage < LB_F64 || lat->storage > LB_BF16DEV)
    return 0;
  return (size_t)lat->n_species * 9 * (size_t)lat->ly * row_pitch(lat->lx) * elem_size(lat->storage);
}

int lb_init(lb_ctx **out, const lb_lattice *lat, const lb_couplings *cpl, const double tau[2],
            const lb_psi_params *psi, const double *rho_init, void *pop_a, void *pop_b, size_t pop_bytes,
            void *hip_stream) {
  if (!out) return fail(nullptr, LB_EINVAL, "null output pointer");
  *out = nullptr;
  std::string msg;
  int rc = validate(lat, cpl, tau, psi, msg);
  if (rc) return fail(nullptr, rc, msg);
  if (!rho_init || !pop_a || !pop_b) return fail(nullptr, LB_EINVAL, "null buffer");
  if (pop_a == pop_b) return fail(nullptr, LB_EINVAL, "pop_a and pop_b must differ");
  const size_t need = lb_pop_bytes(lat);
  if (need >= ((size_t)1 << 32))  // the kernels address a buffer with 32-bit byte offsets
    return fail(nullptr, LB_EINVAL, "lattice too large: one population buffer must stay below 4 GiB");
  if (pop_bytes < need) return fail(nullptr, LB_ENOMEM, "population buffers smaller than lb_pop_bytes()");
  const size_t nsite = (size_t)lat->lx * lat->ly;
  for (size_t i = 0; i < (size_t)lat->n_species * nsite; ++i)
    if (!(rho_init[i] > 0.0) || !std::isfinite(rho_init[i]))
      return fail(nullptr, LB_EINVAL, "rho_init must be finite and > 0 everywhere");

  lb_ctx *c = new (std::nothrow) lb_ctx();
  if (!c) return fail(nullptr, LB_ENOMEM, "context allocation");
  c->lat = *lat;
  c->cpl = *cpl;
  c->psi = *psi;
  c->tau[0] = tau[0];
  c->tau[1] = lat->n_species == 2 ? tau[1] : tau[0];
  normalise(c->lat, c->cpl, c->psi, c->tau);
  c->pop[0] = pop_a;
  c->pop[1] = pop_b;
  c->pop_bytes = pop_bytes;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->pitch = row_pitch(lat->lx);
  c->plane = (long long)lat->ly * c->pitch;
  c->n_cu = device_cu_count();
  default_tile(c);

  hipError_t e;
  if ((e = hipGetDevice(&c->device)) != hipSuccess || (e = static_scratch_setup(c->device)) != hipSuccess) {
    g_init_error = std::string("device scratch lookup: ") + hipGetErrorString(e);
    lb_destroy(c);
    return LB_EDEVICE;
  }
  if ((e = hipMalloc(&c->d_totals, RED_N * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(&c->d_acc, 4 * sizeof(double))) != hipSuccess ||
      (e = hipHostMalloc(&c->h_acc, 4 * sizeof(double), hipHostMallocDefault)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&c->ev, hipEventDisableTiming)) != hipSuccess) {
    g_init_error = std::string("internal allocation: ") + hipGetErrorString(e);
    lb_destroy(c);
    return LB_ENOMEM;
  }
  std::memset(c->h_acc, 0, 4 * sizeof(double));
  // Stage rho_init in pop_b (it is at least as large as n_species * lx * ly doubles).
  const size_t rbytes = (size_t)lat->n_species * nsite * sizeof(double);
  if ((e = launch_fill(c->d_acc, 0.0, 4, c->stream)) != hipSuccess ||
      (e = hipMemcpyAsync(pop_b, rho_init, rbytes, hipMemcpyHostToDevice, c->stream)) != hipSuccess) {
    g_init_error = std::string("initial copy: ") + hipGetErrorString(e);
    lb_destroy(c);
    return LB_EDEVICE;
  }
  LayoutArgs la{};
  la.in = pop_b;
  la.out = pop_a;
  la.plane = c->plane;
  la.lx = lat->lx;
  la.ly = lat->ly;
  la.pitch = c->pitch;
  la.ns = lat->n_species;
  la.rho_ref[0] = c->psi.rho_ref[0];
  la.rho_ref[1] = c->psi.rho_ref[1];
  if ((e = launch_init(lat->storage, lat->walls, la, c->stream)) != hipSuccess ||
      (e = hipStreamSynchronize(c->stream)) != hipSuccess) {
    g_init_error = std::string("init kernel: ") + hipGetErrorString(e);
    lb_destroy(c);
    return LB_EDEVICE;
  }
  *out = c;
  return LB_OK;
}

int lb_step(lb_ctx *c, int64_t n) {
  if (!c) return fail(nullptr, LB_EINVAL, "null context");
  if (n < 0) return fail(c, LB_EINVAL, "n must be >= 0");
  int rc = poll_health(c, false);
  if (rc) return rc;
  bool reduced = false;
  // Without reductions, whole graphs of graph.steps launches (an even number: the state
  // returns to the same buffer) are replayed; the rest is launched one by one.
  if (c->graph.steps > 0 && c->reduce_every == 0) {
    while (n >= c->graph.steps) {
      hipGraphExec_t g = nullptr;
      const int from = c->cur;
      const double *tb = c->rounding == LB_ROUND_STOCHASTIC ? c->d_tbase : nullptr;
      const bool pairs = pairs_on(c);
      hipError_t e = c->graph.get(
          from,
          [&](int k, hipStream_t st) {
            if (!pairs) return launch_plain_step(c, from ^ (k & 1), st, (uint32_t)k, tb);
            // two steps per launch: one launch for each even k, the buffers swap once per launch
            return (k & 1) ? hipSuccess : launch_two_steps(c, from ^ ((k >> 1) & 1), st, (uint32_t)k, tb);
          },
          &g);
      // the replay's steps are t + k: the base goes to device memory (a fill kernel, outside the graph)
      if (e == hipSuccess && tb) e = launch_fill(c->d_tbase, (double)c->t, 1, c->stream);
      if (e == hipSuccess) e = hipGraphLaunch(g, c->stream);
      if (e != hipSuccess) return hip_fail(c, e, "step graph");
      c->t += c->graph.steps;
      if (pairs) c->cur ^= (c->graph.steps >> 1) & 1;
      n -= c->graph.steps;
    }
  }
  if (pairs_on(c) && c->reduce_every == 0) {
    for (; n >= 2; n -= 2) {
      hipError_t e = launch_two_steps(c, c->cur, c->stream, (uint32_t)c->t, nullptr);
      if (e != hipSuccess) return hip_fail(c, e, "two-step kernel launch");
      c->cur ^= 1;
      c->t += 2;
    }
  }
  for (int64_t k = 0; k < n; ++k) {
    const bool red = c->reduce_every > 0 && (c->t % c->reduce_every) == 0;
    rc = run_step_kernel(c, red ? WHAT_STEP_ACCUM : WHAT_STEP, nullptr, nullptr, 0);
    if (rc) return rc;
    reduced |= red;
    c->cur ^= 1;
    ++c->t;
  }
  if (reduced) {
    // one second pass per call: fold the workgroups' running sums, then read back the health
    rc = flush_acc(c);
    if (rc) return rc;
    hipError_t e = hipMemcpyAsync(c->h_acc, c->d_acc, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipEventRecord(c->ev, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "health readback");
    c->check_pending = true;
  }
  return LB_OK;
}

int lb_set_reduce_every(lb_ctx *c, int32_t k) {
  if (!c) return fail(nullptr, LB_EINVAL, "null context");
  if (k < 0) return fail(c, LB_EINVAL, "k must be >= 0");
  c->reduce_every = k;
  return LB_OK;
}

int lb_moments(lb_ctx *c, void *rho, void *u, int32_t dtype) {
  if (!c) return fail(nullptr, LB_EINVAL, "null context");
  if (dtype != LB_OUT_F64 && dtype != LB_OUT_F32) return fail(c, LB_EINVAL, "dtype must be LB_OUT_F64 or LB_OUT_F32");
  if (!rho && !u) return LB_OK;
  return run_step_kernel(c, WHAT_MOMENTS, rho, u, dtype == LB_OUT_F32);
}

int lb_stress_field(lb_ctx *c, void *sigma, int32_t dtype) {
  if (!c) return fail(nullptr, LB_EINVAL, "null context");
  if (!sigma) return fail(c, LB_EINVAL, "null output");
  if (dtype != LB_OUT_F64 && dtype != LB_OUT_F32) return fail(c, LB_EINVAL, "dtype must be LB_OUT_F64 or LB_OUT_F32");
  int nseg = 0;
  const int nb = grid_blocks(c, c->tx, c->sy, &nseg);
  StepArgs a;
  fill_step_args(c, a);
  a.nseg = nseg;
  a.src = c->pop[c->cur];
  a.dst = c->pop[c->cur ^ 1];  // not written
  a.out_sigma = sigma;
  a.out_f32 = dtype == LB_OUT_F32;
  hipError_t e = launch_step(c->lat.storage, c->lat.n_species, c->lat.walls, WHAT_STRESS, c->tx, nb, a, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "stress kernel launch");
  return LB_OK;
}

int lb_wall_stress(lb_ctx *c, double out[2], int32_t reset) {
  if (!c) return fail(nullptr, LB_EINVAL, "null context");
  if (!out) return fail(c, LB_EINVAL, "null output");
  if (!c->lat.walls) return fail(c, LB_ESTATE, "wall stress needs a channel lattice");
  int rc = flush_acc(c);
  if (rc) return rc;
  double h[4];
  hipError_t e = hipMemcpyAsync(h, c->d_acc, sizeof(h), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "wall stress readback");
  if (h[3] > 0.0) c->unstable = true;
  out[0] = h[2] > 0 ? h[0] / h[2] : 0.0;
  out[1] = h[2] > 0 ? h[1] / h[2] : 0.0;
  if (reset) {
    const double keep[4] = {0.0, 0.0, 0.0, h[3]};
    e = hipMemcpyAsync(c->d_acc, keep, sizeof(keep), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "wall stress reset");
  }
  if (c->unstable) return fail(c, LB_EUNSTABLE, "non-finite or non-positive density detected by the reductions");
  return LB_OK;
}

int lb_totals(lb_ctx *c, double mass[2], double momentum[2], double *flow) {
  if (!c) return fail(nullptr, LB_EINVAL, "null context");
  if (!mass || !momentum) return fail(c, LB_EINVAL, "null output");
  int rc = run_step_kernel(c, WHAT_OBSERVE, nullptr, nullptr, 0);
  if (rc) return rc;
  double h[RED_N];
  hipError_t e = hipMemcpyAsync(h, c->d_totals, sizeof(h), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "totals readback");
  mass[0] = h[RED_MASS0];
  mass[1] = h[RED_MASS1];
  momentum[0] = h[RED_PX];
  momentum[1] = h[RED_PY];
  if (flow) *flow = h[RED_FLOW];
  rc = poll_health(c, true);
  if (rc) return rc;
  if (h[RED_BAD] > 0.0) {
    c->unstable = true;
    return fail(c, LB_EUNSTABLE, "non-finite or non-positive density in the current state");
  }
  return LB_OK;
}

int lb_checkpoint(lb_ctx *c, void *dst) {
  if (!c) return fail(nullptr, LB_EINVAL, "null context");
  if (!dst) return fail(c, LB_EINVAL, "null destination");
  LayoutArgs la{};
  la.in = c->pop[c->cur];
  la.out = dst;
  la.plane = c->plane;
  la.lx = c->lat.lx;
  la.ly = c->lat.ly;
  la.pitch = c->pitch;
  la.ns = c->lat.n_species;
  la.rho_ref[0] = c->psi.rho_ref[0];
  la.rho_ref[1] = c->psi.rho_ref[1];
  hipError_t e = launch_checkpoint(c->lat.storage, c->lat.walls, la, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "checkpoint kernel");
  return LB_OK;
}

int lb_restore(lb_ctx *c, const void *src) {
  if (!c) return fail(nullptr, LB_EINVAL, "null context");
  if (!src) return fail(c, LB_EINVAL, "null source");
  // drop any pending health readback: it describes the state being replaced
  if (c->check_pending) {
    (void)hipEventSynchronize(c->ev);
    c->check_pending = false;
  }
  LayoutArgs la{};
  la.in = src;
  la.out = c->pop[c->cur];
  la.plane = c->plane;
  la.lx = c->lat.lx;
  la.ly = c->lat.ly;
  la.pitch = c->pitch;
  la.ns = c->lat.n_species;
  la.rho_ref[0] = c->psi.rho_ref[0];
  la.rho_ref[1] = c->psi.rho_ref[1];
  hipError_t e = launch_restore(c->lat.storage, c->lat.walls, la, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "restore kernel");
  e = launch_fill(c->d_acc, 0.0, 4, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "restore reset");
  c->unstable = false;
  return LB_OK;
}

int64_t lb_time(const lb_ctx *c) { return c ? c->t : -1; }

int lb_set_two_step(lb_ctx *c, int32_t enable, int32_t rows) {
  if (!c) return fail(nullptr, LB_EINVAL, "null context");
  if (enable != LB_TWO_STEP_OFF && enable != LB_TWO_STEP_ON && enable != LB_TWO_STEP_AUTO)
    return fail(c, LB_EINVAL, "enable must be LB_TWO_STEP_OFF, LB_TWO_STEP_ON or LB_TWO_STEP_AUTO");
  if (rows < 0) return fail(c, LB_EINVAL, "rows must be >= 0");
  c->two_step = enable;
  c->sy2 = rows;
  c->graph.clear();  // captured launches change
  return LB_OK;
}

int lb_two_step_active(const lb_ctx *c) { return c ? (pairs_on(c) && c->reduce_every == 0 ? 1 : 0) : -1; }

int lb_set_time(lb_ctx *c, int64_t t) {
  if (!c) return fail(nullptr, LB_EINVAL, "null context");
  if (t < 0) return fail(c, LB_EINVAL, "time must be >= 0");
  c->t = t;
  return LB_OK;
}

int lb_set_tile(lb_ctx *c, int32_t tx, int32_t sy) {
  if (!c) return fail(nullptr, LB_EINVAL, "null context");
  if (tx != 64 && tx != 128 && tx != 256) return fail(c, LB_EINVAL, "tx must be 64, 128 or 256");
  if (sy < 1) return fail(c, LB_EINVAL, "sy must be >= 1");
  if (grid_blocks(c, tx, sy, nullptr) > kMaxBlocks) return fail(c, LB_EINVAL, "too many workgroups");
  c->tx = tx;
  c->sy = std::min<int32_t>(sy, c->lat.ly);
  c->graph.clear();  // captured launches carry the old shape
  return LB_OK;
}

int lb_set_store_policy(lb_ctx *c, int32_t policy) {
  if (!c) return fail(nullptr, LB_EINVAL, "null context");
  if (policy != LB_STORES_AUTO && policy != LB_STORES_WRITE_THROUGH && policy != LB_STORES_STREAMING)
    return fail(c, LB_EINVAL, "policy must be LB_STORES_AUTO, LB_STORES_WRITE_THROUGH or LB_STORES_STREAMING");
  c->store_policy = policy;
  c->graph.clear();  // captured launches carry the old kernel variant
  return LB_OK;
}

int lb_set_rounding(lb_ctx *c, int32_t mode) {
  if (!c) return fail(nullptr, LB_EINVAL, "null context");
  if (mode != LB_ROUND_NEAREST && mode != LB_ROUND_STOCHASTIC)
    return fail(c, LB_EINVAL, "mode must be LB_ROUND_NEAREST or LB_ROUND_STOCHASTIC");
  if (mode == LB_ROUND_STOCHASTIC && c->lat.storage != LB_BF16DEV)
    return fail(c, LB_EINVAL, "stochastic rounding applies to BF16 storage only");
  if (mode == LB_ROUND_STOCHASTIC && !c->d_tbase) {
    hipError_t e = hipMalloc(&c->d_tbase, sizeof(double));
    if (e != hipSuccess) return fail(c, LB_ENOMEM, std::string("step base: ") + hipGetErrorString(e));
  }
  c->rounding = mode;
  c->graph.clear();  // captured launches carry the old kernel variant
  return LB_OK;
}

int lb_set_couplings(lb_ctx *c, const lb_couplings *cpl) {
  if (!c) return fail(nullptr, LB_EINVAL, "null context");
  if (!cpl) return fail(c, LB_EINVAL, "null couplings");
  std::string msg;
  int rc = validate(&c->lat, cpl, c->tau, &c->psi, msg);
  if (rc) return fail(c, rc, msg);
  c->cpl = *cpl;
  normalise(c->lat, c->cpl, c->psi, c->tau);
  c->graph.clear();  // captured launches carry the old couplings
  return LB_OK;
}

namespace {

// The profile pass and its second pass, with `buf` holding the block sums and then the row
// sums ((ncb + 1) * ly * PROF_N doubles).
int profile_into(lb_ctx *c, int nb, int nseg, int ncb, double *buf, double *out) {
  StepArgs a;
  fill_step_args(c, a);
  a.nseg = nseg;
  a.src = c->pop[c->cur];
  a.dst = c->pop[c->cur ^ 1];  // not written
  a.prof = buf;
  a.ncb = ncb;
  hipError_t e = launch_step(c->lat.storage, c->lat.n_species, c->lat.walls, WHAT_PROFILE, c->tx, nb, a, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "profile kernel launch");
  // the walls' share of their momentum exchange: sum_s rho_w,s U / 3 per unit length
  double wb0 = 0.0, wt0 = 0.0;
  if (c->lat.walls)
    for (int s = 0; s < c->lat.n_species; ++s) {
      wb0 += 2.0 * a.wall_mom[0][s];
      wt0 += 2.0 * a.wall_mom[1][s];
    }
  e = launch_profile_finish(buf, ncb, c->lat.lx, c->lat.ly, c->lat.walls, wb0, wt0,
                            buf + (size_t)ncb * c->lat.ly * PROF_N, out, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "profile finish launch");
  return LB_OK;
}

}  // namespace

int lb_profile(lb_ctx *c, double *out) {
  if (!c) return fail(nullptr, LB_EINVAL, "null context");
  if (!out) return fail(c, LB_EINVAL, "null output");
  int nseg = 0;
  const int nb = grid_blocks(c, c->tx, c->sy, &nseg);
  const int ncb = ((c->lat.lx + c->tx - 1) / c->tx) * (c->tx / 64);
  const size_t need = ((size_t)ncb + 1) * c->lat.ly * PROF_N;  // block sums, then the row sums
  if (need > c->prof_cap) {
    if (c->d_prof) (void)hipFree(c->d_prof);
    c->d_prof = nullptr;
    c->prof_cap = 0;
    hipError_t e = hipMalloc(&c->d_prof, need * sizeof(double));
    if (e != hipSuccess) return fail(c, LB_ENOMEM, std::string("profile buffer: ") + hipGetErrorString(e));
    c->prof_cap = need;
  }
  return profile_into(c, nb, nseg, ncb, c->d_prof, out);
}

int lb_profile_noalloc(lb_ctx *c, double *out) {
  if (!c) return fail(nullptr, LB_EINVAL, "null context");
  if (!out) return fail(c, LB_EINVAL, "null output");
  int nseg = 0;
  const int nb = grid_blocks(c, c->tx, c->sy, &nseg);
  const int ncb = ((c->lat.lx + c->tx - 1) / c->tx) * (c->tx / 64);
  const size_t need = ((size_t)ncb + 1) * c->lat.ly * PROF_N;
  if (need > kStaticScratchDoubles)
    return fail(c, LB_EINVAL, "lb_profile_noalloc: this lattice and strip width need " + std::to_string(need) +
                                  " doubles of scratch, the static scratch holds " +
                                  std::to_string(kStaticScratchDoubles) + " (use lb_profile)");
  double *buf = static_scratch(c->device);
  if (!buf) return fail(c, LB_EDEVICE, "lb_profile_noalloc: no static scratch address for this device");
  return profile_into(c, nb, nseg, ncb, buf, out);
}

int lb_profile_stats(lb_ctx *c, const double *samples, int64_t n, int32_t k0, double *out) {
  if (!c) return fail(nullptr, LB_EINVAL, "null context");
  if (!samples || !out) return fail(c, LB_EINVAL, "null argument");
  if (n < 1) return fail(c, LB_EINVAL, "n must be >= 1");
  if (k0 < 0 || k0 > c->lat.ly) return fail(c, LB_EINVAL, "k0 must be in [0, ly]");
  const double ub = c->lat.walls ? c->cpl.wall_velocity[0] : 0.0, ut = c->lat.walls ? c->cpl.wall_velocity[1] : 0.0;
  hipError_t e = launch_profile_stats(samples, (long long)n, c->lat.ly, c->lat.walls, k0, ub, ut, out, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "profile statistics launch");
  return LB_OK;
}

int lb_set_graph(lb_ctx *c, int32_t steps) {
  if (!c) return fail(nullptr, LB_EINVAL, "null context");
  if (steps < 0 || (steps & 1)) return fail(c, LB_EINVAL, "graph steps must be even and >= 0");
  c->graph.clear();
  c->graph.steps = steps;
  return LB_OK;
}

int lb_autotune(lb_ctx *c, int32_t trial_steps, int32_t *tx_out, int32_t *sy_out, double *ms_out) {
  if (!c) return fail(nullptr, LB_EINVAL, "null context");
  if (trial_steps < 1) return fail(c, LB_EINVAL, "trial_steps must be >= 1");
  int rc = poll_health(c, true);
  if (rc) return rc;
  // Every trial launch reads the current state and writes the other buffer, which holds
  // nothing needed: the state is the same before and after tuning.
  const int tx0 = c->tx, sy0 = c->sy;
  int best_tx = tx0, best_sy = sy0;
  double best = -1.0;
  const int txs[3] = {64, 128, 256};
  const int sys[] = {1, 2, 3, 4, 6, 8, 10, 12, 16, 20, 24, 32, 48, 64};
  auto trial = [&](int tx, int sy) -> int {
    if (sy > c->lat.ly || grid_blocks(c, tx, sy, nullptr) > kMaxBlocks) return LB_OK;
    c->tx = tx;
    c->sy = sy;
    const double ms = time_launches(c->stream, 2, trial_steps, [&]() { return launch_plain_step(c, c->cur, c->stream, (uint32_t)c->t, nullptr); });
    if (ms < 0.0) return hip_fail(c, hipGetLastError(), "autotune trial");
    if (best < 0.0 || ms < best) {
      best = ms;
      best_tx = tx;
      best_sy = sy;
    }
    return LB_OK;
  };
  rc = trial(tx0, sy0);  // the default shape competes too
  for (int tx : txs) {
    if (tx > 64 && tx / 2 >= c->lat.lx) continue;  // wider than the lattice needs
    for (int sy : sys)
      if (!rc && !(tx == tx0 && sy == sy0)) rc = trial(tx, sy);
  }
  c->tx = rc ? tx0 : best_tx;
  c->sy = rc ? sy0 : best_sy;
  c->graph.clear();
  if (rc) return rc;
  if (tx_out) *tx_out = c->tx;
  if (sy_out) *sy_out = c->sy;
  if (ms_out) *ms_out = best;
  return LB_OK;
}

int lb_get_tile(const lb_ctx *c, int32_t *tx, int32_t *sy) {
  if (!c || !tx || !sy) return LB_EINVAL;
  *tx = c->tx;
  *sy = c->sy;
  return LB_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------------------
// Adjoint: gradient of L = lw0 <(W_bot + W_top)/2> + lw1 <Q> over T steps.
// ---------------------------------------------------------------------------------------

namespace {

struct AdjLayout {
  int every = 1, ncp = 1;
  bool all = false;  // every == 1: what the reverse step reads of every state, kept by the forward pass
  int64_t per = 1;   // states per segment buffer
  int nbuf = 1;      // segment buffers
  size_t s64 = 0, lamb = 0, nsite = 0, fb = 0, xw = 0;
  size_t corrb = 0, fbb = 0;
  size_t ckpt = 0, seg = 0, fin = 0, lam0 = 0, lam1 = 0, corr0 = 0, corr1 = 0, fields = 0, fbar = 0, partials = 0, acc = 0;
  size_t total = 0;
};

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

bool adjoint_fp64(const lb_ctx *c, int32_t flags) { return c->lat.storage == LB_F64 || (flags & LB_ADJ_FP64); }

AdjLayout adjoint_layout(const lb_ctx *c, int64_t T, int32_t every, int32_t flags) {
  AdjLayout L;
  L.every = every > 0 ? every : std::max<int>(1, (int)std::ceil(std::sqrt((double)T)));
  L.every = (int)std::min<int64_t>(L.every, std::max<int64_t>(T, 1));
  L.ncp = (int)((T + L.every - 1) / L.every);
  L.nsite = (size_t)c->lat.lx * c->lat.ly;
  const size_t rs = adjoint_fp64(c, flags) ? 8 : 4;
  const int ns = c->lat.n_species;
  L.all = L.every == 1;
  // no checkpoints to restore from when every state is kept
  if (L.all) L.ncp = 0;
  // per state: the FP64 populations of the two rows next to the walls, and the fields; with
  // several checkpoint segments, two segment buffers (one is recomputed while the reverse
  // sweep reads the other)
  L.per = L.all ? std::max<int64_t>(T, 1) : L.every;
  L.nbuf = L.ncp > 1 ? 2 : 1;
  const int64_t nstate = L.per * L.nbuf;
  L.s64 = align256((size_t)ns * 9 * L.nsite * 8);
  L.xw = align256((size_t)ns * 9 * 2 * c->lat.lx * 8);
  L.lamb = align256((size_t)ns * 9 * L.nsite * rs);
  L.fb = align256(8 * L.nsite * rs);
  size_t o = 0;
  L.ckpt = o; o += (size_t)L.ncp * L.s64;
  L.seg = o; o += (size_t)nstate * L.xw;
  L.fin = o; o += L.all ? 0 : align256(lb_pop_bytes(&c->lat));
  L.lam0 = o; o += L.lamb;
  L.lam1 = o; o += L.lamb;
  L.corrb = align256((size_t)ns * L.nsite * rs);
  L.corr0 = o; o += L.corrb;
  L.corr1 = o; o += L.corrb;
  L.fields = o; o += (size_t)nstate * L.fb;  // one set per state of a segment (of the run when all)
  L.fbb = align256(8 * L.nsite * rs);
  L.fbar = o; o += 2 * L.fbb;  // ping-pong: a reverse step reads the next step's and writes its own
  L.partials = o; o += align256((size_t)adj_blocks(c->lat.lx, c->lat.ly) * ADJ_N * 8);
  L.acc = o; o += align256(ADJ_N * 8);
  L.total = o;
  return L;
}

AdjArgs adjoint_args(const lb_ctx *c, double lw0, double lw1, int64_t T) {
  AdjArgs a;
  std::memset(&a, 0, sizeof(a));
  a.lx = c->lat.lx;
  a.ly = c->lat.ly;
  a.cross_psi = c->cpl.cross_uses_psi;
  for (int s = 0; s < 2; ++s) {
    for (int q = 0; q < 5; ++q) a.K[s][q] = c->cpl.g1[s] * c->cpl.w[q] + c->cpl.g2[s] * c->cpl.p[q];
    a.g1[s] = c->cpl.g1[s];
    a.g2[s] = c->cpl.g2[s];
    a.body[s] = c->cpl.body_force[s];
    a.tau[s] = c->tau[s];
    a.omega[s] = 1.0 / c->tau[s];
    a.rho_w[s] = c->cpl.rho_wall[s];
    a.psi_w[s] = c->psi.psi0 * (1.0 - std::exp(-c->cpl.rho_wall[s] / c->psi.rho0));
  }
  for (int q = 0; q < 5; ++q) {
    a.w[q] = c->cpl.w[q];
    a.p[q] = c->cpl.p[q];
  }
  a.t[0] = c->cpl.t[0];
  a.t[1] = c->cpl.t[1];
  a.gab = c->cpl.g_ab;
  a.psi0 = c->psi.psi0;
  a.irho0 = 1.0 / c->psi.rho0;
  a.ilx = 1.0 / (double)c->lat.lx;
  a.ilxf = 1.0f / (float)c->lat.lx;
  a.cW = lw0 / (double)T;
  a.cQ = lw1 / (double)T;
  a.u_wall[0] = c->lat.walls ? c->cpl.wall_velocity[0] : 0.0;
  a.u_wall[1] = c->lat.walls ? c->cpl.wall_velocity[1] : 0.0;
  return a;
}

}  // namespace

extern "C" {

size_t lb_adjoint_workspace_bytes(const lb_ctx *c, int64_t T, int32_t every, int32_t flags) {
  if (!c || T < 1) return 0;
  return adjoint_layout(c, T, every, flags).total;
}

int lb_adjoint(lb_ctx *c, int64_t T, int32_t every, int32_t flags, const double loss_weights[2], double *loss,
               double grad[7], void *workspace, size_t workspace_bytes) {
  if (!c) return fail(nullptr, LB_EINVAL, "null context");
  if (T < 1) return fail(c, LB_EINVAL, "T must be >= 1");
  if (!loss_weights || !grad) return fail(c, LB_EINVAL, "null argument");
  if (!workspace) return fail(c, LB_EINVAL, "null workspace");
  if (flags & ~LB_ADJ_FP64) return fail(c, LB_EINVAL, "unknown adjoint flags");
  if (c->rounding != LB_ROUND_NEAREST)
    return fail(c, LB_EINVAL, "the adjoint recomputes states and needs round-to-nearest storage");
  const AdjLayout L = adjoint_layout(c, T, every, flags);
  if (workspace_bytes < L.total) return fail(c, LB_ENOMEM, "workspace smaller than lb_adjoint_workspace_bytes()");
  int rc = poll_health(c, true);
  if (rc) return rc;
  char *ws = static_cast<char *>(workspace);
  const int64_t t0 = c->t;
  const int keep_reduce = c->reduce_every;
  c->reduce_every = 0;
  auto done = [&](int code) {
    c->reduce_every = keep_reduce;
    return code;
  };
  const int fp64 = adjoint_fp64(c, flags) ? 1 : 0;
  hipError_t e = hipSuccess;
  if (L.all) {
    // forward pass keeping what the reverse step reads of every state: no recompute later
    for (int64_t t = 0; t < T && e == hipSuccess; ++t) {
      e = launch_plain_step_fields(c, c->cur, ws + L.seg + (size_t)t * L.xw, ws + L.fields + (size_t)t * L.fb, fp64,
                                   c->stream);
      c->cur ^= 1;
      ++c->t;
    }
    if (e != hipSuccess) return done(hip_fail(c, e, "adjoint forward pass"));
  } else {
    // forward pass with a checkpoint every L.every steps
    for (int k = 0; k < L.ncp; ++k) {
      if ((rc = lb_checkpoint(c, ws + L.ckpt + (size_t)k * L.s64))) return done(rc);
      if ((rc = lb_step(c, std::min<int64_t>(L.every, T - (int64_t)k * L.every)))) return done(rc);
    }
  }
  // the final state, bit for bit (the context continues from it; the checkpointed sweep
  // overwrites the population buffers while recomputing)
  const int cur_final = c->cur;
  const size_t popb = lb_pop_bytes(&c->lat);
  if (!L.all) e = hipMemcpyAsync(ws + L.fin, c->pop[cur_final], popb, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) e = launch_zero(ws + L.lam1, L.lamb, c->stream);
  if (e == hipSuccess) e = launch_zero(ws + L.corr1, L.corrb, c->stream);
  if (e == hipSuccess) e = launch_zero(ws + L.acc, ADJ_N * 8, c->stream);
  if (e == hipSuccess)
    e = launch_zero(ws + L.partials, (size_t)adj_blocks(c->lat.lx, c->lat.ly) * ADJ_N * 8, c->stream);
  if (e != hipSuccess) return done(hip_fail(c, e, "adjoint setup"));
  // reverse sweep: over the whole run when every state was kept, else one checkpoint segment at
  // a time
  AdjArgs a = adjoint_args(c, loss_weights[0], loss_weights[1], T);
  a.partials = reinterpret_cast<double *>(ws + L.partials);
  double *acc = reinterpret_cast<double *>(ws + L.acc);
  // lambda(t+1) is lam_buf[q] + corr_buf[q], lambda(t) lam_buf[q ^ 1] + corr_buf[q ^ 1]
  char *lam_buf[2] = {ws + L.lam1, ws + L.lam0};
  char *corr_buf[2] = {ws + L.corr1, ws + L.corr0};
  // psi_s Fbar_s and r_s Fbar_s of step t + 1 in fbar_buf[q], of step t in fbar_buf[q ^ 1]
  char *fbar_buf[2] = {ws + L.fbar, ws + L.fbar + L.fbb};
  int q = 0;
  // what the reverse step reads of state jj of segment buffer b
  auto seg_x = [&](int b, int jj) { return ws + L.seg + ((size_t)b * L.per + jj) * L.xw; };
  auto seg_f = [&](int b, int jj) { return ws + L.fields + ((size_t)b * L.per + jj) * L.fb; };
  // A recompute that runs beside the reverse sweep takes at most one workgroup per CU (taller
  // segments), leaving the rest of the chip to the reverse kernels; measured 5% faster on the
  // 512 x 256 channel than the resident grid of the context's launch shape.
  int rsy = c->sy;
  if (L.nbuf == 2) {
    const int nstrip = (c->lat.lx + c->tx - 1) / c->tx;
    const int nseg = std::max(1, c->n_cu / nstrip);
    rsy = std::min(c->lat.ly, std::max(c->sy, (c->lat.ly + nseg - 1) / nseg));
  }
  auto recompute = [&](int from, int len, int b, hipStream_t st) -> hipError_t {
    hipError_t er = hipSuccess;
    // every state but the last is stepped from, which writes its fields on the way; the last
    // one's fields come from a pass of their own
    for (int jj = 0; jj < len && er == hipSuccess; ++jj) {
      if (jj + 1 < len) er = launch_plain_step_fields(c, from ^ (jj & 1), seg_x(b, jj), seg_f(b, jj), fp64, st, rsy);
      else er = launch_checkpoint_fields_from(c, from ^ (jj & 1), seg_x(b, jj), seg_f(b, jj), fp64, st);
    }
    return er;
  };
  // FP32 sweeps: inside a segment the local pass gathers the common term of lambda(t+1)
  // itself, from the next step's fbar and the next state's fields in the same segment buffer;
  // the first reverse step of a segment reads it from memory, written by the gather pass that
  // follows the last reverse step of the segment after it (zero for lambda(T)).  FP64 sweeps
  // keep the separate gather pass after every local pass: their gather inside the local pass
  // (LDS traffic of the halo) measured no faster, and its LDS footprint left less room for the
  // recompute running beside it.
  const bool fuse_gather = !fp64;
  auto reverse = [&](int q0, int len, int b, hipStream_t st) -> hipError_t {
    hipError_t er = hipSuccess;
    int qq = q0;
    for (int jj = len - 1; jj >= 0 && er == hipSuccess; --jj) {
      const int gin = fuse_gather && jj + 1 < len ? 1 : 0, gout = !fuse_gather || jj == 0 ? 1 : 0;
      a.x = reinterpret_cast<const double *>(seg_x(b, jj));
      a.fields = seg_f(b, jj);
      a.fields_next = gin ? seg_f(b, jj + 1) : nullptr;
      a.lam_next = lam_buf[qq];
      a.corr_next = corr_buf[qq];
      a.lam = lam_buf[qq ^ 1];
      a.corr = corr_buf[qq ^ 1];
      a.fbar_next = fbar_buf[qq];
      a.fbar = fbar_buf[qq ^ 1];
      er = launch_adjoint_step(fp64, c->lat.n_species, c->lat.walls, a, gin, gout, st);
      qq ^= 1;
    }
    return er;
  };
  // With several segments the reverse sweep runs on a second stream, one segment behind the
  // recompute on the context's stream: segment k's reverse steps overlap segment k - 1's
  // recompute into the other buffer.  Events order the two (a recompute waits until the
  // reverse sweep that read its buffer has finished), so every kernel reads what it read
  // with one stream, and the result is bitwise the same.  A full segment's recompute and its
  // reverse sweep are the same launches for every full segment up to the buffer and the
  // ping-pong parities: each is captured once per combination as a HIP graph and replayed; a
  // shorter last segment runs eagerly.
  GraphCache g_fwd[2], g_rev[2];
  for (int b = 0; b < 2; ++b) g_fwd[b].steps = g_rev[b].steps = 1;
  hipStream_t rst = c->stream;
  hipEvent_t ev_rec[2] = {nullptr, nullptr}, ev_rev[2] = {nullptr, nullptr};
  const bool two = L.nbuf == 2;
  auto release = [&]() {
    if (rst != c->stream) (void)hipStreamSynchronize(rst);
    for (int b = 0; b < 2; ++b) {
      g_fwd[b].destroy();
      g_rev[b].destroy();
      if (ev_rec[b]) (void)hipEventDestroy(ev_rec[b]);
      if (ev_rev[b]) (void)hipEventDestroy(ev_rev[b]);
      ev_rec[b] = ev_rev[b] = nullptr;
    }
    if (rst != c->stream) (void)hipStreamDestroy(rst);
    rst = c->stream;
  };
  auto graphs_done = [&](int code) {
    // nothing of this call is left in flight on the caller's workspace
    (void)hipStreamSynchronize(c->stream);
    release();
    return done(code);
  };
  if (two) {
    e = hipStreamCreateWithFlags(&rst, hipStreamNonBlocking);
    if (e != hipSuccess) rst = c->stream;
    for (int b = 0; b < 2 && e == hipSuccess; ++b) {
      e = hipEventCreateWithFlags(&ev_rec[b], hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_rev[b], hipEventDisableTiming);
    }
    if (e != hipSuccess) return graphs_done(hip_fail(c, e, "adjoint streams"));
  }
  if (L.all) {
    // every state was kept: one reverse sweep over the whole run
    e = reverse(q, (int)T, 0, c->stream);
    if (e != hipSuccess) return graphs_done(hip_fail(c, e, "adjoint sweep"));
  }
  auto seg_len = [&](int k) { return (int)std::min<int64_t>(L.every, T - (int64_t)k * L.every); };
  // restore checkpoint k and recompute its segment into buffer k % nbuf (context's stream)
  auto recompute_segment = [&](int k) -> int {
    const int len = seg_len(k), b = k % L.nbuf;
    int r = lb_restore(c, ws + L.ckpt + (size_t)k * L.s64);
    if (r) return r;
    hipError_t er = hipSuccess;
    if (two && k + 2 < L.ncp) er = hipStreamWaitEvent(c->stream, ev_rev[b], 0);
    const int from = c->cur;
    if (er == hipSuccess) {
      if (len == L.every) {
        hipGraphExec_t gf = nullptr;
        er = g_fwd[b].get(from, [&](int, hipStream_t st) { return recompute(from, len, b, st); }, &gf);
        if (er == hipSuccess) er = hipGraphLaunch(gf, c->stream);
      } else {
        er = recompute(from, len, b, c->stream);
      }
    }
    if (er == hipSuccess && two) er = hipEventRecord(ev_rec[b], c->stream);
    if (er != hipSuccess) return hip_fail(c, er, "adjoint recompute");
    c->cur = from ^ ((len - 1) & 1);
    return LB_OK;
  };
  // the reverse steps of segment k (second stream, after its recompute)
  auto reverse_segment = [&](int k) -> int {
    const int len = seg_len(k), b = k % L.nbuf, q0 = q;
    hipError_t er = two ? hipStreamWaitEvent(rst, ev_rec[b], 0) : hipSuccess;
    if (er == hipSuccess) {
      if (len == L.every) {
        hipGraphExec_t gr = nullptr;
        er = g_rev[b].get(q0, [&](int, hipStream_t st) { return reverse(q0, len, b, st); }, &gr);
        if (er == hipSuccess) er = hipGraphLaunch(gr, rst);
      } else {
        er = reverse(q0, len, b, rst);
      }
    }
    if (er == hipSuccess && two) er = hipEventRecord(ev_rev[b], rst);
    if (er != hipSuccess) return hip_fail(c, er, "adjoint sweep");
    q ^= (len & 1);
    return LB_OK;
  };
  if (L.ncp > 0 && (rc = recompute_segment(L.ncp - 1))) return graphs_done(rc);
  for (int k = L.ncp - 1; k >= 0; --k) {
    if (k > 0 && (rc = recompute_segment(k - 1))) return graphs_done(rc);
    if ((rc = reverse_segment(k))) return graphs_done(rc);
  }
  e = launch_adjoint_reduce(a.partials, c->lat.lx, c->lat.ly, acc, rst);
  // the context's stream continues after the reverse sweep
  if (e == hipSuccess && two) e = hipEventRecord(ev_rev[0], rst);
  if (e == hipSuccess && two) e = hipStreamWaitEvent(c->stream, ev_rev[0], 0);
  if (e != hipSuccess) return graphs_done(hip_fail(c, e, "adjoint reduction"));
  release();
  // back to the state after T steps
  if (!L.all) e = hipMemcpyAsync(c->pop[cur_final], ws + L.fin, popb, hipMemcpyDeviceToDevice, c->stream);
  double h[ADJ_N];
  if (e == hipSuccess) e = hipMemcpyAsync(h, acc, sizeof(h), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return done(hip_fail(c, e, "adjoint readback"));
  c->cur = cur_final;
  c->t = t0 + T;
  for (int k = 0; k < 7; ++k) grad[k] = h[k];
  if (loss) *loss = h[ADJ_LW] + h[ADJ_LQ];
  if (!std::isfinite(h[ADJ_LW] + h[ADJ_LQ])) return done(fail(c, LB_EUNSTABLE, "non-finite loss"));
  return done(LB_OK);
}

const char *lb_last_error(const lb_ctx *c) { return c ? c->err.c_str() : g_init_error.c_str(); }

void lb_destroy(lb_ctx *c) {
  if (!c) return;
  if (c->check_pending && c->ev) (void)hipEventSynchronize(c->ev);
  (void)hipStreamSynchronize(c->stream);
  if (c->d_partials) (void)hipFree(c->d_partials);
  if (c->d_prof) (void)hipFree(c->d_prof);
  if (c->d_tbase) (void)hipFree(c->d_tbase);
  if (c->d_totals) (void)hipFree(c->d_totals);
  if (c->d_acc) (void)hipFree(c->d_acc);
  if (c->d_accrows) (void)hipFree(c->d_accrows);
  if (c->h_acc) (void)hipHostFree(c->h_acc);
  if (c->ev) (void)hipEventDestroy(c->ev);
  c->graph.destroy();
  delete c;
}

}  // extern "C"
