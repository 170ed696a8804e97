// Host runtime of the batched calls of include/lb.h: many independent lattices of uneven
// sizes and couplings (one kernel template: same storage, species count and wall mode),
// stepped together by one persistent launch per time step, optionally replayed from a
// captured HIP graph, with the tile shape picked by an autotuner.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lb_host.hpp"
#include "lb_internal.hpp"

using namespace lb355;
using namespace lb355::host;

namespace {
thread_local std::string g_batch_init_error;
constexpr size_t kInstanceAlign = 256;  // bytes between instances in a population buffer
}  // namespace

struct lb_batch {
  int n = 0;
  int storage = 0, ns = 1, walls = 0;
  std::vector<lb_lattice> lat;
  std::vector<lb_couplings> cpl;
  std::vector<lb_psi_params> psi;
  std::vector<double> tau;         // [n][2]
  std::vector<size_t> off;         // byte offset of each instance in a population buffer
  std::vector<StepArgs> args;      // host copy of d_args
  std::vector<TileDesc> tiles;     // host copy of d_tiles
  std::vector<int> tile0, ntile;   // tiles of instance i: [tile0[i], tile0[i] + ntile[i])
  void *pop[2]{nullptr, nullptr};
  int cur = 0;
  size_t pop_bytes = 0;
  size_t footprint = 0;  // lb_batch_pop_bytes of the instances (one buffer)
  hipStream_t stream = nullptr;
  int tx = 256, sy = 8, grid = 0;  // grid: persistent workgroups (0: one per tile)
  int n_cu = 256;
  int reduce_every = 0;
  int64_t t = 0;
  int rounding = LB_ROUND_NEAREST;  // BF16 stores: nearest or stochastic
  double *d_tbase = nullptr;        // step at which a graph replay starts (stochastic rounding)
  StepArgs *d_args = nullptr;
  TileDesc *d_tiles = nullptr;
  ReduceJob *d_jobs = nullptr;
  double *d_partials = nullptr;  // [tiles][RED_N]
  double *d_accrows = nullptr;   // [tiles][ACC_N]: running sums of reducing steps (zero after a flush)
  double *d_prof = nullptr;      // profile pass of one instance: block sums, then row sums
  size_t prof_cap = 0;           // doubles
  int64_t acc_pending = 0;       // reducing launches since the last flush
  double *d_totals = nullptr;    // [n][RED_N]
  double *d_acc = nullptr;       // [n][4]: wall stress sums (bot, top), count, bad
  double *h_acc = nullptr;       // pinned copy of d_acc
  size_t tile_cap = 0;
  hipEvent_t ev = nullptr;
  bool check_pending = false;
  bool unstable = false;
  GraphCache graph;
  std::string err;
};

namespace {

int bfail(lb_batch *b, int code, const std::string &msg) {
  if (b) b->err = msg;
  else g_batch_init_error = msg;
  return code;
}

int bhip(lb_batch *b, hipError_t e, const char *what) {
  return bfail(b, LB_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

int count_tiles(const lb_batch *b, int tx, int sy) {
  long long n = 0;
  for (int i = 0; i < b->n; ++i)
    n += (long long)((b->lat[i].lx + tx - 1) / tx) * ((b->lat[i].ly + sy - 1) / sy);
  return n > kMaxBlocks ? -1 : (int)n;
}

// Resident workgroups of the batch kernel on the whole device at strip width tx.
int resident(const lb_batch *b, int tx) { return step_blocks_per_cu(b->storage, b->ns, b->walls, tx) * b->n_cu; }

// Build the tile table (band-major within each instance), per-instance arguments and
// reduction jobs for shape (tx, sy) and upload them.  Synchronises the stream.
int build_tiles(lb_batch *b, int tx, int sy) {
  const int nt = count_tiles(b, tx, sy);
  if (nt < 0) return bfail(b, LB_EINVAL, "too many tiles");
  std::vector<TileDesc> tiles;
  tiles.reserve(nt);
  std::vector<ReduceJob> jobs(b->n);
  std::vector<int> t0(b->n), ntl(b->n);
  std::vector<StepArgs> args(b->n);
  for (int i = 0; i < b->n; ++i) {
    const lb_lattice &L = b->lat[i];
    const int pitch = row_pitch(L.lx);
    const long long plane = (long long)L.ly * pitch;
    const int syi = std::min(sy, L.ly);
    args[i] = make_step_args(L, b->cpl[i], b->psi[i], &b->tau[2 * i], pitch, plane, syi);
    args[i].stream_stores = streaming_stores(b->footprint);
    const int nstrip = (L.lx + tx - 1) / tx, nseg = (L.ly + syi - 1) / syi;
    args[i].nseg = nseg;
    args[i].offset = (long long)b->off[i];
    t0[i] = (int)tiles.size();
    for (int seg = 0; seg < nseg; ++seg)
      for (int strip = 0; strip < nstrip; ++strip) {
        TileDesc d;
        d.inst = i;
        d.strip = strip;
        d.seg = seg;
        d.part = (int)tiles.size();
        tiles.push_back(d);
      }
    ntl[i] = (int)tiles.size() - t0[i];
    jobs[i].p0 = t0[i];
    jobs[i].n = ntl[i];
    jobs[i].inv_lx = 1.0 / L.lx;
  }
  hipError_t e = hipStreamSynchronize(b->stream);  // no launch may still read the old tables
  if (e != hipSuccess) return bhip(b, e, "tile table");
  if ((size_t)nt > b->tile_cap) {
    if (b->d_tiles) (void)hipFree(b->d_tiles);
    if (b->d_partials) (void)hipFree(b->d_partials);
    if (b->d_accrows) (void)hipFree(b->d_accrows);
    b->d_tiles = nullptr;
    b->d_partials = nullptr;
    b->d_accrows = nullptr;
    b->tile_cap = 0;
    if ((e = hipMalloc(&b->d_tiles, (size_t)nt * sizeof(TileDesc))) != hipSuccess ||
        (e = hipMalloc(&b->d_partials, (size_t)nt * RED_N * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&b->d_accrows, (size_t)nt * ACC_N * sizeof(double))) != hipSuccess ||
        (e = launch_fill(b->d_accrows, 0.0, nt * ACC_N, b->stream)) != hipSuccess)
      return bfail(b, LB_ENOMEM, std::string("tile table: ") + hipGetErrorString(e));
    b->tile_cap = nt;
  }
  if ((e = hipMemcpyAsync(b->d_tiles, tiles.data(), (size_t)nt * sizeof(TileDesc), hipMemcpyHostToDevice,
                          b->stream)) != hipSuccess ||
      (e = hipMemcpyAsync(b->d_args, args.data(), (size_t)b->n * sizeof(StepArgs), hipMemcpyHostToDevice,
                          b->stream)) != hipSuccess ||
      (e = hipMemcpyAsync(b->d_jobs, jobs.data(), (size_t)b->n * sizeof(ReduceJob), hipMemcpyHostToDevice,
                          b->stream)) != hipSuccess ||
      (e = hipStreamSynchronize(b->stream)) != hipSuccess)
    return bhip(b, e, "tile table upload");
  b->tiles.swap(tiles);
  b->args.swap(args);
  b->tile0.swap(t0);
  b->ntile.swap(ntl);
  b->tx = tx;
  b->sy = sy;
  b->graph.clear();
  return LB_OK;
}

int flush_acc(lb_batch *b) {
  if (b->acc_pending == 0) return LB_OK;
  hipError_t e = launch_batch_flush(b->d_accrows, b->d_jobs, b->n, b->d_acc, (double)b->acc_pending, b->stream);
  if (e != hipSuccess) return bhip(b, e, "reduction flush");
  b->acc_pending = 0;
  return LB_OK;
}

int launch_grid(const lb_batch *b, int ntiles) {
  const int g = b->grid > 0 ? b->grid : ntiles;
  return std::max(1, std::min(g, ntiles));
}

// One launch over tiles [first, first + count) from buffer `from` to the other one.
hipError_t launch_tiles(const lb_batch *b, int what, int from, int first, int count, hipStream_t st,
                        void *out_rho = nullptr, void *out_u = nullptr, int out_f32 = 0, uint32_t t_step = 0,
                        const double *t_base = nullptr) {
  BatchArgs a;
  std::memset(&a, 0, sizeof(a));
  a.inst = b->d_args;
  a.tiles = b->d_tiles;
  a.tile0 = first;
  a.ntiles = count;
  a.src = static_cast<const char *>(b->pop[from]);
  a.dst = static_cast<char *>(b->pop[from ^ 1]);
  a.partials = b->d_partials;
  a.accrows = b->d_accrows;
  a.out_rho = out_rho;
  a.out_u = out_u;
  a.out_f32 = out_f32;
  a.stream_stores = streaming_stores(b->footprint);
  a.t_step = t_step;
  a.t_base = t_base;
  const int mode = b->storage == LB_BF16DEV && b->rounding == LB_ROUND_STOCHASTIC ? MODE_BF16SR : b->storage;
  return launch_batch_step(mode, b->ns, b->walls, what, b->tx, launch_grid(b, count), a, st);
}

int poll(lb_batch *b, bool wait) {
  if (b->check_pending) {
    hipError_t e = wait ? hipEventSynchronize(b->ev) : hipEventQuery(b->ev);
    if (e == hipSuccess) {
      b->check_pending = false;
      for (int i = 0; i < b->n; ++i)
        if (b->h_acc[4 * i + 3] > 0.0) b->unstable = true;
    } else if (e != hipErrorNotReady) {
      return bhip(b, e, "health check");
    }
  }
  if (b->unstable) return bfail(b, LB_EUNSTABLE, "non-finite or non-positive density in an instance");
  return LB_OK;
}

int check_index(lb_batch *b, int32_t i) {
  if (i < 0 || i >= b->n) return bfail(b, LB_EINVAL, "instance index out of range");
  return LB_OK;
}

LayoutArgs layout_args(const lb_batch *b, int i) {
  LayoutArgs la{};
  const int pitch = row_pitch(b->lat[i].lx);
  la.plane = (long long)b->lat[i].ly * pitch;
  la.lx = b->lat[i].lx;
  la.ly = b->lat[i].ly;
  la.pitch = pitch;
  la.ns = b->ns;
  la.rho_ref[0] = b->psi[i].rho_ref[0];
  la.rho_ref[1] = b->psi[i].rho_ref[1];
  return la;
}

}  // namespace

extern "C" {

size_t lb_batch_pop_bytes(int32_t n, const lb_lattice *lats) {
  if (n < 1 || !lats) return 0;
  size_t total = 0;
  for (int i = 0; i < n; ++i) {
    const size_t bi = lb_pop_bytes(&lats[i]);
    if (bi == 0) return 0;
    total += (bi + kInstanceAlign - 1) / kInstanceAlign * kInstanceAlign;
  }
  return total;
}

int lb_batch_init(lb_batch **out, int32_t n, const lb_lattice *lats, const lb_couplings *cpls, const double *tau,
                  const lb_psi_params *psis, const double *const *rho_init, void *pop_a, void *pop_b,
                  size_t pop_bytes, void *hip_stream) {
  if (!out) return bfail(nullptr, LB_EINVAL, "null output pointer");
  *out = nullptr;
  if (n < 1 || !lats || !cpls || !tau || !psis || !rho_init) return bfail(nullptr, LB_EINVAL, "null argument or n < 1");
  if (!pop_a || !pop_b || pop_a == pop_b) return bfail(nullptr, LB_EINVAL, "pop_a and pop_b must be distinct buffers");
  for (int i = 0; i < n; ++i) {
    std::string msg;
    int rc = validate(&lats[i], &cpls[i], &tau[2 * i], &psis[i], msg);
    if (rc) return bfail(nullptr, rc, "instance " + std::to_string(i) + ": " + msg);
    if (lats[i].storage != lats[0].storage || lats[i].n_species != lats[0].n_species ||
        lats[i].walls != lats[0].walls)
      return bfail(nullptr, LB_EINVAL, "all instances must share storage, n_species and walls");
    if (lb_pop_bytes(&lats[i]) >= ((size_t)1 << 32))
      return bfail(nullptr, LB_EINVAL, "instance " + std::to_string(i) + ": population buffer must stay below 4 GiB");
    if (!rho_init[i]) return bfail(nullptr, LB_EINVAL, "null rho_init");
    const size_t cnt = (size_t)lats[i].n_species * lats[i].lx * lats[i].ly;
    for (size_t k = 0; k < cnt; ++k)
      if (!(rho_init[i][k] > 0.0) || !std::isfinite(rho_init[i][k]))
        return bfail(nullptr, LB_EINVAL, "instance " + std::to_string(i) + ": rho_init must be finite and > 0");
  }
  const size_t need = lb_batch_pop_bytes(n, lats);
  if (pop_bytes < need) return bfail(nullptr, LB_ENOMEM, "population buffers smaller than lb_batch_pop_bytes()");

  lb_batch *b = new (std::nothrow) lb_batch();
  if (!b) return bfail(nullptr, LB_ENOMEM, "context allocation");
  b->n = n;
  b->storage = lats[0].storage;
  b->ns = lats[0].n_species;
  b->walls = lats[0].walls;
  b->lat.assign(lats, lats + n);
  b->cpl.assign(cpls, cpls + n);
  b->psi.assign(psis, psis + n);
  b->tau.assign(tau, tau + 2 * n);
  b->off.resize(n);
  size_t o = 0;
  for (int i = 0; i < n; ++i) {
    normalise(b->lat[i], b->cpl[i], b->psi[i], &b->tau[2 * i]);
    b->off[i] = o;
    o += (lb_pop_bytes(&lats[i]) + kInstanceAlign - 1) / kInstanceAlign * kInstanceAlign;
  }
  b->pop[0] = pop_a;
  b->pop[1] = pop_b;
  b->pop_bytes = pop_bytes;
  b->footprint = need;
  b->stream = static_cast<hipStream_t>(hip_stream);
  b->n_cu = device_cu_count();

  hipError_t e;
  if ((e = hipMalloc(&b->d_args, (size_t)n * sizeof(StepArgs))) != hipSuccess ||
      (e = hipMalloc(&b->d_jobs, (size_t)n * sizeof(ReduceJob))) != hipSuccess ||
      (e = hipMalloc(&b->d_totals, (size_t)n * RED_N * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(&b->d_acc, (size_t)n * 4 * sizeof(double))) != hipSuccess ||
      (e = hipHostMalloc(&b->h_acc, (size_t)n * 4 * sizeof(double), hipHostMallocDefault)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&b->ev, hipEventDisableTiming)) != hipSuccess) {
    g_batch_init_error = std::string("internal allocation: ") + hipGetErrorString(e);
    lb_batch_destroy(b);
    return LB_ENOMEM;
  }
  std::memset(b->h_acc, 0, (size_t)n * 4 * sizeof(double));
  // Default shape: widest strip the widest instance fills, 8-row segments, a persistent
  // grid of as many workgroups as are resident at once.
  int maxlx = 0;
  for (int i = 0; i < n; ++i) maxlx = std::max(maxlx, b->lat[i].lx);
  const int tx = maxlx >= 256 ? 256 : (maxlx >= 128 ? 128 : 64);
  b->grid = resident(b, tx);
  int rc = build_tiles(b, tx, 8);
  if (rc) {
    g_batch_init_error = b->err;
    lb_batch_destroy(b);
    return rc;
  }
  // Initial state: stage each instance's rho_init in its slice of pop_b, then lay out rest
  // equilibrium populations into pop_a.
  if ((e = launch_fill(b->d_acc, 0.0, 4 * n, b->stream)) != hipSuccess) {
    g_batch_init_error = std::string("init: ") + hipGetErrorString(e);
    lb_batch_destroy(b);
    return LB_EDEVICE;
  }
  for (int i = 0; i < n; ++i) {
    char *pa = static_cast<char *>(pop_a) + b->off[i];
    char *pb = static_cast<char *>(pop_b) + b->off[i];
    const size_t rbytes = (size_t)b->ns * b->lat[i].lx * b->lat[i].ly * sizeof(double);
    LayoutArgs la = layout_args(b, i);
    la.in = pb;
    la.out = pa;
    if ((e = hipMemcpyAsync(pb, rho_init[i], rbytes, hipMemcpyHostToDevice, b->stream)) != hipSuccess ||
        (e = launch_init(b->storage, b->walls, la, b->stream)) != hipSuccess) {
      g_batch_init_error = std::string("init: ") + hipGetErrorString(e);
      lb_batch_destroy(b);
      return LB_EDEVICE;
    }
  }
  if ((e = hipStreamSynchronize(b->stream)) != hipSuccess) {
    g_batch_init_error = std::string("init: ") + hipGetErrorString(e);
    lb_batch_destroy(b);
    return LB_EDEVICE;
  }
  *out = b;
  return LB_OK;
}

int lb_batch_step(lb_batch *b, int64_t n) {
  if (!b) return bfail(nullptr, LB_EINVAL, "null context");
  if (n < 0) return bfail(b, LB_EINVAL, "n must be >= 0");
  int rc = poll(b, false);
  if (rc) return rc;
  const int nt = (int)b->tiles.size();
  if (b->graph.steps > 0 && b->reduce_every == 0) {
    while (n >= b->graph.steps) {
      hipGraphExec_t g = nullptr;
      const int from = b->cur;
      const double *tb = b->rounding == LB_ROUND_STOCHASTIC ? b->d_tbase : nullptr;
      hipError_t e = b->graph.get(
          from,
          [&](int k, hipStream_t st) {
            return launch_tiles(b, WHAT_STEP, from ^ (k & 1), 0, nt, st, nullptr, nullptr, 0, (uint32_t)k, tb);
          },
          &g);
      // the replay's steps are t + k: the base goes to device memory (a fill kernel, outside the graph)
      if (e == hipSuccess && tb) e = launch_fill(b->d_tbase, (double)b->t, 1, b->stream);
      if (e == hipSuccess) e = hipGraphLaunch(g, b->stream);
      if (e != hipSuccess) return bhip(b, e, "step graph");
      b->t += b->graph.steps;
      n -= b->graph.steps;
    }
  }
  bool reduced = false;
  for (int64_t k = 0; k < n; ++k) {
    const bool red = b->reduce_every > 0 && (b->t % b->reduce_every) == 0;
    hipError_t e = launch_tiles(b, red ? WHAT_STEP_ACCUM : WHAT_STEP, b->cur, 0, nt, b->stream, nullptr, nullptr, 0,
                                (uint32_t)b->t);
    if (e != hipSuccess) return bhip(b, e, "batch step launch");
    reduced |= red;
    if (red) ++b->acc_pending;
    b->cur ^= 1;
    ++b->t;
  }
  if (reduced) {
    // one second pass per call: fold every tile's running sums into its instance
    int rc = flush_acc(b);
    if (rc) return rc;
    hipError_t e = hipMemcpyAsync(b->h_acc, b->d_acc, (size_t)b->n * 4 * sizeof(double), hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipEventRecord(b->ev, b->stream);
    if (e != hipSuccess) return bhip(b, e, "health readback");
    b->check_pending = true;
  }
  return LB_OK;
}

int lb_batch_set_reduce_every(lb_batch *b, int32_t k) {
  if (!b) return bfail(nullptr, LB_EINVAL, "null context");
  if (k < 0) return bfail(b, LB_EINVAL, "k must be >= 0");
  b->reduce_every = k;
  return LB_OK;
}

int lb_batch_set_rounding(lb_batch *b, int32_t mode) {
  if (!b) return bfail(nullptr, LB_EINVAL, "null context");
  if (mode != LB_ROUND_NEAREST && mode != LB_ROUND_STOCHASTIC)
    return bfail(b, LB_EINVAL, "mode must be LB_ROUND_NEAREST or LB_ROUND_STOCHASTIC");
  if (mode == LB_ROUND_STOCHASTIC && b->storage != LB_BF16DEV)
    return bfail(b, LB_EINVAL, "stochastic rounding applies to BF16 storage only");
  if (mode == LB_ROUND_STOCHASTIC && !b->d_tbase) {
    hipError_t e = hipMalloc(&b->d_tbase, sizeof(double));
    if (e != hipSuccess) return bfail(b, LB_ENOMEM, std::string("step base: ") + hipGetErrorString(e));
  }
  b->rounding = mode;
  b->graph.clear();  // captured launches carry the old kernel variant
  return LB_OK;
}

int lb_batch_set_graph(lb_batch *b, int32_t steps) {
  if (!b) return bfail(nullptr, LB_EINVAL, "null context");
  if (steps < 0 || (steps & 1)) return bfail(b, LB_EINVAL, "graph steps must be even and >= 0");
  b->graph.clear();
  b->graph.steps = steps;
  return LB_OK;
}

int lb_batch_set_tile(lb_batch *b, int32_t tx, int32_t sy, int32_t grid) {
  if (!b) return bfail(nullptr, LB_EINVAL, "null context");
  if (tx != 64 && tx != 128 && tx != 256) return bfail(b, LB_EINVAL, "tx must be 64, 128 or 256");
  if (sy < 1) return bfail(b, LB_EINVAL, "sy must be >= 1");
  if (grid < 0 || grid > kMaxBlocks) return bfail(b, LB_EINVAL, "grid must be in [0, 2^20]");
  b->grid = grid;
  return build_tiles(b, tx, sy);
}

int lb_batch_get_tile(const lb_batch *b, int32_t *tx, int32_t *sy, int32_t *grid) {
  if (!b || !tx || !sy || !grid) return LB_EINVAL;
  *tx = b->tx;
  *sy = b->sy;
  *grid = b->grid;
  return LB_OK;
}

int lb_batch_autotune(lb_batch *b, int32_t trial_steps, int32_t out[3], double *ms_out) {
  if (!b) return bfail(nullptr, LB_EINVAL, "null context");
  if (trial_steps < 1) return bfail(b, LB_EINVAL, "trial_steps must be >= 1");
  int rc = poll(b, true);
  if (rc) return rc;
  // As for one lattice: trial launches read the current state and write the other buffer.
  const int tx0 = b->tx, sy0 = b->sy, g0 = b->grid;
  int btx = tx0, bsy = sy0, bg = g0;
  double best = -1.0;
  int maxlx = 0, maxly = 0;
  for (int i = 0; i < b->n; ++i) {
    maxlx = std::max(maxlx, b->lat[i].lx);
    maxly = std::max(maxly, b->lat[i].ly);
  }
  const int txs[3] = {64, 128, 256};
  const int sys[] = {2, 4, 6, 8, 12, 16, 24, 32};
  for (int tx : txs) {
    if (tx > 64 && tx / 2 >= maxlx) continue;
    for (int sy : sys) {
      if (sy > maxly) continue;
      for (int persistent = 0; persistent < 2 && !rc; ++persistent) {
        b->grid = persistent ? resident(b, tx) : 0;
        if ((rc = build_tiles(b, tx, sy))) break;
        const int nt = (int)b->tiles.size();
        const double ms =
            time_launches(b->stream, 2, trial_steps, [&]() { return launch_tiles(b, WHAT_STEP, b->cur, 0, nt, b->stream); });
        if (ms < 0.0) {
          rc = bhip(b, hipGetLastError(), "autotune trial");
          break;
        }
        if (best < 0.0 || ms < best) {
          best = ms;
          btx = tx;
          bsy = sy;
          bg = b->grid;
        }
      }
      if (rc) break;
    }
    if (rc) break;
  }
  b->grid = rc ? g0 : bg;
  const int rc2 = build_tiles(b, rc ? tx0 : btx, rc ? sy0 : bsy);
  if (rc) return rc;
  if (rc2) return rc2;
  if (out) {
    out[0] = b->tx;
    out[1] = b->sy;
    out[2] = b->grid;
  }
  if (ms_out) *ms_out = best;
  return LB_OK;
}

int lb_batch_moments(lb_batch *b, int32_t i, void *rho, void *u, int32_t dtype) {
  if (!b) return bfail(nullptr, LB_EINVAL, "null context");
  int rc = check_index(b, i);
  if (rc) return rc;
  if (dtype != LB_OUT_F64 && dtype != LB_OUT_F32) return bfail(b, LB_EINVAL, "dtype must be LB_OUT_F64 or LB_OUT_F32");
  if (!rho && !u) return LB_OK;
  hipError_t e = launch_tiles(b, WHAT_MOMENTS, b->cur, b->tile0[i], b->ntile[i], b->stream, rho, u, dtype == LB_OUT_F32);
  if (e != hipSuccess) return bhip(b, e, "moments launch");
  return LB_OK;
}

int lb_batch_stress_field(lb_batch *b, int32_t i, void *sigma, int32_t dtype) {
  if (!b) return bfail(nullptr, LB_EINVAL, "null context");
  int rc = check_index(b, i);
  if (rc) return rc;
  if (!sigma) return bfail(b, LB_EINVAL, "null output");
  if (dtype != LB_OUT_F64 && dtype != LB_OUT_F32) return bfail(b, LB_EINVAL, "dtype must be LB_OUT_F64 or LB_OUT_F32");
  hipError_t e = launch_tiles(b, WHAT_STRESS, b->cur, b->tile0[i], b->ntile[i], b->stream, sigma, nullptr,
                              dtype == LB_OUT_F32);
  if (e != hipSuccess) return bhip(b, e, "stress launch");
  return LB_OK;
}

int lb_batch_profile(lb_batch *b, int32_t i, double *out) {
  if (!b) return bfail(nullptr, LB_EINVAL, "null context");
  int rc = check_index(b, i);
  if (rc) return rc;
  if (!out) return bfail(b, LB_EINVAL, "null output");
  const lb_lattice &L = b->lat[i];
  const int ncb = ((L.lx + b->tx - 1) / b->tx) * (b->tx / 64);
  const size_t need = ((size_t)ncb + 1) * L.ly * PROF_N;
  if (need > b->prof_cap) {
    (void)hipStreamSynchronize(b->stream);
    if (b->d_prof) (void)hipFree(b->d_prof);
    b->d_prof = nullptr;
    b->prof_cap = 0;
    hipError_t e = hipMalloc(&b->d_prof, need * sizeof(double));
    if (e != hipSuccess) return bfail(b, LB_ENOMEM, std::string("profile buffer: ") + hipGetErrorString(e));
    b->prof_cap = need;
  }
  hipError_t e = launch_tiles(b, WHAT_PROFILE, b->cur, b->tile0[i], b->ntile[i], b->stream, b->d_prof);
  double wb0 = 0.0, wt0 = 0.0;
  if (b->walls)
    for (int s = 0; s < b->ns; ++s) {
      wb0 += 2.0 * b->args[i].wall_mom[0][s];
      wt0 += 2.0 * b->args[i].wall_mom[1][s];
    }
  if (e == hipSuccess)
    e = launch_profile_finish(b->d_prof, ncb, L.lx, L.ly, b->walls, wb0, wt0, b->d_prof + (size_t)ncb * L.ly * PROF_N,
                              out, b->stream);
  if (e != hipSuccess) return bhip(b, e, "profile launch");
  return LB_OK;
}

int lb_batch_totals(lb_batch *b, double *out) {
  if (!b) return bfail(nullptr, LB_EINVAL, "null context");
  if (!out) return bfail(b, LB_EINVAL, "null output");
  const int nt = (int)b->tiles.size();
  hipError_t e = launch_tiles(b, WHAT_OBSERVE, b->cur, 0, nt, b->stream);
  if (e == hipSuccess) e = launch_batch_reduce(b->d_partials, b->d_jobs, b->n, b->d_totals, b->d_acc, 0, b->stream);
  std::vector<double> h((size_t)b->n * RED_N);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h.data(), b->d_totals, h.size() * sizeof(double), hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return bhip(b, e, "totals");
  bool bad = false;
  for (int i = 0; i < b->n; ++i) {
    const double *t = &h[(size_t)i * RED_N];
    out[5 * i + 0] = t[RED_MASS0];
    out[5 * i + 1] = t[RED_MASS1];
    out[5 * i + 2] = t[RED_PX];
    out[5 * i + 3] = t[RED_PY];
    out[5 * i + 4] = t[RED_FLOW];
    bad |= t[RED_BAD] > 0.0;
  }
  int rc = poll(b, true);
  if (rc) return rc;
  if (bad) {
    b->unstable = true;
    return bfail(b, LB_EUNSTABLE, "non-finite or non-positive density in the current state of an instance");
  }
  return LB_OK;
}

int lb_batch_wall_stress(lb_batch *b, double *out, int32_t reset) {
  if (!b) return bfail(nullptr, LB_EINVAL, "null context");
  if (!out) return bfail(b, LB_EINVAL, "null output");
  if (!b->walls) return bfail(b, LB_ESTATE, "wall stress needs channel lattices");
  int rc = flush_acc(b);
  if (rc) return rc;
  std::vector<double> h((size_t)b->n * 4);
  hipError_t e = hipMemcpyAsync(h.data(), b->d_acc, h.size() * sizeof(double), hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return bhip(b, e, "wall stress readback");
  for (int i = 0; i < b->n; ++i) {
    const double *a = &h[4 * i];
    if (a[3] > 0.0) b->unstable = true;
    out[2 * i + 0] = a[2] > 0 ? a[0] / a[2] : 0.0;
    out[2 * i + 1] = a[2] > 0 ? a[1] / a[2] : 0.0;
  }
  if (reset) {
    for (int i = 0; i < b->n; ++i) h[4 * i] = h[4 * i + 1] = h[4 * i + 2] = 0.0;  // keep the health count
    e = hipMemcpyAsync(b->d_acc, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bhip(b, e, "wall stress reset");
  }
  if (b->unstable) return bfail(b, LB_EUNSTABLE, "non-finite or non-positive density in an instance");
  return LB_OK;
}

int lb_batch_checkpoint(lb_batch *b, int32_t i, void *dst) {
  if (!b) return bfail(nullptr, LB_EINVAL, "null context");
  int rc = check_index(b, i);
  if (rc) return rc;
  if (!dst) return bfail(b, LB_EINVAL, "null destination");
  LayoutArgs la = layout_args(b, i);
  la.in = static_cast<const char *>(b->pop[b->cur]) + b->off[i];
  la.out = dst;
  hipError_t e = launch_checkpoint(b->storage, b->walls, la, b->stream);
  if (e != hipSuccess) return bhip(b, e, "checkpoint kernel");
  return LB_OK;
}

int lb_batch_restore(lb_batch *b, int32_t i, const void *src) {
  if (!b) return bfail(nullptr, LB_EINVAL, "null context");
  int rc = check_index(b, i);
  if (rc) return rc;
  if (!src) return bfail(b, LB_EINVAL, "null source");
  if (b->check_pending) {
    (void)hipEventSynchronize(b->ev);
    b->check_pending = false;
  }
  LayoutArgs la = layout_args(b, i);
  la.in = src;
  la.out = static_cast<char *>(b->pop[b->cur]) + b->off[i];
  hipError_t e = launch_restore(b->storage, b->walls, la, b->stream);
  if (e == hipSuccess) e = launch_fill(b->d_acc + 4 * (size_t)i, 0.0, 4, b->stream);
  if (e != hipSuccess) return bhip(b, e, "restore kernel");
  // the latch clears once no instance reports a bad site any more
  std::vector<double> h((size_t)b->n * 4);
  e = hipMemcpyAsync(h.data(), b->d_acc, h.size() * sizeof(double), hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return bhip(b, e, "restore");
  bool bad = false;
  for (int k = 0; k < b->n; ++k) bad |= h[4 * k + 3] > 0.0;
  b->unstable = bad;
  return LB_OK;
}

int64_t lb_batch_time(const lb_batch *b) { return b ? b->t : -1; }

int lb_batch_set_time(lb_batch *b, int64_t t) {
  if (!b) return bfail(nullptr, LB_EINVAL, "null context");
  if (t < 0) return bfail(b, LB_EINVAL, "time must be >= 0");
  b->t = t;
  return LB_OK;
}

const char *lb_batch_last_error(const lb_batch *b) { return b ? b->err.c_str() : g_batch_init_error.c_str(); }

void lb_batch_destroy(lb_batch *b) {
  if (!b) return;
  if (b->check_pending && b->ev) (void)hipEventSynchronize(b->ev);
  (void)hipStreamSynchronize(b->stream);
  for (void *p : {(void *)b->d_args, (void *)b->d_tiles, (void *)b->d_jobs, (void *)b->d_partials, (void *)b->d_accrows,
                  (void *)b->d_prof,
                  (void *)b->d_totals, (void *)b->d_acc})
    if (p) (void)hipFree(p);
  if (b->h_acc) (void)hipHostFree(b->h_acc);
  if (b->ev) (void)hipEventDestroy(b->ev);
  b->graph.destroy();
  if (b->d_tbase) (void)hipFree(b->d_tbase);
  delete b;
}

}  // extern "C"
