// Kernels around the fused step: the second reduction passes, the layout kernels (canonical
// FP64 populations <-> the stored form), fills, the streaming copy, the profile passes, and
// the dispatch of the step launchers to the translation unit of each storage mode.
// The fused step itself is in lb_step.hpp.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "lb_internal.hpp"
#include "lb_step.hpp"
#include "lb_tables.hpp"

namespace lb355 {

// Second reduction pass: fixed-order sum of the per-workgroup partials (deterministic).
__device__ __forceinline__ void reduce_block(const double *partials, int nblocks, double *totals, double *acc,
                                             int accumulate, double inv_lx) {
  __shared__ double sm[256][RED_N];
  const int tid = threadIdx.x;
  double v[RED_N];
#pragma unroll
  for (int k = 0; k < RED_N; ++k) v[k] = 0.0;
  for (int b = tid; b < nblocks; b += 256)
#pragma unroll
    for (int k = 0; k < RED_N; ++k) v[k] += partials[(size_t)b * RED_N + k];
#pragma unroll
  for (int k = 0; k < RED_N; ++k) sm[tid][k] = v[k];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h)
#pragma unroll
      for (int k = 0; k < RED_N; ++k) sm[tid][k] += sm[tid + h][k];
    __syncthreads();
  }
  if (tid == 0) {
    double t[RED_N];
#pragma unroll
    for (int k = 0; k < RED_N; ++k) t[k] = sm[0][k];
    t[RED_WBOT] *= inv_lx;
    t[RED_WTOP] *= inv_lx;
    t[RED_FLOW] *= inv_lx;
#pragma unroll
    for (int k = 0; k < RED_N; ++k) totals[k] = t[k];
    if (accumulate) {
      acc[0] += t[RED_WBOT];
      acc[1] += t[RED_WTOP];
      acc[2] += 1.0;
      acc[3] += t[RED_BAD];
    }
  }
}

__global__ __launch_bounds__(256) void reduce_kernel(const double *partials, int nblocks, double *totals, double *acc,
                                                     int accumulate, double inv_lx) {
  reduce_block(partials, nblocks, totals, acc, accumulate, inv_lx);
}

// Second pass of the stepping sums: rows [nrows][ACC_N] of running sums (one per workgroup of
// the reducing launches since the last flush) are summed in fixed order into acc (wall stress
// sums per unit length, reduced-step count, bad-site count) and cleared.  One workgroup.
__device__ __forceinline__ void flush_block(double *rows, int nrows, double *acc, double count, double inv_lx) {
  __shared__ double sm[256][ACC_N];
  const int tid = threadIdx.x;
  double v[ACC_N] = {0.0, 0.0, 0.0};
  for (int b = tid; b < nrows; b += 256) {
#pragma unroll
    for (int k = 0; k < ACC_N; ++k) {
      v[k] += rows[(size_t)b * ACC_N + k];
      rows[(size_t)b * ACC_N + k] = 0.0;
    }
  }
#pragma unroll
  for (int k = 0; k < ACC_N; ++k) sm[tid][k] = v[k];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h)
#pragma unroll
      for (int k = 0; k < ACC_N; ++k) sm[tid][k] += sm[tid + h][k];
    __syncthreads();
  }
  if (tid == 0) {
    acc[0] += sm[0][0] * inv_lx;
    acc[1] += sm[0][1] * inv_lx;
    acc[2] += count;
    acc[3] += sm[0][2];
  }
}

__global__ __launch_bounds__(256) void flush_kernel(double *rows, int nrows, double *acc, double count,
                                                    double inv_lx) {
  flush_block(rows, nrows, acc, count, inv_lx);
}

// The same for a batch, one workgroup per instance (its tiles' rows are a contiguous range).
__global__ __launch_bounds__(256) void batch_flush_kernel(double *rows, const ReduceJob *jobs, double *acc,
                                                          double count) {
  const ReduceJob j = jobs[blockIdx.x];
  flush_block(rows + (size_t)j.p0 * ACC_N, j.n, acc + (size_t)blockIdx.x * 4, count, j.inv_lx);
}

// One workgroup per instance of a batch: its tiles' partials are a contiguous range.
__global__ __launch_bounds__(256) void batch_reduce_kernel(const double *partials, const ReduceJob *jobs,
                                                           double *totals, double *acc, int accumulate) {
  const ReduceJob j = jobs[blockIdx.x];
  reduce_block(partials + (size_t)j.p0 * RED_N, j.n, totals + (size_t)blockIdx.x * RED_N,
               acc + (size_t)blockIdx.x * 4, accumulate, j.inv_lx);
}

// ---------------------------------------------------------------------------------------
// Layout kernels: canonical pre-collision f(t) <-> internal post-collision buffer.
// Streaming with bounce-back is a permutation of population slots:
//   f_l(x) = g_l(x - c_l) if x - c_l is fluid, else g_opp(l)(x)
// and its inverse g_l(z) = f_l(z + c_l) if z + c_l is fluid, else f_opp(l)(z).
// ---------------------------------------------------------------------------------------

// Element index of population l of species s at (x, y): layout [y][l][pitch][species].
__device__ inline long long pop_index(int s, int l, int y, int x, int pitch, int ns) {
  return (((long long)y * 9 + l) * pitch + x) * ns + s;
}

template <int MODE, bool WALLS>
__global__ void init_kernel(LayoutArgs a) {  // in: rho [ns][ly][lx] (FP64)
  using C = Codec<MODE>;
  using S = typename C::S;
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= a.lx) return;
  const double *__restrict__ rho = static_cast<const double *>(a.in);
  S *__restrict__ out = static_cast<S *>(a.out);
  const size_t nsite = (size_t)a.lx * a.ly;
  for (int s = 0; s < a.ns; ++s) {
    // the nine loads first, so that they are in flight together
    double rn[9];
#pragma unroll
    for (int l = 0; l < 9; ++l) {
      int zx = x + CXS[l], zy = y + CYS[l];
      if (WALLS && (zy < 0 || zy >= a.ly)) {
        zx = x;
        zy = y;
      } else {
        zx = wrapi(zx, a.lx);
        zy = wrapi(zy, a.ly);
      }
      rn[l] = rho[s * nsite + (size_t)zy * a.lx + zx];
    }
#pragma unroll
    for (int l = 0; l < 9; ++l)
      C::store(out + pop_index(s, l, y, x, a.pitch, a.ns), WD2Q9[l] * rn[l], WD2Q9[l] * a.rho_ref[s]);
  }
}

template <int MODE, bool WALLS>
__global__ void restore_kernel(LayoutArgs a) {  // in: canonical f [ns][9][ly][lx] (FP64)
  using C = Codec<MODE>;
  using S = typename C::S;
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= a.lx) return;
  const double *__restrict__ f = static_cast<const double *>(a.in);
  S *__restrict__ out = static_cast<S *>(a.out);
  const size_t nsite = (size_t)a.lx * a.ly;
  for (int s = 0; s < a.ns; ++s) {
    // the nine loads first, so that they are in flight together
    double v[9];
#pragma unroll
    for (int l = 0; l < 9; ++l) {
      int zx = x + CXS[l], zy = y + CYS[l], lsrc = l;
      if (WALLS && (zy < 0 || zy >= a.ly)) {
        zx = x;
        zy = y;
        lsrc = OPPS[l];
      } else {
        zx = wrapi(zx, a.lx);
        zy = wrapi(zy, a.ly);
      }
      v[l] = f[(size_t)(s * 9 + lsrc) * nsite + (size_t)zy * a.lx + zx];
    }
#pragma unroll
    for (int l = 0; l < 9; ++l) C::store(out + pop_index(s, l, y, x, a.pitch, a.ns), v[l], WD2Q9[l] * a.rho_ref[s]);
  }
}

template <int MODE, bool WALLS>
__global__ void checkpoint_kernel(LayoutArgs a) {  // out: canonical f [ns][9][ly][lx] (FP64)
  using C = Codec<MODE>;
  using S = typename C::S;
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= a.lx) return;
  const S *__restrict__ in = static_cast<const S *>(a.in);
  double *__restrict__ f = static_cast<double *>(a.out);
  const size_t nsite = (size_t)a.lx * a.ly;
  for (int s = 0; s < a.ns; ++s) {
    // the nine pulls first, so that their loads are in flight together
    double v[9];
#pragma unroll
    for (int l = 0; l < 9; ++l) {
      int zx = x - CXS[l], zy = y - CYS[l], lsrc = l;
      if (WALLS && (zy < 0 || zy >= a.ly)) {
        zx = x;
        zy = y;
        lsrc = OPPS[l];
      } else {
        zx = wrapi(zx, a.lx);
        zy = wrapi(zy, a.ly);
      }
      v[l] = C::load(in + pop_index(s, lsrc, zy, zx, a.pitch, a.ns), WD2Q9[lsrc] * a.rho_ref[s]);
    }
#pragma unroll
    for (int l = 0; l < 9; ++l) f[(size_t)(s * 9 + l) * nsite + (size_t)y * a.lx + x] = v[l];
  }
}

// What the adjoint's reverse step reads of a state: the canonical populations of the rows next
// to the walls (bottom row, then top row; the wall stress needs them), and the moments and
// pseudopotential of every site
// (rho_s = sum_l f_l, psi_s = psi0 (1 - exp(-rho_s / rho0)), j_s = sum_l c_l f_l), summed in
// l order in the adjoint's precision RA.
template <int MODE, bool WALLS, typename RA>
__global__ void checkpoint_fields_kernel(LayoutArgs a) {
  using C = Codec<MODE>;
  using S = typename C::S;
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= a.lx) return;
  const S *__restrict__ in = static_cast<const S *>(a.in);
  double *__restrict__ f = static_cast<double *>(a.out);
  RA *__restrict__ fl = static_cast<RA *>(a.fields);
  const size_t nsite = (size_t)a.lx * a.ly;
  const size_t i = (size_t)y * a.lx + x;
  // the reverse step reads the populations themselves only on the rows next to a wall (for
  // the wall stress); elsewhere the fields suffice
  const bool wall_row = WALLS && (y == 0 || y == a.ly - 1);
  for (int s = 0; s < a.ns; ++s) {
    // the nine pulls first, so that their loads are in flight together
    double fp[9];
#pragma unroll
    for (int l = 0; l < 9; ++l) {
      int zx = x - CXS[l], zy = y - CYS[l], lsrc = l;
      if (WALLS && (zy < 0 || zy >= a.ly)) {
        zx = x;
        zy = y;
        lsrc = OPPS[l];
      } else {
        zx = wrapi(zx, a.lx);
        zy = wrapi(zy, a.ly);
      }
      fp[l] = C::load(in + pop_index(s, lsrc, zy, zx, a.pitch, a.ns), WD2Q9[lsrc] * a.rho_ref[s]);
    }
    RA r = 0, jx = 0, jy = 0;
#pragma unroll
    for (int l = 0; l < 9; ++l) {
      const double fv = fp[l];
      if (wall_row) f[((size_t)(s * 9 + l) * 2 + (y == 0 ? 0 : 1)) * a.lx + x] = fv;
      const RA g = RA(fv);
      r += g;
      jx += RA(CXS[l]) * g;
      jy += RA(CYS[l]) * g;
    }
    fl[(size_t)(0 * 2 + s) * nsite + i] = r;
    fl[(size_t)(1 * 2 + s) * nsite + i] = RA(a.psi0) * (RA(1) - exp(-r * RA(a.irho0)));
    fl[(size_t)(2 * 2 + s) * nsite + i] = jx;
    fl[(size_t)(3 * 2 + s) * nsite + i] = jy;
  }
}

// ---------------------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------------------

size_t step_lds_bytes(int mode, int ns, int tx) {
  const size_t r = mode == MODE_F64 ? 8 : 4;
  return 6 * (size_t)(tx + 4) * ns * r * (ns == 2 ? 2 : 1) + 7 * 36 * (size_t)ns * r;  // rings + halo staging
}

hipError_t launch_batch_step(int mode, int ns, int walls, int what, int tx, int grid, const BatchArgs &b,
                             hipStream_t st) {
  switch (mode) {
    case MODE_F64: return launch_batch_f64(ns, walls, what, tx, grid, b, st);
    case MODE_F32: return launch_batch_f32(ns, walls, what, tx, grid, b, st);
    case MODE_BF16: return launch_batch_bf16(false, ns, walls, what, tx, grid, b, st);
    case MODE_BF16SR: return launch_batch_bf16(true, ns, walls, what, tx, grid, b, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_batch_reduce(const double *partials, const ReduceJob *jobs, int njobs, double *totals, double *acc,
                               int accumulate, hipStream_t st) {
  if (njobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(batch_reduce_kernel, dim3(njobs), dim3(256), 0, st, partials, jobs, totals, acc, accumulate);
  return hipGetLastError();
}


hipError_t launch_step2(int mode, int ns, int walls, int nb, const StepArgs &a, hipStream_t st) {
  switch (mode) {
    case MODE_F64: return launch_step2_f64(ns, walls, nb, a, st);
    case MODE_F32: return launch_step2_f32(ns, walls, nb, a, st);
    case MODE_BF16: return launch_step2_bf16(false, ns, walls, nb, a, st);
    case MODE_BF16SR: return launch_step2_bf16(true, ns, walls, nb, a, st);
  }
  return hipErrorInvalidValue;
}

int step_blocks_per_cu(int mode, int ns, int walls, int tx) {
  switch (mode) {
    case MODE_F64: return blocks_per_cu_f64(ns, walls, tx);
    case MODE_F32: return blocks_per_cu_f32(ns, walls, tx);
    case MODE_BF16: return blocks_per_cu_bf16(ns, walls, tx);
  }
  return 1;
}

hipError_t launch_step(int mode, int ns, int walls, int what, int tx, int nb, const StepArgs &a, hipStream_t st) {
  switch (mode) {
    case MODE_F64: return launch_step_f64(ns, walls, what, tx, nb, a, st);
    case MODE_F32: return launch_step_f32(ns, walls, what, tx, nb, a, st);
    case MODE_BF16: return launch_step_bf16(false, ns, walls, what, tx, nb, a, st);
    case MODE_BF16SR: return launch_step_bf16(true, ns, walls, what, tx, nb, a, st);
  }
  return hipErrorInvalidValue;
}

__global__ void fill_kernel(double *p, double v, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Profile second pass, part 1: the per-row sums rows[y][slot] = sum over the 64-column
// blocks b of prof[b][y][slot], in increasing b (one thread per row and slot).
__global__ void profile_rows_kernel(const double *prof, int ncb, int ly, double *rows) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ly * PROF_N) return;
  const size_t stride = (size_t)ly * PROF_N;
  double v = 0.0;
  for (int b = 0; b < ncb; ++b) v += prof[b * stride + i];
  rows[i] = v;
}

// Part 2, one thread per row y (ubar) and per line k (sigma).  Line k lies between rows
// k-1 and k; its stress is
//   sigma(k) = (I1(k-1) + I2(k-2) - Kup(k-1) + Kdn(k)) / lx
// (pair forces across the line on the rows below it, minus the x-momentum streaming up
// across it), with rows wrapping on periodic lattices.  On channels, sigma(0) and sigma(ly)
// are the walls' momentum exchange: 2 Kdn(0) / lx - wb0 and -(2 Kup(ly-1) / lx - wt0).
__global__ void profile_finish_kernel(const double *rows, int lx, int ly, int walls, double wb0, double wt0,
                                      double *out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k > ly) return;
  auto row = [&](int y, int slot) { return rows[(size_t)y * PROF_N + slot]; };
  const double ilx = 1.0 / lx;
  if (k < ly) {
    out[k] = row(k, PROF_U) * ilx;
    out[2 * ly + 1 + k] = row(k, PROF_RA) * ilx;
    out[3 * ly + 1 + k] = row(k, PROF_RB) * ilx;
  }
  double sig;
  if (walls && k == 0) {
    sig = 2.0 * row(0, PROF_KDN) * ilx - wb0;
  } else if (walls && k == ly) {
    sig = -(2.0 * row(ly - 1, PROF_KUP) * ilx - wt0);
  } else {
    const int kk = k == ly ? 0 : k;  // periodic: line ly is line 0
    const int ym1 = kk - 1 < 0 ? kk - 1 + ly : kk - 1;
    const int ym2 = kk - 2 < 0 ? kk - 2 + ly : kk - 2;
    double i = row(ym1, PROF_I1);
    if (!walls || kk >= 2) i += row(ym2, PROF_I2);  // on channels a partner two rows down is a wall
    sig = (i - row(ym1, PROF_KUP) + row(kk, PROF_KDN)) * ilx;
  }
  out[ly + k] = sig;
}

// Time statistics of n profile samples [n][2 ly + 1], one thread per row / line; the
// covariances are taken about the means (two passes over the samples).
__global__ void profile_stats_kernel(const double *smp, long long n, int ly, int walls, int k0, double u_bot,
                                     double u_top, double *out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k > ly) return;
  const size_t len = 4 * (size_t)ly + 1;
  const double in = 1.0 / (double)n;
  double su = 0.0, ss = 0.0, sf = 0.0, s0 = 0.0, sa = 0.0, sb = 0.0;
  for (long long t = 0; t < n; ++t) {
    const double *p = smp + (size_t)t * len;
    const double sig = p[ly + k];
    if (k < ly) {
      su += p[k];
      sa += p[2 * ly + 1 + k];
      sb += p[3 * ly + 1 + k];
    }
    ss += sig;
    s0 += p[ly + k0];
    double du;
    if (walls && k == 0) du = 2.0 * (p[0] - u_bot);
    else if (walls && k == ly) du = 2.0 * (u_top - p[ly - 1]);
    else {
      const int kk = k == ly ? 0 : k;
      du = p[kk] - p[kk == 0 ? ly - 1 : kk - 1];
    }
    sf += du / sig;
  }
  const double mk = ss * in, m0 = s0 * in;
  double c00 = 0.0, ck0 = 0.0;
  for (long long t = 0; t < n; ++t) {
    const double *p = smp + (size_t)t * len;
    const double d0 = p[ly + k0] - m0;
    c00 += d0 * d0;
    ck0 += (p[ly + k] - mk) * d0;
  }
  if (k < ly) {
    out[k] = su * in;
    out[4 * ly + 3 + k] = sa * in;
    out[5 * ly + 3 + k] = sb * in;
  }
  out[ly + k] = mk;
  out[2 * ly + 1 + k] = sf * in;
  out[3 * ly + 2 + k] = c00 > 0.0 ? ck0 / c00 : NAN;
}

hipError_t launch_profile_finish(const double *prof, int ncb, int lx, int ly, int walls, double wb0, double wt0,
                                 double *rows, double *out, hipStream_t st) {
  hipLaunchKernelGGL(profile_rows_kernel, dim3((ly * PROF_N + 255) / 256), dim3(256), 0, st, prof, ncb, ly, rows);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(profile_finish_kernel, dim3((ly + 1 + 255) / 256), dim3(256), 0, st, rows, lx, ly, walls, wb0,
                     wt0, out);
  return hipGetLastError();
}

hipError_t launch_profile_stats(const double *samples, long long n, int ly, int walls, int k0, double u_bot,
                                double u_top, double *out, hipStream_t st) {
  hipLaunchKernelGGL(profile_stats_kernel, dim3((ly + 1 + 255) / 256), dim3(256), 0, st, samples, n, ly, walls, k0,
                     u_bot, u_top, out);
  return hipGetLastError();
}

hipError_t launch_flush(double *rows, int nrows, double *acc, double count, double inv_lx, hipStream_t st) {
  hipLaunchKernelGGL(flush_kernel, dim3(1), dim3(256), 0, st, rows, nrows, acc, count, inv_lx);
  return hipGetLastError();
}

hipError_t launch_batch_flush(double *rows, const ReduceJob *jobs, int njobs, double *acc, double count,
                              hipStream_t st) {
  if (njobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(batch_flush_kernel, dim3(njobs), dim3(256), 0, st, rows, jobs, acc, count);
  return hipGetLastError();
}

// Streaming copy (the benchmark's bandwidth reference): 16-byte accesses in a grid-stride
// loop over n16 elements, non-temporal when NT.
using u32x4v = unsigned int __attribute__((ext_vector_type(4)));
template <int NT>
__global__ void stream_copy_kernel(const u32x4v *__restrict__ src, u32x4v *__restrict__ dst, size_t n16) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) {
    if (NT) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
    else dst[i] = src[i];
  }
}

hipError_t launch_stream_copy(void *dst, const void *src, size_t n16, int nontemporal, int blocks, hipStream_t st) {
  if (n16 == 0) return hipSuccess;
  const auto *s = static_cast<const u32x4v *>(src);
  auto *d = static_cast<u32x4v *>(dst);
  if (nontemporal) hipLaunchKernelGGL(stream_copy_kernel<1>, dim3(blocks), dim3(256), 0, st, s, d, n16);
  else hipLaunchKernelGGL(stream_copy_kernel<0>, dim3(blocks), dim3(256), 0, st, s, d, n16);
  return hipGetLastError();
}

hipError_t launch_fill(double *p, double v, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}

hipError_t launch_reduce(const double *partials, int nblocks, double *totals, double *acc, int accumulate,
                         double inv_lx, hipStream_t st) {
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(256), 0, st, partials, nblocks, totals, acc, accumulate, inv_lx);
  return hipGetLastError();
}

#define LB_LAYOUT_LAUNCHER(NAME, KERNEL)                                                            \
  template <int MODE>                                                                              \
  static hipError_t NAME##_m(int walls, const LayoutArgs &a, hipStream_t st) {                     \
    const dim3 grid((a.lx + 127) / 128, a.ly), block(128);                                         \
    if (walls) hipLaunchKernelGGL((KERNEL<MODE, true>), grid, block, 0, st, a);                    \
    else hipLaunchKernelGGL((KERNEL<MODE, false>), grid, block, 0, st, a);                         \
    return hipGetLastError();                                                                      \
  }                                                                                                \
  hipError_t NAME(int mode, int walls, const LayoutArgs &a, hipStream_t st) {                      \
    switch (mode) {                                                                                \
      case MODE_F64: return NAME##_m<MODE_F64>(walls, a, st);                                      \
      case MODE_F32: return NAME##_m<MODE_F32>(walls, a, st);                                      \
      case MODE_BF16: return NAME##_m<MODE_BF16>(walls, a, st);                                    \
    }                                                                                              \
    return hipErrorInvalidValue;                                                                   \
  }

LB_LAYOUT_LAUNCHER(launch_init, init_kernel)
LB_LAYOUT_LAUNCHER(launch_restore, restore_kernel)
LB_LAYOUT_LAUNCHER(launch_checkpoint, checkpoint_kernel)

template <int MODE, typename RA>
static hipError_t launch_checkpoint_fields_m(int walls, const LayoutArgs &a, hipStream_t st) {
  const dim3 grid((a.lx + 127) / 128, a.ly), block(128);
  if (walls) hipLaunchKernelGGL((checkpoint_fields_kernel<MODE, true, RA>), grid, block, 0, st, a);
  else hipLaunchKernelGGL((checkpoint_fields_kernel<MODE, false, RA>), grid, block, 0, st, a);
  return hipGetLastError();
}

hipError_t launch_checkpoint_fields(int mode, int walls, int fp64, const LayoutArgs &a, hipStream_t st) {
  switch (mode) {
    case MODE_F64:
      return fp64 ? launch_checkpoint_fields_m<MODE_F64, double>(walls, a, st)
                  : launch_checkpoint_fields_m<MODE_F64, float>(walls, a, st);
    case MODE_F32:
      return fp64 ? launch_checkpoint_fields_m<MODE_F32, double>(walls, a, st)
                  : launch_checkpoint_fields_m<MODE_F32, float>(walls, a, st);
    case MODE_BF16:
      return fp64 ? launch_checkpoint_fields_m<MODE_BF16, double>(walls, a, st)
                  : launch_checkpoint_fields_m<MODE_BF16, float>(walls, a, st);
  }
  return hipErrorInvalidValue;
}

#undef LB_LAYOUT_LAUNCHER

}  // namespace lb355
