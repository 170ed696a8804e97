// Hand-written adjoint (reverse-time) step of the two-belt pseudopotential lattice
// Boltzmann map, for gradients of the time-averaged wall stress and flow rate with respect
// to the couplings G_ss,1, G_ss,2, G_AB and the body force g.
//
// Forward map of one step (state x = pre-collision populations f(t), canonical layout):
//   rho_s = sum_l x_l,  j_s = sum_l c_l x_l,  psi_s = psi0 (1 - exp(-rho_s / rho0))
//   F_s   = -psi_s sum_h K_s(q) c (psi_s(x+c) - psi_s(x-c))              (eq. (FORCE))
//           -G_AB r_s sum_{h in belt 1} t(q) c (r_sbar(x+c) - r_sbar(x-c)) (r = rho or psi)
//           +rho_s g
//   u'    = sum_s omega_s j_s / sum_s omega_s rho_s,   u_s = u' + tau_s F_s / rho_s
//   y_l   = (1 - omega_s) x_l + omega_s f^eq_l(rho_s, u_s)                 (eq. (LB))
//   x'_l(x) = y_l(x - c_l), or y_opp(l)(x) when x - c_l is a wall row      (streaming)
// Loss of one step (weights cW = lw0 / T, cQ = lw1 / T):
//   cW (W_bot + W_top) / 2,  W_bot = (1/lx) sum_x sum_s sum_{c_ly = -1} 2 c_lx y_l(x, 0)
//   cQ Q,  Q = (1/lx) sum_x u_x,  u = (sum_s j_s + F_s / 2) / sum_s rho_s
//
// Reverse step, given lambda' = dL/dx(t+1):
//   a_l(x)   = lambda'_l(x + c_l), or lambda'_opp(l)(x) when x + c_l is a wall row (the
//              transpose of streaming), plus the wall-stress source on the wall rows;
//   then the chain rule through the collision, the velocity shift and u' per site gives
//   the local part of lambda(t), the force adjoint Fbar_s and the parameter sensitivities
//   Fbar_s . dF_s/dtheta; finally the force's dependence on the neighbours' psi (and rho)
//   is a gather with the same stencil:
//     psibar_s(y) += sum_h K_s(q) c . (A_s(y+c) - A_s(y-c)),   A_s = psi_s Fbar_s
//     rbar_sbar(y) += G_AB sum_{h in belt 1} t(q) c . (B_s(y+c) - B_s(y-c)),  B_s = r_s Fbar_s
//   and rhobar = psi'(rho) psibar enters every lambda_l(t).
// All three kernels work on canonical-layout arrays [..][y][x], one thread per site.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

#include "lb_internal.hpp"
#include "lb_tables.hpp"

namespace lb355 {

namespace {

__device__ inline int wrapx(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

template <typename R>
struct AdjView {
  const AdjArgs &a;
  int lx, ly;
  size_t n;  // sites
  __device__ AdjView(const AdjArgs &aa) : a(aa), lx(aa.lx), ly(aa.ly), n((size_t)aa.lx * aa.ly) {}
  __device__ R *fields() const { return static_cast<R *>(a.fields); }
  // field k (0 rho, 1 psi, 2 jx, 3 jy) of species s at site i
  __device__ R fld(int k, int s, size_t i) const { return fields()[((size_t)k * 2 + s) * n + i]; }
  __device__ R &fldw(int k, int s, size_t i) const { return fields()[((size_t)k * 2 + s) * n + i]; }
};

// Calls f(std::integral_constant<int, i>{}) for i = 0, 1, ..., N - 1 in order, so that the stencil
// constants indexed by i are compile-time values inside f.
template <typename F, int... I>
__device__ inline void each_index(F &f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ inline void each_index(F &&f) {
  each_index(f, std::make_integer_sequence<int, N>{});
}

// C v for a stencil constant C in {-2, ..., 2}, C != 0: +-1 are a copy or a negation.  Terms
// whose constant is zero are left out of the sums below altogether: they only add a signed
// zero, which leaves a sum unchanged.
template <int C, typename R>
__device__ inline R cmul(R v) {
  static_assert(C != 0, "zero terms are left out");
  if constexpr (C == 1) return v;
  else if constexpr (C == -1) return -v;
  else return R(C) * v;
}

// The equilibrium polynomial's derivative along one axis, 3 c + 9 (c_l . u) c - 3 u_a for
// c = c_l,a, grouped as ((3 c) + (9 (c_l . u)) c) - 3 u_a.
template <int C, typename R>
__device__ inline R eq_grad(R cu, R ua) {
  if constexpr (C == 0) return -(R(3) * ua);
  else return (R(3 * C) + cmul<C>(R(9) * cu)) - R(3) * ua;
}

// c . d for a half-link c = (CX, CY), zero components left out.
template <int CX, int CY, typename R>
__device__ inline R pair_dot(R dx, R dy) {
  if constexpr (CX != 0 && CY != 0) return cmul<CX>(dx) + cmul<CY>(dy);
  else if constexpr (CX != 0) return cmul<CX>(dx);
  else return cmul<CY>(dy);
}

template <typename T>
__device__ inline T block_sum(T v, T *sm) {
  // wave reduction, then across the waves of the block (sm: one slot per wave)
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sm[wv] = v;
  __syncthreads();
  T r = 0;
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) r += sm[k];
  return r;
}

}  // namespace

// The two reverse kernels work on 64 x 4 tiles of sites (one wave per tile row, 256 threads).
// Everything a site reads from its two-belt neighbourhood (psi and rho of the forward state
// for the force, psi_s Fbar_s and r_s Fbar_s for the gather) is first staged for the tile plus
// a halo of two sites into LDS, so each neighbour value is fetched from memory once per tile
// instead of once per reader.
constexpr int ATX = 64, ATY = 4, AHX = ATX + 4, AHY = ATY + 4;

// Site index of lattice point (x, y) for staging, any distance outside the lattice (x always
// periodic; y periodic unless walls, where rows outside are not sites).
template <bool WALLS>
__device__ inline bool stage_site(int x, int y, int lx, int ly, size_t &i) {
  if (WALLS && (y < 0 || y >= ly)) return false;
  const int xi = ((x % lx) + lx) % lx;
  const int yi = WALLS ? y : ((y % ly) + ly) % ly;
  i = (size_t)yi * lx + xi;
  return true;
}

// Per-tile sums of the nine sensitivities and loss terms: a wave reduction each, then the
// four waves in order (one barrier), added to this tile's own row of running sums.
__device__ inline void tile_accumulate(const double (&vals)[ADJ_N], double (*sm)[ADJ_N], double *row) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < ADJ_N; ++k) {
    double v = vals[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) sm[wv][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < ADJ_N) {
    const int k = threadIdx.x;
    row[k] += ((sm[0][k] + sm[1][k]) + sm[2][k]) + sm[3][k];
  }
}

// The term of lambda common to every l at one site: the force's dependence on the
// neighbours' psi (and rho), gathered with the forward stencil from A_s = psi_s Fbar_s and
// B_s = r_s Fbar_s.  ab(which, s, dx, dy, bx, by) gives A_s (which = 0) or B_s (which = 1) at
// the neighbour (dx, dy), zero off the lattice; rho holds the site's densities.
template <typename R, int NS, typename AB>
__device__ inline void gather_corr(const AdjArgs &a, const AB &ab, const R (&rho)[2], R (&corr)[2]) {
  R psib[2] = {0, 0}, rbar[2] = {0, 0};
  for (int s = 0; s < NS; ++s) {
    R Kq[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) Kq[q] = R(a.K[s][q]);
    R acc = 0;
    each_index<NHALF>([&](auto H) {
      constexpr int h = decltype(H)::value, hx = HX[h], hy = HY[h];
      R px, py, mx, my;
      ab(0, s, hx, hy, px, py);
      ab(0, s, -hx, -hy, mx, my);
      acc += Kq[HQ[h]] * pair_dot<hx, hy>(px - mx, py - my);
    });
    psib[s] += acc;
  }
  if (NS == 2) {
    for (int s = 0; s < 2; ++s) {  // species s's force depends on species o = 1 - s's field
      const int o = 1 - s;
      R acc = 0;
      each_index<4>([&](auto H) {
        constexpr int h = decltype(H)::value, hx = HX[h], hy = HY[h];
        R px, py, mx, my;
        ab(1, s, hx, hy, px, py);
        ab(1, s, -hx, -hy, mx, my);
        acc += R(a.t[HQ[h]]) * pair_dot<hx, hy>(px - mx, py - my);
      });
      // B_s uses species s's own r (r_s Fbar_s); it lands on the other species' field
      if (a.cross_psi) psib[o] += R(a.gab) * acc;
      else rbar[o] += R(a.gab) * acc;
    }
  }
  for (int s = 0; s < NS; ++s) corr[s] = rbar[s] + psib[s] * R(a.psi0) * R(a.irho0) * exp(-rho[s] * R(a.irho0));
}

// Local part of the reverse step: force recompute, transposed streaming, the collision's
// and velocity shift's adjoints; writes lam (the local part of lambda(t)), Fbar and per-tile
// partial sums.
//
// GIN: the common term of lambda(t+1) is not read from memory but gathered here, for the tile
// plus a halo of one, from A_s and B_s of step t + 1 (tile plus a halo of three) and the
// densities of state t + 1: the separate gather of step t + 1 is not needed.
template <typename R, int NS, bool WALLS, bool GIN>
__global__ __launch_bounds__(256) void adj_local_kernel(AdjArgs a) {
  AdjView<R> v(a);
  constexpr int GX = ATX + 6, GY = ATY + 6;  // A_s, B_s of step t + 1 staged with a halo of three
  __shared__ R sps[2][AHY][AHX];  // psi of the forward state, tile + halo
  __shared__ R srh[2][AHY][AHX];  // rho
  __shared__ R scn[2][ATY + 2][ATX + 2];  // corr of lambda(t+1), tile + halo of one
  __shared__ R sab[GIN ? 2 : 1][GIN ? 4 : 1][GIN ? GY : 1][GIN ? GX : 1];
  __shared__ double sm[4][ADJ_N];
  const R *corr_next = static_cast<const R *>(a.corr_next);
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int x0 = blockIdx.x * ATX, y0 = blockIdx.y * ATY;
  const bool live = x0 + tx < v.lx && y0 + ty < v.ly;
  // memory accesses of lanes past the lattice's end use its last site (results discarded)
  const int xs = min(x0 + tx, v.lx - 1), y = min(y0 + ty, v.ly - 1);
  const size_t i = (size_t)y * v.lx + xs;
  const R *lam_next = static_cast<const R *>(a.lam_next);
  R *lamout = static_cast<R *>(a.lam);
  R *fbar = static_cast<R *>(a.fbar);

  // Every load of the pass is issued before its first use, with no branch between the
  // requests, so that they are in flight together (a wave holds one tile row and has nothing
  // else to overlap them with).  First what the site reads outside the staged neighbourhood:
  // j_s, and lambda(t+1) at the transposed-streaming sources.  The population leaving x along
  // c_l arrives at x + c_l, or bounces back into opp(l) at x when x + c_l is a wall row; the
  // bounce is folded into the address (y is the same across a wave, so is the bounce).
  R rho[2], jx[2], jy[2], psi[2], Fx[2], Fy[2];
  R lsrc[2][Q];
  for (int s = 0; s < NS; ++s) {
    jx[s] = v.fld(2, s, i);
    jy[s] = v.fld(3, s, i);
  }
  each_index<Q>([&](auto L) {
    constexpr int l = decltype(L)::value, cx = CXS[l], cy = CYS[l];
    const int yn = y + cy;
    const bool bounce = WALLS && cy != 0 && (yn < 0 || yn >= v.ly);
    const size_t j = bounce ? i : (size_t)(WALLS ? yn : wrapx(yn, v.ly)) * v.lx + wrapx(xs + cx, v.lx);
    const int pl = bounce ? OPPS[l] : l;
    for (int s = 0; s < NS; ++s) lsrc[s][l] = lam_next[((size_t)s * Q + pl) * v.n + j];
  });
  // and, on the two wall rows, their pre-collision populations (the wall stress's source)
  R xwr[2][Q];
  if constexpr (WALLS) {
    if (y == 0 || y == v.ly - 1) {
      each_index<Q>([&](auto L) {
        constexpr int l = decltype(L)::value, cy = CYS[l];
        if constexpr (cy != 0)
          for (int s = 0; s < NS; ++s) xwr[s][l] = R(a.x[((size_t)(s * Q + l) * 2 + (cy < 0 ? 0 : 1)) * v.lx + xs]);
      });
    }
  }
  // Then the staging: psi and rho of the tile plus a halo of two, the common term of
  // lambda(t+1) plus a halo of one.  Points that are not sites (past a wall, or past the end of
  // the staging range) load site 0 and store the wall value or zero instead.
  constexpr int NPS = (AHX * AHY + 255) / 256, NCN = ((ATX + 2) * (ATY + 2) + 255) / 256;
  R vps[NPS][2], vrh[NPS][2], vcn[NCN][2];
  bool inps[NPS], incn[NCN];
#pragma unroll
  for (int it = 0; it < NPS; ++it) {
    const int k = threadIdx.x + it * 256, hx = k % AHX, hy = k / AHX;
    size_t j = 0;
    inps[it] = k < AHX * AHY && stage_site<WALLS>(x0 - 2 + hx, y0 - 2 + hy, v.lx, v.ly, j);
    if (!inps[it]) j = 0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      vps[it][s] = v.fld(1, s, j);
      vrh[it][s] = v.fld(0, s, j);
    }
  }
  // with GIN: A_s, B_s of step t + 1 (tile + halo of three), and in vcn the densities of state
  // t + 1 at the points where the common term is gathered; else the common term itself
  constexpr int NAB = GIN ? (GX * GY + 255) / 256 : 1;
  R vab[NAB][2][4];
  bool inab[NAB];
  const R *fbar_next = static_cast<const R *>(a.fbar_next);
  const R *rho_next = static_cast<const R *>(a.fields_next);  // field 0 (rho) of state t + 1
  if constexpr (GIN) {
#pragma unroll
    for (int it = 0; it < NAB; ++it) {
      const int k = threadIdx.x + it * 256, hx = k % GX, hy = k / GX;
      size_t j = 0;
      inab[it] = k < GX * GY && stage_site<WALLS>(x0 - 3 + hx, y0 - 3 + hy, v.lx, v.ly, j);
      if (!inab[it]) j = 0;
#pragma unroll
      for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int c = 0; c < 4; ++c) vab[it][s][c] = fbar_next[((size_t)s * 4 + c) * v.n + j];
    }
  }
#pragma unroll
  for (int it = 0; it < NCN; ++it) {
    const int k = threadIdx.x + it * 256, hx = k % (ATX + 2), hy = k / (ATX + 2);
    size_t j = 0;
    incn[it] = k < (ATX + 2) * (ATY + 2) && stage_site<WALLS>(x0 - 1 + hx, y0 - 1 + hy, v.lx, v.ly, j);
    if (!incn[it]) j = 0;
#pragma unroll
    for (int s = 0; s < NS; ++s) vcn[it][s] = GIN ? rho_next[(size_t)s * v.n + j] : corr_next[(size_t)s * v.n + j];
  }
#pragma unroll
  for (int it = 0; it < NPS; ++it) {
    const int k = threadIdx.x + it * 256, hx = k % AHX, hy = k / AHX;
    if (k < AHX * AHY) {
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        sps[s][hy][hx] = inps[it] ? vps[it][s] : R(a.psi_w[s]);
        srh[s][hy][hx] = inps[it] ? vrh[it][s] : R(a.rho_w[s]);
      }
    }
  }
  if constexpr (GIN) {
#pragma unroll
    for (int it = 0; it < NAB; ++it) {
      const int k = threadIdx.x + it * 256, hx = k % GX, hy = k / GX;
      if (k < GX * GY) {
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
          for (int c = 0; c < 4; ++c) sab[s][c][hy][hx] = inab[it] ? vab[it][s][c] : R(0);
      }
    }
    __syncthreads();
    // the common term of lambda(t+1) at the tile + halo of one, exactly as the gather pass
    // computes it at those sites (zero at points that are not sites)
#pragma unroll
    for (int it = 0; it < NCN; ++it) {
      const int k = threadIdx.x + it * 256, hx = k % (ATX + 2), hy = k / (ATX + 2);
      if (k < (ATX + 2) * (ATY + 2)) {
        auto ab = [&](int which, int s, int dx, int dy, R &bx, R &by) {
          bx = sab[s][2 * which + 0][hy + 2 + dy][hx + 2 + dx];
          by = sab[s][2 * which + 1][hy + 2 + dy][hx + 2 + dx];
        };
        R rn[2] = {vcn[it][0], NS == 2 ? vcn[it][NS - 1] : R(0)}, cn[2];
        gather_corr<R, NS>(a, ab, rn, cn);
#pragma unroll
        for (int s = 0; s < NS; ++s) scn[s][hy][hx] = incn[it] ? cn[s] : R(0);
      }
    }
  } else {
#pragma unroll
    for (int it = 0; it < NCN; ++it) {
      const int k = threadIdx.x + it * 256, hx = k % (ATX + 2), hy = k / (ATX + 2);
      if (k < (ATX + 2) * (ATY + 2)) {
#pragma unroll
        for (int s = 0; s < NS; ++s) scn[s][hy][hx] = incn[it] ? vcn[it][s] : R(0);
      }
    }
  }
  __syncthreads();

  auto psi_at = [&](int s, int dx, int dy) -> R { return sps[s][ty + 2 + dy][tx + 2 + dx]; };
  auto rho_at = [&](int s, int dx, int dy) -> R { return srh[s][ty + 2 + dy][tx + 2 + dx]; };

  R s1x[2], s1y[2], s2x[2], s2y[2], xx[2], xy[2], self[2];
  for (int s = 0; s < NS; ++s) {
    rho[s] = rho_at(s, 0, 0);
    psi[s] = psi_at(s, 0, 0);
    // two-belt sums with the attractive (w) and repulsive (p) shell weights
    R ax = 0, ay = 0, bx = 0, by = 0;
    each_index<NHALF>([&](auto H) {
      constexpr int h = decltype(H)::value, hx = HX[h], hy = HY[h];
      const R d = psi_at(s, hx, hy) - psi_at(s, -hx, -hy);
      const R wq = R(a.w[HQ[h]]), pq = R(a.p[HQ[h]]);
      if constexpr (hx != 0) {
        ax += cmul<hx>(wq) * d;
        bx += cmul<hx>(pq) * d;
      }
      if constexpr (hy != 0) {
        ay += cmul<hy>(wq) * d;
        by += cmul<hy>(pq) * d;
      }
    });
    s1x[s] = ax; s1y[s] = ay; s2x[s] = bx; s2y[s] = by;
    Fx[s] = -psi[s] * (R(a.g1[s]) * ax + R(a.g2[s]) * bx);
    Fy[s] = -psi[s] * (R(a.g1[s]) * ay + R(a.g2[s]) * by);
    xx[s] = 0; xy[s] = 0; self[s] = 0;
  }
  if (NS == 2) {
    for (int s = 0; s < 2; ++s) {
      const int o = 1 - s;
      R cx = 0, cy = 0;
      each_index<4>([&](auto H) {
        constexpr int h = decltype(H)::value, hx = HX[h], hy = HY[h];
        const R d = a.cross_psi ? psi_at(o, hx, hy) - psi_at(o, -hx, -hy) : rho_at(o, hx, hy) - rho_at(o, -hx, -hy);
        const R tq = R(a.t[HQ[h]]);
        if constexpr (hx != 0) cx += cmul<hx>(tq) * d;
        if constexpr (hy != 0) cy += cmul<hy>(tq) * d;
      });
      xx[s] = cx;
      xy[s] = cy;
      self[s] = a.cross_psi ? psi[s] : rho[s];
      Fx[s] -= R(a.gab) * self[s] * cx;
      Fy[s] -= R(a.gab) * self[s] * cy;
    }
  }
  for (int s = 0; s < NS; ++s) {
    Fx[s] += rho[s] * R(a.body[0]);
    Fy[s] += rho[s] * R(a.body[1]);
  }

  // common velocity and the shifted equilibrium velocities
  R nx = 0, ny = 0, den = 0, rtot = 0, mx = 0, my = 0;
  for (int s = 0; s < NS; ++s) {
    const R om = R(a.omega[s]);
    nx += om * jx[s];
    ny += om * jy[s];
    den += om * rho[s];
    rtot += rho[s];
    mx += jx[s] + R(0.5) * Fx[s];
    my += jy[s] + R(0.5) * Fy[s];
  }
  // reciprocals taken once per site: the rest of the pass multiplies
  // 1 / lx comes from the host, rounded in R as a division here would round it
  const R iden = R(1) / den, irt = R(1) / rtot, ilx = sizeof(R) == 8 ? R(a.ilx) : R(a.ilxf);
  const R upx = nx * iden, upy = ny * iden;
  const R urx = mx * irt;  // reported (half-force) velocity, x component
  const R ilr = ilx * irt;  // 1 / (lx rho_tot)

  // adjoint sources of this step's loss
  const R cW = R(a.cW), cQ = R(a.cQ);
  double loss_w = 0.0;  // summed over the wall row's links, divided by lx once
  const double loss_q = live ? double(cQ * urx) / v.lx : 0.0;

  R ubx = 0, uby = 0;  // adjoint of u'
  R rbar[2], jbx[2], jby[2], fbx[2], fby[2];
  R lp[2][Q];
  for (int s = 0; s < NS; ++s) {
    const R om = R(a.omega[s]), tau = R(a.tau[s]);
    const R ir = R(1) / rho[s];
    const R ux = upx + tau * Fx[s] * ir, uy = upy + tau * Fy[s] * ir;
    const R uu = ux * ux + uy * uy;
    R rb = 0, bx = 0, by = 0;
    each_index<Q>([&](auto L) {
      constexpr int l = decltype(L)::value, cx = CXS[l], cy = CYS[l];
      // lambda(t+1) at the transposed-streaming source (loaded above) and its common term
      const bool bounce = WALLS && cy != 0 && (y + cy < 0 || y + cy >= v.ly);
      R al = lsrc[s][l] + (bounce ? scn[s][ty + 1][tx + 1] : scn[s][ty + 1 + cy][tx + 1 + cx]);
      R cu = R(0);  // c_l . u
      if constexpr (cx != 0 && cy != 0) cu = cmul<cx>(ux) + cmul<cy>(uy);
      else if constexpr (cx != 0) cu = cmul<cx>(ux);
      else if constexpr (cy != 0) cu = cmul<cy>(uy);
      const R wl = R(WD2Q9[l]);
      const R poly = R(1) + R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu;  // f^eq_l / (W_l rho_s)
      const R feq = wl * rho[s] * poly;
      if constexpr (WALLS && cy != 0) {
        if (y == (cy < 0 ? 0 : v.ly - 1)) {
          // wall stress: d/dy_l of cW (1/2)(1/lx) (2 c_lx y_l - 6 W_l rho_w c_lx^2 U); the
          // moving wall's share is constant
          if constexpr (cx != 0) al += cmul<cx>(cW) * ilx;
          // post-collision population leaving the wall row
          const R yl = (R(1) - om) * xwr[s][l] + om * feq;
          const R mw = R(3) * wl * R(a.rho_w[s]) * R(cx * cx) * R(cy < 0 ? a.u_wall[0] : a.u_wall[1]);
          if (live) loss_w += double(cW * (R(cx) * yl - mw));
        }
      }
      lp[s][l] = (R(1) - om) * al;
      rb += om * al * wl * poly;  // omega al f^eq / rho
      const R k = om * al * wl * rho[s];
      bx += k * eq_grad<cx>(cu, ux);
      by += k * eq_grad<cy>(cu, uy);
    });
    // u_s = u' + tau F_s / rho_s
    ubx += bx;
    uby += by;
    fbx[s] = tau * bx * ir;
    fby[s] = tau * by * ir;
    rb -= tau * (Fx[s] * bx + Fy[s] * by) * (ir * ir);
    rbar[s] = rb;
  }
  for (int s = 0; s < NS; ++s) {
    const R om = R(a.omega[s]);
    // u' = sum omega j / sum omega rho
    jbx[s] = om * ubx * iden;
    jby[s] = om * uby * iden;
    rbar[s] -= om * (upx * ubx + upy * uby) * iden;
    // flow rate: Q = (1/lx) sum (sum_s j_s + F_s / 2)_x / sum_s rho_s
    jbx[s] += cQ * ilr;
    fbx[s] += R(0.5) * cQ * ilr;
    rbar[s] -= cQ * urx * ilr;
  }
  // force: F_s = -psi_s S_s - G_AB self_s X_s + rho_s g
  double dg1[2] = {0, 0}, dg2[2] = {0, 0}, dgab = 0, dgx = 0, dgy = 0;
  R psib[2] = {0, 0};
  for (int s = 0; s < NS; ++s) {
    const R Sx = R(a.g1[s]) * s1x[s] + R(a.g2[s]) * s2x[s], Sy = R(a.g1[s]) * s1y[s] + R(a.g2[s]) * s2y[s];
    psib[s] -= fbx[s] * Sx + fby[s] * Sy;
    rbar[s] += fbx[s] * R(a.body[0]) + fby[s] * R(a.body[1]);
    if (NS == 2) {
      const R cb = -R(a.gab) * (fbx[s] * xx[s] + fby[s] * xy[s]);
      if (a.cross_psi) psib[s] += cb;
      else rbar[s] += cb;
    }
    if (live) {
      dg1[s] = double(-psi[s] * (fbx[s] * s1x[s] + fby[s] * s1y[s]));
      dg2[s] = double(-psi[s] * (fbx[s] * s2x[s] + fby[s] * s2y[s]));
      dgab += double(-self[s] * (fbx[s] * xx[s] + fby[s] * xy[s]));
      dgx += double(fbx[s] * rho[s]);
      dgy += double(fby[s] * rho[s]);
    }
    // psi'(rho) = (psi0 / rho0) exp(-rho / rho0)
    rbar[s] += psib[s] * R(a.psi0) * R(a.irho0) * exp(-rho[s] * R(a.irho0));
  }
  if (live) {
    for (int s = 0; s < NS; ++s) {
      each_index<Q>([&](auto L) {
        constexpr int l = decltype(L)::value, cx = CXS[l], cy = CYS[l];
        R lam_l = lp[s][l] + rbar[s];
        if constexpr (cx != 0) lam_l += cmul<cx>(jbx[s]);
        if constexpr (cy != 0) lam_l += cmul<cy>(jby[s]);
        lamout[((size_t)s * Q + l) * v.n + i] = lam_l;
      });
      // what the gather needs of this site: A_s = psi_s Fbar_s, B_s = r_s Fbar_s
      fbar[((size_t)s * 4 + 0) * v.n + i] = psi[s] * fbx[s];
      fbar[((size_t)s * 4 + 1) * v.n + i] = psi[s] * fby[s];
      fbar[((size_t)s * 4 + 2) * v.n + i] = self[s] * fbx[s];
      fbar[((size_t)s * 4 + 3) * v.n + i] = self[s] * fby[s];
    }
  }
  // per-tile partial sums, accumulated over the reverse steps in each tile's own row
  // (fixed order: waves, then steps, then tiles in the final pass)
  if (WALLS) loss_w /= v.lx;
  double vals[ADJ_N] = {dg1[0], dg1[1], dg2[0], dg2[1], dgab, dgx, dgy, loss_w, loss_q};
  const size_t blk = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
  tile_accumulate(vals, sm, a.partials + blk * ADJ_N);
}

// Nonlocal part: the force's dependence on the neighbours' psi (and rho), gathered with the
// forward stencil; writes corr, the term of lambda(t) common to every l (the next reverse step
// adds it to lam as it reads lambda).
template <typename R, int NS, bool WALLS>
__global__ __launch_bounds__(256) void adj_gather_kernel(AdjArgs a) {
  AdjView<R> v(a);
  // per species: psi_s Fbar_s (x, y) and r_s Fbar_s (x, y) of tile + halo, zero off the lattice
  __shared__ R sab[2][4][AHY][AHX];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int x0 = blockIdx.x * ATX, y0 = blockIdx.y * ATY;
  const R *fbar = static_cast<const R *>(a.fbar);
  const int x = x0 + tx, y = y0 + ty;
  const bool live = x < v.lx && y < v.ly;
  const size_t i = live ? (size_t)y * v.lx + x : 0;
  // every load is issued before the barrier, together: rho_s of this site, then the staged
  // values (points that are not sites load site 0 and store zero)
  R rho[2];
  for (int s = 0; s < NS; ++s) rho[s] = v.fld(0, s, i);
  constexpr int NST = (AHX * AHY + 255) / 256;
  R vab[NST][2][4];
  bool in[NST];
#pragma unroll
  for (int it = 0; it < NST; ++it) {
    const int k = threadIdx.x + it * 256, hx = k % AHX, hy = k / AHX;
    size_t j = 0;
    in[it] = k < AHX * AHY && stage_site<WALLS>(x0 - 2 + hx, y0 - 2 + hy, v.lx, v.ly, j);
    if (!in[it]) j = 0;
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int c = 0; c < 4; ++c) vab[it][s][c] = fbar[((size_t)s * 4 + c) * v.n + j];
  }
#pragma unroll
  for (int it = 0; it < NST; ++it) {
    const int k = threadIdx.x + it * 256, hx = k % AHX, hy = k / AHX;
    if (k < AHX * AHY) {
#pragma unroll
      for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int c = 0; c < 4; ++c) sab[s][c][hy][hx] = in[it] ? vab[it][s][c] : R(0);
    }
  }
  __syncthreads();
  if (!live) return;  // after the kernel's only barrier
  R *corr = static_cast<R *>(a.corr);
  // A_s = psi_s Fbar_s (which = 0) or B_s = r_s Fbar_s (which = 1) at a neighbour
  auto ab = [&](int which, int s, int dx, int dy, R &bx, R &by) {
    bx = sab[s][2 * which + 0][ty + 2 + dy][tx + 2 + dx];
    by = sab[s][2 * which + 1][ty + 2 + dy][tx + 2 + dx];
  };
  R cn[2];
  gather_corr<R, NS>(a, ab, rho, cn);
  for (int s = 0; s < NS; ++s) corr[(size_t)s * v.n + i] = cn[s];
}

// acc[k] += sum over blocks of partials[block][k], in block order (deterministic).
__global__ __launch_bounds__(256) void adj_reduce_kernel(const double *partials, int nblocks, double *acc) {
  __shared__ double sm[4];
  for (int k = 0; k < ADJ_N; ++k) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) v += partials[(size_t)b * ADJ_N + k];
    const double t = block_sum(v, sm);
    if (threadIdx.x == 0) acc[k] += t;
  }
}

__global__ void zero_kernel(uint32_t *p, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

int adj_blocks(int lx, int ly) { return ((lx + ATX - 1) / ATX) * ((ly + ATY - 1) / ATY); }

template <typename R, int NS, bool WALLS>
static hipError_t adj_step_t(const AdjArgs &a, int gin, int gout, hipStream_t st) {
  const dim3 tiles((a.lx + ATX - 1) / ATX, (a.ly + ATY - 1) / ATY), block(ATX * ATY);
  if (gin) hipLaunchKernelGGL((adj_local_kernel<R, NS, WALLS, true>), tiles, block, 0, st, a);
  else hipLaunchKernelGGL((adj_local_kernel<R, NS, WALLS, false>), tiles, block, 0, st, a);
  if (gout) hipLaunchKernelGGL((adj_gather_kernel<R, NS, WALLS>), tiles, block, 0, st, a);
  return hipGetLastError();
}

template <typename R>
static hipError_t adj_step_r(int ns, int walls, const AdjArgs &a, int gin, int gout, hipStream_t st) {
  if (ns == 1) return walls ? adj_step_t<R, 1, true>(a, gin, gout, st) : adj_step_t<R, 1, false>(a, gin, gout, st);
  return walls ? adj_step_t<R, 2, true>(a, gin, gout, st) : adj_step_t<R, 2, false>(a, gin, gout, st);
}

hipError_t launch_adjoint_step(int fp64, int ns, int walls, const AdjArgs &a, int gather_in, int gather_out,
                               hipStream_t st) {
  return fp64 ? adj_step_r<double>(ns, walls, a, gather_in, gather_out, st)
              : adj_step_r<float>(ns, walls, a, gather_in, gather_out, st);
}

hipError_t launch_adjoint_reduce(const double *partials, int lx, int ly, double *acc, hipStream_t st) {
  hipLaunchKernelGGL(adj_reduce_kernel, dim3(1), dim3(256), 0, st, partials, adj_blocks(lx, ly), acc);
  return hipGetLastError();
}

hipError_t launch_zero(void *p, size_t bytes, hipStream_t st) {
  const size_t n = bytes / 4;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, static_cast<uint32_t *>(p), n);
  return hipGetLastError();
}

}  // namespace lb355
