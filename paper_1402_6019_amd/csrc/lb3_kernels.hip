// Device kernels of the three-dimensional (D3Q19) two-belt pseudopotential step (gfx950).
//
// One launch of step3_kernel performs one time step of eq. (LB) on a 3-D lattice:
//   pull streaming (halfway bounce-back at the y walls) -> moments -> psi -> eq. (FORCE) over the
//   92 links of the 5x5x5 cube, the A-B repulsion over the D3Q19 links and the body force ->
//   velocity shift -> BGK collision with the rest-population closure -> store.
//
// Layout in HBM: [z][y][l][pitch][species], species fastest, so one row (z, y) is one
// contiguous run of its 19 plane rows, and both species of a site move in one access.  Every
// load and store goes through a buffer descriptor whose base is one z-plane of the buffer, so a
// buffer may exceed 4 GiB (one z-plane may not).
//
// Work decomposition: a workgroup owns a tile of 64 columns (x, one wave per row) by ty rows (y)
// and marches +z through a segment of sz planes.  The force at plane z needs psi at planes
// z-2..z+2 and at x +- 2, y +- 2, so the workgroup keeps a six-plane ring of psi_s (and rho_s for
// the A-B term) over the (64 + 4) x (ty + 4) sites of its tile and halo in LDS.  Each iteration
// pulls the lead plane z + 2 (its own sites, then the halo ring around the tile, spread one site
// per thread), turns it into psi and rho in the ring, synchronises once, and updates plane z.  Six
// slots make one barrier per plane sufficient: the slot written in iteration i + 1 is not among
// the five that iteration i reads.  The populations of the updated site are pulled again at the
// update (issued before the lead plane's work so their latency is hidden); they were pulled two
// iterations earlier for psi, so the second read is served by the caches.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "lb3_internal.hpp"
#include "lb_step.hpp"

namespace lb355 {

namespace d3 {

// D3Q19 in the canonical order of lb3.h; opposite links are adjacent (1-2, 3-4, ...).
__device__ constexpr int CX[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
__device__ constexpr int CY[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
__device__ constexpr int CZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

constexpr int opp(int l) { return l == 0 ? 0 : (l & 1 ? l + 1 : l - 1); }
constexpr int cx(int l) { return l == 1 || l == 7 || l == 9 || l == 11 || l == 13 ? 1 : (l == 2 || l == 8 || l == 10 || l == 12 || l == 14 ? -1 : 0); }
constexpr int cy(int l) { return l == 3 || l == 7 || l == 10 || l == 15 || l == 17 ? 1 : (l == 4 || l == 8 || l == 9 || l == 16 || l == 18 ? -1 : 0); }
constexpr int cz(int l) { return l == 5 || l == 11 || l == 14 || l == 15 || l == 18 ? 1 : (l == 6 || l == 12 || l == 13 || l == 16 || l == 17 ? -1 : 0); }

__device__ inline int wrap(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

}  // namespace d3

extern __shared__ __attribute__((aligned(16))) unsigned char lb3_smem[];

// Byte geometry of one population buffer.
struct Geo3 {
  uint32_t site_b, plane_b, row_b;  // bytes per site (both species), per plane row, per (z, y) row
  uint64_t zplane_b;                // bytes per z-plane
};

// Descriptor of z-plane z of buffer p.
__device__ inline Rsrc zplane_rsrc(const void *p, const Geo3 &g, int z) {
  const char *b = static_cast<const char *>(p) + (uint64_t)(uint32_t)z * g.zplane_b;
  return make_rsrc(b, (uint32_t)g.zplane_b);
}

// The 46 half-links of the 92-link cube stencil (one of each +-c pair), grouped by shell:
// c = (dx, dy, dz) with dz > 0, or dz == 0 and dy > 0, or dz == dy == 0 and dx > 0.
#define LB3_HALF_LINKS(X)                                                                        \
  /* shell 1 */ X(0, 1, 0, 0) X(0, 0, 1, 0) X(0, 0, 0, 1)                                       \
  /* shell 2 */ X(1, 1, 1, 0) X(1, -1, 1, 0) X(1, 1, 0, 1) X(1, -1, 0, 1) X(1, 0, 1, 1) X(1, 0, -1, 1) \
  /* shell 3 */ X(2, 1, 1, 1) X(2, -1, 1, 1) X(2, 1, -1, 1) X(2, -1, -1, 1)                      \
  /* shell 4 */ X(3, 2, 0, 0) X(3, 0, 2, 0) X(3, 0, 0, 2)                                        \
  /* shell 5 */ X(4, 2, 1, 0) X(4, -2, 1, 0) X(4, 1, 2, 0) X(4, -1, 2, 0) X(4, 2, 0, 1) X(4, -2, 0, 1) \
                X(4, 0, 2, 1) X(4, 0, -2, 1) X(4, 1, 0, 2) X(4, -1, 0, 2) X(4, 0, 1, 2) X(4, 0, -1, 2) \
  /* shell 6 */ X(5, 2, 1, 1) X(5, -2, 1, 1) X(5, 2, -1, 1) X(5, -2, -1, 1) X(5, 1, 2, 1) X(5, -1, 2, 1) \
                X(5, 1, -2, 1) X(5, -1, -2, 1) X(5, 1, 1, 2) X(5, -1, 1, 2) X(5, 1, -1, 2) X(5, -1, -1, 2) \
  /* shell 8 */ X(6, 2, 2, 0) X(6, -2, 2, 0) X(6, 2, 0, 2) X(6, -2, 0, 2) X(6, 0, 2, 2) X(6, 0, -2, 2)

template <int MODE, int NS, bool WALLS, int WHAT>
__global__ __launch_bounds__(MODE == MODE_F64 ? 256 : 512) __attribute__((amdgpu_waves_per_eu(MODE == MODE_F64 ? 1 : 2))) void step3_kernel(Lb3Args a) {
  using C = Codec<MODE>;
  using R = typename C::R;
  using S = typename C::S;
  using L = typename C::L;
  using V = Vec<R, NS>;
  constexpr bool STORE = WHAT == WHAT_STEP;
  constexpr bool OBSERVE = WHAT == WHAT_OBSERVE;
  constexpr int TX = 64;
  constexpr int W4 = TX + 4;

  const int TY = (int)blockDim.x >> 6;
  const int H4 = TY + 4;
  const int SLOT = W4 * H4;
  V *psi_ring = reinterpret_cast<V *>(lb3_smem);   // [6][H4][W4]
  V *rho_ring = psi_ring + 6 * SLOT;              // [6][H4][W4] (two species)
  __shared__ double red_lds[8][RED3_N];

  const int lx = a.lx, ly = a.ly, lz = a.lz;
  Geo3 g;
  g.site_b = (uint32_t)(NS * sizeof(S));
  g.plane_b = (uint32_t)a.pitch * g.site_b;
  g.row_b = 19u * g.plane_b;
  g.zplane_b = (uint64_t)g.row_b * (uint32_t)ly;

  const int logical = xcd_remap(blockIdx.x, gridDim.x);
  const int per_seg = a.nstrip * a.nband;
  const int seg = logical / per_seg;
  const int rem = logical - seg * per_seg;
  const int band = rem / a.nstrip;
  const int strip = rem - band * a.nstrip;
  const int tid = threadIdx.x, lane = tid & 63, wv = (int)uni((uint32_t)(tid >> 6));
  const int x0 = strip * TX, y0 = band * TY;
  const int x = x0 + lane;
  const int y = y0 + wv;  // uniform per wave
  const bool row_ok = y < ly;
  const bool col_ok = row_ok && x < lx;
  const int zA = seg * a.sz, zB = min(zA + a.sz, lz);

  R K[NS][7], tau[NS], om[NS], rref[NS], psiw[NS], rhow[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
#pragma unroll
    for (int q = 0; q < 7; ++q) K[s][q] = R(a.K[s][q]);
    tau[s] = R(a.tau[s]);
    om[s] = R(a.omega[s]);
    rref[s] = R(a.rho_ref[s]);
    psiw[s] = R(a.psi_w[s]);
    rhow[s] = R(a.rho_w[s]);
  }
  const R T1 = R(a.T[0]), T2 = R(a.T[1]);
  const R gx = R(a.body[0]), gy = R(a.body[1]), gz = R(a.body[2]);
  const R psi0 = R(a.psi0), nirho0 = R(-a.irho0);

  // Interior site of this thread, wrapped onto the lattice: lanes past a ragged strip or band
  // hold the periodic images (or, beyond a wall, the ghost row) in the ring, compute on them and
  // store nothing.  Column bytes of x, x - 1, x + 1 and the row (uniform per wave).
  const int xc = x % lx;
  const bool y_solid = WALLS && y >= ly;
  const int yc = WALLS ? min(y, ly - 1) : y % ly;
  const uint32_t colb[3] = {(uint32_t)d3::wrap(xc - 1, lx) * g.site_b, (uint32_t)xc * g.site_b,
                            (uint32_t)d3::wrap(xc + 1, lx) * g.site_b};

  // Pull of the interior site (xc, yc) at plane z: f_l = f*_l(x - c_l), or f*_opp(l)(x) off a wall.
  auto pull_own = [&](int z, L (&f)[NS][19]) {
    const Rsrc rz[3] = {zplane_rsrc(a.src, g, d3::wrap(z + 1, lz)), zplane_rsrc(a.src, g, z),
                        zplane_rsrc(a.src, g, d3::wrap(z - 1, lz))};
#pragma unroll
    for (int l = 0; l < 19; ++l) {
      const int sy = yc - d3::cy(l);
      const bool bb = WALLS && (sy < 0 || sy >= ly);
      uint32_t soff, voff;
      int zi;
      if (bb) {
        soff = (uint32_t)yc * g.row_b + (uint32_t)d3::opp(l) * g.plane_b;
        voff = colb[1];
        zi = 1;
      } else {
        soff = (uint32_t)d3::wrap(sy, ly) * g.row_b + (uint32_t)l * g.plane_b;
        voff = colb[1 - d3::cx(l)];
        zi = 1 + d3::cz(l);  // source plane z - c_z: rz[0] = z + 1 (c_z = -1), rz[2] = z - 1 (c_z = +1)
      }
      if (NS == 2) C::bload2(rz[zi], voff, uni(soff), f[0][l], f[NS - 1][l]);
      else f[0][l] = C::bload(rz[zi], voff, uni(soff));
    }
  };

  // Halo sites of the ring: the (TX + 4) x (TY + 4) sites less the tile, numbered h = 0 ..
  // nhalo - 1 over the two rows above and below the tile, then the two columns left and right of
  // its rows; thread t handles h = t, t + blockDim.x, ... (nhalo = 4 TY + 272 exceeds the
  // workgroup's 64 TY threads).
  const int nhalo = SLOT - TX * TY;
  const int nthreads = (int)blockDim.x;
  auto halo_site = [&](int h, int &hdx, int &hdy) {
    const int top = 2 * W4;
    if (h < 2 * top) {  // rows -2, -1 (h < top) and TY, TY + 1
      const int r = h / W4;
      hdx = h - r * W4 - 2;
      hdy = r < 2 ? r - 2 : TY + (r - 2);
    } else {
      const int k = h - 2 * top;  // 4 columns per tile row
      hdy = k >> 2;
      const int c = k & 3;
      hdx = c < 2 ? c - 2 : TX + (c - 2);
    }
  };

  // psi and rho of the site whose pulled populations are f.
  auto site_psi = [&](const L (&f)[NS][19], V &ps, V &rh) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      R sum = C::dec(f[s][0], s);
#pragma unroll
      for (int l = 1; l < 19; ++l) sum += C::dec(f[s][l], s);
      rh.v[s] = rref[s] + sum;
      ps.v[s] = psi0 * (R(1) - C::expo(rh.v[s] * nirho0));
    }
  };

  // Pulls of halo site h of plane z, its ring index, and whether it lies past a wall.  Rows are
  // clamped onto the lattice, so every load has a valid address and a caller may issue them
  // unconditionally (a solid site's values are discarded).
  auto halo_pull = [&](int h, int z, L (&f)[NS][19], bool &solid, int &hi) {
    int hdx, hdy;
    halo_site(h, hdx, hdy);
    const int hx = ((x0 + hdx) % lx + lx) % lx;
    const int hy_raw = y0 + hdy;
    solid = WALLS && (hy_raw < 0 || hy_raw >= ly);
    const int hy = WALLS ? min(max(hy_raw, 0), ly - 1) : ((hy_raw % ly) + ly) % ly;
    const uint32_t hcol[3] = {(uint32_t)d3::wrap(hx - 1, lx) * g.site_b, (uint32_t)hx * g.site_b,
                              (uint32_t)d3::wrap(hx + 1, lx) * g.site_b};
    const Rsrc rz[3] = {zplane_rsrc(a.src, g, d3::wrap(z + 1, lz)), zplane_rsrc(a.src, g, z),
                        zplane_rsrc(a.src, g, d3::wrap(z - 1, lz))};
#pragma unroll
    for (int l = 0; l < 19; ++l) {
      const int sy = hy - d3::cy(l);
      const bool bb = WALLS && (sy < 0 || sy >= ly);
      uint32_t off;
      int zi;
      if (bb) {
        off = (uint32_t)hy * g.row_b + (uint32_t)d3::opp(l) * g.plane_b + hcol[1];
        zi = 1;
      } else {
        off = (uint32_t)d3::wrap(sy, ly) * g.row_b + (uint32_t)l * g.plane_b + hcol[1 - d3::cx(l)];
        zi = 1 + d3::cz(l);
      }
      if (NS == 2) C::bload2(rz[zi], off, 0u, f[0][l], f[NS - 1][l]);
      else f[0][l] = C::bload(rz[zi], off, 0u);
    }
    hi = (hdy + 2) * W4 + (hdx + 2);
  };
  // psi and rho of a site from its pulls, or the wall's values past a wall
  auto ring_value = [&](bool solid, const L (&f)[NS][19], V &vp, V &vr) {
    if (solid) {
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        vp.v[s] = psiw[s];
        vr.v[s] = rhow[s];
      }
    } else {
      site_psi(f, vp, vr);
    }
  };

  // Lead plane p into ring slot sl: the tile's own sites, then the halo, and with pull_u the
  // update's own pull of plane zu into fu.  FP32: the loads of the own sites, of the first halo
  // round (one site per thread) and of the update's pull are issued together before any of them
  // is waited for, so three memory latencies overlap instead of following each other.  FP64
  // keeps them in turn: its three sets of pulls would take 228 of its 256 registers.
  auto ring_plane = [&](int p, int sl, bool pull_u, int zu, L (&fu)[NS][19]) {
    const int z = d3::wrap(d3::wrap(p, lz), lz);
    V *ps = psi_ring + sl * SLOT;
    V *rh = rho_ring + sl * SLOT;
    if constexpr (MODE == MODE_F64) {
      {
        L fo[NS][19];
        pull_own(z, fo);
        V vp, vr;
        ring_value(y_solid, fo, vp, vr);
        const int i = (wv + 2) * W4 + lane + 2;
        ps[i] = vp;
        if (NS == 2) rh[i] = vr;
      }
      for (int h = tid; h < nhalo; h += nthreads) {
        L f2[NS][19];
        bool hs = false;
        int hi = 0;
        halo_pull(h, z, f2, hs, hi);
        V vp, vr;
        ring_value(hs, f2, vp, vr);
        ps[hi] = vp;
        if (NS == 2) rh[hi] = vr;
      }
      if (pull_u) pull_own(zu, fu);  // its latency overlaps the barrier
      return;
    }
    L fo[NS][19], fh[NS][19];
    pull_own(z, fo);
    bool hsolid = false;
    int hi0 = 0;
    halo_pull(min(tid, nhalo - 1), z, fh, hsolid, hi0);
    if (pull_u) pull_own(zu, fu);
    {
      V vp, vr;
      ring_value(y_solid, fo, vp, vr);
      const int i = (wv + 2) * W4 + lane + 2;
      ps[i] = vp;
      if (NS == 2) rh[i] = vr;
    }
    if (tid < nhalo) {
      V vp, vr;
      ring_value(hsolid, fh, vp, vr);
      ps[hi0] = vp;
      if (NS == 2) rh[hi0] = vr;
    }
    for (int h = tid + nthreads; h < nhalo; h += nthreads) {
      L f2[NS][19];
      bool hs = false;
      int hi = 0;
      halo_pull(h, z, f2, hs, hi);
      V vp, vr;
      ring_value(hs, f2, vp, vr);
      ps[hi] = vp;
      if (NS == 2) rh[hi] = vr;
    }
  };

  double acc[RED3_N];
#pragma unroll
  for (int k = 0; k < RED3_N; ++k) acc[k] = 0.0;

  // Prologue: planes zA - 2 .. zA + 1 into slots 0..3 (plane p lives in slot (p - zA + 2) mod 6).
  {
    L unused[NS][19];
    for (int k = 0; k < 4; ++k) ring_plane(zA - 2 + k, k, false, 0, unused);
  }

  for (int z = zA; z < zB; ++z) {
    const int k0 = z - zA;  // slot of plane z - 2
    L f[NS][19];  // the site to update, pulled together with the lead plane
    ring_plane(z + 2, (k0 + 4) % 6, true, z, f);
    __syncthreads();

    // ---- update plane z ---------------------------------------------------------------
    R fd[NS][19];
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int l = 0; l < 19; ++l) fd[s][l] = C::dec(f[s][l], s);
    R drho[NS], rho[NS], jx[NS], jy[NS], jz[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      R sum = fd[s][0];
#pragma unroll
      for (int l = 1; l < 19; ++l) sum += fd[s][l];
      drho[s] = sum;
      rho[s] = rref[s] + sum;
      jx[s] = ((fd[s][1] + fd[s][7]) + (fd[s][9] + fd[s][11]) + fd[s][13]) -
              ((fd[s][2] + fd[s][8]) + (fd[s][10] + fd[s][12]) + fd[s][14]);
      jy[s] = ((fd[s][3] + fd[s][7]) + (fd[s][10] + fd[s][15]) + fd[s][17]) -
              ((fd[s][4] + fd[s][8]) + (fd[s][9] + fd[s][16]) + fd[s][18]);
      jz[s] = ((fd[s][5] + fd[s][11]) + (fd[s][14] + fd[s][15]) + fd[s][18]) -
              ((fd[s][6] + fd[s][12]) + (fd[s][13] + fd[s][16]) + fd[s][17]);
    }

    // ring planes z - 2 .. z + 2 in slots (k0 + m) % 6
    const V *pl[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) pl[m] = psi_ring + ((k0 + m) % 6) * SLOT + (wv + 2) * W4 + lane + 2;
#define PSI3(dx, dy, dz) (pl[(dz) + 2][(dy) * W4 + (dx)])
    const V pc = PSI3(0, 0, 0);
    R Fx[NS], Fy[NS], Fz[NS];
    {
      // eq. (FORCE) as antisymmetric pair differences over the half links:
      // sum_c K(|c|^2) c psi(x + c) = sum_{half links} K(|c|^2) c (psi(x + c) - psi(x - c))
      R ax[NS], ay[NS], az[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) ax[s] = ay[s] = az[s] = R(0);
#define LB3_ACC(q, dx, dy, dz)                                                   \
  {                                                                              \
    const V pp = PSI3(dx, dy, dz), pm = PSI3(-(dx), -(dy), -(dz));               \
    _Pragma("unroll") for (int s = 0; s < NS; ++s) {                             \
      const R kd = K[s][q] * (pp.v[s] - pm.v[s]);                                \
      if ((dx) != 0) ax[s] = fmadd(R(dx), kd, ax[s]);                            \
      if ((dy) != 0) ay[s] = fmadd(R(dy), kd, ay[s]);                            \
      if ((dz) != 0) az[s] = fmadd(R(dz), kd, az[s]);                            \
    }                                                                            \
  }
      LB3_HALF_LINKS(LB3_ACC)
#undef LB3_ACC
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        Fx[s] = fmadd(-pc.v[s], ax[s], rho[s] * gx);
        Fy[s] = fmadd(-pc.v[s], ay[s], rho[s] * gy);
        Fz[s] = fmadd(-pc.v[s], az[s], rho[s] * gz);
      }
    }
#undef PSI3
    if (NS == 2) {
      // A-B repulsion over the D3Q19 links, between densities (or psi)
      const V *base = a.cross_psi ? psi_ring : rho_ring;
      const V *xr[3];
#pragma unroll
      for (int m = 0; m < 3; ++m) xr[m] = base + ((k0 + 1 + m) % 6) * SLOT + (wv + 2) * W4 + lane + 2;
#define XR3(dx, dy, dz) (xr[(dz) + 1][(dy) * W4 + (dx)])
      const V c0 = XR3(0, 0, 0);
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int o = 1 - s;
        const R ex = XR3(1, 0, 0).v[o] - XR3(-1, 0, 0).v[o];
        const R ey = XR3(0, 1, 0).v[o] - XR3(0, -1, 0).v[o];
        const R ez = XR3(0, 0, 1).v[o] - XR3(0, 0, -1).v[o];
        const R pxy = XR3(1, 1, 0).v[o] - XR3(-1, -1, 0).v[o], mxy = XR3(1, -1, 0).v[o] - XR3(-1, 1, 0).v[o];
        const R pxz = XR3(1, 0, 1).v[o] - XR3(-1, 0, -1).v[o], mxz = XR3(1, 0, -1).v[o] - XR3(-1, 0, 1).v[o];
        const R pyz = XR3(0, 1, 1).v[o] - XR3(0, -1, -1).v[o], myz = XR3(0, 1, -1).v[o] - XR3(0, -1, 1).v[o];
        const R cxs = fmadd(T1, ex, T2 * ((pxy + mxy) + (pxz + mxz)));
        const R cys = fmadd(T1, ey, T2 * ((pxy - mxy) + (pyz + myz)));
        const R czs = fmadd(T1, ez, T2 * ((pxz - mxz) + (pyz - myz)));
        Fx[s] = fmadd(-c0.v[s], cxs, Fx[s]);
        Fy[s] = fmadd(-c0.v[s], cys, Fy[s]);
        Fz[s] = fmadd(-c0.v[s], czs, Fz[s]);
      }
#undef XR3
    }

    // common velocity u' = sum_s (j_s / tau_s) / sum_s (rho_s / tau_s)
    R nux = jx[0] * om[0], nuy = jy[0] * om[0], nuz = jz[0] * om[0], den = rho[0] * om[0];
#pragma unroll
    for (int s = 1; s < NS; ++s) {
      nux = fmadd(jx[s], om[s], nux);
      nuy = fmadd(jy[s], om[s], nuy);
      nuz = fmadd(jz[s], om[s], nuz);
      den = fmadd(rho[s], om[s], den);
    }
    const R iden = C::rcp(den);
    const R upx = nux * iden, upy = nuy * iden, upz = nuz * iden;

    if (WHAT == WHAT_MOMENTS && col_ok) {
      R sr = rho[0], mx = jx[0] + R(0.5) * Fx[0], my = jy[0] + R(0.5) * Fy[0], mz = jz[0] + R(0.5) * Fz[0];
#pragma unroll
      for (int s = 1; s < NS; ++s) {
        sr += rho[s];
        mx += jx[s] + R(0.5) * Fx[s];
        my += jy[s] + R(0.5) * Fy[s];
        mz += jz[s] + R(0.5) * Fz[s];
      }
      const size_t nsite = (size_t)lx * ly * lz;
      const size_t site = ((size_t)z * ly + y) * lx + x;
      if (a.out_rho) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          if (a.out_f32) static_cast<float *>(a.out_rho)[s * nsite + site] = float(rho[s]);
          else static_cast<double *>(a.out_rho)[s * nsite + site] = double(rho[s]);
        }
      }
      if (a.out_u) {
        const R ux = mx / sr, uy = my / sr, uz = mz / sr;
        if (a.out_f32) {
          float *u = static_cast<float *>(a.out_u);
          u[site] = float(ux);
          u[nsite + site] = float(uy);
          u[2 * nsite + site] = float(uz);
        } else {
          double *u = static_cast<double *>(a.out_u);
          u[site] = double(ux);
          u[nsite + site] = double(uy);
          u[2 * nsite + site] = double(uz);
        }
      }
    }

    if (OBSERVE && col_ok) {
      R sr = rho[0], mx = jx[0] + R(0.5) * Fx[0];
      bool bad = !(rho[0] > R(0) && rho[0] < R(INFINITY));
#pragma unroll
      for (int s = 1; s < NS; ++s) {
        sr += rho[s];
        mx += jx[s] + R(0.5) * Fx[s];
        bad = bad || !(rho[s] > R(0) && rho[s] < R(INFINITY));
      }
      acc[RED3_MASS0] += double(rho[0]);
      if (NS == 2) acc[RED3_MASS1] += double(rho[NS - 1]);
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        acc[RED3_PX] += double(jx[s]);
        acc[RED3_PY] += double(jy[s]);
        acc[RED3_PZ] += double(jz[s]);
      }
      acc[RED3_FLOW] += double(mx / sr);
      acc[RED3_BAD] += bad ? 1.0 : 0.0;
    }

    if (STORE) {
      R fs[NS][19];
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const R ir = C::rcp(rho[s]);
        const R ux = fmadd(tau[s] * Fx[s], ir, upx);
        const R uy = fmadd(tau[s] * Fy[s], ir, upy);
        const R uz = fmadd(tau[s] * Fz[s], ir, upz);
        // f^eq_l - W_l rho_ref = W_l (drho - 3/2 rho u.u) + W_l rho cu (3 + 9/2 cu)
        const R m15 = R(-1.5) * fmadd(ux, ux, fmadd(uy, uy, uz * uz));
        const R r18 = rho[s] * R(1.0 / 18.0), r36 = rho[s] * R(1.0 / 36.0);
        const R b18 = fmadd(r18, m15, drho[s] * R(1.0 / 18.0)), b36 = fmadd(r36, m15, drho[s] * R(1.0 / 36.0));
        const R o = om[s];
        auto relax = [o](R fl, R b, R r, R cu) { return fmadd(o, fmadd(r, cu * fmadd(R(4.5), cu, R(3)), b) - fl, fl); };
        fs[s][1] = relax(fd[s][1], b18, r18, ux);
        fs[s][2] = relax(fd[s][2], b18, r18, -ux);
        fs[s][3] = relax(fd[s][3], b18, r18, uy);
        fs[s][4] = relax(fd[s][4], b18, r18, -uy);
        fs[s][5] = relax(fd[s][5], b18, r18, uz);
        fs[s][6] = relax(fd[s][6], b18, r18, -uz);
        fs[s][7] = relax(fd[s][7], b36, r36, ux + uy);
        fs[s][8] = relax(fd[s][8], b36, r36, -(ux + uy));
        fs[s][9] = relax(fd[s][9], b36, r36, ux - uy);
        fs[s][10] = relax(fd[s][10], b36, r36, -(ux - uy));
        fs[s][11] = relax(fd[s][11], b36, r36, ux + uz);
        fs[s][12] = relax(fd[s][12], b36, r36, -(ux + uz));
        fs[s][13] = relax(fd[s][13], b36, r36, ux - uz);
        fs[s][14] = relax(fd[s][14], b36, r36, -(ux - uz));
        fs[s][15] = relax(fd[s][15], b36, r36, uy + uz);
        fs[s][16] = relax(fd[s][16], b36, r36, -(uy + uz));
        fs[s][17] = relax(fd[s][17], b36, r36, uy - uz);
        fs[s][18] = relax(fd[s][18], b36, r36, -(uy - uz));
        // rest population closes the mass balance: d*_0 = drho - sum_{l>0} d*_l
        R t = fs[s][1];
#pragma unroll
        for (int l = 2; l < 19; ++l) t += fs[s][l];
        fs[s][0] = drho[s] - t;
      }
      if (col_ok) {
        const Rsrc rd = zplane_rsrc(a.dst, g, z);
        const uint32_t rb = (uint32_t)y * g.row_b;
#pragma unroll
        for (int l = 0; l < 19; ++l) {
          if (NS == 2) C::template bstore2<kStoreWriteThrough>(rd, colb[1], uni(rb + (uint32_t)l * g.plane_b), fs[0][l], fs[NS - 1][l]);
          else C::template bstore<kStoreWriteThrough>(rd, colb[1], uni(rb + (uint32_t)l * g.plane_b), fs[0][l]);
        }
      }
    }
  }

  if (OBSERVE) {
    const int nw = (int)blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < RED3_N; ++k) {
      const double v = wave_sum(acc[k]);
      if (lane == 0) red_lds[wv][k] = v;
    }
    __syncthreads();
    if (tid < RED3_N) {
      double v = 0.0;
      for (int i = 0; i < nw; ++i) v += red_lds[i][tid];
      a.partials[(size_t)blockIdx.x * RED3_N + tid] = v;
    }
  }
}

size_t step3_lds_bytes(int mode, int ns, int ty) {
  const size_t r = mode == MODE_F64 ? 8 : 4;
  return 2 * 6 * (size_t)(64 + 4) * (ty + 4) * ns * r;
}

template <int MODE, int NS, bool WALLS>
static hipError_t launch3_t(int what, int ty, int nb, const Lb3Args &a, hipStream_t st) {
  const size_t lds = step3_lds_bytes(MODE, NS, ty);
  const dim3 grid(nb), block(64 * ty);
  switch (what) {
    case WHAT_STEP: hipLaunchKernelGGL((step3_kernel<MODE, NS, WALLS, WHAT_STEP>), grid, block, lds, st, a); break;
    case WHAT_MOMENTS: hipLaunchKernelGGL((step3_kernel<MODE, NS, WALLS, WHAT_MOMENTS>), grid, block, lds, st, a); break;
    case WHAT_OBSERVE: hipLaunchKernelGGL((step3_kernel<MODE, NS, WALLS, WHAT_OBSERVE>), grid, block, lds, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int MODE>
static hipError_t launch3_m(int ns, int walls, int what, int ty, int nb, const Lb3Args &a, hipStream_t st) {
  if (ns == 1) return walls ? launch3_t<MODE, 1, true>(what, ty, nb, a, st) : launch3_t<MODE, 1, false>(what, ty, nb, a, st);
  return walls ? launch3_t<MODE, 2, true>(what, ty, nb, a, st) : launch3_t<MODE, 2, false>(what, ty, nb, a, st);
}

hipError_t launch_step3(int mode, int ns, int walls, int what, int ty, int nb, const Lb3Args &a, hipStream_t st) {
  switch (mode) {
    case MODE_F64: return launch3_m<MODE_F64>(ns, walls, what, ty, nb, a, st);
    case MODE_F32: return launch3_m<MODE_F32>(ns, walls, what, ty, nb, a, st);
  }
  return hipErrorInvalidValue;
}

template <int MODE, int NS, bool WALLS>
static int blocks3_t(int ty) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step3_kernel<MODE, NS, WALLS, WHAT_STEP>, 64 * ty,
                                                   step3_lds_bytes(MODE, NS, ty)) != hipSuccess)
    return 1;
  return n > 0 ? n : 1;
}

int step3_blocks_per_cu(int mode, int ns, int walls, int ty) {
  if (mode == MODE_F64) {
    if (ns == 1) return walls ? blocks3_t<MODE_F64, 1, true>(ty) : blocks3_t<MODE_F64, 1, false>(ty);
    return walls ? blocks3_t<MODE_F64, 2, true>(ty) : blocks3_t<MODE_F64, 2, false>(ty);
  }
  if (ns == 1) return walls ? blocks3_t<MODE_F32, 1, true>(ty) : blocks3_t<MODE_F32, 1, false>(ty);
  return walls ? blocks3_t<MODE_F32, 2, true>(ty) : blocks3_t<MODE_F32, 2, false>(ty);
}

// Second pass of lb3_totals: fixed-order sum of the per-workgroup partials.
__global__ __launch_bounds__(256) void reduce3_kernel(const double *partials, int nblocks, double *totals) {
  __shared__ double sm[256][RED3_N];
  const int tid = threadIdx.x;
  double v[RED3_N];
#pragma unroll
  for (int k = 0; k < RED3_N; ++k) v[k] = 0.0;
  for (int b = tid; b < nblocks; b += 256)
#pragma unroll
    for (int k = 0; k < RED3_N; ++k) v[k] += partials[(size_t)b * RED3_N + k];
#pragma unroll
  for (int k = 0; k < RED3_N; ++k) sm[tid][k] = v[k];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h)
#pragma unroll
      for (int k = 0; k < RED3_N; ++k) sm[tid][k] += sm[tid + h][k];
    __syncthreads();
  }
  if (tid < RED3_N) totals[tid] = sm[0][tid];
}

hipError_t launch_reduce3(const double *partials, int nblocks, double *totals, hipStream_t st) {
  hipLaunchKernelGGL(reduce3_kernel, dim3(1), dim3(256), 0, st, partials, nblocks, totals);
  return hipGetLastError();
}

// Layout kernels: canonical pre-collision f[s][l][z][y][x] (FP64) <-> the stored
// post-collision form [z][y][l][pitch][s].  Streaming with bounce-back is a permutation:
//   f_l(x) = g_l(x - c_l) if x - c_l is fluid, else g_opp(l)(x); inverse g_l(w) = f_l(w + c_l)
// if w + c_l is fluid, else f_opp(l)(w).
__device__ inline size_t pop3_index(int s, int l, int z, int y, int x, int ly, int pitch, int ns) {
  return ((((size_t)z * ly + y) * 19 + l) * pitch + x) * ns + s;
}

template <int MODE, bool WALLS>
__global__ void init3_kernel(Lb3Layout a) {  // in: rho [ns][lz][ly][lx] FP64; state at rest
  using C = Codec<MODE>;
  using S = typename C::S;
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
  if (x >= a.lx) return;
  const double *rho = static_cast<const double *>(a.in);
  S *out = static_cast<S *>(a.out);
  const size_t nsite = (size_t)a.lx * a.ly * a.lz;
  for (int s = 0; s < a.ns; ++s)
    for (int l = 0; l < 19; ++l) {
      int wx = x + d3::CX[l], wy = y + d3::CY[l], wz = z + d3::CZ[l];
      if (WALLS && (wy < 0 || wy >= a.ly)) {
        wx = x; wy = y; wz = z;
      } else {
        wx = d3::wrap(wx, a.lx); wy = d3::wrap(wy, a.ly); wz = d3::wrap(wz, a.lz);
      }
      const double W = l == 0 ? 1.0 / 3.0 : (l <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
      const double v = W * rho[s * nsite + ((size_t)wz * a.ly + wy) * a.lx + wx];
      C::store(out + pop3_index(s, l, z, y, x, a.ly, a.pitch, a.ns), v, W * a.rho_ref[s]);
    }
}

template <int MODE, bool WALLS>
__global__ void restore3_kernel(Lb3Layout a) {  // in: canonical f (FP64)
  using C = Codec<MODE>;
  using S = typename C::S;
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
  if (x >= a.lx) return;
  const double *f = static_cast<const double *>(a.in);
  S *out = static_cast<S *>(a.out);
  const size_t nsite = (size_t)a.lx * a.ly * a.lz;
  for (int s = 0; s < a.ns; ++s)
    for (int l = 0; l < 19; ++l) {
      // g_l at w = (x, y, z) is f_l(w + c_l), or f_opp(l)(w) when w + c_l is solid
      int vx = x + d3::CX[l], vy = y + d3::CY[l], vz = z + d3::CZ[l];
      int lsrc = l;
      if (WALLS && (vy < 0 || vy >= a.ly)) {
        vx = x; vy = y; vz = z;
        lsrc = d3::opp(l);
      } else {
        vx = d3::wrap(vx, a.lx); vy = d3::wrap(vy, a.ly); vz = d3::wrap(vz, a.lz);
      }
      const double W = l == 0 ? 1.0 / 3.0 : (l <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
      const double v = f[((size_t)s * 19 + lsrc) * nsite + ((size_t)vz * a.ly + vy) * a.lx + vx];
      C::store(out + pop3_index(s, l, z, y, x, a.ly, a.pitch, a.ns), v, W * a.rho_ref[s]);
    }
}

template <int MODE, bool WALLS>
__global__ void checkpoint3_kernel(Lb3Layout a) {  // out: canonical f (FP64)
  using C = Codec<MODE>;
  using S = typename C::S;
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
  if (x >= a.lx) return;
  const S *g = static_cast<const S *>(a.in);
  double *f = static_cast<double *>(a.out);
  const size_t nsite = (size_t)a.lx * a.ly * a.lz;
  for (int s = 0; s < a.ns; ++s)
    for (int l = 0; l < 19; ++l) {
      // f_l(x) = g_l(x - c_l), or g_opp(l)(x) when x - c_l is solid
      int wx = x - d3::CX[l], wy = y - d3::CY[l], wz = z - d3::CZ[l];
      int lsrc = l;
      if (WALLS && (wy < 0 || wy >= a.ly)) {
        wx = x; wy = y; wz = z;
        lsrc = d3::opp(l);
      } else {
        wx = d3::wrap(wx, a.lx); wy = d3::wrap(wy, a.ly); wz = d3::wrap(wz, a.lz);
      }
      const double W = l == 0 ? 1.0 / 3.0 : (l <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
      const double v = C::load(g + pop3_index(s, lsrc, wz, wy, wx, a.ly, a.pitch, a.ns), W * a.rho_ref[s]);
      f[((size_t)s * 19 + l) * nsite + ((size_t)z * a.ly + y) * a.lx + x] = double(v);
    }
}

template <template <int, bool> class K>
struct Dummy;

hipError_t launch_layout3(int kind, int mode, int walls, const Lb3Layout &a, hipStream_t st) {
  const dim3 grid((a.lx + 63) / 64, a.ly, a.lz), block(64);
#define LB3_LAYOUT(KERN)                                                                                  \
  if (mode == MODE_F64) {                                                                                 \
    if (walls) hipLaunchKernelGGL((KERN<MODE_F64, true>), grid, block, 0, st, a);                         \
    else hipLaunchKernelGGL((KERN<MODE_F64, false>), grid, block, 0, st, a);                              \
  } else {                                                                                                \
    if (walls) hipLaunchKernelGGL((KERN<MODE_F32, true>), grid, block, 0, st, a);                         \
    else hipLaunchKernelGGL((KERN<MODE_F32, false>), grid, block, 0, st, a);                              \
  }
  switch (kind) {
    case 0: LB3_LAYOUT(init3_kernel) break;
    case 1: LB3_LAYOUT(restore3_kernel) break;
    case 2: LB3_LAYOUT(checkpoint3_kernel) break;
    default: return hipErrorInvalidValue;
  }
#undef LB3_LAYOUT
  return hipGetLastError();
}

}  // namespace lb355
