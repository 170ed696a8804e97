// Two time steps per launch: temporal blocking of the fused step, one wave per workgroup.
//
// A launch reads the post-collision populations f*(t - 1) from HBM, advances every site
// through steps t and t + 1, and writes f*(t + 1): the intermediate f*(t) never leaves the
// chip, so the populations cross HBM once per two steps.  The per-site arithmetic is the
// single-step kernel's, operation for operation (same expressions, same order, the
// intermediate rounded to the storage format exactly as a store and a load would round it),
// so the result is bitwise that of two single steps.
//
// Work decomposition: a wave owns a strip of 54 output columns and a segment of rows, and
// its 64 lanes cover the strip plus 5 columns on each side (lane i is column x0 - 5 + i).
// The first step (L1) is valid on lanes 2..61 (its force needs psi two columns away), the
// pull of the second step (L2) on lanes 3..60, and L2's force on lanes 5..58, the 54
// output columns.  The wave marches its segment row by row (up, or down in odd segments; the
// offsets below are for the upward march and change sign downward); in the iteration of lead
// row r:
//   (a) psi(t), rho(t) of row r (from the pulled populations of r, loaded three iterations
//       earlier into a register FIFO) into the L1 ring;
//   (b) L1 update of row r - 2 (force from the L1 ring, collision) -> f*(t) of that row,
//       rounded as the storage rounds, into the L2 input ring (three rows, in LDS);
//   (c) L2 pull of row r - 3 from the input ring (neighbouring lanes and rows; bounce-back
//       from the same site), its psi(t+1), rho(t+1) into the L2 ring, the pulled values
//       into a second register FIFO;
//   (d) L2 update of row r - 5 (force from the L2 ring, collision) and the store of f*(t+1).
// The wave is alone in its workgroup, so no barrier is needed: its own LDS writes and reads
// are ordered.  Columns beyond the strip are computed twice (by the neighbouring wave too)
// and rows beyond the segment ends are recomputed by the neighbouring segments: the cost of
// keeping f*(t) on chip.

#pragma once

#include <type_traits>

#include "lb_step.hpp"

namespace lb355 {

constexpr int kStrip2 = 54;  // output columns per wave
constexpr int kPad2 = 5;     // lanes left of the first output column

// LDS of one two-step workgroup, sized so that eight fit in the 160 KB of a compute unit in FP32
// and BF16 (two waves per SIMD), four in FP64 (one wave per SIMD, whose 512 registers, 256 of
// them accumulation registers, hold the FP64 register FIFOs).  Rings of psi (five rows) and
// rho (four rows) for both steps: rows of 64 entries laid end to end with two spare entries at
// each end, so a lane's neighbours two columns away fall on the adjacent row's edge lanes (only
// lanes whose results are discarded read them).  The input ring of the second step keeps each
// row of f*(t) only as long as its planes are pulled: planes 0, 1, 3 (pulled in place) and 4, 7,
// 8 (pulled from the row above) for two rows, planes 2, 5, 6 (pulled from the row below) for
// three; a plane row has 64 entries and the pull's neighbouring lane wraps round (again only for
// discarded lanes).
constexpr int kRing2Psi = 5 * 64 + 4, kRing2Rho = 4 * 64 + 4, kIn2Rows = 21;
inline size_t step2_lds_bytes(int mode, int ns) {
  const size_t r = mode == MODE_F64 ? 8 : 4;
  return (2 * kRing2Psi + 2 * kRing2Rho + kIn2Rows * 64) * (size_t)ns * r;
}

// Plane row of the input ring holding plane l of f*(t) at row r, for a wave marching in
// direction dir (see step2_lds_bytes): the planes pulled from the row behind the march are kept
// one row longer.
__device__ inline int in2_row(int l, int r, int dir) {
  // group of the plane: 0 {0, 1, 3} two slots; 1 {2, 5, 6} (pulled from the row below) and
  // 2 {4, 7, 8} (from the row above): three slots for the one behind the march, two for the other
  const int g = (l == 0 || l == 1 || l == 3) ? 0 : ((l == 2 || l == 5 || l == 6) ? 1 : 2);
  const int pos = (l == 0 || l == 2 || l == 4) ? 0 : ((l == 1 || l == 5 || l == 7) ? 1 : 2);
  const int n1 = dir > 0 ? 3 : 2;
  const int base = g == 0 ? 0 : (g == 1 ? 6 : 6 + 3 * n1);
  const int ns = g == 0 ? 2 : (g == 1 ? n1 : 5 - n1);
  const int slot = ((r % ns) + ns) % ns;
  return base + slot * 3 + pos;
}

template <int MODE, int NS, bool WALLS, int STP>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(MODE == MODE_F64 ? 1 : 2))) void step2_kernel(StepArgs a) {
  using C = Codec<MODE>;
  using R = typename C::R;
  using S = typename C::S;
  using L = typename C::L;
  using V = Vec<R, NS>;
  V *ring1 = reinterpret_cast<V *>(lb_smem);  // psi(t): row slot k, lane j at entry 64 k + 2 + j
  V *rho1 = ring1 + kRing2Psi;                // rho(t), four row slots
  V *ring2 = rho1 + kRing2Rho;                // psi(t+1)
  V *rho2 = ring2 + kRing2Psi;                // rho(t+1)
  V *inr = rho2 + kRing2Rho;                  // f*(t): [21 plane rows][64]

  const int lx = a.lx, ly = a.ly;
  const uint32_t site_b = (uint32_t)(NS * sizeof(S));
  const uint32_t plane_b = (uint32_t)a.pitch * site_b;
  const uint32_t row_b = 9u * plane_b;
  const uint32_t buf_b = 9u * (uint32_t)a.plane * site_b;
  const int nstrip = (int)gridDim.x / a.nseg;
  const int logical = xcd_remap(blockIdx.x, gridDim.x);
  const int seg = logical / nstrip;
  const int strip = logical - seg * nstrip;
  const int lane = threadIdx.x;
  const int x0 = strip * kStrip2;
  const int yA = seg * a.sy, yB = min(yA + a.sy, ly);


  // this lane's column (wrapped onto the lattice) and whether it stores an output column
  const int xs = x0 - kPad2 + lane;
  const int xc = ((xs % lx) + lx) % lx;
  const bool out_lane = lane >= kPad2 && lane < kPad2 + kStrip2 && xs < lx;
  const LaneCols pcc = {(uint32_t)xc * site_b, (uint32_t)wrapi(xc - 1, lx) * site_b,
                        (uint32_t)wrapi(xc + 1, lx) * site_b};

  uint32_t tseed1 = 0, tseed2 = 0;
  if constexpr (MODE == MODE_BF16SR) {
    const uint32_t t0 = launch_step_index<MODE>(a.t_step, a.t_base);
    tseed1 = uni(mix32(t0 * 0x9e3779b9u + 0x632be5abu));
    tseed2 = uni(mix32((t0 + 1u) * 0x9e3779b9u + 0x632be5abu));
  }

  R K1[NS], K2[NS], K4[NS], K5[NS], K8[NS], tau[NS], om[NS], rref[NS], psiw[NS], rhow[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    K1[s] = R(a.K[s][0]);
    K2[s] = R(a.K[s][1]);
    K4[s] = R(2.0 * a.K[s][2]);
    K5[s] = R(a.K[s][3]);
    K8[s] = R(2.0 * a.K[s][4]);
    tau[s] = R(a.tau[s]);
    om[s] = R(a.omega[s]);
    psiw[s] = R(a.psi_w[s]);
    rhow[s] = R(a.rho_w[s]);
    rref[s] = R(a.rho_ref[s]);
  }
  const R T1 = R(a.T[0]), T2 = R(a.T[1]);
  const R gx = R(a.body[0]), gy = R(a.body[1]);
  const R psi0 = R(a.psi0), nirho0 = R(-a.irho0);

  auto slot5 = [](int r) { return (int)uni((uint32_t)(((r % 5) + 5) % 5)); };
  auto slot4 = [](int r) { return (int)uni((uint32_t)(((r % 4) + 4) % 4)); };

  // psi and rho of a site from its pulled (decoded) populations, as the single-step ring does
  auto site_ring = [&](V *ps_row, V *rh_row, int r, const R (&f)[NS][9]) {
    V ps, rh;
    if (!row_fluid<WALLS>(r, ly)) {
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        ps.v[s] = psiw[s];
        rh.v[s] = rhow[s];
      }
    } else {
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        rh.v[s] = rref[s] + sum9(f[s]);
        ps.v[s] = psi0 * (R(1) - C::expo(rh.v[s] * nirho0));
      }
    }
    ps_row[lane + 2] = ps;
    if (NS == 2) rh_row[lane + 2] = rh;
  };

  // Force, velocity shift and collision of row y (the single-step update, expression for
  // expression): f = the site's pulled populations (decoded), psi rows y-2..y+2 and rho (or
  // psi) rows y-1..y+1 of the ring.  Writes the post-collision deviations to fsa, including the
  // moving walls' momentum on the populations they reflect.
  auto update = [&](int y, const R (&f)[NS][9], V *const *prow, V *const *xrow, R (&fsa)[NS][9]) {
    R drho[NS], rho[NS], jx[NS], jy[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      drho[s] = sum9(f[s]);
      rho[s] = rref[s] + drho[s];
      jx[s] = (f[s][1] + f[s][5] + f[s][8]) - (f[s][3] + f[s][6] + f[s][7]);
      jy[s] = (f[s][2] + f[s][5] + f[s][6]) - (f[s][4] + f[s][7] + f[s][8]);
    }
#define PS2(dx, dy) (prow[(dy) + 2][lane + 2 + (dx)])
    const V pc = PS2(0, 0);
    const V e1 = PS2(1, 0), w1 = PS2(-1, 0), n1 = PS2(0, 1), s1 = PS2(0, -1);
    const V ne = PS2(1, 1), sw = PS2(-1, -1), se = PS2(1, -1), nw = PS2(-1, 1);
    const V e2 = PS2(2, 0), w2 = PS2(-2, 0), n2 = PS2(0, 2), s2 = PS2(0, -2);
    const V qa = PS2(2, 1), qA = PS2(-2, -1), qb = PS2(2, -1), qB = PS2(-2, 1);
    const V qc = PS2(1, 2), qC = PS2(-1, -2), qd = PS2(1, -2), qD = PS2(-1, 2);
    const V d8a = PS2(2, 2), d8A = PS2(-2, -2), d8b = PS2(2, -2), d8B = PS2(-2, 2);
#undef PS2
    R Fx[NS], Fy[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const R dE = e1.v[s] - w1.v[s], dN = n1.v[s] - s1.v[s];
      const R dd1 = ne.v[s] - sw.v[s], dd2 = se.v[s] - nw.v[s];
      const R d4x = e2.v[s] - w2.v[s], d4y = n2.v[s] - s2.v[s];
      const R da = qa.v[s] - qA.v[s], db = qb.v[s] - qB.v[s];
      const R dc = qc.v[s] - qC.v[s], dd = qd.v[s] - qD.v[s];
      const R ea = d8a.v[s] - d8A.v[s], eb = d8b.v[s] - d8B.v[s];
      const R sx = fmadd(K1[s], dE, fmadd(K2[s], dd1 + dd2, fmadd(K4[s], d4x,
                   fmadd(K5[s], R(2) * (da + db) + (dc + dd), K8[s] * (ea + eb)))));
      const R sy = fmadd(K1[s], dN, fmadd(K2[s], dd1 - dd2, fmadd(K4[s], d4y,
                   fmadd(K5[s], (da - db) + R(2) * (dc - dd), K8[s] * (ea - eb)))));
      Fx[s] = fmadd(-pc.v[s], sx, rho[s] * gx);
      Fy[s] = fmadd(-pc.v[s], sy, rho[s] * gy);
    }
    if (NS == 2) {
#define XR2(dx, dy) (xrow[(dy) + 1][lane + 2 + (dx)])
      const V c0 = XR2(0, 0);
      const V xe = XR2(1, 0), xw = XR2(-1, 0), xn = XR2(0, 1), xs2 = XR2(0, -1);
      const V xne = XR2(1, 1), xsw = XR2(-1, -1), xse = XR2(1, -1), xnw = XR2(-1, 1);
#undef XR2
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int o = 1 - s;
        const R t1 = xne.v[o] - xsw.v[o], t2 = xse.v[o] - xnw.v[o];
        const R cx = fmadd(T1, xe.v[o] - xw.v[o], T2 * (t1 + t2));
        const R cy = fmadd(T1, xn.v[o] - xs2.v[o], T2 * (t1 - t2));
        Fx[s] = fmadd(-c0.v[s], cx, Fx[s]);
        Fy[s] = fmadd(-c0.v[s], cy, Fy[s]);
      }
    }
    R nux = jx[0] * om[0], nuy = jy[0] * om[0], den = rho[0] * om[0];
#pragma unroll
    for (int s = 1; s < NS; ++s) {
      nux = fmadd(jx[s], om[s], nux);
      nuy = fmadd(jy[s], om[s], nuy);
      den = fmadd(rho[s], om[s], den);
    }
    const R iden = C::rcp(den);
    const R upx = nux * iden, upy = nuy * iden;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const R ir = C::rcp(rho[s]);
      const R ux = fmadd(tau[s] * Fx[s], ir, upx);
      const R uy = fmadd(tau[s] * Fy[s], ir, upy);
      const R m15 = R(-1.5) * fmadd(ux, ux, uy * uy);
      const R r9 = rho[s] * R(1.0 / 9.0), r36 = rho[s] * R(1.0 / 36.0);
      const R b9 = fmadd(r9, m15, drho[s] * R(1.0 / 9.0)), b36 = fmadd(r36, m15, drho[s] * R(1.0 / 36.0));
      const R o = om[s];
      auto relax = [o](R fl, R b, R r, R cu) { return fmadd(o, fmadd(r, cu * fmadd(R(4.5), cu, R(3)), b) - fl, fl); };
      R (&fs)[9] = fsa[s];
      fs[1] = relax(f[s][1], b9, r9, ux);
      fs[3] = relax(f[s][3], b9, r9, -ux);
      fs[2] = relax(f[s][2], b9, r9, uy);
      fs[4] = relax(f[s][4], b9, r9, -uy);
      fs[5] = relax(f[s][5], b36, r36, ux + uy);
      fs[7] = relax(f[s][7], b36, r36, -(ux + uy));
      fs[6] = relax(f[s][6], b36, r36, uy - ux);
      fs[8] = relax(f[s][8], b36, r36, -(uy - ux));
      fs[0] = drho[s] - ((((fs[1] + fs[2]) + (fs[3] + fs[4])) + ((fs[5] + fs[6]) + (fs[7] + fs[8]))));
    }
    if (WALLS && a.moving) {
      if (y == 0) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          fsa[s][7] += R(a.wall_mom[0][s]);
          fsa[s][8] -= R(a.wall_mom[0][s]);
        }
      }
      if (y == ly - 1) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          fsa[s][6] += R(a.wall_mom[1][s]);
          fsa[s][5] -= R(a.wall_mom[1][s]);
        }
      }
    }
  };

  // The value a store of v (species s, plane l) followed by a load returns: the storage's
  // rounding of the intermediate step, bit for bit.
  auto stored = [&](R v, int s, int l, uint32_t hs) -> R {
    if constexpr (MODE == MODE_BF16SR) {
      const uint32_t rnd = mix32(hs + (uint32_t)l * 0x9e3779b9u);
      const uint32_t h = C::round_sr(v, s == 0 ? (rnd & 0xffffu) : (rnd >> 16)) & 0xffffu;
      return C::decode(h);
    } else if constexpr (MODE == MODE_BF16) {
      return C::decode(C::encode(v));
    } else {
      return v;
    }
  };

  // The march, for each direction as its own code: odd segments march down, so two neighbouring
  // segments pull their shared lead rows at the same time (both at their start or both at their
  // end) and L2 serves the second pull.  The direction is a compile-time constant of each copy:
  // as a run-time value it costs the registers that the march cannot spare.
  auto march = [&](auto dirc) {
    constexpr int dir = decltype(dirc)::value;
    auto inrow = [&](int l, int r) { return inr + (int)uni((uint32_t)in2_row(l, r, dir)) * 64; };

    // Register FIFO of pulled f(t) rows (6 rows: lead row r + 3 in flight ... row r - 2 held for
    // its L1 update) and of pulled f(t+1) rows (3 rows: r - 3 .. r - 5).
    constexpr int D1 = 6, D2 = 3;
    L B1[D1][NS][9];
    R B2[D2][NS][9];
    // lead rows of the segment's iterations: yA - 5 .. yB + 4, in march order from rstart
    const int rlo = yA - 5, rhi = yB + 4;
    const int rstart = dir > 0 ? rlo : rhi;
    auto in_range = [](int v, int lo, int hi) { return v >= lo && v <= hi; };
    auto load_row = [&](int r, L (&dstb)[NS][9]) {
      const RowOffs pr = row_pull<WALLS>(lead_row<WALLS>(r, ly), ly, row_b);
      load_pull<C, NS>(a.src, buf_b, plane_b, pcc, pr, dstb);
    };
#pragma unroll
    for (int m = 0; m < 3; ++m) load_row(rstart + dir * m, B1[m]);

    const int niter = rhi - rlo + 1;
    auto iteration = [&](const int r_in, L (&FL)[NS][9], const L (&FR)[NS][9], const L (&FU)[NS][9],
                         R (&P2)[NS][9], const R (&P2old)[NS][9]) {
      const int r = (int)uni((uint32_t)r_in);
      // issue the loads of lead row r + 3
      if (in_range(r + 3 * dir, rlo, rhi)) load_row(r + 3 * dir, FL);

      // (a) psi(t), rho(t) of lead row r
      {
        R f[NS][9];
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
          for (int l = 0; l < 9; ++l) f[s][l] = C::dec(FR[s][l], s);
        site_ring(ring1 + slot5(r) * 64, rho1 + slot4(r) * 64, r, f);
      }

      // (b) L1 update of row r - 2 -> the input ring
      const int u1 = r - 2 * dir;
      if (in_range(u1, yA - 3, yB + 2) && row_fluid<WALLS>(u1, ly)) {
        R f[NS][9];
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
          for (int l = 0; l < 9; ++l) f[s][l] = C::dec(FU[s][l], s);
        V *prow[5];
        V *xrow[3];
#pragma unroll
        for (int k = 0; k < 5; ++k) prow[k] = ring1 + slot5(u1 - 2 + k) * 64;
#pragma unroll
        for (int k = 0; k < 3; ++k)
          xrow[k] = a.cross_psi ? ring1 + slot5(u1 - 1 + k) * 64 : rho1 + slot4(u1 - 1 + k) * 64;
        R fsa[NS][9];
        update(u1, f, prow, xrow, fsa);
        const int yw = WALLS ? u1 : wrapi(u1, ly);
        uint32_t hs = 0;
        if constexpr (MODE == MODE_BF16SR) hs = mix32((uint32_t)(yw * lx + xc) ^ tseed1);
#pragma unroll
        for (int l = 0; l < 9; ++l) {
          V v;
#pragma unroll
          for (int s = 0; s < NS; ++s) v.v[s] = stored(fsa[s][l], s, l, hs);
          inrow(l, u1)[lane] = v;
        }
      }

      // (c) L2 pull of row r - 3 from the input ring; psi(t+1), rho(t+1) into the L2 ring
      const int p2 = r - 3 * dir;
      if (in_range(p2, yA - 2, yB + 1)) {
        if (row_fluid<WALLS>(p2, ly)) {
          const bool lo = WALLS && p2 == 0, hi = WALLS && p2 == ly - 1;
          const int lm = (lane - 1) & 63, lp = (lane + 1) & 63;  // pull from x - 1 / x + 1
          V g[9];
          g[0] = inrow(0, p2)[lane];
          g[1] = inrow(1, p2)[lm];
          g[3] = inrow(3, p2)[lp];
          // c_y = +1 from the row below, or reflected off the wall below (planes 4, 7, 8 in place)
          g[2] = lo ? inrow(4, p2)[lane] : inrow(2, p2 - 1)[lane];
          g[5] = lo ? inrow(7, p2)[lane] : inrow(5, p2 - 1)[lm];
          g[6] = lo ? inrow(8, p2)[lane] : inrow(6, p2 - 1)[lp];
          // c_y = -1 from the row above, or reflected off the wall above (planes 2, 5, 6 in place)
          g[4] = hi ? inrow(2, p2)[lane] : inrow(4, p2 + 1)[lane];
          g[7] = hi ? inrow(5, p2)[lane] : inrow(7, p2 + 1)[lp];
          g[8] = hi ? inrow(6, p2)[lane] : inrow(8, p2 + 1)[lm];
#pragma unroll
          for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int l = 0; l < 9; ++l) P2[s][l] = g[l].v[s];
        }
        site_ring(ring2 + slot5(p2) * 64, rho2 + slot4(p2) * 64, p2, P2);
      }

      // (d) L2 update of row r - 5 and the store of f*(t+1)
      const int u2 = r - 5 * dir;
      if (in_range(u2, yA, yB - 1)) {
        V *prow[5];
        V *xrow[3];
#pragma unroll
        for (int k = 0; k < 5; ++k) prow[k] = ring2 + slot5(u2 - 2 + k) * 64;
#pragma unroll
        for (int k = 0; k < 3; ++k)
          xrow[k] = a.cross_psi ? ring2 + slot5(u2 - 1 + k) * 64 : rho2 + slot4(u2 - 1 + k) * 64;
        R fsa[NS][9];
        update(u2, P2old, prow, xrow, fsa);
        if (out_lane) {
          const Rsrc rd = make_rsrc(a.dst, buf_b);
          const uint32_t rb0 = (uint32_t)u2 * row_b;
          const uint32_t sto = (uint32_t)xc * site_b;
          if constexpr (MODE == MODE_BF16SR) {
            const uint32_t hs = mix32((uint32_t)(u2 * lx + xc) ^ tseed2);
#pragma unroll
            for (int l = 0; l < 9; ++l) {
              const uint32_t rnd = mix32(hs + (uint32_t)l * 0x9e3779b9u);
              if (NS == 2) C::template bstore2_sr<STP>(rd, sto, uni(rb0 + (uint32_t)l * plane_b), fsa[0][l], fsa[NS - 1][l], rnd);
              else C::template bstore_sr<STP>(rd, sto, uni(rb0 + (uint32_t)l * plane_b), fsa[0][l], rnd);
            }
          } else {
#pragma unroll
            for (int l = 0; l < 9; ++l) {
              if (NS == 2) C::template bstore2<STP>(rd, sto, uni(rb0 + (uint32_t)l * plane_b), fsa[0][l], fsa[NS - 1][l]);
              else C::template bstore<STP>(rd, sto, uni(rb0 + (uint32_t)l * plane_b), fsa[0][l]);
            }
          }
        }
      }
    };

    // Rows: lead row r = rstart + dir i lives in B1[i mod 6]; the pulled f(t+1) of row p2 = r - 3 dir
    // in B2[i mod 3] (its update, three iterations later, reads B2[(i + 0) mod 3] again).
    for (int i0 = 0; i0 < niter; i0 += 6) {
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        if (i0 + k < niter) {
          iteration(rstart + dir * (i0 + k), B1[(k + 3) % D1], B1[k % D1], B1[(k + 4) % D1], B2[k % D2],
                    B2[(k + 1) % D2]);
        }
      }
    }
  };
  if (seg & 1) march(std::integral_constant<int, -1>{});
  else march(std::integral_constant<int, 1>{});
}

}  // namespace lb355
