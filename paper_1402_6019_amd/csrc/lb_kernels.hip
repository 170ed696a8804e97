// Device kernels of the two-belt pseudopotential D2Q9 lattice Boltzmann step (gfx950).
//
// One launch of step_kernel performs one full time step of eq. (LB) for every site:
//   pull streaming (with halfway bounce-back at channel walls)  ->  moments rho_s, j_s
//   ->  psi_s = psi0 (1 - exp(-rho_s / rho0))  ->  eq. (FORCE) two-belt force, A-B repulsion,
//   body force  ->  velocity shift u_eq,s = u' + tau_s F_s / rho_s  ->  BGK collision
//   ->  store of the post-collision populations (unshifted; the next step pulls them).
//
// Layout in HBM: populations as planes [species][l][y][pitch], x fastest (SoA), so every
// load and store of a wavefront touches 64 consecutive elements of one row.
//
// Work decomposition: a workgroup owns a strip of tx columns (one thread per column) and a
// segment of sy rows, and marches down its rows.  The force at row y needs psi at rows
// y-2..y+2 and columns x-2..x+2, so the workgroup keeps a six-row ring of psi_s (and rho_s
// for the A-B term) for its tx + 4 columns in LDS: each iteration computes the leading row
// r = y + 2 of the ring (the pulled moments of tx + 4 sites), synchronises once, then
// updates row y from the ring.  Interior columns are computed once per row; only the two
// halo columns on each side and four extra rows per segment are recomputed by neighbours.
// Six ring slots make one barrier per row sufficient: the slot written in iteration r+1 is
// never among the five slots read in iteration r.
//
// Workgroups are dispatched round-robin over the eight XCDs; xcd_remap() gives each XCD a
// contiguous range of (strip, segment) tiles, segments fastest, so the halo rows shared by
// consecutive segments are re-read from that XCD's own L2.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "lb_internal.hpp"
#include "lb_tables.hpp"

namespace lb355 {

extern __shared__ __attribute__((aligned(16))) unsigned char lb_smem[];

// ---------------------------------------------------------------------------------------
// Storage codecs.  Populations are read and written through raw buffer instructions: the
// buffer descriptor (one per species, SGPRs) holds the base address, the row and plane
// offset is a uniform SGPR and only the column byte offset lives in a VGPR, so a load or
// store costs no vector address arithmetic.  Each species' nine planes must span < 4 GiB.
// ---------------------------------------------------------------------------------------

using Rsrc = __amdgpu_buffer_rsrc_t;
using u32x2 = unsigned int __attribute__((ext_vector_type(2)));

// Base addresses and row offsets are uniform by construction (they depend only on the
// workgroup and the row index); readfirstlane states that to the compiler, which otherwise
// may keep them in VGPRs and wrap every buffer access in a per-lane loop.
__device__ inline uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ inline Rsrc make_rsrc(const void *p, uint32_t bytes) {
  const uint64_t u = reinterpret_cast<uint64_t>(p);
  const uint64_t b = ((uint64_t)uni((uint32_t)(u >> 32)) << 32) | uni((uint32_t)u);
  return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void *>(b), (short)0, (int)uni(bytes), 0x00020000);
}

template <int MODE> struct Codec;

// Every storage mode holds deviations d_l = f_l - W_l rho_ref from the rest equilibrium of a
// per-species reference density.  load/store (layout kernels) convert to and from f; the
// step works on deviations directly (bload/bstore), which costs nothing and keeps the
// rounding of each stored value relative to |d_l| instead of |f_l|.
template <> struct Codec<MODE_F64> {
  using S = double;
  using R = double;
  __device__ static R load(const S *p, R wref) { return *p + wref; }
  __device__ static void store(S *p, R v, R wref) { *p = v - wref; }
  __device__ static R bload(Rsrc r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  }
  __device__ static void bstore(Rsrc r, uint32_t voff, uint32_t soff, R v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 0);
  }
  __device__ static R expo(R v) { return exp(v); }
  __device__ static R rcp(R v) { return 1.0 / v; }
};

template <> struct Codec<MODE_F32> {
  using S = float;
  using R = float;
  __device__ static R load(const S *p, R wref) { return *p + wref; }
  __device__ static void store(S *p, R v, R wref) { *p = v - wref; }
  __device__ static R bload(Rsrc r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
  }
  __device__ static void bstore(Rsrc r, uint32_t voff, uint32_t soff, R v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, voff, soff, 0);
  }
  __device__ static R expo(R v) { return __expf(v); }
  __device__ static R rcp(R v) { return __builtin_amdgcn_rcpf(v); }  // 1 ulp
};

// BF16: stored value = bf16(d_l), arithmetic in FP32.
template <> struct Codec<MODE_BF16> {
  using S = uint16_t;
  using R = float;
  __device__ static R decode(uint32_t h) { return __uint_as_float(h << 16); }
  __device__ static uint16_t encode(R v) {
    const uint32_t b = __float_as_uint(v);
    // round to nearest even; NaN stays NaN
    const uint32_t r = (b & 0x7f800000u) == 0x7f800000u && (b & 0x007fffffu) ? (b | 0x00400000u)
                                                                              : b + 0x7fffu + ((b >> 16) & 1u);
    return uint16_t(r >> 16);
  }
  __device__ static R load(const S *p, R wref) { return decode(*p) + wref; }
  __device__ static void store(S *p, R v, R wref) { *p = encode(v - wref); }
  __device__ static R bload(Rsrc r, uint32_t voff, uint32_t soff) {
    return decode(__builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0));
  }
  __device__ static void bstore(Rsrc r, uint32_t voff, uint32_t soff, R v) {
    __builtin_amdgcn_raw_buffer_store_b16(encode(v), r, voff, soff, 0);
  }
  __device__ static R expo(R v) { return __expf(v); }
  __device__ static R rcp(R v) { return __builtin_amdgcn_rcpf(v); }  // 1 ulp
};

template <typename R, int NS>
struct alignas(sizeof(R) * NS) Vec {
  R v[NS];
};

__device__ inline int xcd_remap(int b, int nb) {
  constexpr int NX = 8;
  const int q = nb / NX, r = nb % NX;
  const int xcd = b % NX, k = b / NX;
  return (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + k;
}

__device__ inline int wrapi(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

// Where the nine populations pulled into one site come from:
//   f_l(x, y) = f*_l(x - c_l, y - c_l), or f*_opp(l)(x, y) when (x - c_l, y - c_l) is a wall.
// A load address is  species base (buffer descriptor) + row offset (SGPR) + lane offset
// (VGPR).  The lane offset folds in the plane, l * plane_bytes + column bytes of x - c_lx,
// and is fixed for the whole kernel; only the three row offsets change from row to row.
struct RowOffs {
  uint32_t m, o, p;  // byte offsets of rows y-1, y, y+1 (or y where reflected)
  bool lo, hi;       // row y-1 / y+1 is a wall
};

struct LaneOffs {
  uint32_t ld[9];  // l * plane_bytes + bytes of column x - c_lx
  uint32_t bb[4];  // (5..8) * plane_bytes + bytes of column x: reflected sources
};

__device__ inline LaneOffs lane_offsets(int x, int xm, int xp, uint32_t es, uint32_t plane_b) {
  LaneOffs o;
  const uint32_t xb = (uint32_t)x * es, xmb = (uint32_t)xm * es, xpb = (uint32_t)xp * es;
  const uint32_t colb[9] = {xb, xmb, xb, xpb, xb, xmb, xpb, xpb, xmb};  // column of x - c_lx
#pragma unroll
  for (int l = 0; l < 9; ++l) o.ld[l] = (uint32_t)l * plane_b + colb[l];
#pragma unroll
  for (int k = 0; k < 4; ++k) o.bb[k] = (uint32_t)(5 + k) * plane_b + xb;
  return o;
}

template <class C, int NS>
__device__ inline void load_pull(const void *base, uint32_t spec_b, const LaneOffs &lo_, const RowOffs &r,
                                 typename C::R (&f)[NS][9]) {
  // source of each population: (lane offset, row offset)
  uint32_t vo[9], so[9];
  vo[0] = lo_.ld[0]; so[0] = r.o;
  vo[1] = lo_.ld[1]; so[1] = r.o;
  vo[3] = lo_.ld[3]; so[3] = r.o;
  // c_y = +1 populations come from the row below, or bounce back off the wall below
  vo[2] = r.lo ? lo_.ld[4] : lo_.ld[2]; so[2] = r.lo ? r.o : r.m;  // reflected: plane 4 at x
  vo[5] = r.lo ? lo_.bb[2] : lo_.ld[5]; so[5] = r.lo ? r.o : r.m;  // plane 7 at x
  vo[6] = r.lo ? lo_.bb[3] : lo_.ld[6]; so[6] = r.lo ? r.o : r.m;  // plane 8 at x
  // c_y = -1 populations come from the row above, or bounce back off the wall above
  vo[4] = r.hi ? lo_.ld[2] : lo_.ld[4]; so[4] = r.hi ? r.o : r.p;  // plane 2 at x
  vo[7] = r.hi ? lo_.bb[0] : lo_.ld[7]; so[7] = r.hi ? r.o : r.p;  // plane 5 at x
  vo[8] = r.hi ? lo_.bb[1] : lo_.ld[8]; so[8] = r.hi ? r.o : r.p;  // plane 6 at x
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const Rsrc rs = make_rsrc(static_cast<const char *>(base) + (uint64_t)s * spec_b, spec_b);
#pragma unroll
    for (int l = 0; l < 9; ++l)  // W_opp(l) = W_l: a reflected deviation is still a deviation
      f[s][l] = C::bload(rs, vo[l], uni(so[l]));
  }
}

// Row geometry: fluid rows wrap (periodic) or are bounded by walls (channel).
template <bool WALLS>
__device__ inline bool row_fluid(int r, int ly) { return !WALLS || (r >= 0 && r < ly); }

template <bool WALLS>
__device__ inline int lead_row(int r, int ly) { return WALLS ? min(max(r, 0), ly - 1) : r; }

template <bool WALLS>
__device__ inline RowOffs row_pull(int r, int ly, uint32_t pitch_b) {
  RowOffs o;
  const int rw = WALLS ? r : wrapi(r, ly);
  o.lo = WALLS && rw == 0;
  o.hi = WALLS && rw == ly - 1;
  o.o = (uint32_t)rw * pitch_b;
  o.m = o.lo ? o.o : (uint32_t)wrapi(rw - 1, ly) * pitch_b;
  o.p = o.hi ? o.o : (uint32_t)wrapi(rw + 1, ly) * pitch_b;
  return o;
}

template <typename R>
__device__ inline R sum9(const R f[9]) {
  R r = f[0];
#pragma unroll
  for (int l = 1; l < 9; ++l) r += f[l];
  return r;
}

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------------------------------
// Fused step
// ---------------------------------------------------------------------------------------
//
// Software pipeline of one row iteration r (lead row r, output row y = r - 2):
//   1. psi, rho of lead row r from populations already in registers  -> LDS ring slot
//   2. issue the loads of output row y (stage 2 input)
//   3. issue the loads of lead row r + 1 (next iteration's step 1)
//   4. barrier
//   5. force + collision of row y from the ring and the stage-2 registers, store
// so the memory latency of both load batches overlaps the arithmetic of steps 1 and 5.

template <int MODE, int NS, bool WALLS, int WHAT>
__global__ __launch_bounds__(256) void step_kernel(StepArgs a) {
  using C = Codec<MODE>;
  using R = typename C::R;
  using S = typename C::S;
  using V = Vec<R, NS>;
  constexpr bool STORE = (WHAT == WHAT_STEP || WHAT == WHAT_STEP_REDUCE);
  constexpr bool REDUCE = (WHAT == WHAT_STEP_REDUCE || WHAT == WHAT_OBSERVE);

  const int TX = blockDim.x;
  const int W4 = TX + 4;
  V *psi_ring = reinterpret_cast<V *>(lb_smem);      // [6][W4]
  V *rho_ring = psi_ring + 6 * W4;                   // [6][W4] (two species only)
  __shared__ double red_lds[4][RED_N];

  const int logical = xcd_remap(blockIdx.x, gridDim.x);
  const int strip = logical / a.nseg;
  const int seg = logical - strip * a.nseg;
  const int lx = a.lx, ly = a.ly;
  const uint32_t pitch_b = (uint32_t)a.pitch * sizeof(S);
  const uint32_t plane_b = (uint32_t)a.plane * (uint32_t)sizeof(S);
  const int x0 = strip * TX;
  const int w = min(TX, lx - x0);
  const int yA = seg * a.sy;
  const int yB = min(yA + a.sy, ly);
  const int tid = threadIdx.x;

  // Per-species constants in the arithmetic type.
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
  const void *const src = a.src;
  void *const dst = a.dst;

  // Interior column of this thread (ring slot tid + 2) and, for threads 0..3, one halo
  // column (ring slots 0, 1, w+2, w+3 = columns x0-2, x0-1, x0+w, x0+w+1).
  const bool col_ok = tid < w;
  const int xc = x0 + (col_ok ? tid : 0);
  const uint32_t es = (uint32_t)sizeof(S);
  const uint32_t spec_b = 9u * plane_b;
  const LaneOffs pcc = lane_offsets(xc, wrapi(xc - 1, lx), wrapi(xc + 1, lx), es, plane_b);
  // Store column: lanes past a ragged strip's end write into the row padding (the row
  // pitch is a multiple of the widest strip), which no kernel ever reads.
  uint32_t sto[9];
#pragma unroll
  for (int l = 0; l < 9; ++l) sto[l] = (uint32_t)l * plane_b + (uint32_t)(x0 + tid) * es;
  const bool halo = tid < 4;
  const int hslot = tid < 2 ? tid : w + tid;
  const int xh = wrapi(x0 - 2 + hslot, lx);
  const int xhm = wrapi(xh - 1, lx), xhp = wrapi(xh + 1, lx);

  double acc[RED_N];
#pragma unroll
  for (int k = 0; k < RED_N; ++k) acc[k] = 0.0;

  // Stage 1: psi_s and rho_s of lead row r into ring slot `slot` (interior and halo columns)
  // from the pulled populations A (interior column) and H (halo column).
  auto ring_row = [&](int slot, int r, const R (&A)[NS][9], const R (&H)[NS][9]) {
    V *prow = psi_ring + slot * W4;
    V *rrow = rho_ring + slot * W4;
    if (!row_fluid<WALLS>(r, ly)) {
      V ps, rh;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        ps.v[s] = psiw[s];
        rh.v[s] = rhow[s];
      }
      if (col_ok) {
        prow[tid + 2] = ps;
        if (NS == 2) rrow[tid + 2] = rh;
      }
      if (halo) {
        prow[hslot] = ps;
        if (NS == 2) rrow[hslot] = rh;
      }
    } else {
      if (col_ok) {
        V ps, rh;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          rh.v[s] = rref[s] + sum9(A[s]);
          ps.v[s] = psi0 * (R(1) - C::expo(rh.v[s] * nirho0));
        }
        prow[tid + 2] = ps;
        if (NS == 2) rrow[tid + 2] = rh;
      }
      if (halo) {
        V ps, rh;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          rh.v[s] = rref[s] + sum9(H[s]);
          ps.v[s] = psi0 * (R(1) - C::expo(rh.v[s] * nirho0));
        }
        prow[hslot] = ps;
        if (NS == 2) rrow[hslot] = rh;
      }
    }
  };

  // Register FIFO of pulled populations.  The populations of lead row y+3, loaded in the
  // iteration of output row y to compute its psi, are the stage-2 input of row y+3 three
  // iterations later; four row buffers (the main loop is unrolled by four so their roles
  // rotate statically) mean every population is loaded once per step, one iteration of
  // arithmetic ahead of its first use.
  R B[4][NS][9];
  R FH[NS][9];  // halo column of the lead row (threads 0..3)

  // Prologue: ring rows yA-2 .. yA+2, loads one row ahead.  Rows yA, yA+1, yA+2 stay in
  // B[1], B[2], B[3] for the first three output rows.
  {
    R PH[2][NS][9];
    constexpr int buf_of[5] = {0, 3, 1, 2, 3};
    {
      const RowOffs pr = row_pull<WALLS>(lead_row<WALLS>(yA - 2, ly), ly, pitch_b);
      if (halo) load_pull<C, NS>(src, spec_b, lane_offsets(xh, xhm, xhp, es, plane_b), pr, PH[0]);
      load_pull<C, NS>(src, spec_b, pcc, pr, B[buf_of[0]]);
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      if (k < 4) {
        const RowOffs pr = row_pull<WALLS>(lead_row<WALLS>(yA - 1 + k, ly), ly, pitch_b);
        if (halo)
          load_pull<C, NS>(src, spec_b, lane_offsets(xh, xhm, xhp, es, plane_b), pr, PH[(k + 1) & 1]);
        load_pull<C, NS>(src, spec_b, pcc, pr, B[buf_of[k + 1]]);
      }
      ring_row(k, yA - 2 + k, B[buf_of[k]], PH[k & 1]);
    }
  }

  // One output row y: issue the loads of lead row y+3 (halo batch first: it is the only one
  // under a lane condition) -> barrier -> force + collision of row y from the ring and the
  // FIFO, store -> ring row y+3.  Stores carry no condition either: lanes past a ragged
  // strip's end write into the row padding.  The ring slot written last, (y+3) mod 6, is
  // not among the rows y-2..y+2 that slower waves may still be reading.
  auto step_row = [&](const int y_in, const int lead_slot_in, R (&FL)[NS][9], const R (&f)[NS][9]) {
    // the row index is uniform; saying so keeps every row and plane offset in SGPRs
    const int y = (int)uni((uint32_t)y_in);
    const int lead_slot = (int)uni((uint32_t)lead_slot_in);
    const int rlead = y + 3;
    const uint32_t rb0 = (uint32_t)y * pitch_b;
    {
      const RowOffs pr = row_pull<WALLS>(lead_row<WALLS>(rlead, ly), ly, pitch_b);
      if (halo) load_pull<C, NS>(src, spec_b, lane_offsets(xh, xhm, xhp, es, plane_b), pr, FH);
      load_pull<C, NS>(src, spec_b, pcc, pr, FL);
    }

    __syncthreads();

    // ---- update row y ---------------------------------------------------------------------
    // ring rows y-2 .. y+2 occupy slots lead_slot-5 .. lead_slot-1 (mod 6)
    R drho[NS], rho[NS], jx[NS], jy[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      drho[s] = sum9(f[s]);
      rho[s] = rref[s] + drho[s];
      jx[s] = (f[s][1] + f[s][5] + f[s][8]) - (f[s][3] + f[s][6] + f[s][7]);
      jy[s] = (f[s][2] + f[s][5] + f[s][6]) - (f[s][4] + f[s][7] + f[s][8]);
    }

    // ring rows y-2 .. y+2
    const V *rows[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      int sl = lead_slot + 1 + k;
      sl = sl >= 6 ? sl - 6 : sl;
      sl = sl >= 6 ? sl - 6 : sl;
      rows[k] = psi_ring + sl * W4 + tid + 2;
    }
#define PS(dx, dy) (rows[(dy) + 2][(dx)])
    const V pc = PS(0, 0);
    const V e1 = PS(1, 0), w1 = PS(-1, 0), n1 = PS(0, 1), s1 = PS(0, -1);
    const V ne = PS(1, 1), sw = PS(-1, -1), se = PS(1, -1), nw = PS(-1, 1);
    const V e2 = PS(2, 0), w2 = PS(-2, 0), n2 = PS(0, 2), s2 = PS(0, -2);
    const V qa = PS(2, 1), qA = PS(-2, -1), qb = PS(2, -1), qB = PS(-2, 1);
    const V qc = PS(1, 2), qC = PS(-1, -2), qd = PS(1, -2), qD = PS(-1, 2);
    const V d8a = PS(2, 2), d8A = PS(-2, -2), d8b = PS(2, -2), d8B = PS(-2, 2);
#undef PS
    R Fx[NS], Fy[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      // eq. (FORCE) regrouped into antisymmetric pairs over one link of each +-c pair:
      // sum_l K(q_l) psi(x + c_l) c_l = sum_half K(q) c (psi(x + c) - psi(x - c)).
      const R dE = e1.v[s] - w1.v[s], dN = n1.v[s] - s1.v[s];
      const R dd1 = ne.v[s] - sw.v[s], dd2 = se.v[s] - nw.v[s];
      const R d4x = e2.v[s] - w2.v[s], d4y = n2.v[s] - s2.v[s];
      const R da = qa.v[s] - qA.v[s], db = qb.v[s] - qB.v[s];
      const R dc = qc.v[s] - qC.v[s], dd = qd.v[s] - qD.v[s];
      const R ea = d8a.v[s] - d8A.v[s], eb = d8b.v[s] - d8B.v[s];
      const R sx = K1[s] * dE + K2[s] * (dd1 + dd2) + K4[s] * d4x + K5[s] * (R(2) * (da + db) + (dc + dd)) +
                   K8[s] * (ea + eb);
      const R sy = K1[s] * dN + K2[s] * (dd1 - dd2) + K4[s] * d4y + K5[s] * ((da - db) + R(2) * (dc - dd)) +
                   K8[s] * (ea - eb);
      Fx[s] = -pc.v[s] * sx + rho[s] * gx;
      Fy[s] = -pc.v[s] * sy + rho[s] * gy;
    }
    if (NS == 2) {
      // A-B repulsion over the first belt between the densities (or psi) of both species.
      const V *xr[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const V *base = a.cross_psi ? psi_ring : rho_ring;
        int sl = lead_slot + 2 + k;
        sl = sl >= 6 ? sl - 6 : sl;
        sl = sl >= 6 ? sl - 6 : sl;
        xr[k] = base + sl * W4 + tid + 2;
      }
#define XR(dx, dy) (xr[(dy) + 1][(dx)])
      const V c0 = XR(0, 0);
      const V xe = XR(1, 0), xw = XR(-1, 0), xn = XR(0, 1), xs = XR(0, -1);
      const V xne = XR(1, 1), xsw = XR(-1, -1), xse = XR(1, -1), xnw = XR(-1, 1);
#undef XR
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int o = 1 - s;
        const R t1 = xne.v[o] - xsw.v[o], t2 = xse.v[o] - xnw.v[o];
        const R cx = T1 * (xe.v[o] - xw.v[o]) + T2 * (t1 + t2);
        const R cy = T1 * (xn.v[o] - xs.v[o]) + T2 * (t1 - t2);
        Fx[s] -= c0.v[s] * cx;
        Fy[s] -= c0.v[s] * cy;
      }
    }

    // common velocity u' = sum_s (j_s / tau_s) / sum_s (rho_s / tau_s)
    R nux = jx[0] * om[0], nuy = jy[0] * om[0], den = rho[0] * om[0];
#pragma unroll
    for (int s = 1; s < NS; ++s) {
      nux += jx[s] * om[s];
      nuy += jy[s] * om[s];
      den += rho[s] * om[s];
    }
    const R iden = C::rcp(den);
    const R upx = nux * iden, upy = nuy * iden;

    if (WHAT == WHAT_MOMENTS && col_ok) {
      R sr = rho[0], mx = jx[0] + R(0.5) * Fx[0], my = jy[0] + R(0.5) * Fy[0];
#pragma unroll
      for (int s = 1; s < NS; ++s) {
        sr += rho[s];
        mx += jx[s] + R(0.5) * Fx[s];
        my += jy[s] + R(0.5) * Fy[s];
      }
      const size_t site = (size_t)y * lx + xc;
      const size_t nsite = (size_t)lx * ly;
      if (a.out_rho) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          if (a.out_f32) static_cast<float *>(a.out_rho)[s * nsite + site] = float(rho[s]);
          else static_cast<double *>(a.out_rho)[s * nsite + site] = double(rho[s]);
        }
      }
      if (a.out_u) {
        const R ux = mx / sr, uy = my / sr;
        if (a.out_f32) {
          static_cast<float *>(a.out_u)[site] = float(ux);
          static_cast<float *>(a.out_u)[nsite + site] = float(uy);
        } else {
          static_cast<double *>(a.out_u)[site] = double(ux);
          static_cast<double *>(a.out_u)[nsite + site] = double(uy);
        }
      }
    }

    if (WHAT != WHAT_MOMENTS) {
    double wb = 0.0, wt = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const R ir = C::rcp(rho[s]);
      const R ux = upx + tau[s] * Fx[s] * ir;
      const R uy = upy + tau[s] * Fy[s] * ir;
      // Deviation form of f^eq_l = W_l rho (1 + 3 cu + 9/2 cu^2 - 3/2 u.u):
      //   f^eq_l - W_l rho_ref = W_l (drho - 3/2 rho u.u) + W_l rho cu (3 + 9/2 cu)
      const R m15 = R(-1.5) * (ux * ux + uy * uy);
      const R r9 = rho[s] * R(1.0 / 9.0), r36 = rho[s] * R(1.0 / 36.0);
      const R b9 = drho[s] * R(1.0 / 9.0) + r9 * m15, b36 = drho[s] * R(1.0 / 36.0) + r36 * m15;
      const R o = om[s];
      R fs[9];
      {
        const R cu = ux;
        fs[1] = f[s][1] + o * (b9 + r9 * (cu * (R(3) + R(4.5) * cu)) - f[s][1]);
        fs[3] = f[s][3] + o * (b9 - r9 * (cu * (R(3) - R(4.5) * cu)) - f[s][3]);
      }
      {
        const R cu = uy;
        fs[2] = f[s][2] + o * (b9 + r9 * (cu * (R(3) + R(4.5) * cu)) - f[s][2]);
        fs[4] = f[s][4] + o * (b9 - r9 * (cu * (R(3) - R(4.5) * cu)) - f[s][4]);
      }
      {
        const R cu = ux + uy;
        fs[5] = f[s][5] + o * (b36 + r36 * (cu * (R(3) + R(4.5) * cu)) - f[s][5]);
        fs[7] = f[s][7] + o * (b36 - r36 * (cu * (R(3) - R(4.5) * cu)) - f[s][7]);
      }
      {
        const R cu = uy - ux;
        fs[6] = f[s][6] + o * (b36 + r36 * (cu * (R(3) + R(4.5) * cu)) - f[s][6]);
        fs[8] = f[s][8] + o * (b36 - r36 * (cu * (R(3) - R(4.5) * cu)) - f[s][8]);
      }
      // rest population closes the mass balance exactly: d*_0 = drho - sum_{l>0} d*_l
      fs[0] = drho[s] - ((((fs[1] + fs[2]) + (fs[3] + fs[4])) + ((fs[5] + fs[6]) + (fs[7] + fs[8]))));

      if (STORE) {
#pragma unroll
        for (int l = 0; l < 9; ++l)
          C::bstore(make_rsrc(static_cast<char *>(dst) + (uint64_t)s * spec_b, spec_b), sto[l], uni(rb0), fs[l]);
      }
      if (REDUCE && WALLS && col_ok) {
        if (y == 0) wb += 2.0 * (double(fs[8]) - double(fs[7]));
        if (y == ly - 1) wt += 2.0 * (double(fs[5]) - double(fs[6]));
      }
    }

    if (REDUCE && col_ok) {
      R sr = rho[0], mx = jx[0] + R(0.5) * Fx[0];
      bool bad = !(rho[0] > R(0) && rho[0] < R(INFINITY));
#pragma unroll
      for (int s = 1; s < NS; ++s) {
        sr += rho[s];
        mx += jx[s] + R(0.5) * Fx[s];
        bad = bad || !(rho[s] > R(0) && rho[s] < R(INFINITY));
      }
      acc[RED_MASS0] += double(rho[0]);
      if (NS == 2) acc[RED_MASS1] += double(rho[NS - 1]);
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        acc[RED_PX] += double(jx[s]);
        acc[RED_PY] += double(jy[s]);
      }
      acc[RED_WBOT] += wb;
      acc[RED_WTOP] += wt;
      acc[RED_FLOW] += double(mx / sr);
      acc[RED_BAD] += bad ? 1.0 : 0.0;
    }
    }  // WHAT != WHAT_MOMENTS

    // ---- ring row y + 3 from the loads issued at the top of this iteration -----------------
    ring_row(lead_slot, y + 3, FL, FH);
  };

  int lead_slot = 5;
  auto next_slot = [](int sl) { return sl == 5 ? 0 : sl + 1; };
  for (int y = yA; y < yB;) {
    step_row(y, lead_slot, B[0], B[1]);
    lead_slot = next_slot(lead_slot);
    if (++y >= yB) break;
    step_row(y, lead_slot, B[1], B[2]);
    lead_slot = next_slot(lead_slot);
    if (++y >= yB) break;
    step_row(y, lead_slot, B[2], B[3]);
    lead_slot = next_slot(lead_slot);
    if (++y >= yB) break;
    step_row(y, lead_slot, B[3], B[0]);
    lead_slot = next_slot(lead_slot);
    ++y;
  }

  if (REDUCE) {
    const int lane = tid & 63, wv = tid >> 6;
#pragma unroll
    for (int k = 0; k < RED_N; ++k) {
      const double v = wave_sum(acc[k]);
      if (lane == 0) red_lds[wv][k] = v;
    }
    __syncthreads();
    if (tid < RED_N) {
      double v = 0.0;
      const int nw = (TX + 63) >> 6;
      for (int i = 0; i < nw; ++i) v += red_lds[i][tid];
      a.partials[(size_t)blockIdx.x * RED_N + tid] = v;
    }
  }
}

// Second reduction pass: fixed-order sum of the per-workgroup partials (deterministic).
__global__ __launch_bounds__(256) void reduce_kernel(const double *partials, int nblocks, double *totals, double *acc,
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

// ---------------------------------------------------------------------------------------
// Layout kernels: canonical pre-collision f(t) <-> internal post-collision buffer.
// Streaming with bounce-back is a permutation of population slots:
//   f_l(x) = g_l(x - c_l) if x - c_l is fluid, else g_opp(l)(x)
// and its inverse g_l(z) = f_l(z + c_l) if z + c_l is fluid, else f_opp(l)(z).
// ---------------------------------------------------------------------------------------

template <int MODE, bool WALLS>
__global__ void init_kernel(LayoutArgs a) {  // in: rho [ns][ly][lx] (FP64)
  using C = Codec<MODE>;
  using S = typename C::S;
  using R = typename C::R;
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= a.lx) return;
  const double *rho = static_cast<const double *>(a.in);
  S *out = static_cast<S *>(a.out);
  const size_t nsite = (size_t)a.lx * a.ly;
  for (int s = 0; s < a.ns; ++s)
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
      const double v = WD2Q9[l] * rho[s * nsite + (size_t)zy * a.lx + zx];
      C::store(out + (long long)(s * 9 + l) * a.plane + (long long)y * a.pitch + x, R(v),
               R(WD2Q9[l] * a.rho_ref[s]));
    }
}

template <int MODE, bool WALLS>
__global__ void restore_kernel(LayoutArgs a) {  // in: canonical f [ns][9][ly][lx] (FP64)
  using C = Codec<MODE>;
  using S = typename C::S;
  using R = typename C::R;
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= a.lx) return;
  const double *f = static_cast<const double *>(a.in);
  S *out = static_cast<S *>(a.out);
  const size_t nsite = (size_t)a.lx * a.ly;
  for (int s = 0; s < a.ns; ++s)
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
      const double v = f[(size_t)(s * 9 + lsrc) * nsite + (size_t)zy * a.lx + zx];
      C::store(out + (long long)(s * 9 + l) * a.plane + (long long)y * a.pitch + x, R(v),
               R(WD2Q9[l] * a.rho_ref[s]));
    }
}

template <int MODE, bool WALLS>
__global__ void checkpoint_kernel(LayoutArgs a) {  // out: canonical f [ns][9][ly][lx] (FP64)
  using C = Codec<MODE>;
  using S = typename C::S;
  using R = typename C::R;
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= a.lx) return;
  const S *in = static_cast<const S *>(a.in);
  double *f = static_cast<double *>(a.out);
  const size_t nsite = (size_t)a.lx * a.ly;
  for (int s = 0; s < a.ns; ++s)
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
      const R v = C::load(in + (long long)(s * 9 + lsrc) * a.plane + (long long)zy * a.pitch + zx,
                          R(WD2Q9[lsrc] * a.rho_ref[s]));
      f[(size_t)(s * 9 + l) * nsite + (size_t)y * a.lx + x] = double(v);
    }
}

// ---------------------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------------------

size_t step_lds_bytes(int mode, int ns, int tx) {
  const size_t r = mode == MODE_F64 ? 8 : 4;
  return 6 * (size_t)(tx + 4) * ns * r * (ns == 2 ? 2 : 1);
}

template <int MODE, int NS, bool WALLS>
static hipError_t launch_step_t(int what, int tx, int nb, const StepArgs &a, hipStream_t st) {
  const size_t lds = step_lds_bytes(MODE, NS, tx);
  switch (what) {
    case WHAT_STEP: hipLaunchKernelGGL((step_kernel<MODE, NS, WALLS, WHAT_STEP>), dim3(nb), dim3(tx), lds, st, a); break;
    case WHAT_STEP_REDUCE:
      hipLaunchKernelGGL((step_kernel<MODE, NS, WALLS, WHAT_STEP_REDUCE>), dim3(nb), dim3(tx), lds, st, a);
      break;
    case WHAT_MOMENTS:
      hipLaunchKernelGGL((step_kernel<MODE, NS, WALLS, WHAT_MOMENTS>), dim3(nb), dim3(tx), lds, st, a);
      break;
    case WHAT_OBSERVE:
      hipLaunchKernelGGL((step_kernel<MODE, NS, WALLS, WHAT_OBSERVE>), dim3(nb), dim3(tx), lds, st, a);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int MODE>
static hipError_t launch_step_m(int ns, int walls, int what, int tx, int nb, const StepArgs &a, hipStream_t st) {
  if (ns == 1) return walls ? launch_step_t<MODE, 1, true>(what, tx, nb, a, st) : launch_step_t<MODE, 1, false>(what, tx, nb, a, st);
  return walls ? launch_step_t<MODE, 2, true>(what, tx, nb, a, st) : launch_step_t<MODE, 2, false>(what, tx, nb, a, st);
}

hipError_t launch_step(int mode, int ns, int walls, int what, int tx, int nb, const StepArgs &a, hipStream_t st) {
  switch (mode) {
    case MODE_F64: return launch_step_m<MODE_F64>(ns, walls, what, tx, nb, a, st);
    case MODE_F32: return launch_step_m<MODE_F32>(ns, walls, what, tx, nb, a, st);
    case MODE_BF16: return launch_step_m<MODE_BF16>(ns, walls, what, tx, nb, a, st);
  }
  return hipErrorInvalidValue;
}

__global__ void fill_kernel(double *p, double v, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
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

#undef LB_LAYOUT_LAUNCHER

}  // namespace lb355
