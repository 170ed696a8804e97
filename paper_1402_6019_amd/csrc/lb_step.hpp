#pragma once
// Device code of the fused step: storage codecs, the row-marching tile (run_tile), the
// single-lattice and batched step kernels, and templated launchers.  Included by one
// translation unit per storage mode (lb_step_f64.hip, lb_step_f32.hip, lb_step_bf16.hip), which
// instantiate the kernels of that mode, and by lb_kernels.hip for the codecs of the layout
// kernels.
//
// Device kernels of the two-belt pseudopotential D2Q9 lattice Boltzmann step (gfx950).
//
// One launch of step_kernel performs one full time step of eq. (LB) for every site:
//   pull streaming (with halfway bounce-back at channel walls)  ->  moments rho_s, j_s
//   ->  psi_s = psi0 (1 - exp(-rho_s / rho0))  ->  eq. (FORCE) two-belt force, A-B repulsion,
//   body force  ->  velocity shift u_eq,s = u' + tau_s F_s / rho_s  ->  BGK collision
//   ->  store of the post-collision populations (unshifted; the next step pulls them).
//
// Layout in HBM: [y][l][pitch][species], species fastest: the two species' populations of a
// site are adjacent, so one load or store instruction moves both (8 bytes per lane in FP32),
// and the nine plane rows of a lattice row follow each other as one contiguous run.
//
// Work decomposition: a workgroup owns a strip of tx columns (one thread per column) and a
// segment of sy rows, and marches through its rows, down for even segments and up for odd
// ones.  The force at row y needs psi at rows y-2..y+2 and columns x-2..x+2, so the
// workgroup keeps a six-row ring of psi_s (and rho_s for the A-B term) for its tx + 4
// columns in LDS: each iteration synchronises once, computes the leading row of the ring
// (the pulled moments of tx + 4 sites), then updates row y from the ring.  Interior columns
// are computed once per row; only the two halo columns on each side and three rows beyond
// each end of a segment are pulled again by the neighbours.  Six ring slots make one
// barrier per row sufficient: the slot written in iteration r+1 is never among the five
// slots read in iteration r.
//
// Those overlaps are read twice from L2 but once from memory when both readers run on the
// same XCD at the same time.  Workgroups are dispatched round-robin over the eight XCDs;
// xcd_remap() gives each XCD a contiguous range of tiles in band-major order (all strips
// of a band of rows, then the next band), so horizontal neighbours share an XCD and reach
// the same row together; and since neighbouring segments march in opposite directions,
// both reach their common boundary rows at the same time (together at the start, or
// together at the end of the march).

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "lb_internal.hpp"
#include "lb_tables.hpp"

namespace lb355 {

extern __shared__ __attribute__((aligned(16))) unsigned char lb_smem[];

// ---------------------------------------------------------------------------------------
// Storage codecs.  Populations are read and written through raw buffer instructions: the
// buffer descriptor (SGPRs) holds the base address, the row and plane offset is a uniform
// SGPR and only the column byte offset lives in a VGPR, so a load or store costs no vector
// address arithmetic.  A population buffer must span < 4 GiB.
// ---------------------------------------------------------------------------------------

using Rsrc = __amdgpu_buffer_rsrc_t;
using u32x2 = unsigned int __attribute__((ext_vector_type(2)));
using u32x4 = unsigned int __attribute__((ext_vector_type(4)));

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

// Cache policy of the population stores (the buffer instructions' cache-policy operand):
// SC1 (bit 4) gives the store device scope, so it is written through the XCD's L2 instead
// of staying there dirty, which leaves L2 to the rows and halo columns that neighbouring
// workgroups read twice; NT (bit 1) additionally marks it non-temporal, so it does not
// displace the next step's reads from the Infinity Cache.  That pays when both population
// buffers together exceed the Infinity Cache (the state cannot stay resident anyway) and
// costs when they fit (the next step would have read them from it), so the host picks the
// kernel instantiation per lattice from the footprint.  The streaming instantiation also
// issues its tail rows' loads without a branch (see the lead-row loads in run_tile).
constexpr int kStoreWriteThrough = 16;      // SC1
constexpr int kStoreStreaming = 16 | 2;     // SC1 | NT

// Every storage mode holds deviations d_l = f_l - W_l rho_ref from the rest equilibrium of a
// per-species reference density.  load/store (layout kernels) convert to and from the canonical
// FP64 f with wref = W_l rho_ref in FP64 arithmetic, so a checkpoint (f = d + wref) restores to
// the stored d exactly whenever the sum is exact in FP64 (for FP32, |d| >= 2^-29 |wref|; BF16
// always); the step works on deviations directly (bload/bstore), which costs nothing and keeps
// the rounding of each stored value relative to |d_l| instead of |f_l|.
// L is the type a pulled population is held in between its load and its use (the register
// FIFO of the step); dec(v, s) turns it into species s's value in the arithmetic type.
template <> struct Codec<MODE_F64> {
  using S = double;
  using R = double;
  using L = double;
  __device__ static R dec(L v, int) { return v; }
  __device__ static double load(const S *p, double wref) { return *p + wref; }
  __device__ static void store(S *p, double v, double wref) { *p = v - wref; }
  __device__ static L bload(Rsrc r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  }
  template <int AUX>
  __device__ static void bstore(Rsrc r, uint32_t voff, uint32_t soff, R v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, AUX);
  }
  // both species of a site (adjacent in memory) in one access
  __device__ static void bload2(Rsrc r, uint32_t voff, uint32_t soff, L &a, L &b) {
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
    a = __builtin_bit_cast(double, u32x2{v[0], v[1]});
    b = __builtin_bit_cast(double, u32x2{v[2], v[3]});
  }
  template <int AUX>
  __device__ static void bstore2(Rsrc r, uint32_t voff, uint32_t soff, R a, R b) {
    const u32x2 ua = __builtin_bit_cast(u32x2, a), ub = __builtin_bit_cast(u32x2, b);
    __builtin_amdgcn_raw_buffer_store_b128(u32x4{ua.x, ua.y, ub.x, ub.y}, r, voff, soff, AUX);
  }
  __device__ static R expo(R v) { return exp(v); }
  __device__ static R rcp(R v) { return 1.0 / v; }
};

template <> struct Codec<MODE_F32> {
  using S = float;
  using R = float;
  using L = float;
  __device__ static R dec(L v, int) { return v; }
  __device__ static double load(const S *p, double wref) { return double(*p) + wref; }
  __device__ static void store(S *p, double v, double wref) { *p = float(v - wref); }
  __device__ static L bload(Rsrc r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
  }
  template <int AUX>
  __device__ static void bstore(Rsrc r, uint32_t voff, uint32_t soff, R v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, voff, soff, AUX);
  }
  __device__ static void bload2(Rsrc r, uint32_t voff, uint32_t soff, L &a, L &b) {
    // element access by index: with .x / .y and bit_cast this compiler narrowed the load
    // to its first dword
    const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
    a = __uint_as_float(v[0]);
    b = __uint_as_float(v[1]);
  }
  template <int AUX>
  __device__ static void bstore2(Rsrc r, uint32_t voff, uint32_t soff, R a, R b) {
    __builtin_amdgcn_raw_buffer_store_b64(u32x2{__builtin_bit_cast(unsigned int, a), __builtin_bit_cast(unsigned int, b)},
                                          r, voff, soff, AUX);
  }
  __device__ static R expo(R v) { return __expf(v); }
  __device__ static R rcp(R v) { return __builtin_amdgcn_rcpf(v); }  // 1 ulp
};

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// Integer hash for the stochastic rounding bits (a 32-bit xorshift-multiply mixer; any
// well-mixed function of (site, plane, step) would do).
__device__ inline uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}
typedef float f32x2 __attribute__((ext_vector_type(2)));

// BF16: stored value = bf16(d_l), arithmetic in FP32.
// BF16: the FIFO keeps the raw 32-bit word that holds both species of a site (one register
// for the pair: bload2 hands the same word to both), decoded where used: species 0 is the low
// half, species 1 the high half.
template <> struct Codec<MODE_BF16> {
  static constexpr bool kStochastic = false;
  using S = uint16_t;
  using R = float;
  using L = uint32_t;
  __device__ static R dec(L v, int s) { return __uint_as_float(s == 0 ? v << 16 : v & 0xffff0000u); }
  __device__ static R decode(uint32_t h) { return __uint_as_float(h << 16); }
  // the hardware conversion (v_cvt_pk_bf16_f32): round to nearest even, NaN stays NaN
  __device__ static uint16_t encode(R v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }
  __device__ static double load(const S *p, double wref) { return double(decode(*p)) + wref; }
  __device__ static void store(S *p, double v, double wref) { *p = encode(float(v - wref)); }
  __device__ static L bload(Rsrc r, uint32_t voff, uint32_t soff) {
    return __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0);
  }
  template <int AUX>
  __device__ static void bstore(Rsrc r, uint32_t voff, uint32_t soff, R v) {
    __builtin_amdgcn_raw_buffer_store_b16(encode(v), r, voff, soff, AUX);
  }
  __device__ static R expo(R v) { return __expf(v); }
  __device__ static R rcp(R v) { return __builtin_amdgcn_rcpf(v); }  // 1 ulp
  __device__ static void bload2(Rsrc r, uint32_t voff, uint32_t soff, L &a, L &b) {
    const uint32_t v = __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
    a = v;
    b = v;
  }
  template <int AUX>
  __device__ static void bstore2(Rsrc r, uint32_t voff, uint32_t soff, R a, R b) {
    // both values in one packed conversion
    const f32x2 v = {a, b};
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2)), r, voff,
                                          soff, AUX);
  }
};

// BF16 with stochastic rounding at the population stores: 16 random bits are added to the 16
// bits that BF16 drops before they are cut off, so a value rounds away from zero with
// probability equal to the dropped fraction.  The rounding is unbiased, so increments far
// below one BF16 step (a weak body force) still accumulate on average.
// The hardware conversion (v_cvt_sr_bf16_f32) does this: it adds the high 16 bits of its random
// operand to the float's bits and keeps the top 16, (bits + r16) >> 16 for a finite value (checked
// bit for bit against that expression over a million random values and random bits); a value
// rounds away from zero with probability equal to the dropped fraction, and infinities stay
// infinite.
template <> struct Codec<MODE_BF16SR> : Codec<MODE_BF16> {
  static constexpr bool kStochastic = true;
  // bits of bf16(v) rounded with the 16 random bits r16
  __device__ static uint32_t round_sr(float v, uint32_t r16) {
    const bf16x2 z = {};
    return __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_sr_bf16_f32(z, v, r16 << 16, false)) & 0xffffu;
  }
  template <int AUX>
  __device__ static void bstore_sr(Rsrc r, uint32_t voff, uint32_t soff, R v, uint32_t rnd) {
    __builtin_amdgcn_raw_buffer_store_b16((uint16_t)round_sr(v, rnd & 0xffffu), r, voff, soff, AUX);
  }
  // both species in one word: a rounded with the low 16 random bits, b with the high 16
  template <int AUX>
  __device__ static void bstore2_sr(Rsrc r, uint32_t voff, uint32_t soff, R a, R b, uint32_t rnd) {
    bf16x2 w = {};
    w = __builtin_amdgcn_cvt_sr_bf16_f32(w, a, rnd << 16, false);
    w = __builtin_amdgcn_cvt_sr_bf16_f32(w, b, rnd & 0xffff0000u, true);
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, w), r, voff, soff, AUX);
  }
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
// A load address is  buffer base (descriptor) + row and plane offset (SGPR) + column
// offset (VGPR).  Only the column bytes of x, x - 1 and x + 1 live in VGPRs, fixed for the
// whole kernel; the plane and the source row go into the uniform offset.
struct RowOffs {
  uint32_t m, o, p;  // byte offsets of rows y-1, y, y+1 (or y where reflected)
  bool lo, hi;       // row y-1 / y+1 is a wall
};

struct LaneCols {
  uint32_t c, m, p;  // bytes of columns x, x - 1, x + 1 (periodic wrap folded in)
};

template <class C, int NS>
__device__ inline void load_pull(const void *base, uint32_t buf_b, uint32_t plane_b, const LaneCols &col,
                                 const RowOffs &r, typename C::L (&f)[NS][9]) {
  // source of each population: (column offset, row + plane offset)
  const uint32_t P1 = plane_b, P2 = 2 * plane_b, P3 = 3 * plane_b, P4 = 4 * plane_b, P5 = 5 * plane_b,
                 P6 = 6 * plane_b, P7 = 7 * plane_b, P8 = 8 * plane_b;
  uint32_t vo[9], so[9];
  vo[0] = col.c; so[0] = r.o;
  vo[1] = col.m; so[1] = r.o + P1;
  vo[3] = col.p; so[3] = r.o + P3;
  // c_y = +1 populations come from the row below, or bounce back off the wall below
  vo[2] = col.c;                  so[2] = r.lo ? r.o + P4 : r.m + P2;  // reflected: plane 4 at x
  vo[5] = r.lo ? col.c : col.m;   so[5] = r.lo ? r.o + P7 : r.m + P5;  // plane 7 at x
  vo[6] = r.lo ? col.c : col.p;   so[6] = r.lo ? r.o + P8 : r.m + P6;  // plane 8 at x
  // c_y = -1 populations come from the row above, or bounce back off the wall above
  vo[4] = col.c;                  so[4] = r.hi ? r.o + P2 : r.p + P4;  // plane 2 at x
  vo[7] = r.hi ? col.c : col.p;   so[7] = r.hi ? r.o + P5 : r.p + P7;  // plane 5 at x
  vo[8] = r.hi ? col.c : col.m;   so[8] = r.hi ? r.o + P6 : r.p + P8;  // plane 6 at x
  const Rsrc rs = make_rsrc(base, buf_b);
#pragma unroll
  for (int l = 0; l < 9; ++l) {  // W_opp(l) = W_l: a reflected deviation is still a deviation
    if (NS == 2) C::bload2(rs, vo[l], uni(so[l]), f[0][l], f[NS - 1][l]);
    else f[0][l] = C::bload(rs, vo[l], uni(so[l]));
  }
}

// Row geometry: fluid rows wrap (periodic) or are bounded by walls (channel).
template <bool WALLS>
__device__ inline bool row_fluid(int r, int ly) { return !WALLS || (r >= 0 && r < ly); }

template <bool WALLS>
__device__ inline int lead_row(int r, int ly) { return WALLS ? min(max(r, 0), ly - 1) : r; }

template <bool WALLS>
__device__ inline RowOffs row_pull(int r, int ly, uint32_t row_b) {
  RowOffs o;
  const int rw = WALLS ? r : wrapi(r, ly);
  o.lo = WALLS && rw == 0;
  o.hi = WALLS && rw == ly - 1;
  o.o = (uint32_t)rw * row_b;
  o.m = o.lo ? o.o : (uint32_t)wrapi(rw - 1, ly) * row_b;
  o.p = o.hi ? o.o : (uint32_t)wrapi(rw + 1, ly) * row_b;
  return o;
}

// One pulled population (both species) of a halo column: lane offsets (plane and column
// folded in) for the direct and the reflected source, and masks for c_y = +1 / -1 (all ones or 0;
// mask arithmetic instead of a three-way choice, which the compiler would otherwise turn
// into a lookup table in scratch memory).
struct HaloItem {
  uint32_t direct, reflected;
  uint32_t up, dn;
};

__device__ inline HaloItem halo_item(int l, int xh, int lx, uint32_t site_b, uint32_t plane_b) {
  int cx = 0, cy = 0, op = 0;
  switch (l) {  // D2Q9 velocities and opposites
    case 0: cx = 0; cy = 0; op = 0; break;
    case 1: cx = 1; cy = 0; op = 3; break;
    case 2: cx = 0; cy = 1; op = 4; break;
    case 3: cx = -1; cy = 0; op = 1; break;
    case 4: cx = 0; cy = -1; op = 2; break;
    case 5: cx = 1; cy = 1; op = 7; break;
    case 6: cx = -1; cy = 1; op = 8; break;
    case 7: cx = -1; cy = -1; op = 5; break;
    default: cx = 1; cy = -1; op = 6; break;
  }
  HaloItem h;
  h.direct = (uint32_t)l * plane_b + (uint32_t)wrapi(xh - cx, lx) * site_b;
  h.reflected = (uint32_t)op * plane_b + (uint32_t)xh * site_b;
  h.up = cy == 1 ? 0xffffffffu : 0u;
  h.dn = cy == -1 ? 0xffffffffu : 0u;
  return h;
}

// Byte offset of a halo item in lead row r: source row r - c_y, or the item's reflected
// source in row r when that row is a wall.
__device__ inline uint32_t halo_offset(const HaloItem &h, const RowOffs &r) {
  const uint32_t lo = r.lo ? 0xffffffffu : 0u, hi = r.hi ? 0xffffffffu : 0u;
  const uint32_t bb = (h.up & lo) | (h.dn & hi);
  const uint32_t row = r.o ^ ((r.m ^ r.o) & h.up) ^ ((r.p ^ r.o) & h.dn);
  return (bb & (h.reflected + r.o)) | (~bb & (h.direct + row));
}

// Fused multiply-add where the arithmetic asks for one.  Device code is compiled without
// floating-point contraction, so every rounding is fixed by the source: every kernel and
// every unrolled copy of the row update computes bitwise the same result.
__device__ inline double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ inline float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

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
// Software pipeline of one row iteration, output row y (rows named in march order):
//   1. stage the halo items of lead row y+3 (loaded in the previous iteration) in LDS
//   2. issue the loads of lead row y+4 (populations and halo items) into the register FIFO
//   3. barrier
//   4. psi, rho of lead row y+3 from the FIFO (and the staged halo items) -> LDS ring slot
//   5. force + collision of row y from the ring and row y's populations in the FIFO, store
// Every population is loaded once, an iteration before its first use in step 4, and stays in
// the FIFO until its own row is updated, so the loads' latency overlaps steps 3 to 5.

// One tile: strip `strip` (tx = blockDim.x columns) and segment `seg` (a.sy rows) of the
// lattice described by a, read from src and written to dst.  part: this tile's row of
// reduction partials; out0: the output of a pass beside the populations (WHAT_STEP_FIELDS*:
// the reverse step's fields) or of one that stores nothing (WHAT_MOMENTS: rho;
// WHAT_STRESS: the pressure tensor; WHAT_PROFILE: the [64-column block][row][PROF_N] sums);
// out_u: the WHAT_MOMENTS velocity, or the WHAT_STEP_FIELDS* wall-row populations.
template <int MODE, int NS, bool WALLS, int WHAT, int STP>
__device__ __forceinline__ void run_tile(const StepArgs &a, const void *const src, void *const dst, const int strip,
                                         const int seg, double *const part, void *const out0,
                                         void *const out_u, const int out_f32, const uint32_t tstep) {
  using C = Codec<MODE>;
  using R = typename C::R;
  using S = typename C::S;
  using L = typename C::L;
  using V = Vec<R, NS>;
  constexpr bool FIELDS = (WHAT == WHAT_STEP_FIELDS || WHAT == WHAT_STEP_FIELDS32);
  constexpr bool STORE = (WHAT == WHAT_STEP || WHAT == WHAT_STEP_ACCUM || FIELDS);
  constexpr bool REDUCE = (WHAT == WHAT_OBSERVE || WHAT == WHAT_STEP_ACCUM);
  // WHAT_STEP_ACCUM keeps only what stepping averages (wall stress) and the health count,
  // added to this workgroup's own row of running sums; the second pass runs when the host
  // reads them, not every step
  constexpr bool ACCUM = (WHAT == WHAT_STEP_ACCUM);
  constexpr bool PROFILE = (WHAT == WHAT_PROFILE);

  const int TX = blockDim.x;
  const int W4 = TX + 4;
  V *psi_ring = reinterpret_cast<V *>(lb_smem);      // [6][W4]
  V *rho_ring = psi_ring + 6 * W4;                   // [6][W4] (two species only)
  __shared__ double red_lds[4][RED_N];

  const int lx = a.lx, ly = a.ly;
  // Layout [y][l][pitch][species]: site_b bytes per site (both species), plane_b: byte
  // stride between planes l and l+1 of one row, row_b: between rows, buf_b: the buffer.
  const uint32_t site_b = (uint32_t)(NS * sizeof(S));
  const uint32_t pitch_b = (uint32_t)a.pitch * site_b;
  const uint32_t plane_b = pitch_b;
  const uint32_t row_b = 9u * pitch_b;
  const int x0 = strip * TX;
  const int w = min(TX, lx - x0);
  const int yA = seg * a.sy;
  const int yB = min(yA + a.sy, ly);
  // march direction and first output row: rows y0, y0 + dir, ..., through the segment
  const int dir = (seg & 1) ? -1 : 1;
  const int y0 = dir > 0 ? yA : yB - 1;
  // last lead row the march needs (two beyond the segment's far end)
  const int ylast = dir > 0 ? yB + 1 : yA - 2;
  const int tid = threadIdx.x;
  // stochastic rounding: a seed per time step
  uint32_t tseed = 0;
  if constexpr (MODE == MODE_BF16SR) tseed = uni(mix32(tstep * 0x9e3779b9u + 0x632be5abu));

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

  // Interior column of this thread (ring slot tid + 2).
  const bool col_ok = tid < w;
  const int xc = x0 + (col_ok ? tid : 0);
  const uint32_t buf_b = 9u * (uint32_t)a.plane * site_b;
  // A wave whose every lane lies past a ragged strip's last column loads and stores through
  // a zero-length range (loads return zeros, stores are dropped): it moves no bytes, yet
  // takes every barrier of the tile like the others.  Wave 0 always holds column x0.
  const bool wave_idle = (int)uni((uint32_t)(tid & ~63)) >= w;
  const uint32_t ld_b = wave_idle ? 0u : buf_b;
  const LaneCols pcc = {(uint32_t)xc * site_b, (uint32_t)wrapi(xc - 1, lx) * site_b,
                        (uint32_t)wrapi(xc + 1, lx) * site_b};
  // Store column: lanes past a ragged strip's end write into the row padding (the row
  // pitch is a multiple of the widest strip), which no kernel ever reads.
  const uint32_t sto = (uint32_t)(x0 + tid) * site_b;

  // Halo columns x0-2, x0-1, x0+w, x0+w+1 (ring slots 0, 1, w+2, w+3).  Their 4 x 9 pulled
  // sites per lead row ("halo items", item it: column it / 9, plane it % 9, both species in
  // one load) are spread over the workgroup, one per thread (threads past the 36 items
  // re-load item 0, so no load sits under a lane condition); staged in LDS and summed in
  // plane order by one lane per (column, species) in every wave -- the same sum, in the
  // same order, as for an interior column.
  constexpr int NI = 36;
  R *hstage = reinterpret_cast<R *>(psi_ring + (NS == 2 ? 12 : 6) * W4);  // [7][NI][NS]
  const int xhc0 = wrapi(x0 - 2, lx), xhc1 = wrapi(x0 - 1, lx), xhc2 = wrapi(x0 + w, lx),
            xhc3 = wrapi(x0 + w + 1, lx);
  HaloItem hitem;
  {
    const int it = tid < NI ? tid : 0;
    const int hc = it / 9, l = it % 9;
    const int xh = hc == 0 ? xhc0 : (hc == 1 ? xhc1 : (hc == 2 ? xhc2 : xhc3));
    hitem = halo_item(l, xh, lx, site_b, plane_b);
  }

  double acc[RED_N];
#pragma unroll
  for (int k = 0; k < RED_N; ++k) acc[k] = 0.0;

  // Stage 1, interior columns: psi_s and rho_s of lead row r into ring slot `slot` from the
  // pulled populations A of this thread's column.
  auto ring_row = [&](int slot, int r, const L (&A)[NS][9]) {
    if (!col_ok) return;
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
        R a9[9];
#pragma unroll
        for (int l = 0; l < 9; ++l) a9[l] = C::dec(A[s][l], s);
        rh.v[s] = rref[s] + sum9(a9);
        ps.v[s] = psi0 * (R(1) - C::expo(rh.v[s] * nirho0));
      }
    }
    psi_ring[slot * W4 + tid + 2] = ps;
    if (NS == 2) rho_ring[slot * W4 + tid + 2] = rh;
  };

  // Stage 1, halo columns: load (one item per thread), stage into LDS buffer `buf`, and
  // finish (after a barrier) into ring slot `slot`.
  auto halo_load = [&](const RowOffs &r, L (&hv)[2], uint32_t nbytes) {
    const Rsrc rs = make_rsrc(src, nbytes);
    if (NS == 2) C::bload2(rs, halo_offset(hitem, r), 0u, hv[0], hv[1]);
    else hv[0] = C::bload(rs, halo_offset(hitem, r), 0u);
  };
  auto halo_stage = [&](int buf, const L (&hv)[2]) {
    if (tid < NI) {
#pragma unroll
      for (int s = 0; s < NS; ++s) hstage[(buf * NI + tid) * NS + s] = C::dec(hv[s], s);
    }
  };
  auto halo_finish = [&](int buf, int slot, int r) {
    const int lane = tid & 63, wv = tid >> 6, nw = TX >> 6;
    if (lane >= NS) return;
    const int sp = lane;
    const bool fluid = row_fluid<WALLS>(r, ly);
    const R rr = sp == 0 ? rref[0] : rref[NS - 1];
    for (int hc = wv; hc < 4; hc += nw) {
      R rh, ps;
      if (!fluid) {
        rh = sp == 0 ? rhow[0] : rhow[NS - 1];
        ps = sp == 0 ? psiw[0] : psiw[NS - 1];
      } else {
        const R *q = hstage + (buf * NI + hc * 9) * NS + sp;
        R sum = q[0];
#pragma unroll
        for (int l = 1; l < 9; ++l) sum += q[l * NS];
        rh = rr + sum;
        ps = psi0 * (R(1) - C::expo(rh * nirho0));
      }
      const int hsl = hc < 2 ? hc : w + hc;
      reinterpret_cast<R *>(psi_ring + slot * W4 + hsl)[sp] = ps;
      if (NS == 2) reinterpret_cast<R *>(rho_ring + slot * W4 + hsl)[sp] = rh;
    }
  };

  // Register FIFO of pulled populations, D row buffers.  Rows are named in march order below
  // (y + 4 means y + 4 dir); row y0 + m lives in B[m mod D].  The populations of row y+D-1
  // are loaded in the iteration of output row y, turned into psi D-4 iterations later (as
  // ring row y'+3 of output row y' = y+D-4) and are the stage-2 input of their own row D-1
  // iterations after loading: every population is loaded once per step, D-4 full
  // iterations before its first use.  The halo items of a lead row are held in registers
  // for the same D-4 iterations (NHV sets).  D = 5: six or eight rows (two or four
  // iterations of lead, with D a multiple of NHV) measured no faster in any storage mode,
  // FP64 included, where the extra rows cost no occupancy.
  constexpr int D = 5;
  constexpr int NHV = D - 4;
  L B[D][NS][9];
  L HV[NHV][2];

  // Prologue: ring rows y0-2 .. y0+2 (slots 0..4) from B[D-1] (row y0-2), B[D-2] (row y0-1,
  // then reloaded with row y0+D-2) and B[0..2]; rows y0+3 .. y0+D-3 go to B[3..D-3] with
  // their halo items in HV[0..D-6], and row y0+D-2's halo items to HV[D-5].
  {
    L HP[5][2];
    auto load_row = [&](int r, L (&dstb)[NS][9], L (&hv)[2]) {
      const RowOffs pr = row_pull<WALLS>(lead_row<WALLS>(r, ly), ly, row_b);
      load_pull<C, NS>(src, ld_b, plane_b, pcc, pr, dstb);
      halo_load(pr, hv, ld_b);
    };
    load_row(y0 - 2 * dir, B[D - 1], HP[0]);
    load_row(y0 - dir, B[D - 2], HP[1]);
#pragma unroll
    for (int m = 0; m < 3; ++m) load_row(y0 + dir * m, B[m], HP[m + 2]);
#pragma unroll
    for (int m = 3; m <= D - 3; ++m) load_row(y0 + dir * m, B[m], HV[m - 3]);
    ring_row(0, y0 - 2 * dir, B[D - 1]);
    halo_stage(0, HP[0]);
    ring_row(1, y0 - dir, B[D - 2]);
    halo_stage(1, HP[1]);
    load_row(y0 + dir * (D - 2), B[D - 2], HV[D - 5]);
#pragma unroll
    for (int k = 2; k < 5; ++k) {
      ring_row(k, y0 + dir * (k - 2), B[k - 2]);
      halo_stage(k, HP[k]);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 5; ++k) halo_finish(k, k, y0 + dir * (k - 2));
  }

  // One output row y (march order; FIFO roles: FL <- lead row y+D-1, f = row y, FR = lead
  // row y+3, hv: halo items of row y+3 in, of row y+D-1 out):
  //   stage the halo items of lead row y+3 -> issue the loads of lead row y+D-1 -> barrier ->
  //   ring row y+3 (interior and halo) -> force + collision of row y, store.
  // Loads and stores carry no lane or row conditions (lanes past a ragged strip's end store
  // into the row padding), so every wait covers exactly the batch it needs.  The ring slot
  // written last, (y+3) mod 6, is not among the rows y-2..y+2 that slower waves may still
  // read, and the halo staging buffers alternate between iterations.
  auto step_row = [&](const int y_in, const int lead_slot_in, const int hbuf_in, L (&FL)[NS][9],
                      const L (&fraw)[NS][9], const L (&FR)[NS][9], L (&hv)[2]) {
    // the row index is uniform; saying so keeps every row offset in SGPRs
    const int y = (int)uni((uint32_t)y_in);
    const int lead_slot = (int)uni((uint32_t)lead_slot_in);
    const int hbuf = (int)uni((uint32_t)hbuf_in);
    const uint32_t rb0 = (uint32_t)y * row_b;
    halo_stage(hbuf, hv);
    // Lead rows past the last one the segment needs are not fetched; their buffers then feed
    // only ring rows that no output row reads.
    const int rl = y + dir * (D - 1);
    const bool past = dir > 0 ? rl > ylast : rl < ylast;
    if (STP == kStoreStreaming) {
      // Footprint beyond the Infinity Cache: the loads are issued for every row, those of a
      // row past the end through a zero-length buffer range (they return zeros and touch no
      // memory).  With no branch around them the compiler counts outstanding loads exactly
      // and no longer waits for the previous row's stores before the ring row, which pays
      // once HBM serves the traffic; with cache-resident buffers the extra issue costs more.
      const RowOffs pr = row_pull<WALLS>(lead_row<WALLS>(past ? ylast : rl, ly), ly, row_b);
      const uint32_t nb = past ? 0u : ld_b;
      load_pull<C, NS>(src, nb, plane_b, pcc, pr, FL);
      halo_load(pr, hv, nb);
    } else if (!past) {  // uniform branch
      const RowOffs pr = row_pull<WALLS>(lead_row<WALLS>(rl, ly), ly, row_b);
      load_pull<C, NS>(src, ld_b, plane_b, pcc, pr, FL);
      halo_load(pr, hv, ld_b);
    }

    __syncthreads();

    // ---- ring row y + 3 from the loads issued in the previous iteration ----------------------
    // (slot (y+3) mod 6 is not among the rows y-2..y+2 read below; doing it first lets its
    // LDS round trips overlap the update of row y)
    ring_row(lead_slot, y + 3 * dir, FR);
    halo_finish(hbuf, lead_slot, y + 3 * dir);

    // ---- update row y ---------------------------------------------------------------------
    // the ring holds rows y + dir (m - 2), m = 0..4, in slots lead_slot + 1 + m (mod 6): the
    // row at physical offset d is in slot lead_slot + 3 + dir d
    R f[NS][9];
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int l = 0; l < 9; ++l) f[s][l] = C::dec(fraw[s][l], s);
    if constexpr (FIELDS) {
      // the reverse step's inputs, from the pulled (pre-collision) populations of this row, as
      // a checkpoint of the state would give them: f_l = d_l + W_l rho_ref in FP64, then rho,
      // j summed in l order and psi in the adjoint's precision RA
      using RA = typename std::conditional<WHAT == WHAT_STEP_FIELDS, double, float>::type;
      if (col_ok) {
        const size_t site = (size_t)y * lx + xc, nsite = (size_t)lx * ly;
        RA *fl = static_cast<RA *>(out0);
        double *xw = static_cast<double *>(out_u);
        const bool wall_row = WALLS && (y == 0 || y == ly - 1);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          RA r = 0, px = 0, py = 0;
#pragma unroll
          for (int l = 0; l < 9; ++l) {
            const double fv = double(f[s][l]) + WD2Q9[l] * a.rho_ref[s];
            if (wall_row) xw[((size_t)(s * 9 + l) * 2 + (y == 0 ? 0 : 1)) * lx + xc] = fv;
            const RA g = RA(fv);
            r += g;
            px += RA(CXS[l]) * g;
            py += RA(CYS[l]) * g;
          }
          fl[(size_t)(0 * 2 + s) * nsite + site] = r;
          fl[(size_t)(1 * 2 + s) * nsite + site] = RA(a.psi0) * (RA(1) - exp(-r * RA(a.irho0)));
          fl[(size_t)(2 * 2 + s) * nsite + site] = px;
          fl[(size_t)(3 * 2 + s) * nsite + site] = py;
        }
      }
    }
    R drho[NS], rho[NS], jx[NS], jy[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      drho[s] = sum9(f[s]);
      rho[s] = rref[s] + drho[s];
      jx[s] = (f[s][1] + f[s][5] + f[s][8]) - (f[s][3] + f[s][6] + f[s][7]);
      jy[s] = (f[s][2] + f[s][5] + f[s][6]) - (f[s][4] + f[s][7] + f[s][8]);
    }

    // ring rows y-2 .. y+2 (physical order)
    const V *rows[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      int sl = lead_slot + 3 + dir * (k - 2);
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
      const R sx = fmadd(K1[s], dE, fmadd(K2[s], dd1 + dd2, fmadd(K4[s], d4x,
                   fmadd(K5[s], R(2) * (da + db) + (dc + dd), K8[s] * (ea + eb)))));
      const R sy = fmadd(K1[s], dN, fmadd(K2[s], dd1 - dd2, fmadd(K4[s], d4y,
                   fmadd(K5[s], (da - db) + R(2) * (dc - dd), K8[s] * (ea - eb)))));
      Fx[s] = fmadd(-pc.v[s], sx, rho[s] * gx);
      Fy[s] = fmadd(-pc.v[s], sy, rho[s] * gy);
    }
    if (NS == 2) {
      // A-B repulsion over the first belt between the densities (or psi) of both species.
      const V *xr[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const V *base = a.cross_psi ? psi_ring : rho_ring;
        int sl = lead_slot + 3 + dir * (k - 1);
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
        const R cx = fmadd(T1, xe.v[o] - xw.v[o], T2 * (t1 + t2));
        const R cy = fmadd(T1, xn.v[o] - xs.v[o], T2 * (t1 - t2));
        Fx[s] = fmadd(-c0.v[s], cx, Fx[s]);
        Fy[s] = fmadd(-c0.v[s], cy, Fy[s]);
      }
    }

    // common velocity u' = sum_s (j_s / tau_s) / sum_s (rho_s / tau_s)
    R nux = jx[0] * om[0], nuy = jy[0] * om[0], den = rho[0] * om[0];
#pragma unroll
    for (int s = 1; s < NS; ++s) {
      nux = fmadd(jx[s], om[s], nux);
      nuy = fmadd(jy[s], om[s], nuy);
      den = fmadd(rho[s], om[s], den);
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
      if (out0) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          if (out_f32) static_cast<float *>(out0)[s * nsite + site] = float(rho[s]);
          else static_cast<double *>(out0)[s * nsite + site] = double(rho[s]);
        }
      }
      if (out_u) {
        const R ux = mx / sr, uy = my / sr;
        if (out_f32) {
          static_cast<float *>(out_u)[site] = float(ux);
          static_cast<float *>(out_u)[nsite + site] = float(uy);
        } else {
          static_cast<double *>(out_u)[site] = double(ux);
          static_cast<double *>(out_u)[nsite + site] = double(uy);
        }
      }
    }

    if (WHAT == WHAT_STRESS && col_ok) {
      // Pressure tensor of the lattice stress section, per site: sum over species of
      // c_s^2 rho_s delta + sigma^(int)_s + (tau_s - 1/2)^2 F_s F_s / rho_s, plus the A-B pair
      // stress.  sigma^(int) follows Appendix A shell by shell (K(q) = G_1 w(q) + G_2 p(q)):
      //   shells 1, 2: K/2 psi(x) sum psi(x + c) c c
      //   shells 4, 8: K/4 sum [psi(x) psi(x + c) + psi(x - c/2) psi(x + c/2)] c c
      //   shell 5:     K/4 psi(x) sum psi(x + c) c c, plus K/4 (psi(x + c_a) psi(x + c_b) + ...) c c
      //                over the first-belt pairs whose difference is c13, c14, c15 or c16
      double sxx = 0.0, sxy = 0.0, syy = 0.0;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const R k1 = R(a.K[s][0]) * R(0.5), k2 = R(a.K[s][1]) * R(0.5), k4 = R(a.K[s][2]);
        const R k5 = R(a.K[s][3]) * R(0.25), k8 = R(a.K[s][4]);
        const R p0 = pc.v[s];
        const R E = e1.v[s], W = w1.v[s], N = n1.v[s], S = s1.v[s];
        const R NE = ne.v[s], NW = nw.v[s], SE = se.v[s], SW = sw.v[s];
        const R diag = (NE + SW) + (NW + SE), dxy = (NE + SW) - (NW + SE);
        const R d8 = (d8a.v[s] + d8A.v[s]) + (d8b.v[s] + d8B.v[s]), d8xy = (d8a.v[s] + d8A.v[s]) - (d8b.v[s] + d8B.v[s]);
        const R mid8 = R(2) * (NE * SW + NW * SE), mid8xy = R(2) * (NE * SW - NW * SE);
        const R qx = (qa.v[s] + qA.v[s]) + (qb.v[s] + qB.v[s]);  // |c_x| = 2
        const R qy = (qc.v[s] + qC.v[s]) + (qd.v[s] + qD.v[s]);  // |c_y| = 2
        const R qxy = ((qa.v[s] + qA.v[s]) + (qc.v[s] + qC.v[s])) - ((qb.v[s] + qB.v[s]) + (qd.v[s] + qD.v[s]));
        const R e13 = NE * W + E * SW, e14 = NE * S + N * SW, e15 = N * SE + NW * S, e16 = NW * E + W * SE;
        R xx = k1 * p0 * (E + W) + k2 * p0 * diag + k4 * (p0 * (e2.v[s] + w2.v[s]) + R(2) * (E * W)) +
               k8 * (p0 * d8 + mid8) + k5 * (p0 * (R(4) * qx + qy) + (R(4) * (e13 + e16) + (e14 + e15)));
        R yy = k1 * p0 * (N + S) + k2 * p0 * diag + k4 * (p0 * (n2.v[s] + s2.v[s]) + R(2) * (N * S)) +
               k8 * (p0 * d8 + mid8) + k5 * (p0 * (qx + R(4) * qy) + ((e13 + e16) + R(4) * (e14 + e15)));
        R xy = k2 * p0 * dxy + k8 * (p0 * d8xy + mid8xy) + k5 * R(2) * (p0 * qxy + ((e13 + e14) - (e15 + e16)));
        // ideal gas and the discrete forcing correction
        const R cr = (tau[s] - R(0.5)) * (tau[s] - R(0.5)) / rho[s];
        xx += rho[s] * R(1.0 / 3.0) + cr * Fx[s] * Fx[s];
        yy += rho[s] * R(1.0 / 3.0) + cr * Fy[s] * Fy[s];
        xy += cr * Fx[s] * Fy[s];
        sxx += double(xx);
        sxy += double(xy);
        syy += double(yy);
      }
      if (NS == 2) {
        // A-B repulsion: (G_AB / 2) sum_l t(q) [r_A(x) r_B(x + c) + r_B(x) r_A(x + c)] c c
        const V *base = a.cross_psi ? psi_ring : rho_ring;
        const V *xr[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          int sl = lead_slot + 3 + dir * (k - 1);
          sl = sl >= 6 ? sl - 6 : sl;
          xr[k] = base + sl * W4 + tid + 2;
        }
        const V c0 = xr[1][0];
        R xx = 0, xy = 0, yy = 0;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const int o = 1 - s;
          const R ax = xr[1][1].v[o] + xr[1][-1].v[o], ay = xr[2][0].v[o] + xr[0][0].v[o];
          const R dg = (xr[2][1].v[o] + xr[0][-1].v[o]) + (xr[2][-1].v[o] + xr[0][1].v[o]);
          const R dgxy = (xr[2][1].v[o] + xr[0][-1].v[o]) - (xr[2][-1].v[o] + xr[0][1].v[o]);
          xx += c0.v[s] * (T1 * ax + T2 * dg);
          yy += c0.v[s] * (T1 * ay + T2 * dg);
          xy += c0.v[s] * (T2 * dgxy);
        }
        sxx += double(R(0.5) * xx);
        sxy += double(R(0.5) * xy);
        syy += double(R(0.5) * yy);
      }
      const size_t site = (size_t)y * lx + xc;
      const size_t nsite = (size_t)lx * ly;
      if (out_f32) {
        static_cast<float *>(out0)[site] = float(sxx);
        static_cast<float *>(out0)[nsite + site] = float(sxy);
        static_cast<float *>(out0)[2 * nsite + site] = float(syy);
      } else {
        static_cast<double *>(out0)[site] = sxx;
        static_cast<double *>(out0)[nsite + site] = sxy;
        static_cast<double *>(out0)[2 * nsite + site] = syy;
      }
    }

    if (WHAT != WHAT_MOMENTS && WHAT != WHAT_STRESS) {
    double wb = 0.0, wt = 0.0;
    R fsa[NS][9];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const R ir = C::rcp(rho[s]);
      const R ux = fmadd(tau[s] * Fx[s], ir, upx);
      const R uy = fmadd(tau[s] * Fy[s], ir, upy);
      // Deviation form of f^eq_l = W_l rho (1 + 3 cu + 9/2 cu^2 - 3/2 u.u):
      //   f^eq_l - W_l rho_ref = W_l (drho - 3/2 rho u.u) + W_l rho cu (3 + 9/2 cu)
      const R m15 = R(-1.5) * fmadd(ux, ux, uy * uy);
      const R r9 = rho[s] * R(1.0 / 9.0), r36 = rho[s] * R(1.0 / 36.0);
      const R b9 = fmadd(r9, m15, drho[s] * R(1.0 / 9.0)), b36 = fmadd(r36, m15, drho[s] * R(1.0 / 36.0));
      const R o = om[s];
      // relaxation of one population towards W_l (drho - 3/2 rho u.u) + W_l rho cu (3 + 9/2 cu),
      // cu = c_l . u (r = W_l rho, b = the velocity-independent part); opposite links take -cu
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
      // rest population closes the mass balance exactly: d*_0 = drho - sum_{l>0} d*_l
      fs[0] = drho[s] - ((((fs[1] + fs[2]) + (fs[3] + fs[4])) + ((fs[5] + fs[6]) + (fs[7] + fs[8]))));

      if (REDUCE && WALLS && col_ok) {
        // momentum handed to the wall: c_x f* out minus c_x of the reflected population,
        // which a moving wall raises by 6 W_l rho_w (c_l . U) = +-rho_w U / 6
        if (y == 0) wb += 2.0 * (double(fs[8]) - double(fs[7])) - 2.0 * a.wall_mom[0][s];
        if (y == ly - 1) wt += 2.0 * (double(fs[5]) - double(fs[6])) - 2.0 * a.wall_mom[1][s];
      }
    }
    if (PROFILE) {
      // x-momentum crossing the lines above (c_y = +1) and below (c_y = -1) the row when
      // these populations stream, before any wall term
      double kup = 0.0, kdn = 0.0;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        kup += double(fsa[s][5] - fsa[s][6]);
        kdn += double(fsa[s][8] - fsa[s][7]);
      }
      // pair forces on this site from partners above it, x components: eq. (FORCE) over the
      // links with c_y = 1 (|c|^2 = 2, 5) and c_y = 2 (|c|^2 = 5, 8), and the A-B term over
      // c = (+-1, 1); each +-c_x pair as one difference, as in the force itself
      double i1 = 0.0, i2 = 0.0;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const R up1 = fmadd(K2[s], ne.v[s] - nw.v[s], K5[s] * (R(2) * (qa.v[s] - qB.v[s])));
        const R up2 = fmadd(K5[s], qc.v[s] - qD.v[s], K8[s] * (d8a.v[s] - d8B.v[s]));
        i1 += double(-pc.v[s] * (up1 + up2));
        i2 += double(-pc.v[s] * up2);
      }
      if (NS == 2) {
        const V *base = a.cross_psi ? psi_ring : rho_ring;
        int sl0 = lead_slot + 3, sl1 = lead_slot + 3 + dir;
        sl0 = sl0 >= 6 ? sl0 - 6 : sl0;
        sl1 = sl1 >= 6 ? sl1 - 6 : (sl1 < 0 ? sl1 + 6 : sl1);
        const V c0 = base[sl0 * W4 + tid + 2];
        const V xne = base[sl1 * W4 + tid + 3], xnw = base[sl1 * W4 + tid + 1];
#pragma unroll
        for (int s = 0; s < NS; ++s) i1 += double(-c0.v[s] * (T2 * (xne.v[1 - s] - xnw.v[1 - s])));
      }
      R sr = rho[0], mx = jx[0] + R(0.5) * Fx[0];
#pragma unroll
      for (int s = 1; s < NS; ++s) {
        sr += rho[s];
        mx += jx[s] + R(0.5) * Fx[s];
      }
      double pv[PROF_N] = {double(mx / sr), kup, kdn, i1, i2, double(rho[0]), NS == 2 ? double(rho[NS - 1]) : 0.0};
      const int lane = tid & 63, wv = tid >> 6;
      double *row = static_cast<double *>(out0) + ((size_t)(strip * (TX >> 6) + wv) * ly + y) * PROF_N;
#pragma unroll
      for (int k = 0; k < PROF_N; ++k) {
        const double v = wave_sum(col_ok ? pv[k] : 0.0);
        if (lane == 0) row[k] = v;
      }
    }
    if (STORE && WALLS && a.moving) {
      // reflected populations of a moving wall: the stored outgoing population is only ever
      // pulled back into its opposite at the same site, so the wall's momentum goes in here:
      // f_5 = f*_7 + rho_w U_bot / 6, f_6 = f*_8 - rho_w U_bot / 6 off the bottom wall,
      // f_8 = f*_6 + rho_w U_top / 6, f_7 = f*_5 - rho_w U_top / 6 off the top wall
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
    if (STORE) {
      const Rsrc rd = make_rsrc(dst, ld_b);
      if constexpr (MODE == MODE_BF16SR) {
        // random bits from (site, plane, step): the same for every launch shape
        const uint32_t hs = mix32((uint32_t)(y * lx + (x0 + tid)) ^ tseed);
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

    if (ACCUM && col_ok) {
      bool bad = !(rho[0] > R(0) && rho[0] < R(INFINITY));
#pragma unroll
      for (int s = 1; s < NS; ++s) bad = bad || !(rho[s] > R(0) && rho[s] < R(INFINITY));
      acc[RED_WBOT] += wb;
      acc[RED_WTOP] += wt;
      acc[RED_BAD] += bad ? 1.0 : 0.0;
    }
    if (REDUCE && !ACCUM && col_ok) {
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

  };

  int lead_slot = 5;
  auto next_slot = [](int sl) { return sl == 5 ? 0 : sl + 1; };
  const int nrow = yB - yA;
  // unrolled by D so the FIFO roles are static; the halo staging buffer alternates with the
  // parity of the iteration (a fast wave stages the next row while a slow one may still read
  // the current row's buffer)
  for (int i0 = 0; i0 < nrow; i0 += D) {
#pragma unroll
    for (int k = 0; k < D; ++k) {
      if (i0 + k < nrow) {
        step_row(y0 + dir * (i0 + k), lead_slot, 5 + ((i0 + k) & 1), B[(k + D - 1) % D], B[k], B[(k + 3) % D],
                 HV[k % NHV]);
        lead_slot = next_slot(lead_slot);
      }
    }
  }

  if (ACCUM) {
    const int lane = tid & 63, wv = tid >> 6;
    constexpr int slot[ACC_N] = {RED_WBOT, RED_WTOP, RED_BAD};
#pragma unroll
    for (int k = 0; k < ACC_N; ++k) {
      const double v = wave_sum(acc[slot[k]]);
      if (lane == 0) red_lds[wv][k] = v;
    }
    __syncthreads();
    if (tid < ACC_N) {
      double v = 0.0;
      const int nw = (TX + 63) >> 6;
      for (int i = 0; i < nw; ++i) v += red_lds[i][tid];
      part[tid] += v;  // this workgroup's running sums (ACC_N per row)
    }
  } else if (REDUCE) {
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
      part[tid] = v;
    }
  }
}

// Time step of a launch (read only by the stochastically rounding variant): t_step, plus the
// step a graph replay starts at when t_base is set.
template <int MODE>
__device__ inline uint32_t launch_step_index(uint32_t t_step, const double *t_base) {
  if constexpr (MODE != MODE_BF16SR) return 0u;
  return t_step + (t_base ? (uint32_t)(long long)*t_base : 0u);
}

// One lattice: one workgroup per tile, tiles in band-major order spread over the XCDs.
template <int MODE, int NS, bool WALLS, int WHAT, int STP = kStoreWriteThrough>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MODE == MODE_F64 ? 1 : 2))) void step_kernel(StepArgs a) {
  const int logical = xcd_remap(blockIdx.x, gridDim.x);
  const int nstrip = (int)gridDim.x / a.nseg;
  const int seg = logical / nstrip;
  const int strip = logical - seg * nstrip;
  double *const part = WHAT == WHAT_STEP_ACCUM ? a.accrows + (size_t)blockIdx.x * ACC_N
                                               : a.partials + (size_t)blockIdx.x * RED_N;
  void *const out0 =
      WHAT == WHAT_STRESS ? a.out_sigma : (WHAT == WHAT_PROFILE ? static_cast<void *>(a.prof) : a.out_rho);
  run_tile<MODE, NS, WALLS, WHAT, STP>(a, a.src, a.dst, strip, seg, part, out0, a.out_u, a.out_f32,
                                       launch_step_index<MODE>(a.t_step, a.t_base));
}

// Many independent lattices in one persistent launch.  The host lists every tile of every
// instance (band-major within an instance); the workgroups of the grid take the tiles in
// rounds of gridDim.x, each round spread over the XCDs like the single-lattice grid, and
// read the instance's sizes, couplings and buffer offsets from b.inst.  Tiles of one round
// that neighbour each other share their overlap rows and columns through L2.
template <int MODE, int NS, bool WALLS, int WHAT, int STP = kStoreWriteThrough>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MODE == MODE_F64 ? 1 : 2))) void batch_step_kernel(BatchArgs b) {
  const int G = (int)gridDim.x;
  const int mine = xcd_remap(blockIdx.x, G);
  const uint32_t tstep = launch_step_index<MODE>(b.t_step, b.t_base);
  for (int base = 0; base < b.ntiles; base += G) {
    const int t = base + mine;
    if (t >= b.ntiles) break;  // later rounds are shorter still
    if (base > 0) __syncthreads();  // the previous tile's last ring and staging reads are done
    const int ti = (int)__builtin_amdgcn_readfirstlane((uint32_t)(b.tile0 + t));
    const TileDesc td = b.tiles[ti];
    const StepArgs &a = b.inst[td.inst];
    double *const part = WHAT == WHAT_STEP_ACCUM ? b.accrows + (size_t)td.part * ACC_N
                                                 : b.partials + (size_t)td.part * RED_N;
    run_tile<MODE, NS, WALLS, WHAT, STP>(a, b.src + a.offset, b.dst + a.offset, td.strip, td.seg, part, b.out_rho,
                                         b.out_u, b.out_f32, tstep);
  }
}

// ---------------------------------------------------------------------------------------
// Templated launchers (instantiated per storage mode)
// ---------------------------------------------------------------------------------------

template <int MODE, int NS, bool WALLS>
static hipError_t launch_step_t(int what, int tx, int nb, const StepArgs &a, hipStream_t st) {
  const size_t lds = step_lds_bytes(MODE, NS, tx);
  switch (what) {
    case WHAT_STEP:
      if (a.stream_stores)
        hipLaunchKernelGGL((step_kernel<MODE, NS, WALLS, WHAT_STEP, kStoreStreaming>), dim3(nb), dim3(tx), lds, st, a);
      else
        hipLaunchKernelGGL((step_kernel<MODE, NS, WALLS, WHAT_STEP>), dim3(nb), dim3(tx), lds, st, a);
      break;
    case WHAT_STEP_ACCUM:
      if (a.stream_stores)
        hipLaunchKernelGGL((step_kernel<MODE, NS, WALLS, WHAT_STEP_ACCUM, kStoreStreaming>), dim3(nb), dim3(tx), lds,
                           st, a);
      else
        hipLaunchKernelGGL((step_kernel<MODE, NS, WALLS, WHAT_STEP_ACCUM>), dim3(nb), dim3(tx), lds, st, a);
      break;
    case WHAT_MOMENTS:
      hipLaunchKernelGGL((step_kernel<MODE, NS, WALLS, WHAT_MOMENTS>), dim3(nb), dim3(tx), lds, st, a);
      break;
    case WHAT_OBSERVE:
      hipLaunchKernelGGL((step_kernel<MODE, NS, WALLS, WHAT_OBSERVE>), dim3(nb), dim3(tx), lds, st, a);
      break;
    case WHAT_PROFILE:
      hipLaunchKernelGGL((step_kernel<MODE, NS, WALLS, WHAT_PROFILE>), dim3(nb), dim3(tx), lds, st, a);
      break;
    case WHAT_STRESS:
      hipLaunchKernelGGL((step_kernel<MODE, NS, WALLS, WHAT_STRESS>), dim3(nb), dim3(tx), lds, st, a);
      break;
    case WHAT_STEP_FIELDS:
      hipLaunchKernelGGL((step_kernel<MODE, NS, WALLS, WHAT_STEP_FIELDS>), dim3(nb), dim3(tx), lds, st, a);
      break;
    case WHAT_STEP_FIELDS32:
      hipLaunchKernelGGL((step_kernel<MODE, NS, WALLS, WHAT_STEP_FIELDS32>), dim3(nb), dim3(tx), lds, st, a);
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

template <int MODE, int NS, bool WALLS>
static hipError_t launch_batch_t(int what, int tx, int grid, const BatchArgs &b, hipStream_t st) {
  const size_t lds = step_lds_bytes(MODE, NS, tx);
  switch (what) {
    case WHAT_STEP:
      if (b.stream_stores)
        hipLaunchKernelGGL((batch_step_kernel<MODE, NS, WALLS, WHAT_STEP, kStoreStreaming>), dim3(grid), dim3(tx), lds,
                           st, b);
      else
        hipLaunchKernelGGL((batch_step_kernel<MODE, NS, WALLS, WHAT_STEP>), dim3(grid), dim3(tx), lds, st, b);
      break;
    case WHAT_STEP_ACCUM:
      if (b.stream_stores)
        hipLaunchKernelGGL((batch_step_kernel<MODE, NS, WALLS, WHAT_STEP_ACCUM, kStoreStreaming>), dim3(grid), dim3(tx),
                           lds, st, b);
      else
        hipLaunchKernelGGL((batch_step_kernel<MODE, NS, WALLS, WHAT_STEP_ACCUM>), dim3(grid), dim3(tx), lds, st, b);
      break;
    case WHAT_MOMENTS:
      hipLaunchKernelGGL((batch_step_kernel<MODE, NS, WALLS, WHAT_MOMENTS>), dim3(grid), dim3(tx), lds, st, b);
      break;
    case WHAT_OBSERVE:
      hipLaunchKernelGGL((batch_step_kernel<MODE, NS, WALLS, WHAT_OBSERVE>), dim3(grid), dim3(tx), lds, st, b);
      break;
    case WHAT_PROFILE:
      hipLaunchKernelGGL((batch_step_kernel<MODE, NS, WALLS, WHAT_PROFILE>), dim3(grid), dim3(tx), lds, st, b);
      break;
    case WHAT_STRESS:
      hipLaunchKernelGGL((batch_step_kernel<MODE, NS, WALLS, WHAT_STRESS>), dim3(grid), dim3(tx), lds, st, b);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int MODE>
static hipError_t launch_batch_m(int ns, int walls, int what, int tx, int grid, const BatchArgs &b, hipStream_t st) {
  if (ns == 1) return walls ? launch_batch_t<MODE, 1, true>(what, tx, grid, b, st) : launch_batch_t<MODE, 1, false>(what, tx, grid, b, st);
  return walls ? launch_batch_t<MODE, 2, true>(what, tx, grid, b, st) : launch_batch_t<MODE, 2, false>(what, tx, grid, b, st);
}

template <int NS, bool WALLS>
static hipError_t launch_batch_sr_t(int what, int tx, int grid, const BatchArgs &b, hipStream_t st) {
  constexpr int M = MODE_BF16SR;
  const size_t lds = step_lds_bytes(M, NS, tx);
  switch (what) {
    case WHAT_STEP:
      if (b.stream_stores)
        hipLaunchKernelGGL((batch_step_kernel<M, NS, WALLS, WHAT_STEP, kStoreStreaming>), dim3(grid), dim3(tx), lds, st, b);
      else
        hipLaunchKernelGGL((batch_step_kernel<M, NS, WALLS, WHAT_STEP>), dim3(grid), dim3(tx), lds, st, b);
      break;
    case WHAT_STEP_ACCUM:
      if (b.stream_stores)
        hipLaunchKernelGGL((batch_step_kernel<M, NS, WALLS, WHAT_STEP_ACCUM, kStoreStreaming>), dim3(grid), dim3(tx), lds,
                           st, b);
      else
        hipLaunchKernelGGL((batch_step_kernel<M, NS, WALLS, WHAT_STEP_ACCUM>), dim3(grid), dim3(tx), lds, st, b);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int MODE, int NS, bool WALLS>
static int blocks_per_cu_t(int tx) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_kernel<MODE, NS, WALLS, WHAT_STEP>, tx,
                                                   step_lds_bytes(MODE, NS, tx)) != hipSuccess)
    return 1;
  return n > 0 ? n : 1;
}

template <int MODE>
static int blocks_per_cu_m(int ns, int walls, int tx) {
  if (ns == 1) return walls ? blocks_per_cu_t<MODE, 1, true>(tx) : blocks_per_cu_t<MODE, 1, false>(tx);
  return walls ? blocks_per_cu_t<MODE, 2, true>(tx) : blocks_per_cu_t<MODE, 2, false>(tx);
}

// The stochastically rounding BF16 variant exists for the passes that store populations.
template <int NS, bool WALLS>
static hipError_t launch_step_sr_t(int what, int tx, int nb, const StepArgs &a, hipStream_t st) {
  constexpr int M = MODE_BF16SR;
  const size_t lds = step_lds_bytes(M, NS, tx);
  switch (what) {
    case WHAT_STEP:
      if (a.stream_stores)
        hipLaunchKernelGGL((step_kernel<M, NS, WALLS, WHAT_STEP, kStoreStreaming>), dim3(nb), dim3(tx), lds, st, a);
      else
        hipLaunchKernelGGL((step_kernel<M, NS, WALLS, WHAT_STEP>), dim3(nb), dim3(tx), lds, st, a);
      break;
    case WHAT_STEP_ACCUM:
      if (a.stream_stores)
        hipLaunchKernelGGL((step_kernel<M, NS, WALLS, WHAT_STEP_ACCUM, kStoreStreaming>), dim3(nb), dim3(tx), lds, st, a);
      else
        hipLaunchKernelGGL((step_kernel<M, NS, WALLS, WHAT_STEP_ACCUM>), dim3(nb), dim3(tx), lds, st, a);
      break;
    case WHAT_OBSERVE:
      hipLaunchKernelGGL((step_kernel<M, NS, WALLS, WHAT_OBSERVE>), dim3(nb), dim3(tx), lds, st, a);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace lb355
