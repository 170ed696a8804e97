// Internal declarations shared by the host runtime (lb_api.cpp) and the device kernels
// (lb_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lb355 {

// MODE_BF16SR: BF16 storage whose population stores round stochastically (the step kernels
// only; every other kernel reads and writes it like MODE_BF16).
enum StoreMode { MODE_F64 = 0, MODE_F32 = 1, MODE_BF16 = 2, MODE_BF16SR = 3 };

// What one launch of the fused step kernel does.
enum StepWhat {
  WHAT_STEP = 0,         // stream + force + collide, store f*
  WHAT_MOMENTS = 2,      // write rho_s and the half-force velocity, store nothing
  WHAT_OBSERVE = 3,      // partial sums of the current state, store nothing
  WHAT_PROFILE = 4,      // per-row sums of the current state (velocity, stress parts), store nothing
  WHAT_STRESS = 5,       // write the site pressure tensor of the current state, store nothing
  WHAT_STEP_ACCUM = 6,   // step, adding wall stress and health counts to per-workgroup FP64 running sums
  // step, also writing what the adjoint's reverse step reads of the state it steps from: rho,
  // psi, j of every site (out_rho, [4][2][ly][lx], FP64 / FP32) and the canonical FP64
  // populations of the rows next to the walls (out_u, [s][l][2][lx])
  WHAT_STEP_FIELDS = 7,
  WHAT_STEP_FIELDS32 = 8
};

// Running sums of WHAT_STEP_ACCUM, per workgroup row.
enum AccSlot { ACC_WBOT = 0, ACC_WTOP, ACC_BAD, ACC_N };

// Per-row sums written by a WHAT_PROFILE launch, per 64-column block of a row:
//   PROF_U   sum of the half-force velocity u_x
//   PROF_KUP sum_s (f*_5 - f*_6): x-momentum the populations with c_y = +1 carry up
//   PROF_KDN sum_s (f*_8 - f*_7): x-momentum the populations with c_y = -1 carry down
//   PROF_I1  x-force on the row's sites from partners at c_y >= 1 (pairs crossing line y + 1/2)
//   PROF_I2  the part of PROF_I1 from partners at c_y = 2 (pairs also crossing line y + 3/2)
//   PROF_RA, PROF_RB  sums of the species densities (B zero for one component)
enum ProfSlot { PROF_U = 0, PROF_KUP, PROF_KDN, PROF_I1, PROF_I2, PROF_RA, PROF_RB, PROF_N };

// Partial-sum slots written per workgroup (and totals after the second pass).
enum RedSlot {
  RED_MASS0 = 0, RED_MASS1, RED_PX, RED_PY, RED_WBOT, RED_WTOP, RED_FLOW, RED_BAD, RED_N
};

// Kernel arguments of the fused step (passed by value through the kernarg segment).
struct StepArgs {
  const void *src;      // post-collision populations of the previous step (pull source)
  void *dst;            // post-collision populations of this step
  double *partials;     // [gridDim.x][RED_N] when reducing
  void *out_rho;        // moments: [ns][ly][lx]
  void *out_u;          // moments: [2][ly][lx]
  long long plane;      // elements per (species, l) plane = ly * pitch
  int lx, ly, pitch;    // lattice and row pitch (elements)
  int sy, nseg;         // rows per workgroup, workgroups per strip
  int out_f32;          // moments output type
  int cross_psi;        // A-B term between psi (1) or rho (0)
  double K[2][5];       // folded shell couplings G_ss,1 w(q) + G_ss,2 p(q)
  double T[2];          // G_AB t(1), G_AB t(2)
  double body[2];       // acceleration g
  double tau[2], omega[2];
  double psi0, irho0;
  double rho_w[2], psi_w[2];  // wall ghost rows (channel)
  double rho_ref[2];          // FP32 / BF16 deviation reference
  long long offset;           // batch: byte offset of this instance in each population buffer
  double wall_mom[2][2];      // [bottom, top][species]: rho_w,s U / 6, added on reflection
  int moving;                 // some wall moves (wall_mom != 0)
  int ncb;                    // profile: 64-column blocks per row in prof
  double *prof;               // profile: [ncb][ly][PROF_N]
  int stream_stores;          // both population buffers exceed the Infinity Cache: non-temporal stores
  uint32_t t_step;            // MODE_BF16SR: time step of the launch, plus *t_base when t_base is set
  const double *t_base;       // (graph replays: the step at which the replay starts)
  void *out_sigma;            // stress: [3][ly][lx] (xx, xy, yy)
  double *accrows;            // WHAT_STEP_ACCUM: [gridDim.x][ACC_N] running sums
};

// Batched launches: one tile of one instance.
struct TileDesc {
  int inst;   // instance index (into BatchArgs::inst)
  int strip;  // strip of blockDim.x columns
  int seg;    // segment of StepArgs::sy rows
  int part;   // row of reduction partials this tile writes
};

// Kernel arguments of the batched step: tiles [tile0, tile0 + ntiles) of the table.
struct BatchArgs {
  const StepArgs *inst;  // [n] per-instance arguments (device)
  const TileDesc *tiles; // tile table (device)
  int tile0, ntiles;
  const char *src;       // population buffers holding every instance at StepArgs::offset
  char *dst;
  double *partials;      // [tiles][RED_N]
  void *out_rho, *out_u; // WHAT_MOMENTS (the launch then covers one instance); out_rho is the
                         // output of WHAT_STRESS and WHAT_PROFILE too
  int out_f32;
  int stream_stores;     // non-temporal population stores (see StepArgs)
  double *accrows;       // WHAT_STEP_ACCUM: [tiles][ACC_N] running sums, row TileDesc::part
  uint32_t t_step;       // MODE_BF16SR: time step of the launch (see StepArgs)
  const double *t_base;
};

// Second reduction pass of one batch instance: partial rows [p0, p0 + n).
struct ReduceJob {
  int p0, n;
  double inv_lx;
};

// Arguments of the layout kernels (init / checkpoint / restore).
struct LayoutArgs {
  const void *in;
  void *out;
  long long plane;
  int lx, ly, pitch, ns;
  double rho_ref[2];
  // checkpoint with fields (adjoint): out receives only the canonical populations of the rows
  // next to the walls ([s][l][2][lx], FP64), fields rho, psi, jx, jy of each species of the
  // state, [4][2][ly][lx] in the adjoint's precision
  void *fields;
  double psi0, irho0;
};

// Reverse step of the adjoint (lb_adjoint.hip).  Arrays are canonical [..][y][x]; R is
// double for FP64 contexts and float otherwise.
struct AdjArgs {
  const double *x;       // pre-collision populations f(t) of the rows next to the walls, [s][l][2][x]
                         // (bottom row, then top row), FP64; read with walls only
  // lambda(t) is kept in two parts: lam [s][l][y][x], written by the local pass, and corr
  // [s][y][x], the term common to every l that the gather adds; lambda_l = lam_l + corr.
  const void *lam_next;   // lam of lambda(t+1) (R)
  const void *corr_next;  // corr of lambda(t+1) (R)
  void *lam;              // lam of lambda(t) (R, written)
  void *corr;             // corr of lambda(t) (R, written)
  void *fields;          // [4][2][y][x] (R): rho, psi, jx, jy of f(t)
  void *fbar;            // [2][4][y][x] (R): psi_s Fbar_s and r_s Fbar_s (x, y components), written
  // With the common term of lambda(t+1) gathered in the local pass instead of read from
  // corr_next: fbar of step t + 1 and the fields of f(t + 1).
  const void *fbar_next;
  const void *fields_next;
  double *partials;      // [blocks][ADJ_N]
  int lx, ly;
  int cross_psi, pad_;
  double K[2][5];        // G_ss,1 w(q) + G_ss,2 p(q)
  double w[5], p[5], t[2];
  double g1[2], g2[2], gab;
  double body[2], tau[2], omega[2];
  double psi0, irho0;
  double rho_w[2], psi_w[2];
  double cW, cQ;         // per-step loss weights
  double ilx;            // 1 / lx, and the same rounded from a float division
  float ilxf, pad2_;
  double u_wall[2];      // x-velocity of the bottom and top wall
};

// Per-block partial sums of the adjoint: parameter sensitivities and the loss.
enum AdjSlot { ADJ_G1A = 0, ADJ_G1B, ADJ_G2A, ADJ_G2B, ADJ_GAB, ADJ_GX, ADJ_GY, ADJ_LW, ADJ_LQ, ADJ_N };

int adj_blocks(int lx, int ly);
// One reverse step; adds this step's per-block sensitivities to a.partials.  gather_in: the
// local pass gathers the common term of lambda(t+1) from a.fbar_next and a.fields_next
// instead of reading a.corr_next; gather_out: a gather pass writes a.corr for lambda(t) (the
// next reverse step reads it from memory).
hipError_t launch_adjoint_step(int fp64, int ns, int walls, const AdjArgs &a, int gather_in, int gather_out,
                               hipStream_t st);
// acc[k] += sum over blocks of partials[block][k] (fixed order).
hipError_t launch_adjoint_reduce(const double *partials, int lx, int ly, double *acc, hipStream_t st);
hipError_t launch_zero(void *p, size_t bytes, hipStream_t st);

// Host-side launchers (lb_kernels.hip).  Return hipSuccess or the launch error.
hipError_t launch_step2(int mode, int ns, int walls, int nblocks, const StepArgs &a, hipStream_t st);
hipError_t launch_step(int mode, int ns, int walls, int what, int tx, int nblocks, const StepArgs &a,
                       hipStream_t st);
hipError_t launch_reduce(const double *partials, int nblocks, double *totals, double *acc, int accumulate,
                         double inv_lx, hipStream_t st);
hipError_t launch_init(int mode, int walls, const LayoutArgs &a, hipStream_t st);
hipError_t launch_checkpoint(int mode, int walls, const LayoutArgs &a, hipStream_t st);
// The same, also writing the fields rho, psi, jx, jy (FP64 if fp64, else FP32) to a.fields.
hipError_t launch_checkpoint_fields(int mode, int walls, int fp64, const LayoutArgs &a, hipStream_t st);
hipError_t launch_restore(int mode, int walls, const LayoutArgs &a, hipStream_t st);

hipError_t launch_fill(double *p, double v, int n, hipStream_t st);
// Grid-stride copy of n16 16-byte elements (blocks workgroups of 256), non-temporal if asked.
hipError_t launch_stream_copy(void *dst, const void *src, size_t n16, int nontemporal, int blocks, hipStream_t st);
// acc[0..1] += (column sums of rows' wall stress) * inv_lx, acc[2] += count, acc[3] += bad;
// rows are cleared.
hipError_t launch_flush(double *rows, int nrows, double *acc, double count, double inv_lx, hipStream_t st);
// The same per batch instance: rows of job i into acc[4 i ..].
hipError_t launch_batch_flush(double *rows, const ReduceJob *jobs, int njobs, double *acc, double count,
                              hipStream_t st);

// Profile second pass: out[0..ly) = ubar, out[ly..2ly] = sigma, out[2ly+1..4ly+1) = the
// species densities per row (see lb_profile).  wb0, wt0:
// sum_s rho_w,s U / 3 of the bottom and top wall; rows: scratch of ly * PROF_N doubles.
hipError_t launch_profile_finish(const double *prof, int ncb, int lx, int ly, int walls, double wb0, double wt0,
                                 double *rows, double *out, hipStream_t st);
hipError_t launch_profile_stats(const double *samples, long long n, int ly, int walls, int k0, double u_bot,
                                double u_top, double *out, hipStream_t st);

hipError_t launch_batch_step(int mode, int ns, int walls, int what, int tx, int grid, const BatchArgs &b,
                             hipStream_t st);
hipError_t launch_batch_reduce(const double *partials, const ReduceJob *jobs, int njobs, double *totals, double *acc,
                               int accumulate, hipStream_t st);

size_t step_lds_bytes(int mode, int ns, int tx);

// Static device scratch of the entry points that allocate nothing (lb_static.hip), in doubles.
constexpr size_t kStaticScratchDoubles = (size_t)1 << 19;
// Looks up the scratch array's address on `device` once (makes it current for the lookup).
hipError_t static_scratch_setup(int device);
// That address (nullptr before static_scratch_setup succeeded on the device).
double *static_scratch(int device);

// Per storage mode (lb_step_f64.hip, lb_step_f32.hip, lb_step_bf16.hip): the launchers that
// launch_step / launch_batch_step / step_blocks_per_cu dispatch to.
hipError_t launch_step_f64(int ns, int walls, int what, int tx, int nb, const StepArgs &a, hipStream_t st);
hipError_t launch_step_f32(int ns, int walls, int what, int tx, int nb, const StepArgs &a, hipStream_t st);
hipError_t launch_step_bf16(bool stochastic, int ns, int walls, int what, int tx, int nb, const StepArgs &a,
                            hipStream_t st);
hipError_t launch_batch_f64(int ns, int walls, int what, int tx, int grid, const BatchArgs &b, hipStream_t st);
hipError_t launch_batch_f32(int ns, int walls, int what, int tx, int grid, const BatchArgs &b, hipStream_t st);
hipError_t launch_batch_bf16(bool stochastic, int ns, int walls, int what, int tx, int grid, const BatchArgs &b,
                             hipStream_t st);
int blocks_per_cu_f64(int ns, int walls, int tx);
// Two time steps per launch (lb_step2.hpp): one wave per workgroup, strips of 54 columns,
// nb = strips x segments workgroups, a.sy rows per segment.
hipError_t launch_step2_f64(int ns, int walls, int nb, const StepArgs &a, hipStream_t st);
hipError_t launch_step2_f32(int ns, int walls, int nb, const StepArgs &a, hipStream_t st);
hipError_t launch_step2_bf16(bool stochastic, int ns, int walls, int nb, const StepArgs &a, hipStream_t st);
int blocks2_per_cu_f32(int ns, int walls);  // also BF16 (the same registers and LDS)
int blocks2_per_cu_f64(int ns, int walls);
int blocks_per_cu_f32(int ns, int walls, int tx);
int blocks_per_cu_bf16(int ns, int walls, int tx);
// Workgroups of tx threads of the plain step kernel that one compute unit holds at once.
int step_blocks_per_cu(int mode, int ns, int walls, int tx);

}  // namespace lb355
