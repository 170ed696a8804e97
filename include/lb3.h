/*
 * lb3.h -- C ABI of the three-dimensional extension of the two-belt pseudopotential lattice
 * Boltzmann library (MI355X, gfx950).
 *
 * The paper (Sbragaglia, Benzi, Bernaschi, Succi, arXiv:1402.6019) builds the competing
 * interaction model in two dimensions and, in section "Competing interactions", points to
 * extensions to three dimensions without giving them.  This library's 3-D step is the direct
 * extension:
 *   - BGK equation (LB) on the D3Q19 lattice, second-order Hermite equilibrium, c_s^2 = 1/3,
 *     force applied by the equilibrium-velocity shift u_eq = u' + tau F / rho;
 *   - eq. (FORCE) with the same two belts over the integer vectors of the 5x5x5 cube: the
 *     attractive sum G1 w(|c|^2) over |c|^2 = 1, 2, 3, 4 (32 links) and the repulsive sum
 *     G2 p(|c|^2) over |c|^2 = 1, 2, 3, 4, 5, 6, 8 (92 links); lb3_default_couplings fills the
 *     isotropic weights with E2 = 1/3 (the (BULK) normalisation): w sixth-order isotropic on
 *     four shells, p eighth-order isotropic on seven, both unique;
 *   - two species with the A-B repulsion over the D3Q19 links (D3Q19 weights t) between
 *     densities or pseudopotentials, and the common velocity weighted by 1/tau_s;
 *   - optional channel: halfway bounce-back walls at y = -1/2 and y = ly - 1/2 with wetting
 *     ghost densities and a body force; periodic in x and z.
 *
 * Conventions as in lb.h.  Dense arrays are [...][z][y][x], x fastest.  The canonical
 * population layout of lb3_checkpoint / lb3_restore is f[species][l][z][y][x] (FP64,
 * pre-collision), D3Q19 order c_0..c_18 = (0,0,0), (1,0,0), (-1,0,0), (0,1,0), (0,-1,0),
 * (0,0,1), (0,0,-1), (1,1,0), (-1,-1,0), (1,-1,0), (-1,1,0), (1,0,1), (-1,0,-1), (1,0,-1),
 * (-1,0,1), (0,1,1), (0,-1,-1), (0,1,-1), (0,-1,1).
 * Ownership, errors (enum lb_status) and threading as in lb.h.
 */
#ifndef LB355_LB3_H
#define LB355_LB3_H

#include "lb.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lb3_ctx lb3_ctx;

typedef struct {
  int32_t lx, ly, lz;  /* lx, ly, lz >= 5; lx * ly * lz <= 2^30; one z-plane of one population buffer
                          (ly * 19 * pitch * n_species values) below 4 GiB */
  int32_t n_species;   /* 1 or 2 */
  int32_t walls;       /* 0: periodic in x, y, z; 1: bounce-back walls below row y = 0 and above y = ly - 1 */
  int32_t storage;     /* LB_F64 or LB_F32 (enum lb_storage; BF16 is not offered in 3-D) */
} lb3_lattice;

typedef struct {
  double g1[2], g2[2];  /* G_ss,1 (attractive, < 0) and G_ss,2 (repulsive, > 0) per species */
  double g_ab;          /* A-B repulsion (two species) */
  double w[7], p[7];    /* shell weights for |c|^2 = 1, 2, 3, 4, 5, 6, 8 (w: attractive belt, zero beyond 4) */
  double t[2];          /* A-B weights for |c|^2 = 1, 2 */
  double body_force[3]; /* g; species s feels rho_s g */
  double rho_wall[2];   /* channel: ghost densities of the solid rows (wetting) */
  int32_t cross_uses_psi; /* 0: A-B term between densities, 1: between pseudopotentials */
  int32_t reserved_;
} lb3_couplings;

/* Zero couplings and the isotropic default weights.  Pure host call. */
int lb3_default_couplings(lb3_couplings *c);

/* Bytes of ONE population buffer (two are needed).  0 for an invalid lattice.  Pure host call. */
size_t lb3_pop_bytes(const lb3_lattice *lat);

/* Create a 3-D simulation; validation, ownership and stream as lb_init.  rho_init: host,
   [n_species][lz][ly][lx]; the state starts at rest, f_l = W_l rho_init.  psi->rho_ref: FP32
   deviation reference per species (as in lb.h).  Synchronises the stream once. */
int lb3_init(lb3_ctx **out, const lb3_lattice *lat, const lb3_couplings *cpl, const double tau[2],
             const lb_psi_params *psi, const double *rho_init, void *pop_a, void *pop_b, size_t pop_bytes,
             void *hip_stream);

/* Advance n >= 0 steps of eq. (LB) in 3-D: one fused launch per step (pull streaming with
   bounce-back, moments, psi, the two-belt force of eq. (FORCE) over the cube, the A-B
   repulsion and the body force, the velocity shift, BGK collision with the rest-population
   closure, store).  Asynchronous. */
int lb3_step(lb3_ctx *ctx, int64_t n);

/* Density rho (device [n_species][lz][ly][lx]) and velocity u (device [3][lz][ly][lx]),
   u = (sum_s j_s + F_s / 2) / sum_s rho_s, of the current state (section "Lattice Kinetic
   Theory for non-ideal fluids": the zeroth and first moments of the populations).  dtype:
   enum lb_dtype.  Either pointer may be NULL.  Asynchronous. */
int lb3_moments(lb3_ctx *ctx, void *rho, void *u, int32_t dtype);

/* FP64 totals of the current state (host): species masses, total momentum sum_s j_s (3
   components), the collision invariants of eq. (LB); and, if flow != NULL, the flow rate
   sum u_x / (lx lz) with u as in lb3_moments.  Synchronises; LB_EUNSTABLE on a non-finite or
   non-positive density. */
int lb3_totals(lb3_ctx *ctx, double mass[2], double momentum[3], double *flow);

/* Canonical FP64 pre-collision populations f_l(x, t) of eq. (LB) (layout above) to dst / from
   src (device, n_species * 19 * lz * ly * lx doubles).  lb3_restore keeps the step count.
   Asynchronous. */
int lb3_checkpoint(lb3_ctx *ctx, void *dst_f64);
int lb3_restore(lb3_ctx *ctx, const void *src_f64);

/* Launch shape: ty in {1, 2, 4} rows of 64 columns per workgroup (ty waves), or 8 with FP32
   storage, and sz >= 1 z-planes per workgroup; any shape gives bitwise identical results.
   LB_EINVAL otherwise.  Host call. */
int lb3_set_tile(lb3_ctx *ctx, int32_t ty, int32_t sz);
int lb3_get_tile(const lb3_ctx *ctx, int32_t *ty, int32_t *sz);

int64_t lb3_time(const lb3_ctx *ctx);
const char *lb3_last_error(const lb3_ctx *ctx);
void lb3_destroy(lb3_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* LB355_LB3_H */
