/*
 * lb.h -- C ABI of the MI355X (gfx950) two-belt pseudopotential lattice Boltzmann library.
 *
 * The library advances the one- or two-component D2Q9 BGK lattice Boltzmann equation,
 * eq. (LB) of Sbragaglia, Benzi, Bernaschi, Succi (arXiv:1402.6019), whose forcing term is
 * the two-belt competing pseudopotential force of eq. (FORCE): a short-range attraction
 * (G1 < 0, weights w on links with |c|^2 <= 4) against a mid-range repulsion (G2 > 0,
 * weights p on links with |c|^2 <= 8), with psi(rho) = psi0 (1 - exp(-rho/rho0)) and the
 * force applied by shifting the equilibrium velocity (u_eq -> u_eq + tau F / rho).  For two
 * components (emulsion section of the paper) each species s in {A, B} has its own
 * populations and couplings G_ss,1, G_ss,2, and the species repel each other with strength
 * G_AB over the first belt.  Optional planar channel: halfway bounce-back walls at
 * y = -1/2 and y = ly - 1/2 with a uniform body force (the confined Poiseuille flows), and
 * walls that slide along x (the planar Couette cell, walls moving with +-U_w).
 *
 * Conventions
 *   - Lattice units (dx = dt = 1, c_s^2 = 1/3).  x is the streamwise (periodic) direction,
 *     y the cross-stream direction (the paper's z).
 *   - Device pointers are HIP device addresses (e.g. torch tensors' data_ptr()).  Host
 *     pointers are marked "host".  Dense field arrays are row-major [...][y][x], x fastest.
 *   - Population buffers are opaque: ask lb_pop_bytes() for their size and use
 *     lb_checkpoint()/lb_restore() to read or write populations in the canonical layout
 *     f[species][l][y][x] (FP64, pre-collision, D2Q9 order c_0..c_8 =
 *     (0,0),(1,0),(0,1),(-1,0),(0,-1),(1,1),(-1,1),(-1,-1),(1,-1)).
 *   - All device work is enqueued on the HIP stream given to lb_init / lb_batch_init and is
 *     asynchronous unless a call is documented as synchronising.
 *
 * Ownership: the caller allocates population buffers and output arrays and keeps them alive
 * until lb_destroy(); the context borrows them and never frees caller memory.  The context
 * owns small internal buffers (reduction partials, totals, staging) and frees them in
 * lb_destroy().
 *
 * Errors: every int-returning call returns LB_OK (0) or a negative lb_status.  The reason is
 * available from lb_last_error(ctx) (or lb_last_error(NULL) when no context exists yet).
 * Asynchronous numerical failure (non-finite or non-positive density) is latched on the
 * device by the reductions and reported as LB_EUNSTABLE by the next synchronising call.
 * After an error the context remains valid for lb_restore() and lb_destroy().
 *
 * Threads: a context must not be used from two threads at once.
 */
#ifndef LB355_LB_H
#define LB355_LB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lb_ctx lb_ctx;

enum lb_status {
  LB_OK = 0,
  LB_EINVAL = -1,     /* invalid argument (sizes, tau <= 1/2, non-positive density, ...) */
  LB_ENOMEM = -2,     /* an internal allocation failed, or a caller buffer is too small */
  LB_EDEVICE = -3,    /* a HIP runtime call failed */
  LB_EUNSTABLE = -4,  /* the run produced a non-finite or non-positive density */
  LB_ESTATE = -5      /* call not valid in the current state (e.g. no walls for wall stress) */
};

/* Storage of the populations in HBM. */
enum lb_storage {
  LB_F64 = 0,     /* FP64 populations, FP64 arithmetic */
  LB_F32 = 1,     /* FP32 deviations f_l - W_l rho_ref[s] (see lb_psi_params), FP32 arithmetic */
  LB_BF16DEV = 2  /* BF16 deviations f_l - W_l rho_ref[s], FP32 arithmetic */
};

/* Output type of lb_moments. */
enum lb_dtype { LB_OUT_F64 = 0, LB_OUT_F32 = 1 };

/* Rounding of BF16 population stores (lb_set_rounding). */
enum lb_rounding {
  LB_ROUND_NEAREST = 0,   /* round to nearest even (default) */
  LB_ROUND_STOCHASTIC = 1 /* unbiased random rounding, reproducible from (site, plane, step) */
};

/* Population store policy of the plain and reducing step kernels (lb_set_store_policy). */
enum lb_store_policy {
  LB_STORES_AUTO = 0,          /* by footprint: streaming once both buffers exceed 256 MiB */
  LB_STORES_WRITE_THROUGH = 1, /* stores written through L2 and kept by the Infinity Cache */
  LB_STORES_STREAMING = 2      /* non-temporal stores, lead-row loads issued without a branch */
};

typedef struct {
  int32_t lx, ly;      /* lattice size: lx, ly >= 5, ly <= 65535, lx * ly <= 2^27, and one population
                          buffer (lb_pop_bytes) below 4 GiB */
  int32_t n_species;   /* 1 or 2 */
  int32_t walls;       /* 0: periodic in x and y; 1: channel, bounce-back walls below row 0 and above row ly-1 */
  int32_t storage;     /* enum lb_storage */
} lb_lattice;

typedef struct {
  /* eq. (FORCE) per species s: G_ss,1 (attractive, < 0) and G_ss,2 (repulsive, > 0). */
  double g1[2], g2[2];
  /* A-B repulsion strength G_AB (two components only). */
  double g_ab;
  /* Shell weights for |c|^2 = 1, 2, 4, 5, 8: w on the attractive belt (w[3] = w[4] = 0 in the
     paper's form), p on both belts; t[0], t[1]: A-B cross weights for |c|^2 = 1, 2.
     lb_default_couplings() fills the isotropic sets (E2 = 1/3; w sixth-order, p eighth-order
     isotropic; t = D2Q9 weights). */
  double w[5], p[5], t[2];
  /* Body force per unit mass g = (g_x, g_y); species s feels rho_s g. */
  double body_force[2];
  /* Channel only: densities of the solid ghost rows seen by the force stencil (wetting). */
  double rho_wall[2];
  /* 0: A-B repulsion between densities (default); 1: between pseudopotentials. */
  int32_t cross_uses_psi;
  int32_t reserved_;
  /* Channel only: x-velocity of the bottom and the top wall (planar Couette cell: -U_w, +U_w).
     Bounce-back off a wall moving with velocity U hands the reflected population the momentum
     6 W_l rho_wall[s] (c_l . U): the wall's momentum density is rho_wall[s] U per species, so
     set rho_wall to the densities of the phase that wets the walls (one component: its density).
     Must be 0 on periodic lattices. */
  double wall_velocity[2];
} lb_couplings;

typedef struct {
  double psi0, rho0;   /* psi(rho) = psi0 (1 - exp(-rho / rho0)) */
  double rho_ref[2];   /* LB_F32 / LB_BF16DEV: populations are stored as deviations f_l - W_l rho_ref[s]
                          from the rest state of this reference density per species, so their rounding
                          is relative to the deviation, not to f_l (0: plain populations).  LB_F64 always
                          stores plain populations. */
} lb_psi_params;

/* Streaming copy of `bytes` (a multiple of 16, 16-byte aligned device buffers) from src to
   dst with 16-byte accesses, non-temporal if nontemporal != 0: the bandwidth reference the
   benchmark compares the step against (a plain copy moves the same bytes with no stencil).
   Asynchronous on hip_stream; errors are reported by lb_last_error(NULL). */
int lb_stream_copy(void *dst, const void *src, size_t bytes, int32_t nontemporal, void *hip_stream);

/* Fill *c with zero couplings and the default isotropic weights.  Pure host call. */
int lb_default_couplings(lb_couplings *c);

/* Bytes of ONE population buffer for this lattice (two are needed: ping and pong).
   Returns 0 for an invalid lattice.  Pure host call. */
size_t lb_pop_bytes(const lb_lattice *lat);

/*
 * Create a simulation.  Validates the lattice (lx, ly >= 5, n_species in {1,2}, walls in
 * {0,1}, storage valid), tau[s] > 1/2, psi0 > 0, rho0 > 0, rho_init > 0 and finite, and
 * pop_bytes >= lb_pop_bytes(lat).  rho_init (host, [n_species][ly][lx]) gives the rest
 * equilibrium start f_l = W_l rho_init.  pop_a and pop_b are device buffers of pop_bytes
 * each; the state starts in pop_a.  hip_stream is a hipStream_t (NULL = default stream).
 * Synchronises the stream once (host-to-device copy of rho_init).
 */
int lb_init(lb_ctx **out, const lb_lattice *lat, const lb_couplings *cpl, const double tau[2],
            const lb_psi_params *psi, const double *rho_init, void *pop_a, void *pop_b, size_t pop_bytes,
            void *hip_stream);

/* Advance n >= 0 time steps of eq. (LB) (pull streaming + two-belt force + BGK collision in
   one fused kernel per step).  Asynchronous.  Returns LB_EUNSTABLE if an earlier reduction
   (see lb_set_reduce_every) has already reported a bad density. */
int lb_step(lb_ctx *ctx, int64_t n);

/* Every k-th step (k = 0: never; default 0) also accumulates, in its epilogue, the FP64 wall
   momentum exchange (lb_wall_stress averages over the steps that did) and the count of
   non-finite or non-positive densities (the health latch).  Each workgroup adds to its own row
   of running sums; lb_step folds them once per call, in fixed order, and starts the
   asynchronous health readback.  Masses, momentum and flow rate come from lb_totals.
   Host call. */
int lb_set_reduce_every(lb_ctx *ctx, int32_t k);

/* Density and velocity of the current state (section "Lattice Kinetic Theory for non-ideal
   fluids": the density and momentum are the zeroth and first moments of the populations,
   rho = sum_l f_l, rho u = sum_l c_l f_l; for the mixture the densities of the emulsion
   section's two species and their common flow): rho (device, [n_species][ly][lx]) and
   u (device, [2][ly][lx]) with u = (sum_s j_s + F_s / 2) / sum_s rho_s, the momentum counted
   half-way through the forcing of the step (the paper does not fix which velocity is reported;
   this one is consistent with the (tau - 1/2)^2 forcing term of the lattice stress).  F_s is
   the force of eq. (FORCE) plus the A-B repulsion and the body force.  dtype: lb_dtype.
   Either pointer may be NULL.  Asynchronous. */
int lb_moments(lb_ctx *ctx, void *rho, void *u, int32_t dtype);

/* Pressure tensor of the current state at every site (section "The Stress Field on The
   lattice" and Appendix A): sigma (device, [3][ly][lx], components xx, xy, yy) =
   sum_s [c_s^2 rho_s delta + sigma^(int)_s + (tau_s - 1/2)^2 F_s F_s / rho_s] + sigma^(AB), with
   sigma^(int)_s built shell by shell as Appendix A writes it (G_ss,1 w(q) + G_ss,2 p(q) per
   shell: half of each first- and second-shell pair at its two ends; midpoint terms for shells 4
   and 8; for shell 5 the pair at its ends plus the four extra pair products), and the A-B pair
   stress (G_AB / 2) sum_l t(q) [r_A(x) r_B(x + c_l) + r_B(x) r_A(x + c_l)] c_l c_l over the first
   belt (r = rho, or psi with cross_uses_psi).  Wall ghost rows enter as in the force.  Across a
   relaxed flat interface the normal component is uniform and equals the bulk pressure (BULK).
   dtype: lb_dtype.  One read of the state (a step without the store); the state is not
   changed.  Asynchronous. */
int lb_stress_field(lb_ctx *ctx, void *sigma, int32_t dtype);

/* Time-averaged x-force per unit wall length on the bottom and top walls (host out[2]),
   averaged over the reduced steps since the last reset; momentum exchange of the bounced
   populations, c_x f* out minus c_x of the reflected population (2 c_x f* for walls at rest,
   less rho_wall[s] U / 3 per site and species for a wall moving with U).
   reset != 0 clears the running average after reading.
   Channel lattices only (LB_ESTATE otherwise).  Synchronises. */
int lb_wall_stress(lb_ctx *ctx, double out[2], int32_t reset);

/* FP64 totals of the current state (host outputs): species masses mass[s] and total
   momentum (sum_s j_s), the quantities the collision of eq. (LB) conserves (section "Lattice
   Kinetic Theory for non-ideal fluids"; the emulsion section keeps each species' mass fixed by
   its initial condition); also the flow rate (1/lx) sum u_x of the confined flows (section
   "Numerical simulations of confined pressure-driven flows", u as in lb_moments) if
   flow != NULL.  Sums are FP64 in a fixed order whatever the storage mode.  Launches one
   reduction pass.  Synchronises; returns LB_EUNSTABLE on a bad density. */
int lb_totals(lb_ctx *ctx, double mass[2], double momentum[2], double *flow);

/* Write the current pre-collision populations f(t) in the canonical FP64 layout to dst
   (device, n_species*9*ly*lx doubles): the state of eq. (LB) at time t, the populations f_l(x, t)
   before the collision of step t (section "Lattice Kinetic Theory for non-ideal fluids"), in the
   D2Q9 order of the conventions above, species by species.  Storage modes that keep deviations
   add W_l rho_ref[s] back.  Asynchronous. */
int lb_checkpoint(lb_ctx *ctx, void *dst_f64);

/* Replace the state by canonical FP64 pre-collision populations src (device; the layout of
   lb_checkpoint: f_l(x, t) of eq. (LB) before the collision of step t), converted to the
   storage mode (rounded for LB_F32 / LB_BF16DEV).  The step count is kept (lb_set_time sets
   it).  Clears a latched LB_EUNSTABLE.  Asynchronous. */
int lb_restore(lb_ctx *ctx, const void *src_f64);

/* Number of completed time steps. */
int64_t lb_time(const lb_ctx *ctx);

/* Set the step count t >= 0 (host call).  The count picks the reducing steps
   (lb_set_reduce_every) and seeds the stochastic rounding bits of step t, so a run resumed
   in a new context from lb_checkpoint data continues bit for bit as the uninterrupted run
   when its count is set to the checkpoint's lb_time before stepping.  LB_EINVAL for t < 0. */
int lb_set_time(lb_ctx *ctx, int64_t t);

/* Launch shape of the step kernel: strip width tx in {64, 128, 256} columns (one workgroup
   thread per column) and sy >= 1 rows per workgroup.  Any shape gives bitwise identical
   results.  Host call. */
int lb_set_tile(lb_ctx *ctx, int32_t tx, int32_t sy);
int lb_get_tile(const lb_ctx *ctx, int32_t *tx, int32_t *sy);

/* Choose the step kernel's variant for the population traffic (enum lb_store_policy).  The
   default, LB_STORES_AUTO, takes the streaming variant when both population buffers together
   exceed the 256 MiB Infinity Cache and the write-through one otherwise; the other two values
   force one.  All variants give bitwise identical results; only their speed differs.
   Captured graphs are rebuilt.  Host call; LB_EINVAL for any other value. */
int lb_set_store_policy(lb_ctx *ctx, int32_t policy);

/* Rounding of the population stores of a BF16-deviation context (enum lb_rounding).  With
   LB_ROUND_NEAREST (default) every store rounds to nearest, and an increment below half a
   BF16 step of the stored deviation (a weak body force) is lost at every step.  With
   LB_ROUND_STOCHASTIC each store rounds away from zero with probability equal to the dropped
   fraction, using bits hashed from the site, the plane and the time step: unbiased, and
   bitwise reproducible for any launch shape and under graph replay.  Device memory for one
   double is allocated on first use.  LB_EINVAL for other storage modes; lb_adjoint refuses
   stochastically rounding contexts (it recomputes states).  Host call. */
int lb_set_rounding(lb_ctx *ctx, int32_t mode);

/* Temporal blocking (every storage mode): with LB_TWO_STEP_ON, lb_step advances plain steps
   (no reductions, lb_set_reduce_every k = 0) two at a time, one launch per pair, keeping the
   intermediate post-collision populations on chip, so the populations cross HBM once per two
   steps.  Each wave updates a strip of 54 columns from a 64-column window and a segment of
   `rows` rows (0: the default, sized so the whole grid is resident), recomputing the overlaps.
   The per-site arithmetic and the rounding of the intermediate to the storage format are those
   of two single steps: results are bitwise identical to LB_TWO_STEP_OFF (also with stochastic
   BF16 rounding and under graph replay).  LB_TWO_STEP_AUTO (the default) pairs the steps where
   they measured faster, for lattices whose two population buffers exceed the 256 MiB Infinity
   Cache: walled FP32 and periodic FP64 lattices.  LB_EINVAL for rows < 0.  Host call. */
enum lb_two_step { LB_TWO_STEP_OFF = 0, LB_TWO_STEP_ON = 1, LB_TWO_STEP_AUTO = 2 };
int lb_set_two_step(lb_ctx *ctx, int32_t enable, int32_t rows);

/* 1 if lb_step currently advances plain steps in pairs (lb_set_two_step and the reduction
   setting), 0 if one per launch, -1 for a NULL context.  Pure host call. */
int lb_two_step_active(const lb_ctx *ctx);

/* Replay plain steps from captured HIP graphs: with steps > 0 (even) and no reductions
   (lb_set_reduce_every k = 0), lb_step runs whole groups of `steps` launches as one graph
   launch on the context's stream and the remainder one by one.  Graphs are captured on first
   use on a private stream and rebuilt after lb_set_tile / lb_autotune.  steps = 0 turns
   graphs off.  Host call; results are bitwise those of individual launches. */
int lb_set_graph(lb_ctx *ctx, int32_t steps);

/* Autotuner: time trial_steps launches of each candidate launch shape (tx in {64, 128, 256},
   sy from 1 to 64, and the current shape) with HIP events on the context's stream, keep the
   fastest and return it in *tx, *sy and its time per step in milliseconds in *ms (any
   output may be NULL).  Trial launches read the current state and write the other
   population buffer, so the state is unchanged.  Synchronises. */
int lb_autotune(lb_ctx *ctx, int32_t trial_steps, int32_t *tx, int32_t *sy, double *ms);

/* Replace the couplings (G_ss,1, G_ss,2, G_AB, weights, body force, wall densities and
   velocities) of a running simulation; validated as in lb_init.  Takes effect at the next
   step.  Host call. */
int lb_set_couplings(lb_ctx *ctx, const lb_couplings *cpl);

/*
 * Stream-wise averaged profiles for the rheology of the confined flows (emulsion section:
 * the averaged velocity and density profiles and stress of the pressure-driven channel and of
 * the planar Couette cell, from which the local fluidity f(z) = (du/dz) / sigma and the
 * cooperative length of eq. (fluidity) / eq. (predict) follow; and the stress correlator of
 * eq. (correlator)).
 *
 * lb_profile writes, for the current state at time t, out[0 .. ly-1] = ubar(y), the x-average
 * of the velocity u_x of lb_moments in row y, and out[ly .. 2 ly] = sigma(k), k = 0..ly, the
 * x-averaged shear stress through the horizontal line k between rows k-1 and k: the x-force
 * per unit length that the material above the line exerts on the material below it in step
 * t, i.e. the pair forces of eq. (FORCE) (and of the A-B repulsion) between sites on the two
 * sides, minus the x-momentum the streaming populations carry upward across the line.
 * sigma(0) = W_bot(t) and sigma(ly) = -W_top(t) on channel lattices (the walls' momentum
 * exchange of lb_wall_stress); on periodic lattices sigma(ly) = sigma(0).  Exact lattice
 * momentum balance: the x-momentum of the rows between lines k1 < k2 changes in step t by
 * lx (sigma(k2) - sigma(k1)) + g_x times their mass.  out[2 ly + 1 .. 3 ly] and
 * out[3 ly + 1 .. 4 ly] are the x-averaged densities of species A and B in row y (B zero for
 * one component).  out: device, 4 ly + 1 doubles.
 * One read of the state (a step without the store) plus a small second pass; the state
 * is not changed.  Asynchronous.
 */
int lb_profile(lb_ctx *ctx, double *out);

/*
 * lb_profile without allocation, for callers that cannot allocate device memory (code under
 * HIP graph capture, tight sampling loops, hosts that forbid hipMalloc): the same passes and
 * the same output as lb_profile, bit for bit, but the block sums and row sums go to a static
 * scratch array of 2^19 doubles (4 MiB) in the library's code object on each device, whose
 * address lb_init looks up once per device.  The call allocates nothing.  It needs
 * ((lx + tx - 1) / tx * (tx / 64) + 1) * ly * 7 doubles of scratch (tx: the strip width of
 * lb_set_tile); larger lattices are refused with LB_EINVAL (use lb_profile, or a narrower
 * strip).  Every call on a device shares that device's scratch: calls on one device whose
 * work overlaps (contexts on different streams) race, so order them on one stream or
 * synchronise between them.  Asynchronous.
 */
int lb_profile_noalloc(lb_ctx *ctx, double *out);

/*
 * Time statistics of n >= 1 profile samples (device, [n][4 ly + 1], as written by
 * lb_profile), written to out (device, 6 ly + 3 doubles):
 *   out[0 .. ly-1]             <ubar(y)>
 *   out[ly .. 2ly]             <sigma(k)>, k = 0..ly
 *   out[2ly+1 .. 3ly+1]        <f(k)>, the time average of the local fluidity
 *                              f(k) = (ubar(k) - ubar(k-1)) / sigma(k) at line k; at the walls of a
 *                              channel the velocity difference is taken to the wall, over half a
 *                              site: f(0) = 2 (ubar(0) - U_bot) / sigma(0), f(ly) = 2 (U_top - ubar(ly-1)) / sigma(ly)
 *   out[3ly+2 .. 4ly+2]        C_sigma(k, k0) of eq. (correlator): the covariance of sigma(k) and
 *                              sigma(k0) over the samples divided by the variance of sigma(k0)
 *                              (NaN if that variance is 0)
 *   out[4ly+3 .. 5ly+2]        <rho_A(y)>
 *   out[5ly+3 .. 6ly+2]        <rho_B(y)>
 * with 0 <= k0 <= ly.  Sums run over the samples in order, in FP64.  Asynchronous.
 */
int lb_profile_stats(lb_ctx *ctx, const double *samples, int64_t n, int32_t k0, double *out);

/*
 * Least-squares fit of the cooperative-length prediction, eq. (predict), to a fluidity
 * profile: f(z) = f_b + (f_w - f_b) cosh((z - H/2) / zeta) / cosh(H / (2 zeta)) over the n >= 3
 * points (z[i], f[i]) (host arrays), 0 <= z <= H.  For each zeta the model is linear in f_b and
 * f_w (solved exactly); zeta is searched on a logarithmic grid over [zeta_min, zeta_max]
 * (0 < zeta_min < zeta_max) and refined by golden section.  out (host): zeta, f_b, f_w and
 * the rms residual.  Pure host call.
 */
int lb_fit_cooperative_length(const double *z, const double *f, int32_t n, double H, double zeta_min,
                              double zeta_max, double out[4]);

/*
 * Disjoining pressure of flat films from their film tensions, eq. (doppiasigma) (section "The
 * case of two near-interfaces: emergence of the disjoining pressure"): a flat film of thickness
 * h has the film tension gamma_f(h) (the integral across it of the normal minus the tangential
 * pressure, e.g. the row sum of sigma_xx - sigma_yy from lb_stress_field across a film normal to
 * x), and differentiating eq. (doppiasigma) gives d gamma_f = h d Pi.  With Pi = 0 at the
 * thickest film and gamma_f taken linear between the given thicknesses,
 * Pi(h) = -int_h^h_max gamma_f'(h') / h' dh', integrated exactly on each interval.  h, gamma_f:
 * host arrays of n >= 2 films (any order; thicknesses positive and distinct); pi: host output
 * in the input order.  LB_EINVAL otherwise.  Pure host call.
 */
int lb_disjoining_pressure(const double *h, const double *gamma_f, int32_t n, double *pi);

/*
 * Adjoint (reverse-time) gradient of the time-averaged wall stress and flow rate (emulsion
 * section: Poiseuille flow of a confined emulsion) over the next T >= 1 steps:
 *   L = lw[0] * (1/T) sum_t (W_bot(t) + W_top(t)) / 2  +  lw[1] * (1/T) sum_t Q(t),
 * W_bot/W_top as in lb_wall_stress for step t, Q(t) = (1/lx) sum_x u_x (u as in lb_moments),
 * t running over the T steps from the current state, which is held fixed.  Outputs (host):
 * *loss = L and grad[7] = dL/d(G_AA,1, G_BB,1, G_AA,2, G_BB,2, G_AB, g_x, g_y).
 * The forward pass keeps an FP64 checkpoint of the populations every `every` steps
 * (every <= 0: ceil(sqrt(T))); the reverse sweep recomputes each segment's states from its
 * checkpoint and runs the hand-written reverse step (FP64 for LB_F64 contexts or with
 * flags & LB_ADJ_FP64, FP32 otherwise).  With several segments the reverse steps run on a
 * second stream of the library's own, created and destroyed by the call, one segment behind
 * the recompute on the context's stream (two segment buffers in the workspace); the result
 * does not depend on the overlap.  every = 1 keeps instead what the reverse step reads
 * of every state (moments and pseudopotential of every site, populations of the two rows
 * next to the walls): no recompute, at about T * 64 (FP64 reverse) or T * 32 (FP32) bytes per
 * site of workspace.  workspace: device buffer of
 * lb_adjoint_workspace_bytes(ctx, T, every, flags) bytes,
 * owned by the caller.  On return the context holds the state after T steps, bit for bit as
 * lb_step(ctx, T) would leave it, and lb_time has advanced by T; the running wall-stress
 * average is reset.  Synchronises. */
enum lb_adjoint_flags {
  LB_ADJ_FP64 = 1  /* reverse sweep in FP64 also for FP32 / BF16 contexts (forward stays in the storage mode) */
};
size_t lb_adjoint_workspace_bytes(const lb_ctx *ctx, int64_t T, int32_t every, int32_t flags);
int lb_adjoint(lb_ctx *ctx, int64_t T, int32_t every, int32_t flags, const double loss_weights[2], double *loss,
               double grad[7], void *workspace, size_t workspace_bytes);

/* Message of the last failure on ctx (ctx = NULL: last failure of lb_init in this thread). */
const char *lb_last_error(const lb_ctx *ctx);

/* Release the context's own buffers (not the caller's). */
void lb_destroy(lb_ctx *ctx);

/* ---------------------------------------------------------------------------------------
 * Batches: n independent lattices (e.g. channels of uneven size with their own couplings,
 * relaxation times and body forces) advanced together by one persistent kernel launch per
 * time step.  Each instance evolves exactly as it would in its own lb_init context (same
 * step, bitwise the same per-site arithmetic).  All instances share storage, n_species and
 * walls; sizes, couplings, tau and psi parameters are per instance.
 * Ownership and errors as for lb_ctx; lb_batch_last_error(NULL) reports lb_batch_init.
 * ------------------------------------------------------------------------------------- */
typedef struct lb_batch lb_batch;

/* Bytes of ONE population buffer holding all n instances (each instance's lb_pop_bytes,
   rounded up to 256 bytes).  0 for invalid input.  Pure host call. */
size_t lb_batch_pop_bytes(int32_t n, const lb_lattice *lats);

/* Create a batch.  lats, cpls, psis: host arrays of n; tau: host [n][2]; rho_init: host
   array of n host pointers, instance i [n_species][ly_i][lx_i].  Validation per instance as
   in lb_init.  pop_a, pop_b: device buffers of pop_bytes >= lb_batch_pop_bytes.
   Synchronises the stream. */
int lb_batch_init(lb_batch **out, int32_t n, const lb_lattice *lats, const lb_couplings *cpls, const double *tau,
                  const lb_psi_params *psis, const double *const *rho_init, void *pop_a, void *pop_b,
                  size_t pop_bytes, void *hip_stream);

/* Advance every instance by n >= 0 steps: one launch per step over the tiles of all
   instances (plus one reduction launch on reduced steps).  Asynchronous. */
int lb_batch_step(lb_batch *b, int64_t n);

/* As lb_set_reduce_every, for every instance. */
int lb_batch_set_reduce_every(lb_batch *b, int32_t k);

/* lb_set_rounding for a batch: every instance's BF16 stores rounded to nearest or
   stochastically; an instance's bits equal those of a single context of the same lattice
   (the hash uses the instance's own site indices and the batch's step count). */
int lb_batch_set_rounding(lb_batch *b, int32_t mode);

/* As lb_set_graph: graphs of `steps` batch launches. */
int lb_batch_set_graph(lb_batch *b, int32_t steps);

/* Tile shape of all instances (tx in {64, 128, 256}, sy >= 1) and the persistent grid:
   grid workgroups take the tiles in rounds (grid = 0: one workgroup per tile).  Rebuilds the
   tile table.  Synchronises. */
int lb_batch_set_tile(lb_batch *b, int32_t tx, int32_t sy, int32_t grid);
int lb_batch_get_tile(const lb_batch *b, int32_t *tx, int32_t *sy, int32_t *grid);

/* Autotuner over tx, sy in {2, ..., 32} and grid in {resident workgroups, one per tile}, as
   lb_autotune; out[3] = (tx, sy, grid) and *ms (either may be NULL).  Synchronises. */
int lb_batch_autotune(lb_batch *b, int32_t trial_steps, int32_t out[3], double *ms);

/* Moments of instance i, as lb_moments (device outputs [n_species][ly_i][lx_i] and
   [2][ly_i][lx_i]).  Asynchronous. */
int lb_batch_moments(lb_batch *b, int32_t i, void *rho, void *u, int32_t dtype);

/* Profiles of instance i, as lb_profile (device out, 4 ly_i + 1 doubles); time statistics of
   its samples follow from lb_profile_stats on a context of the same lattice, or directly from
   the samples.  Asynchronous. */
int lb_batch_profile(lb_batch *b, int32_t i, double *out);

/* Site pressure tensor of instance i, as lb_stress_field (device [3][ly_i][lx_i]).
   Asynchronous. */
int lb_batch_stress_field(lb_batch *b, int32_t i, void *sigma, int32_t dtype);

/* FP64 totals of every instance (host out[n][5]: mass A, mass B, momentum x, momentum y,
   flow rate), as lb_totals.  Synchronises. */
int lb_batch_totals(lb_batch *b, double *out);

/* Time-averaged wall stress of every instance (host out[n][2]), as lb_wall_stress.
   Channel batches only.  Synchronises. */
int lb_batch_wall_stress(lb_batch *b, double *out, int32_t reset);

/* Checkpoint / restore instance i in the canonical FP64 layout, as lb_checkpoint /
   lb_restore. */
int lb_batch_checkpoint(lb_batch *b, int32_t i, void *dst_f64);
int lb_batch_restore(lb_batch *b, int32_t i, const void *src_f64);

int64_t lb_batch_time(const lb_batch *b);
/* As lb_set_time, for the batch's common step count. */
int lb_batch_set_time(lb_batch *b, int64_t t);
const char *lb_batch_last_error(const lb_batch *b);
void lb_batch_destroy(lb_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* LB355_LB_H */
