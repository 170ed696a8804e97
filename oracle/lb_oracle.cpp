// Plain FP64 CPU oracle of the two-belt pseudopotential D2Q9 lattice Boltzmann step.
//
// TEST INFRASTRUCTURE ONLY.  This file is the reference the GPU path is checked against.
// Only tests, the smoke check and the CPU-baseline leg of the benchmark may load it; the
// product library never links or calls it, and it shares no code, table or header with the
// GPU path.  It is written for clarity, not speed: every stage is a separate loop over the
// whole lattice, in the order the method states it.
//
// What it computes (Sbragaglia, Benzi, Bernaschi, Succi, arXiv:1402.6019):
//   * BGK lattice Boltzmann equation, eq. (LB), Sec. "Lattice Kinetic Theory for non-ideal
//     fluids": f_l(x+c_l, t+1) - f_l(x,t) = -(f_l - f_l^eq(rho,u))/tau, applied to every l.
//   * Moments rho = sum_l f_l, rho u = sum_l f_l c_l (same section, unnumbered display).
//   * Equilibrium: second-order Hermite D2Q9 form; the paper only fixes its second moment
//     (sum c c f^eq = c_s^2 rho delta + rho u u), so this form is a reading.
//   * Pseudopotential psi = psi0 (1 - exp(-rho/rho0)) (Sec. "Numerical simulations of confined
//     pressure-driven flows": psi = 1 - exp(-rho/rho0), rho0 = 0.83 for the emulsion).
//   * Two-belt competing force, eq. (FORCE), Sec. "Competing interactions":
//       F = -G1 psi(x) sum_{l=1..12} w(|c_l|^2) psi(x+c_l) c_l
//           -G2 psi(x) sum_{l=1..24} p(|c_l|^2) psi(x+c_l) c_l
//     evaluated exactly as written (two separate sums, links in the order of Fig. 1).
//   * Forcing by shifting the equilibrium velocity, u^eq -> u^eq + tau F / rho (same section
//     as eq. (FORCEa)).
//   * Binary mixture (emulsion section): one population set per species, each evolving by
//     (LB); an A-B repulsion proportional to G_AB, read as the Shan-Chen multicomponent form
//       F_s += -G_AB rho_s(x) sum_{l=1..8} t(|c_l|^2) rho_sbar(x+c_l) c_l
//     with D2Q9 weights t; a common velocity u' = sum_s(j_s/tau_s) / sum_s(rho_s/tau_s).
//   * Planar channel (emulsion section: no-slip walls at z=0 and z=H, volume force):
//     halfway bounce-back with walls at y=-1/2 and y=ly-1/2; wall ghost sites carry the
//     densities rho_wall (wetting); body force rho_s g per species.
//   * Planar Couette cell (same section: the walls move with velocities +-U_w along x):
//     bounce-back off a wall moving with velocity U adds 6 W_l rho_w c_l . U to the reflected
//     population (the wall's momentum density is read as rho_wall[s] U per species; the
//     added terms of one site sum to zero, so mass is conserved).
//
// Conventions fixed here (the paper is silent): state = pre-collision populations f(x,t);
// arrays are [species][l][y][x], x fastest; sums run in increasing l.
//
// The scalar type is a template parameter so the same code runs in std::complex<double>
// for complex-step derivatives (every stage is analytic in the couplings).

#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

extern "C" {
typedef struct {
  int32_t lx, ly, ns, walls;   // walls: 0 periodic in y, 1 channel (bounce-back rows)
  double g1[2], g2[2], gab;    // G_ss,1 (attractive, <0), G_ss,2 (repulsive, >0), G_AB
  double w[5], p[5], t[2];     // shell weights for |c|^2 = 1,2,4,5,8 ; cross weights |c|^2 = 1,2
  double body[2];              // acceleration g; force density rho_s g
  double rho_wall[2];          // ghost densities on solid rows (channel only)
  double tau[2];
  double psi0, rho0;
  int32_t cross_psi;           // 0: cross term uses rho (default reading), 1: uses psi
  int32_t pad_;
  double u_wall[2];            // x-velocity of the bottom and the top wall (channel only)
} orc_config;
}

namespace {

// D2Q9 lattice: velocities, weights, opposite directions.
const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
const double WL[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                      1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

// The 24 interaction links of Fig. 1 (two belts), numbered 1..24 as stored at index 0..23.
// Links 1-8 are the D2Q9 links; 9-12 have |c|^2 = 4; 13-20 have |c|^2 = 5 in the order the
// Appendix A extra terms imply (c13 = c5 - c3, c14 = c5 - c4, c15 = c2 - c8, c16 = c6 - c1);
// 21-24 have |c|^2 = 8.
const int LX[24] = {1, 0, -1, 0, 1, -1, -1, 1, 2, 0, -2, 0, 2, 1, -1, -2, -2, -1, 1, 2, 2, -2, -2, 2};
const int LY[24] = {0, 1, 0, -1, 1, 1, -1, -1, 0, 2, 0, -2, 1, 2, 2, 1, -1, -2, -2, -1, 2, 2, -2, -2};

int shell_index(int cx, int cy) {
  switch (cx * cx + cy * cy) {
    case 1: return 0;
    case 2: return 1;
    case 4: return 2;
    case 5: return 3;
    case 8: return 4;
  }
  return -1;
}

inline int wrap(int a, int n) {
  int r = a % n;
  return r < 0 ? r + n : r;
}

template <typename T>
T exp_t(const T &x) { using std::exp; return exp(x); }

template <typename T>
struct Sim {
  int lx, ly, ns, walls, cross_psi;
  size_t nsite;
  // Couplings and parameters in the scalar type (complex-step perturbs them).
  T g1[2], g2[2], gab, body[2], tau[2], psi0, rho0, rho_wall[2];
  double u_wall[2];
  double w[5], p[5], t[2];
  std::vector<T> f, fs;             // pre- and post-collision populations [s][l][y][x]
  std::vector<T> rho, jx, jy, psi;  // [s][y][x]
  std::vector<T> fx, fy;            // force [s][y][x]
  int64_t time = 0;

  explicit Sim(const orc_config &c) {
    lx = c.lx; ly = c.ly; ns = c.ns; walls = c.walls; cross_psi = c.cross_psi;
    nsite = (size_t)lx * ly;
    for (int s = 0; s < 2; ++s) {
      g1[s] = c.g1[s]; g2[s] = c.g2[s]; tau[s] = c.tau[s]; rho_wall[s] = c.rho_wall[s];
      body[s] = c.body[s];
    }
    gab = c.gab; psi0 = c.psi0; rho0 = c.rho0;
    u_wall[0] = c.u_wall[0]; u_wall[1] = c.u_wall[1];
    for (int q = 0; q < 5; ++q) { w[q] = c.w[q]; p[q] = c.p[q]; }
    t[0] = c.t[0]; t[1] = c.t[1];
    f.assign((size_t)ns * 9 * nsite, T(0));
    fs = f;
    rho.assign((size_t)ns * nsite, T(0));
    jx = rho; jy = rho; psi = rho; fx = rho; fy = rho;
  }

  size_t at(int s, int l, int y, int x) const { return (((size_t)s * 9 + l) * ly + y) * lx + x; }
  size_t at(int s, int y, int x) const { return ((size_t)s * ly + y) * lx + x; }

  T pseudo(const T &r) const { return psi0 * (T(1.0) - exp_t(-r / rho0)); }

  // True when (x, y) is a fluid site; returns its wrapped coordinates.
  bool fluid(int x, int y, int &xi, int &yi) const {
    xi = wrap(x, lx);
    if (walls && (y < 0 || y >= ly)) return false;
    yi = wrap(y, ly);
    return true;
  }
  T psi_at(int s, int x, int y) const {
    int xi, yi;
    if (!fluid(x, y, xi, yi)) return pseudo(rho_wall[s]);
    return psi[at(s, yi, xi)];
  }
  T rho_at(int s, int x, int y) const {
    int xi, yi;
    if (!fluid(x, y, xi, yi)) return rho_wall[s];
    return rho[at(s, yi, xi)];
  }

  // Stage 1: moments rho_s, j_s of the pre-collision populations; psi_s(rho_s).
  void moments() {
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ly; ++y)
      for (int s = 0; s < ns; ++s)
        for (int x = 0; x < lx; ++x) {
          T r = 0, ax = 0, ay = 0;
          for (int l = 0; l < 9; ++l) {
            T v = f[at(s, l, y, x)];
            r += v;
            ax += v * double(CX[l]);
            ay += v * double(CY[l]);
          }
          rho[at(s, y, x)] = r;
          jx[at(s, y, x)] = ax;
          jy[at(s, y, x)] = ay;
          psi[at(s, y, x)] = pseudo(r);
        }
  }

  // Stage 2: eq. (FORCE) per species, the A-B repulsion and the body force.
  void forces() {
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ly; ++y)
      for (int s = 0; s < ns; ++s)
        for (int x = 0; x < lx; ++x) {
          T s1x = 0, s1y = 0, s2x = 0, s2y = 0;
          for (int l = 0; l < 12; ++l) {  // attractive sum, links 1..12 (|c|^2 <= 4), weights w
            T nb = psi_at(s, x + LX[l], y + LY[l]);
            double wq = w[shell_index(LX[l], LY[l])];
            s1x += wq * nb * double(LX[l]);
            s1y += wq * nb * double(LY[l]);
          }
          for (int l = 0; l < 24; ++l) {  // repulsive sum, links 1..24 (|c|^2 <= 8), weights p
            T nb = psi_at(s, x + LX[l], y + LY[l]);
            double pq = p[shell_index(LX[l], LY[l])];
            s2x += pq * nb * double(LX[l]);
            s2y += pq * nb * double(LY[l]);
          }
          T ps = psi[at(s, y, x)];
          T Fx = -g1[s] * ps * s1x - g2[s] * ps * s2x;
          T Fy = -g1[s] * ps * s1y - g2[s] * ps * s2y;
          if (ns == 2) {  // A-B repulsion over the first belt (links 1..8)
            int sb = 1 - s;
            T cxs = 0, cys = 0;
            for (int l = 0; l < 8; ++l) {
              T nb = cross_psi ? psi_at(sb, x + LX[l], y + LY[l]) : rho_at(sb, x + LX[l], y + LY[l]);
              double tq = t[shell_index(LX[l], LY[l])];
              cxs += tq * nb * double(LX[l]);
              cys += tq * nb * double(LY[l]);
            }
            T self = cross_psi ? ps : rho[at(s, y, x)];
            Fx += -gab * self * cxs;
            Fy += -gab * self * cys;
          }
          T r = rho[at(s, y, x)];
          Fx += r * body[0];
          Fy += r * body[1];
          fx[at(s, y, x)] = Fx;
          fy[at(s, y, x)] = Fy;
        }
  }

  // Stage 3: BGK collision (LB) towards f^eq(rho_s, u^eq_s), u^eq_s = u' + tau_s F_s / rho_s.
  void collide() {
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ly; ++y)
      for (int x = 0; x < lx; ++x) {
        T num_x = 0, num_y = 0, den = 0;
        for (int s = 0; s < ns; ++s) {
          num_x += jx[at(s, y, x)] / tau[s];
          num_y += jy[at(s, y, x)] / tau[s];
          den += rho[at(s, y, x)] / tau[s];
        }
        T upx = num_x / den, upy = num_y / den;
        for (int s = 0; s < ns; ++s) {
          T r = rho[at(s, y, x)];
          T ux = upx + tau[s] * fx[at(s, y, x)] / r;
          T uy = upy + tau[s] * fy[at(s, y, x)] / r;
          T uu = ux * ux + uy * uy;
          for (int l = 0; l < 9; ++l) {
            T cu = double(CX[l]) * ux + double(CY[l]) * uy;
            T feq = WL[l] * r * (T(1.0) + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
            T v = f[at(s, l, y, x)];
            fs[at(s, l, y, x)] = v - (v - feq) / tau[s];
          }
        }
      }
  }

  // Population that bounces back into direction l (c_ly = +1 off the bottom wall, -1 off
  // the top wall) at a site whose outgoing population was fout: halfway bounce-back plus
  // the momentum the moving wall hands over, 6 W_l rho_w,s (c_l . U).
  T reflected(int s, int l, const T &fout) const {
    const double U = CY[l] > 0 ? u_wall[0] : u_wall[1];
    return fout + 6.0 * WL[l] * rho_wall[s] * (double(CX[l]) * U);
  }

  // Stage 4: streaming f_l(x, t+1) = f*_l(x - c_l, t); halfway bounce-back off solid rows.
  void stream() {
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ly; ++y)
      for (int s = 0; s < ns; ++s)
        for (int l = 0; l < 9; ++l)
          for (int x = 0; x < lx; ++x) {
            int xi, yi;
            if (fluid(x - CX[l], y - CY[l], xi, yi))
              f[at(s, l, y, x)] = fs[at(s, l, yi, xi)];
            else
              f[at(s, l, y, x)] = reflected(s, l, fs[at(s, OPP[l], y, x)]);
          }
  }

  // Observables of the step just collided: [mass_0, mass_1, P_x, P_y, W_bot, W_top, Q, 0].
  //   mass, momentum: of the pre-collision state f(t).
  //   W_bot/W_top: x-momentum per unit wall length handed to the bottom/top wall by the
  //   populations that bounce back in this step: c_x f* of the outgoing population minus
  //   c_x of the reflected one, i.e. 2 c_x f* less what a moving wall adds.
  //   Q: (1/lx) sum_x,y u_x with u = (sum_s j_s + F_s/2) / sum_s rho_s.
  void record(T *out) const {
    T mass[2] = {0, 0}, px = 0, py = 0, wb = 0, wt = 0, q = 0;
    for (int s = 0; s < ns; ++s)
      for (size_t i = 0; i < nsite; ++i) {
        mass[s] += rho[s * nsite + i];
        px += jx[s * nsite + i];
        py += jy[s * nsite + i];
      }
    for (int y = 0; y < ly; ++y)
      for (int x = 0; x < lx; ++x) {
        T num = 0, den = 0;
        for (int s = 0; s < ns; ++s) {
          num += jx[at(s, y, x)] + 0.5 * fx[at(s, y, x)];
          den += rho[at(s, y, x)];
        }
        q += num / den;
      }
    if (walls) {
      for (int s = 0; s < ns; ++s)
        for (int x = 0; x < lx; ++x)
          for (int l = 0; l < 9; ++l) {
            if (CY[l] == -1) {
              const T out = fs[at(s, l, 0, x)];
              wb += double(CX[l]) * out - double(CX[OPP[l]]) * reflected(s, OPP[l], out);
            }
            if (CY[l] == +1) {
              const T out = fs[at(s, l, ly - 1, x)];
              wt += double(CX[l]) * out - double(CX[OPP[l]]) * reflected(s, OPP[l], out);
            }
          }
    }
    out[0] = mass[0]; out[1] = mass[1]; out[2] = px; out[3] = py;
    out[4] = wb / double(lx); out[5] = wt / double(lx); out[6] = q / double(lx); out[7] = 0;
  }

  void step(T *rec) {
    moments();
    forces();
    collide();
    if (rec) record(rec);
    stream();
    ++time;
  }

  // S0: rest equilibrium f_l = W_l rho_init.
  void init_rest(const double *rho_init) {
    for (int s = 0; s < ns; ++s)
      for (int l = 0; l < 9; ++l)
        for (size_t i = 0; i < nsite; ++i) f[((size_t)s * 9 + l) * nsite + i] = WL[l] * rho_init[s * nsite + i];
    time = 0;
  }
};

inline double re(double v) { return v; }
inline double re(const std::complex<double> &v) { return v.real(); }
inline double im(double) { return 0.0; }
inline double im(const std::complex<double> &v) { return v.imag(); }

}  // namespace

extern "C" {

void *orc_create(const orc_config *c) { return new Sim<double>(*c); }
void orc_destroy(void *h) { delete static_cast<Sim<double> *>(h); }

void orc_set_threads(int n) {
#ifdef _OPENMP
  omp_set_num_threads(n > 0 ? n : 1);
#else
  (void)n;
#endif
}
int orc_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_init_rest(void *h, const double *rho_init) { static_cast<Sim<double> *>(h)->init_rest(rho_init); }

void orc_set_f(void *h, const double *f) {
  auto *s = static_cast<Sim<double> *>(h);
  std::memcpy(s->f.data(), f, s->f.size() * sizeof(double));
}
void orc_get_f(void *h, double *f) {
  auto *s = static_cast<Sim<double> *>(h);
  std::memcpy(f, s->f.data(), s->f.size() * sizeof(double));
}
int64_t orc_time(void *h) { return static_cast<Sim<double> *>(h)->time; }

// Advance n steps; rec (n x 8, may be NULL) receives the per-step observables.
void orc_step(void *h, int n, double *rec) {
  auto *s = static_cast<Sim<double> *>(h);
  for (int k = 0; k < n; ++k) s->step(rec ? rec + 8 * (size_t)k : nullptr);
}

// Fields of the current state without advancing it.  Any pointer may be NULL.
//   rho, psi: [ns][ly][lx]; force: [ns][2][ly][lx]; u: [2][ly][lx] (half-force velocity);
//   j: [ns][2][ly][lx]; fstar: [ns][9][ly][lx] post-collision populations of this step.
void orc_fields(void *h, double *rho, double *psi, double *force, double *u, double *j, double *fstar) {
  auto *s = static_cast<Sim<double> *>(h);
  s->moments();
  s->forces();
  const size_t n = s->nsite;
  for (int sp = 0; sp < s->ns; ++sp)
    for (size_t i = 0; i < n; ++i) {
      if (rho) rho[sp * n + i] = s->rho[sp * n + i];
      if (psi) psi[sp * n + i] = s->psi[sp * n + i];
      if (force) {
        force[(2 * sp + 0) * n + i] = s->fx[sp * n + i];
        force[(2 * sp + 1) * n + i] = s->fy[sp * n + i];
      }
      if (j) {
        j[(2 * sp + 0) * n + i] = s->jx[sp * n + i];
        j[(2 * sp + 1) * n + i] = s->jy[sp * n + i];
      }
    }
  if (u)
    for (size_t i = 0; i < n; ++i) {
      double nx = 0, ny = 0, den = 0;
      for (int sp = 0; sp < s->ns; ++sp) {
        nx += s->jx[sp * n + i] + 0.5 * s->fx[sp * n + i];
        ny += s->jy[sp * n + i] + 0.5 * s->fy[sp * n + i];
        den += s->rho[sp * n + i];
      }
      u[i] = nx / den;
      u[n + i] = ny / den;
    }
  if (fstar) {
    s->collide();
    std::memcpy(fstar, s->fs.data(), s->fs.size() * sizeof(double));
  }
}

// Complex-step derivative of the time-averaged loss
//   L = lw[0] * mean_t (W_bot + W_top)/2 + lw[1] * mean_t Q,   t = 0..nsteps-1,
// starting from the pre-collision state f0, with respect to one parameter:
//   0: G1 (G_ss,1 of every species), 1: G2 (G_ss,2 of every species), 2: G_AB, 3: g_x.
// Returns L in *loss and dL/dtheta in *dloss.
void orc_cs_grad(const orc_config *c, const double *f0, int nsteps, const double *lw, int param, double h,
                 double *loss, double *dloss) {
  using C = std::complex<double>;
  Sim<C> s(*c);
  const C ih(0.0, h);
  switch (param) {
    case 0: for (int k = 0; k < 2; ++k) s.g1[k] += ih; break;
    case 1: for (int k = 0; k < 2; ++k) s.g2[k] += ih; break;
    case 2: s.gab += ih; break;
    case 3: s.body[0] += ih; break;
    default: break;
  }
  for (size_t i = 0; i < s.f.size(); ++i) s.f[i] = f0[i];
  C acc_w = 0, acc_q = 0;
  C rec[8];
  for (int k = 0; k < nsteps; ++k) {
    s.step(rec);
    acc_w += 0.5 * (rec[4] + rec[5]);
    acc_q += rec[6];
  }
  C L = lw[0] * acc_w / double(nsteps) + lw[1] * acc_q / double(nsteps);
  *loss = re(L);
  *dloss = im(L) / h;
}

}  // extern "C"
