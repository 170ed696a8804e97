// Plain FP64 CPU oracle of the three-dimensional extension of the two-belt pseudopotential
// lattice Boltzmann step (D3Q19).
//
// TEST INFRASTRUCTURE ONLY.  The reference the GPU path's 3-D step is checked against.  Only
// tests, the smoke check and the CPU-baseline leg of the benchmark may load it; the product
// library never links or calls it, and it shares no code, table or header with the GPU path
// (nor with the two-dimensional oracle).  Written for clarity, not speed: one loop over the
// whole lattice per stage, in the order the method states it.
//
// The paper (Sbragaglia, Benzi, Bernaschi, Succi, arXiv:1402.6019) treats the two-dimensional
// model and, in Sec. "Competing interactions", points to extensions to three dimensions without
// giving them.  This oracle takes the direct extension, fixed here:
//   * BGK equation (LB) on the D3Q19 lattice, second-order Hermite equilibrium, c_s^2 = 1/3;
//   * eq. (FORCE) with the same two belts, now over the integer vectors of the 5x5x5 cube:
//       F = -G1 psi(x) sum_{1 <= |c|^2 <= 4} w(|c|^2) psi(x+c) c
//           -G2 psi(x) sum_{1 <= |c|^2 <= 8} p(|c|^2) psi(x+c) c,
//     shells |c|^2 = 1, 2, 3, 4 (32 links) and 1, 2, 3, 4, 5, 6, 8 (92 links); the weights are
//     inputs (the isotropic sets are derived in weights.py: w sixth-order, p eighth-order,
//     E2 = 1/3 for both, as in two dimensions);
//   * psi = psi0 (1 - exp(-rho/rho0)); forcing by the equilibrium-velocity shift;
//   * two species with the A-B repulsion -G_AB r_s(x) sum_{D3Q19 links} t(|c|^2) r_sbar(x+c) c
//     (r = rho, or psi with cross_psi), t the D3Q19 weights, and the common velocity
//     u' = sum_s (j_s / tau_s) / sum_s (rho_s / tau_s);
//   * optional channel: halfway bounce-back walls at y = -1/2 and y = ly - 1/2, ghost densities
//     rho_wall on the solid rows seen by the force stencils, body force rho_s g; periodic in x
//     and z (and in y without walls).
// Arrays are [species][l][z][y][x], x fastest; sums run in increasing link order.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

extern "C" {
typedef struct {
  int32_t lx, ly, lz, ns, walls, cross_psi;
  double g1[2], g2[2], gab;
  double w[7], p[7];      // shell weights for |c|^2 = 1, 2, 3, 4, 5, 6, 8
  double t[2];            // A-B weights for |c|^2 = 1, 2
  double body[3];
  double rho_wall[2];
  double tau[2];
  double psi0, rho0;
} orc3_config;
}

namespace {

// D3Q19: rest, the six axis links, the twelve face diagonals; opposite links are adjacent.
const int CX[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
const int CY[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
const int CZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
const int OPP[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
double WL(int l) { return l == 0 ? 1.0 / 3.0 : (l <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }

int shell_index(int q) {
  switch (q) {
    case 1: return 0;
    case 2: return 1;
    case 3: return 2;
    case 4: return 3;
    case 5: return 4;
    case 6: return 5;
    case 8: return 6;
  }
  return -1;
}

inline int wrap(int a, int n) {
  int r = a % n;
  return r < 0 ? r + n : r;
}

struct Link { int x, y, z, q; };

struct Sim3 {
  orc3_config c;
  size_t nsite;
  std::vector<Link> links;          // every c with 1 <= |c|^2 <= 8, z outer, x inner, -2..2
  std::vector<double> f, fs;        // [s][l][z][y][x]
  std::vector<double> rho, jx, jy, jz, psi, fx, fy, fz;  // [s][z][y][x]
  int64_t time = 0;

  explicit Sim3(const orc3_config &cfg) : c(cfg) {
    nsite = (size_t)c.lx * c.ly * c.lz;
    for (int z = -2; z <= 2; ++z)
      for (int y = -2; y <= 2; ++y)
        for (int x = -2; x <= 2; ++x) {
          const int q = x * x + y * y + z * z;
          if (q >= 1 && q <= 8 && shell_index(q) >= 0) links.push_back({x, y, z, q});
        }
    f.assign((size_t)c.ns * 19 * nsite, 0.0);
    fs = f;
    rho.assign((size_t)c.ns * nsite, 0.0);
    jx = rho; jy = rho; jz = rho; psi = rho; fx = rho; fy = rho; fz = rho;
  }

  size_t site(int x, int y, int z) const { return ((size_t)z * c.ly + y) * c.lx + x; }
  size_t at(int s, int l, size_t i) const { return ((size_t)s * 19 + l) * nsite + i; }
  size_t at(int s, size_t i) const { return (size_t)s * nsite + i; }

  double pseudo(double r) const { return c.psi0 * (1.0 - std::exp(-r / c.rho0)); }

  // Site index of (x, y, z) after periodic wrapping, or -1 for a solid (wall ghost) site.
  long long fluid(int x, int y, int z) const {
    if (c.walls && (y < 0 || y >= c.ly)) return -1;
    return (long long)site(wrap(x, c.lx), wrap(y, c.ly), wrap(z, c.lz));
  }
  double psi_at(int s, int x, int y, int z) const {
    const long long i = fluid(x, y, z);
    return i < 0 ? pseudo(c.rho_wall[s]) : psi[at(s, (size_t)i)];
  }
  double rho_at(int s, int x, int y, int z) const {
    const long long i = fluid(x, y, z);
    return i < 0 ? c.rho_wall[s] : rho[at(s, (size_t)i)];
  }

  void moments() {
#pragma omp parallel for schedule(static)
    for (int z = 0; z < c.lz; ++z)
      for (int y = 0; y < c.ly; ++y)
        for (int x = 0; x < c.lx; ++x) {
          const size_t i = site(x, y, z);
          for (int s = 0; s < c.ns; ++s) {
            double r = 0, ax = 0, ay = 0, az = 0;
            for (int l = 0; l < 19; ++l) {
              const double v = f[at(s, l, i)];
              r += v;
              ax += v * CX[l];
              ay += v * CY[l];
              az += v * CZ[l];
            }
            rho[at(s, i)] = r;
            jx[at(s, i)] = ax;
            jy[at(s, i)] = ay;
            jz[at(s, i)] = az;
            psi[at(s, i)] = pseudo(r);
          }
        }
  }

  // eq. (FORCE) in three dimensions, the A-B repulsion and the body force.
  void forces() {
#pragma omp parallel for schedule(static)
    for (int z = 0; z < c.lz; ++z)
      for (int y = 0; y < c.ly; ++y)
        for (int x = 0; x < c.lx; ++x) {
          const size_t i = site(x, y, z);
          for (int s = 0; s < c.ns; ++s) {
            double a[3] = {0, 0, 0}, b[3] = {0, 0, 0};
            for (const Link &k : links) {
              const double nb = psi_at(s, x + k.x, y + k.y, z + k.z);
              const int sh = shell_index(k.q);
              if (k.q <= 4) {  // attractive belt, weights w
                a[0] += c.w[sh] * nb * k.x;
                a[1] += c.w[sh] * nb * k.y;
                a[2] += c.w[sh] * nb * k.z;
              }
              b[0] += c.p[sh] * nb * k.x;  // repulsive belt, weights p
              b[1] += c.p[sh] * nb * k.y;
              b[2] += c.p[sh] * nb * k.z;
            }
            const double ps = psi[at(s, i)];
            double F[3];
            for (int d = 0; d < 3; ++d) F[d] = -c.g1[s] * ps * a[d] - c.g2[s] * ps * b[d];
            if (c.ns == 2) {
              const int sb = 1 - s;
              double x3[3] = {0, 0, 0};
              for (int l = 1; l < 19; ++l) {
                const double nb = c.cross_psi ? psi_at(sb, x + CX[l], y + CY[l], z + CZ[l])
                                              : rho_at(sb, x + CX[l], y + CY[l], z + CZ[l]);
                const double tq = l <= 6 ? c.t[0] : c.t[1];
                x3[0] += tq * nb * CX[l];
                x3[1] += tq * nb * CY[l];
                x3[2] += tq * nb * CZ[l];
              }
              const double self = c.cross_psi ? ps : rho[at(s, i)];
              for (int d = 0; d < 3; ++d) F[d] += -c.gab * self * x3[d];
            }
            const double r = rho[at(s, i)];
            fx[at(s, i)] = F[0] + r * c.body[0];
            fy[at(s, i)] = F[1] + r * c.body[1];
            fz[at(s, i)] = F[2] + r * c.body[2];
          }
        }
  }

  // BGK collision (LB) towards f^eq(rho_s, u^eq_s), u^eq_s = u' + tau_s F_s / rho_s.
  void collide() {
#pragma omp parallel for schedule(static)
    for (long long ii = 0; ii < (long long)nsite; ++ii) {
      const size_t i = (size_t)ii;
      double nx = 0, ny = 0, nz = 0, den = 0;
      for (int s = 0; s < c.ns; ++s) {
        nx += jx[at(s, i)] / c.tau[s];
        ny += jy[at(s, i)] / c.tau[s];
        nz += jz[at(s, i)] / c.tau[s];
        den += rho[at(s, i)] / c.tau[s];
      }
      const double upx = nx / den, upy = ny / den, upz = nz / den;
      for (int s = 0; s < c.ns; ++s) {
        const double r = rho[at(s, i)];
        const double ux = upx + c.tau[s] * fx[at(s, i)] / r;
        const double uy = upy + c.tau[s] * fy[at(s, i)] / r;
        const double uz = upz + c.tau[s] * fz[at(s, i)] / r;
        const double uu = ux * ux + uy * uy + uz * uz;
        for (int l = 0; l < 19; ++l) {
          const double cu = CX[l] * ux + CY[l] * uy + CZ[l] * uz;
          const double feq = WL(l) * r * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
          const double v = f[at(s, l, i)];
          fs[at(s, l, i)] = v - (v - feq) / c.tau[s];
        }
      }
    }
  }

  // Streaming f_l(x, t+1) = f*_l(x - c_l, t); halfway bounce-back off the solid rows.
  void stream() {
#pragma omp parallel for schedule(static)
    for (int z = 0; z < c.lz; ++z)
      for (int y = 0; y < c.ly; ++y)
        for (int x = 0; x < c.lx; ++x) {
          const size_t i = site(x, y, z);
          for (int s = 0; s < c.ns; ++s)
            for (int l = 0; l < 19; ++l) {
              const long long src = fluid(x - CX[l], y - CY[l], z - CZ[l]);
              f[at(s, l, i)] = src >= 0 ? fs[at(s, l, (size_t)src)] : fs[at(s, OPP[l], i)];
            }
        }
  }

  // [mass_0, mass_1, P_x, P_y, P_z, W_bot, W_top, Q]: masses and momentum of f(t); wall
  // x-momentum exchange per unit wall area (2 c_x f* of the populations bouncing off each wall);
  // Q = sum u_x / (lx lz) with u = (sum_s j_s + F_s / 2) / sum_s rho_s.
  void record(double *out) const {
    double m[2] = {0, 0}, P[3] = {0, 0, 0}, wb = 0, wt = 0, q = 0;
    for (int s = 0; s < c.ns; ++s)
      for (size_t i = 0; i < nsite; ++i) {
        m[s] += rho[at(s, i)];
        P[0] += jx[at(s, i)];
        P[1] += jy[at(s, i)];
        P[2] += jz[at(s, i)];
      }
    for (size_t i = 0; i < nsite; ++i) {
      double num = 0, den = 0;
      for (int s = 0; s < c.ns; ++s) {
        num += jx[at(s, i)] + 0.5 * fx[at(s, i)];
        den += rho[at(s, i)];
      }
      q += num / den;
    }
    if (c.walls)
      for (int s = 0; s < c.ns; ++s)
        for (int z = 0; z < c.lz; ++z)
          for (int x = 0; x < c.lx; ++x)
            for (int l = 0; l < 19; ++l) {
              if (CY[l] == -1) wb += 2.0 * CX[l] * fs[at(s, l, site(x, 0, z))];
              if (CY[l] == +1) wt += 2.0 * CX[l] * fs[at(s, l, site(x, c.ly - 1, z))];
            }
    const double area = (double)c.lx * c.lz;
    out[0] = m[0]; out[1] = m[1]; out[2] = P[0]; out[3] = P[1]; out[4] = P[2];
    out[5] = wb / area; out[6] = wt / area; out[7] = q / area;
  }

  void step(double *rec) {
    moments();
    forces();
    collide();
    if (rec) record(rec);
    stream();
    ++time;
  }

  void init_rest(const double *rho_init) {
    for (int s = 0; s < c.ns; ++s)
      for (int l = 0; l < 19; ++l)
        for (size_t i = 0; i < nsite; ++i) f[at(s, l, i)] = WL(l) * rho_init[(size_t)s * nsite + i];
    time = 0;
  }
};

}  // namespace

extern "C" {

void *orc3_create(const orc3_config *c) { return new Sim3(*c); }
void orc3_destroy(void *h) { delete static_cast<Sim3 *>(h); }
void orc3_init_rest(void *h, const double *rho) { static_cast<Sim3 *>(h)->init_rest(rho); }
void orc3_set_f(void *h, const double *f) {
  auto *s = static_cast<Sim3 *>(h);
  std::memcpy(s->f.data(), f, s->f.size() * sizeof(double));
}
void orc3_get_f(void *h, double *f) {
  auto *s = static_cast<Sim3 *>(h);
  std::memcpy(f, s->f.data(), s->f.size() * sizeof(double));
}
int64_t orc3_time(void *h) { return static_cast<Sim3 *>(h)->time; }
int orc3_nlinks(void *h) { return (int)static_cast<Sim3 *>(h)->links.size(); }

void orc3_step(void *h, int n, double *rec) {
  auto *s = static_cast<Sim3 *>(h);
  for (int k = 0; k < n; ++k) s->step(rec ? rec + 8 * (size_t)k : nullptr);
}

// Fields of the current state: rho, psi [ns][z][y][x]; force, j [ns][3][z][y][x];
// u [3][z][y][x] (half-force velocity).  Any pointer may be NULL.
void orc3_fields(void *h, double *rho, double *psi, double *force, double *u, double *j) {
  auto *s = static_cast<Sim3 *>(h);
  s->moments();
  s->forces();
  const size_t n = s->nsite;
  for (int sp = 0; sp < s->c.ns; ++sp)
    for (size_t i = 0; i < n; ++i) {
      if (rho) rho[sp * n + i] = s->rho[sp * n + i];
      if (psi) psi[sp * n + i] = s->psi[sp * n + i];
      if (force) {
        force[(3 * sp + 0) * n + i] = s->fx[sp * n + i];
        force[(3 * sp + 1) * n + i] = s->fy[sp * n + i];
        force[(3 * sp + 2) * n + i] = s->fz[sp * n + i];
      }
      if (j) {
        j[(3 * sp + 0) * n + i] = s->jx[sp * n + i];
        j[(3 * sp + 1) * n + i] = s->jy[sp * n + i];
        j[(3 * sp + 2) * n + i] = s->jz[sp * n + i];
      }
    }
  if (u)
    for (size_t i = 0; i < n; ++i) {
      double m[3] = {0, 0, 0}, den = 0;
      for (int sp = 0; sp < s->c.ns; ++sp) {
        m[0] += s->jx[sp * n + i] + 0.5 * s->fx[sp * n + i];
        m[1] += s->jy[sp * n + i] + 0.5 * s->fy[sp * n + i];
        m[2] += s->jz[sp * n + i] + 0.5 * s->fz[sp * n + i];
        den += s->rho[sp * n + i];
      }
      for (int d = 0; d < 3; ++d) u[d * n + i] = m[d] / den;
    }
}

}  // extern "C"
