"""Oracle-side diagnostics from the paper's equilibrium analysis (FP64, numpy).

TEST INFRASTRUCTURE ONLY.  Used by the oracle's self-tests to pin it against what the paper
fixes: the bulk equation of state (BULK), the exact mechanical balance across an interface
(Sec. "The Stress Field on The lattice": the force is the lattice divergence of a stress, so
the normal stress through any plane is uniform at equilibrium), the surface-stress mismatch
of Appendix A and the coefficients C2, C4 (eqs. (C2), (C4), (finale4), (finale6)).

Readings of the paper used here:
  * A0 of Appendix A: the printed -G1(w(1) - 4 w(4)) is read as -G1(w(1) + 4 w(4)); only then
    does a uniform state give sigma_xx = sigma_zz, and the shell-by-shell derivation of
    sigma^(4) gives the same sign.
  * c_s^2 = 1/3 in lattice units.
"""

import numpy as np

from . import CX, CY, WL

CS2 = 1.0 / 3.0

# Interaction links 1..24 in the numbering of Fig. 1 (pinned by the shell-5 extra terms of
# Appendix A: c13 = c5 - c3 = c1 - c7, c14 = c5 - c4 = c2 - c7, c15 = c2 - c8 = c6 - c4,
# c16 = c6 - c1 = c3 - c8).  Index 0 is unused so that LINKS[l] is link l.
LINKS = [None,
         (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1),
         (2, 0), (0, 2), (-2, 0), (0, -2),
         (2, 1), (1, 2), (-1, 2), (-2, 1), (-2, -1), (-1, -2), (1, -2), (2, -1),
         (2, 2), (-2, 2), (-2, -2), (2, -2)]
SHELL_OF = {1: 0, 2: 1, 4: 2, 5: 3, 8: 4}


def pseudo(rho, psi0=1.0, rho0=1.0):
    return psi0 * (1.0 - np.exp(-np.asarray(rho) / rho0))


def bulk_pressure(rho, g_total, psi0=1.0, rho0=1.0):
    """(BULK): P_b = c_s^2 rho + c_s^2 (G1 + G2)/2 psi^2."""
    psi = pseudo(rho, psi0, rho0)
    return CS2 * rho + CS2 * 0.5 * g_total * psi * psi


def bulk_pressure_2c(rho_a, rho_b, params):
    """Two-component extension of (BULK) under the cross-term reading:
    P_b = c_s^2 (rho_A + rho_B) + c_s^2/2 sum_s (G_ss,1 + G_ss,2) psi_s^2 + c_s^2 G_AB rho_A rho_B."""
    P = params
    pa = pseudo(rho_a, P.psi0, P.rho0)
    pb = pseudo(rho_b, P.psi0, P.rho0)
    return (CS2 * (rho_a + rho_b)
            + CS2 * 0.5 * ((P.g1[0] + P.g2[0]) * pa * pa + (P.g1[1] + P.g2[1]) * pb * pb)
            + CS2 * P.gab * rho_a * rho_b)


def normal_pressure_x(fstar, psi, rho, params):
    """Normal stress P_N(x + 1/2) through the plane between columns x and x+1, averaged
    over y, for a periodic lattice.  Kinetic part: momentum carried across the plane by the
    post-collision populations in one streaming step.  Interaction part: minus the x-force
    that the sites right of the plane exert on the sites left of it, from the pair form of
    eq. (FORCE) (and of the A-B repulsion).  Returns an array over x."""
    P = params
    assert P.walls == 0
    ns = P.ns
    out = np.zeros(P.lx)
    right = CX == 1
    left = CX == -1
    for s in range(ns):
        kin = fstar[s, right].sum(axis=0) + np.roll(fstar[s, left].sum(axis=0), -1, axis=1)
        out += kin.mean(axis=0)
        K = P.shell_k(s)
        for l in range(1, 25):
            cx, cy = LINKS[l]
            if cx <= 0:
                continue
            k = K[SHELL_OF[cx * cx + cy * cy]]
            # left site at column X - j (j < cx), partner at X - j + cx, row shifted by cy
            for jj in range(cx):
                a = np.roll(psi[s], jj, axis=1)                           # psi(X - jj, y)
                b = np.roll(np.roll(psi[s], jj - cx, axis=1), -cy, axis=0)  # psi(X - jj + cx, y + cy)
                out += k * cx * (a * b).mean(axis=0)
    if ns == 2 and P.gab != 0.0:
        src = psi if P.cross_psi else rho
        for l in range(1, 9):
            cx, cy = LINKS[l]
            if cx <= 0:
                continue
            t = P.t[SHELL_OF[cx * cx + cy * cy]]
            for s in range(2):
                a = src[s]
                b = np.roll(np.roll(src[1 - s], -cx, axis=1), -cy, axis=0)
                out += P.gab * t * cx * (a * b).mean(axis=0)
    return out


def a_coefficients(g1, g2, w, p):
    """Appendix A coefficients A0..A3 (with the A0 sign reading) for one species."""
    w1, w4 = w[0], w[2]
    p1, p4, p5 = p[0], p[2], p[3]
    a1 = g2 * (p1 / 2 - 3 * p5) + g1 * w1 / 2
    a2 = g2 * (p4 + 1.5 * p5) + g1 * w4
    a0 = g2 * (-p1 - 4 * p4) - g1 * (w1 + 4 * w4)
    a3 = g2 * (2 * p4 + 3 * p5) + 2 * g1 * w4
    return a0, a1, a2, a3


def stress_mismatch_a(psi_x, g1, g2, w, p):
    """(sigma^int_xx - sigma^int_zz)(x) of a 1-D periodic profile psi(x), Appendix A form."""
    a0, a1, a2, a3 = a_coefficients(g1, g2, w, p)
    ps = psi_x
    p1, m1 = np.roll(ps, -1), np.roll(ps, 1)
    p2, m2 = np.roll(ps, -2), np.roll(ps, 2)
    return a1 * ps * (p1 + m1) + a2 * ps * (p2 + m2) + a0 * ps * ps + a3 * p1 * m1


def stress_mismatch_shells(psi_x, g1, g2, w, p):
    """Same quantity built shell by shell from the sigma^(1), sigma^(2), sigma^(4),
    sigma^(5), sigma^(8) expressions of Appendix A (second, independent route)."""
    ps = np.asarray(psi_x)

    def at(off):  # psi(x + off) for an integer or half-integer offset given as 2*off
        return np.roll(ps, -off)

    def half(c):  # psi(x - c/2) psi(x + c/2) for even c_x
        return np.roll(ps, c // 2) * np.roll(ps, -c // 2)

    def dxz(c):
        return c[0] * c[0] - c[1] * c[1]

    out = np.zeros_like(ps)
    for G, W in ((g1, w), (g2, p)):
        # shells 1 and 2: (G/2) W psi(x) sum psi(x+c) c c
        for l in range(1, 9):
            c = LINKS[l]
            q = SHELL_OF[c[0] ** 2 + c[1] ** 2]
            out += 0.5 * G * W[q] * ps * at(c[0]) * dxz(c)
        # shells 4 and 8: (G/4) W [psi(x) psi(x+c) + psi(x-c/2) psi(x+c/2)] c c
        for l in list(range(9, 13)) + list(range(21, 25)):
            c = LINKS[l]
            q = SHELL_OF[c[0] ** 2 + c[1] ** 2]
            out += 0.25 * G * W[q] * (ps * at(c[0]) + half(c[0])) * dxz(c)
        # shell 5: (G/4) W(5) psi(x) psi(x+c) c c over links 13..20, plus the extra pairs
        for l in range(13, 21):
            c = LINKS[l]
            out += 0.25 * G * W[3] * ps * at(c[0]) * dxz(c)
        extra = {13: ((5, 3), (1, 7)), 14: ((5, 4), (2, 7)), 15: ((2, 8), (6, 4)), 16: ((6, 1), (3, 8))}
        for l, pairs in extra.items():
            c = LINKS[l]
            acc = np.zeros_like(ps)
            for a, b in pairs:
                acc += at(LINKS[a][0]) * at(LINKS[b][0])
            out += 0.25 * G * W[3] * acc * dxz(c)
    return out


def c2_c4_formula(g1, g2, e4w, e4p, e6w, e6p):
    """(C2), (C4)."""
    return -0.5 * g1 * e4w - 0.5 * g2 * e4p, 0.25 * g1 * e6w + 0.25 * g2 * e6p


def c2_c4_from_a(g1, g2, w, p):
    """C2 = -A1 - 4A2 - 2A3, C4 = A1/12 + 4A2/3 + 2A3/3 (Appendix A)."""
    _, a1, a2, a3 = a_coefficients(g1, g2, w, p)
    return -a1 - 4 * a2 - 2 * a3, a1 / 12 + 4 * a2 / 3 + 2 * a3 / 3


def droplet_radius(rho, rho_in, rho_out):
    """Equimolar radius of a single circular droplet: area = (M - rho_out A) / (rho_in - rho_out)."""
    area = (rho.sum() - rho_out * rho.size) / (rho_in - rho_out)
    return np.sqrt(abs(area) / np.pi)


def shear_profile(orc, parts=False):
    """Stream-wise averaged velocity and shear stress of the current state of an Oracle
    (emulsion section: the averaged profiles ubar_x(z) and sigma(z) of the confined flows,
    from which the local fluidity of eq. (fluidity) / eq. (predict) is taken).

    Returns (ubar [ly], sigma [ly + 1]):
      ubar(y)  = (1/lx) sum_x u_x(x, y), u the half-force velocity of the oracle's fields;
      sigma(k) = x-force per unit length exerted, in this step, by everything above the
                 horizontal line k (between rows k-1 and k) on everything below it: the pair
                 forces of eq. (FORCE) and of the A-B repulsion between fluid sites on either
                 side of the line, minus the x-momentum that streaming carries up across the
                 line (post-collision populations with c_y = +1 below it, minus those with
                 c_y = -1 above it).  On a channel, sigma(0) and sigma(ly) are the momentum
                 exchanged with the bottom wall (W_bot, force on the wall) and the top wall
                 (-W_top, force of the wall on the fluid), moving walls included.  On a
                 periodic lattice sigma(ly) = sigma(0).
    Every pair is enumerated explicitly (no regrouping).  With parts=True also returns the
    pair-force part of sigma alone (zero on wall lines)."""
    P = orc.params
    fl = orc.fields(fstar=True)
    fs, psi, rho, u = fl["fstar"], fl["psi"], fl["rho"], fl["u"]
    ns, ly, lx = P.ns, P.ly, P.lx
    walls = bool(P.walls)
    ubar = u[0].sum(axis=1) / lx

    # x-momentum of the populations leaving each row upward / downward, summed over x
    kup = np.zeros(ly)
    kdn = np.zeros(ly)
    for s in range(ns):
        for l in range(9):
            if CY[l] == 1:
                kup += CX[l] * fs[s, l].sum(axis=1)
            if CY[l] == -1:
                kdn += CX[l] * fs[s, l].sum(axis=1)

    cross = P.ns == 2 and P.gab != 0.0
    rsrc = psi if P.cross_psi else rho

    def pair_force(k):
        """x-force on the fluid rows below line k from the fluid rows above it."""
        tot = 0.0
        for ay in (k - 1, k - 2):
            if walls and ay < 0:
                continue
            ayw = ay % ly
            for li in range(1, 25):
                cx, cy = LINKS[li]
                if cy < 1 or ay + cy < k:
                    continue
                by = ay + cy
                if walls and by > ly - 1:
                    continue  # partner is a wall ghost: wall force, not fluid stress
                byw = by % ly
                q = SHELL_OF[cx * cx + cy * cy]
                for s in range(ns):
                    Ks = P.shell_k(s)[q]
                    a_val = psi[s, ayw]
                    b_val = np.roll(psi[s, byw], -cx)  # psi(x + cx, by)
                    tot += -Ks * cx * float((a_val * b_val).sum())
                    if cross and li <= 8:
                        t = P.t[q]
                        a_r = rsrc[s, ayw]
                        b_r = np.roll(rsrc[1 - s, byw], -cx)
                        tot += -P.gab * t * cx * float((a_r * b_r).sum())
        return tot

    sigma = np.zeros(ly + 1)
    pair = np.zeros(ly + 1)
    lines = range(1, ly) if walls else range(0, ly)
    for k in lines:
        below, above = (k - 1) % ly, k % ly
        pair[k] = pair_force(k) / lx
        sigma[k] = (pair_force(k) - kup[below] + kdn[above]) / lx
    if walls:
        # reflected population off a wall moving with U: f*_out + 6 W_l rho_w (c_l . U)
        wb = wt = 0.0
        for s in range(ns):
            for l in range(9):
                lo = int(np.nonzero((CX == -CX[l]) & (CY == -CY[l]))[0][0])
                if CY[l] == -1:
                    out = fs[s, l, 0]
                    refl = out + 6.0 * WL[lo] * P.rho_wall[s] * (CX[lo] * P.u_wall[0])
                    wb += float((CX[l] * out - CX[lo] * refl).sum())
                if CY[l] == 1:
                    out = fs[s, l, ly - 1]
                    refl = out + 6.0 * WL[lo] * P.rho_wall[s] * (CX[lo] * P.u_wall[1])
                    wt += float((CX[l] * out - CX[lo] * refl).sum())
        sigma[0] = wb / lx
        sigma[ly] = -wt / lx
    else:
        sigma[ly] = sigma[0]
        pair[ly] = pair[0]
    if parts:
        return ubar, sigma, pair
    return ubar, sigma


def _at(a, dx, dy, walls, fill):
    """a(x + dx, y + dy) for a field a[ly, lx]: periodic in x; in y periodic, or the wall
    ghost value `fill` beyond the rows of a channel."""
    b = np.roll(a, -dx, axis=1)
    if not walls:
        return np.roll(b, -dy, axis=0)
    out = np.full_like(b, fill)
    ly = a.shape[0]
    if dy >= 0:
        out[:ly - dy] = b[dy:]
    else:
        out[-dy:] = b[:ly + dy]
    return out


def stress_field(orc):
    """Pressure tensor of section "The Stress Field on The lattice" at every site of the
    current state: sigma_ij = sum_s [c_s^2 rho_s delta_ij + sigma^(int)_s,ij
    + (tau_s - 1/2)^2 F_s,i F_s,j / rho_s] + sigma^(AB)_ij.  Returns (sxx, sxy, syy), each
    [ly, lx].

    sigma^(int) follows Appendix A shell by shell, with G_1 w(q) + G_2 p(q) per shell (the
    long-range terms replace w by p and G_1 by G_2, and both add):
      shells 1, 2: (G/2) W psi(x) sum_l psi(x + c_l) c_l c_l
      shells 4, 8: (G/4) W sum_l [psi(x) psi(x + c_l) + psi(x - c_l/2) psi(x + c_l/2)] c_l c_l
      shell 5:     (G/4) p(5) sum_{l=13..20} psi(x) psi(x + c_l) c_l c_l plus, for l = 13..16,
                   (G/4) p(5) (psi(x + c_a) psi(x + c_b) + psi(x + c_a') psi(x + c_b')) c_l c_l
                   over the two pairs of first-belt links whose difference is c_l.
    The A-B repulsion (the cross-term reading: Shan-Chen form over the first belt) adds, by
    the same construction as shells 1 and 2, (G_AB / 2) sum_{l=1..8} t(q)
    [r_A(x) r_B(x + c_l) + r_B(x) r_A(x + c_l)] c_l c_l.  On channels the solid ghost rows carry
    the wall densities, as in the force."""
    P = orc.params
    fl = orc.fields()
    psi, rho, F = fl["psi"], fl["rho"], fl["force"]
    walls = bool(P.walls)
    ly, lx = P.ly, P.lx
    comps = ((0, 0), (0, 1), (1, 1))
    out = [np.zeros((ly, lx)) for _ in comps]

    def add(val, c, coef):
        for k, (i, j) in enumerate(comps):
            out[k] += coef * c[i] * c[j] * val

    extra = {13: ((5, 3), (1, 7)), 14: ((5, 4), (2, 7)), 15: ((2, 8), (6, 4)), 16: ((6, 1), (3, 8))}
    for s in range(P.ns):
        K = P.shell_k(s)
        ps = psi[s]
        pw = pseudo(P.rho_wall[s], P.psi0, P.rho0)

        def at(dx, dy):
            return _at(ps, dx, dy, walls, pw)

        for l in range(1, 25):
            c = LINKS[l]
            q = SHELL_OF[c[0] * c[0] + c[1] * c[1]]
            if q in (0, 1):
                add(ps * at(*c), c, 0.5 * K[q])
            elif q in (2, 4):
                add(ps * at(*c), c, 0.25 * K[q])
                add(at(-c[0] // 2, -c[1] // 2) * at(c[0] // 2, c[1] // 2), c, 0.25 * K[q])
            else:
                add(ps * at(*c), c, 0.25 * K[q])
        for l, pairs in extra.items():
            v = sum(at(*LINKS[a]) * at(*LINKS[b]) for a, b in pairs)
            add(v, LINKS[l], 0.25 * K[3])
        # ideal part and the discrete forcing correction
        r = rho[s]
        out[0] += CS2 * r
        out[2] += CS2 * r
        corr = (P.tau[s] - 0.5) ** 2 / r
        out[0] += corr * F[s, 0] * F[s, 0]
        out[1] += corr * F[s, 0] * F[s, 1]
        out[2] += corr * F[s, 1] * F[s, 1]
    if P.ns == 2 and P.gab != 0.0:
        src = psi if P.cross_psi else rho
        fills = [pseudo(P.rho_wall[s], P.psi0, P.rho0) if P.cross_psi else P.rho_wall[s] for s in range(2)]
        for l in range(1, 9):
            c = LINKS[l]
            t = P.t[SHELL_OF[c[0] * c[0] + c[1] * c[1]]]
            v = (src[0] * _at(src[1], c[0], c[1], walls, fills[1]) + src[1] * _at(src[0], c[0], c[1], walls, fills[0]))
            add(v, c, 0.5 * P.gab * t)
    return out[0], out[1], out[2]


def fluidity(ubar, sigma, walls=True, u_wall=(0.0, 0.0)):
    """Local fluidity at the lines k = 0..ly: the velocity difference across the line over
    the stress through it, f(k) = (ubar(k) - ubar(k-1)) / sigma(k); at a wall the difference
    is taken to the wall velocity over half a site (periodic lattices wrap)."""
    ly = len(ubar)
    f = np.empty(ly + 1)
    for k in range(ly + 1):
        if walls and k == 0:
            du = 2.0 * (ubar[0] - u_wall[0])
        elif walls and k == ly:
            du = 2.0 * (u_wall[1] - ubar[ly - 1])
        else:
            kk = k % ly
            du = ubar[kk] - ubar[(kk - 1) % ly]
        f[k] = du / sigma[k]
    return f


def cooperative_shape(z, H, zeta):
    """Right-hand side of eq. (predict): cosh((z - H/2) / zeta) / cosh(H / (2 zeta))."""
    return np.cosh((np.asarray(z) - H / 2.0) / zeta) / np.cosh(H / (2.0 * zeta))
