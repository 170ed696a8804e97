"""Seeded synthetic inputs for the lattice Boltzmann runs (initial density fields and
per-instance parameter draws).

This module holds geometry and random draws only -- none of the method's arithmetic -- so
that the GPU path and the CPU oracle can be fed identical inputs without sharing code.
All randomness is numpy's PCG64 with an explicit seed.

The paper's own packings (its Figs. 4-5) are not available; the emulsion generator stands in
for them with the same structure: polydisperse droplets of an A-rich phase
(rho_A, rho_B) ~ (1.2, 0.2) in a B-rich continuous phase (0.2, 1.2), dense enough at high
packing fraction to form a foam-like network of thin B films.
"""

import math

import numpy as np

EMULSION_RICH = (1.2, 0.2)
EMULSION_POOR = (0.2, 1.2)


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def uniform_noise(lx, ly, rho0=1.0, amp=0.01, seed=1):
    """rho = rho0 (1 + amp U(-1, 1)) per site, shape [ly, lx]."""
    g = rng(seed)
    return rho0 * (1.0 + amp * g.uniform(-1.0, 1.0, size=(ly, lx)))


def flat_slab(lx, ly, rho_in, rho_out, x0, x1):
    """Columns [x0, x1) at rho_in, the rest at rho_out (an interface normal to x)."""
    r = np.full((ly, lx), float(rho_out))
    r[:, x0:x1] = rho_in
    return r


def disc(lx, ly, radius, rho_in, rho_out, cx=None, cy=None):
    """A sharp disc of rho_in in rho_out, centred on (cx, cy) (default: the lattice centre)."""
    cx = (lx - 1) / 2.0 if cx is None else cx
    cy = (ly - 1) / 2.0 if cy is None else cy
    y, x = np.mgrid[0:ly, 0:lx]
    inside = (x - cx) ** 2 + (y - cy) ** 2 <= radius * radius
    return np.where(inside, float(rho_in), float(rho_out))


def facing_bubbles(lx, ly, radius, gap, rho_in=0.28, rho_out=1.39, width=1.5):
    """Two half-discs of the gas phase (rho_in) in the liquid (rho_out), their flat faces
    facing each other across a liquid gap of `gap` sites at the lattice centre (the thin-film
    setup: two bubbles pressed against each other with a film between them).  The bubble
    centres of curvature are at (lx/2 -+ gap/2, ly/2); the profile is a tanh of the signed
    distance to the nearer half-disc, of width `width`.  Shape [ly, lx]."""
    y, x = np.mgrid[0:ly, 0:lx] + 0.5
    xl, xr, cy = lx / 2.0 - gap / 2.0, lx / 2.0 + gap / 2.0, ly / 2.0
    dl = np.maximum(np.hypot(x - xl, y - cy) - radius, x - xl)
    dr = np.maximum(np.hypot(x - xr, y - cy) - radius, xr - x)
    d = np.minimum(dl, dr)
    return rho_in + (rho_out - rho_in) * 0.5 * (1.0 + np.tanh(d / width))


def flat_film(lx, ly, thickness, rho_gas=0.28, rho_liq=1.39, width=1.5):
    """A flat liquid film (rho_liq) of `thickness` sites centred at x = lx/2, uniform in y, in
    the gas (rho_gas): the flat counterpart of the film between two bubbles, whose film
    tension gives the theoretical disjoining pressure.  tanh walls of width `width`.
    Shape [ly, lx]."""
    x = np.arange(lx, dtype=np.float64)
    x1, x2 = lx / 2.0 - thickness / 2.0, lx / 2.0 + thickness / 2.0
    prof = rho_gas + (rho_liq - rho_gas) * 0.5 * (np.tanh((x - x1) / width) - np.tanh((x - x2) / width))
    return np.broadcast_to(prof, (ly, lx)).copy()


def _expected_area(rmin, rmax):
    er2 = (rmax ** 3 - rmin ** 3) / (3.0 * (rmax - rmin))
    return math.pi * er2


def emulsion(lx, ly, fraction=0.8, seed=2, walls=False, rmin=8.0, rmax=24.0, gap=2.0,
             rich=EMULSION_RICH, poor=EMULSION_POOR):
    """Polydisperse packed emulsion.

    round(fraction * lx * ly / E[pi r^2]) centres uniform in the box with radii U(rmin, rmax).
    Every site belongs to the centre of smallest power distance |x - x_i|^2 - r_i^2 (periodic
    in x, and in y unless walls).  A site is A-rich when it lies within lam * r_i of its centre
    and at least gap/2 from the boundary of its power cell (and, with walls, at least gap/2
    from the wall rows); lam is set by bisection so that the A-rich volume fraction is
    `fraction`.  Dense packings turn into polygonal cells separated by films of width ~gap.
    When the films leave less than `fraction` of the box (small droplets, wide gap) the result
    is the densest packing the cells allow, and info['volume_fraction'] reports what it reached.

    Returns (rho[2, ly, lx], info) with info = {n_drops, volume_fraction, mass_fraction, lam}.
    """
    from scipy.spatial import cKDTree

    g = rng(seed)
    n = max(1, int(round(fraction * lx * ly / _expected_area(rmin, rmax))))
    cxs = g.uniform(0.0, lx, n)
    cys = g.uniform(0.0, ly, n)
    rad = g.uniform(rmin, rmax, n)

    # Power distance as a Euclidean distance in one extra dimension:
    # |x - c|^2 + (R^2 - r^2) differs from |x - c|^2 - r^2 by the constant R^2.
    big = rmax
    lift = np.sqrt(big * big - rad * rad)
    shifts_x = (-lx, 0, lx)
    shifts_y = (0,) if walls else (-ly, 0, ly)
    pts, owner = [], []
    for sx in shifts_x:
        for sy in shifts_y:
            pts.append(np.stack([cxs + sx, cys + sy, lift], axis=1))
            owner.append(np.arange(n))
    pts = np.concatenate(pts)
    owner = np.concatenate(owner)
    tree = cKDTree(pts)

    yy, xx = np.mgrid[0:ly, 0:lx]
    q = np.stack([xx.ravel().astype(np.float64), yy.ravel().astype(np.float64), np.zeros(xx.size)], axis=1)
    k = 4
    d, idx = tree.query(q, k=k)
    pd = d * d  # power distance + R^2
    c0 = pts[idx[:, 0]]
    dist_c = np.sqrt((q[:, 0] - c0[:, 0]) ** 2 + (q[:, 1] - c0[:, 1]) ** 2)
    r0 = rad[owner[idx[:, 0]]]
    bdist = np.full(q.shape[0], np.inf)
    for j in range(1, k):
        cj = pts[idx[:, j]]
        sep = np.sqrt((c0[:, 0] - cj[:, 0]) ** 2 + (c0[:, 1] - cj[:, 1]) ** 2)
        same = owner[idx[:, j]] == owner[idx[:, 0]]
        with np.errstate(divide="ignore", invalid="ignore"):
            bj = np.where(same | (sep == 0), np.inf, (pd[:, j] - pd[:, 0]) / (2.0 * sep))
        bdist = np.minimum(bdist, bj)
    ok = bdist >= gap / 2.0
    if walls:
        ok &= (q[:, 1] >= gap / 2.0) & (q[:, 1] <= ly - 1 - gap / 2.0)
    ratio = dist_c / r0

    def frac(lam):
        return np.count_nonzero(ok & (ratio < lam)) / q.shape[0]

    lo, hi = 0.0, 8.0
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if frac(mid) < fraction:
            lo = mid
        else:
            hi = mid
    lam = hi
    a_rich = (ok & (ratio < lam)).reshape(ly, lx)
    rho = np.empty((2, ly, lx))
    rho[0] = np.where(a_rich, rich[0], poor[0])
    rho[1] = np.where(a_rich, rich[1], poor[1])
    ma, mb = rho[0].sum(), rho[1].sum()
    info = dict(n_drops=n, volume_fraction=float(a_rich.mean()), mass_fraction=float(ma / (ma + mb)), lam=lam)
    return rho, info


def emulsion3d(lx, ly, lz, fraction=0.5, seed=2, walls=False, rmin=4.0, rmax=8.0, gap=2.0,
               rich=EMULSION_RICH, poor=EMULSION_POOR):
    """Polydisperse packed emulsion in a box of lx x ly x lz sites, the 3-D counterpart of
    emulsion(): round(fraction * V / E[4/3 pi r^3]) centres uniform in the box with radii
    U(rmin, rmax); every site belongs to the centre of smallest power distance (periodic in x
    and z, and in y unless walls); it is A-rich when within lam * r_i of that centre and at least
    gap/2 from its power cell's boundary (and from the wall rows); lam is set by bisection to
    reach the volume fraction.  Returns (rho[2, lz, ly, lx], info)."""
    from scipy.spatial import cKDTree

    g = rng(seed)
    er3 = (rmax ** 4 - rmin ** 4) / (4.0 * (rmax - rmin))
    n = max(1, int(round(fraction * lx * ly * lz / (4.0 / 3.0 * math.pi * er3))))
    cen = np.stack([g.uniform(0.0, lx, n), g.uniform(0.0, ly, n), g.uniform(0.0, lz, n)], axis=1)
    rad = g.uniform(rmin, rmax, n)
    lift = np.sqrt(rmax * rmax - rad * rad)
    pts, owner = [], []
    for sx in (-lx, 0, lx):
        for sy in ((0,) if walls else (-ly, 0, ly)):
            for sz in (-lz, 0, lz):
                pts.append(np.concatenate([cen + np.array([sx, sy, sz]), lift[:, None]], axis=1))
                owner.append(np.arange(n))
    pts = np.concatenate(pts)
    owner = np.concatenate(owner)
    tree = cKDTree(pts)
    zz, yy, xx = np.mgrid[0:lz, 0:ly, 0:lx]
    q = np.stack([xx.ravel(), yy.ravel(), zz.ravel(), np.zeros(xx.size)], axis=1).astype(np.float64)
    k = 4
    d, idx = tree.query(q, k=k)
    pd = d * d
    c0 = pts[idx[:, 0]]
    dist_c = np.sqrt(((q[:, :3] - c0[:, :3]) ** 2).sum(axis=1))
    r0 = rad[owner[idx[:, 0]]]
    bdist = np.full(q.shape[0], np.inf)
    for j in range(1, k):
        cj = pts[idx[:, j]]
        sep = np.sqrt(((c0[:, :3] - cj[:, :3]) ** 2).sum(axis=1))
        same = owner[idx[:, j]] == owner[idx[:, 0]]
        with np.errstate(divide="ignore", invalid="ignore"):
            bj = np.where(same | (sep == 0), np.inf, (pd[:, j] - pd[:, 0]) / (2.0 * sep))
        bdist = np.minimum(bdist, bj)
    ok = bdist >= gap / 2.0
    if walls:
        ok &= (q[:, 1] >= gap / 2.0) & (q[:, 1] <= ly - 1 - gap / 2.0)
    ratio = dist_c / r0
    lo, hi = 0.0, 8.0
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if np.count_nonzero(ok & (ratio < mid)) / q.shape[0] < fraction:
            lo = mid
        else:
            hi = mid
    a_rich = (ok & (ratio < hi)).reshape(lz, ly, lx)
    rho = np.empty((2, lz, ly, lx))
    rho[0] = np.where(a_rich, rich[0], poor[0])
    rho[1] = np.where(a_rich, rich[1], poor[1])
    ma, mb = rho[0].sum(), rho[1].sum()
    return rho, dict(n_drops=n, volume_fraction=float(a_rich.mean()), mass_fraction=float(ma / (ma + mb)), lam=hi)


# Emulsion couplings of the confined-flow simulations (emulsion section of the paper).
EMULSION_G1 = (-9.0, -8.0)
EMULSION_G2 = (8.1, 7.1)
EMULSION_GAB = 0.587
EMULSION_RHO0 = 0.83
# Single-component frustrated couplings of the thin-film (disjoining pressure) runs.
FILM_G1 = -20.4
FILM_G2 = 16.0


def batch_specs(n=64, seed=4, ly_range=(64, 512), lx_range=(256, 2048)):
    """Per-instance draws for a sweep of independent emulsion channels: sizes
    Ly ~ U{ly_range}, Lx ~ U{lx_range}; couplings scattered around the emulsion values
    (G_ss,k x (1 + 0.05 U(-1,1)), G_AB x (1 + 0.1 U(-1,1))); body force g ~ 1e-6 U(0.5, 2).
    Instance i's initial field uses seed seed * 1000 + i."""
    g = rng(seed)
    specs = []
    for i in range(n):
        ly = int(g.integers(ly_range[0], ly_range[1] + 1))
        lx = int(g.integers(lx_range[0], lx_range[1] + 1))
        e1 = g.uniform(-1.0, 1.0, 2)
        e2 = g.uniform(-1.0, 1.0, 2)
        eab = g.uniform(-1.0, 1.0)
        gx = 1e-6 * g.uniform(0.5, 2.0)
        specs.append(dict(
            lx=lx, ly=ly,
            g1=tuple(EMULSION_G1[s] * (1.0 + 0.05 * e1[s]) for s in range(2)),
            g2=tuple(EMULSION_G2[s] * (1.0 + 0.05 * e2[s]) for s in range(2)),
            gab=EMULSION_GAB * (1.0 + 0.1 * eab),
            body=(gx, 0.0),
            seed=seed * 1000 + i,
        ))
    return specs
