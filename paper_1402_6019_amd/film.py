"""Thin-film observables of the disjoining-pressure experiment (section "The case of two
near-interfaces: emergence of the disjoining pressure"): two bubbles pressed against each
other leave a liquid film between them; in mechanical equilibrium the disjoining pressure of
that film equals the capillary pressure between the bulk inside a bubble and the bulk outside.

The theoretical side follows eq. (doppiasigma): a flat film of thickness h has a film tension
gamma_f(h), the integral of the mismatch between the normal and tangential components of the
pressure tensor across it, and differentiating (doppiasigma) gives d gamma_f = h dPi, so
Pi(h) = -int_h^inf gamma_f'(h') / h' dh' with Pi(inf) = 0 and gamma_f(inf) = 2 gamma.

Every field comes from the GPU (lb_moments for the density along the axis through the film,
lb_stress_field for the pressure tensor), and the integration of eq. (doppiasigma) runs in the
library (lb_disjoining_pressure); the host reads a few values of the fields, sums one row of the
tensor (a few hundred numbers) and interpolates the two crossings that bound the film.
"""

import numpy as np


def _crossing(line, start, step, level):
    """First position from `start` going in direction `step` where `line` drops below
    `level`, linearly interpolated between the two sites that bracket it (None if none)."""
    n = len(line)
    i = start
    while 0 <= i + step < n:
        j = i + step
        if line[j] < level <= line[i]:
            return i + step * (line[i] - level) / (line[i] - line[j])
        i = j
    return None


def film_observables(sim, axis_row, film_x, bubble_x, outer_xy):
    """Film thickness and pressures of the current state of `sim` (one component).

    axis_row: the row through both bubble centres and the film; film_x: a column inside the
    film; bubble_x: a column deep inside one bubble on that row; outer_xy: (x, y) of a site in
    the bulk outside the bubbles.  Returns a dict:
      h             distance between the two crossings of the mid density (half-way between the
                    bubble and outer bulk densities) that bound the film on the axis (0 if the
                    film has ruptured, i.e. the film column is below the mid density)
      p_bubble      (sigma_xx + sigma_yy) / 2 at (bubble_x, axis_row)
      p_outer       the same at outer_xy
      pi_capillary  p_bubble - p_outer: the disjoining pressure of the film at equilibrium
      pn_film       sigma_xx at (film_x, axis_row) - p_outer: the film's normal stress above the
                    outer pressure
    """
    rho, _ = sim.moments()
    line = rho[:, axis_row, :].sum(dim=0).cpu().numpy()
    sig = sim.stress_field()
    ox, oy = outer_xy
    pick = sig[:, [axis_row, axis_row, oy], [bubble_x, film_x, ox]].cpu().numpy()
    p_bubble = 0.5 * (pick[0, 0] + pick[2, 0])
    p_outer = 0.5 * (pick[0, 2] + pick[2, 2])
    rho_b = float(line[bubble_x])
    rho_o = float(rho[:, oy, ox].sum().item())
    mid = 0.5 * (rho_b + rho_o)
    h = 0.0
    if line[film_x] >= mid:
        left = _crossing(line, film_x, -1, mid)
        right = _crossing(line, film_x, +1, mid)
        if left is not None and right is not None:
            h = right - left
    return dict(h=float(h), p_bubble=float(p_bubble), p_outer=float(p_outer),
                pi_capillary=float(p_bubble - p_outer), pn_film=float(pick[0, 1] - p_outer),
                rho_bubble=rho_b, rho_outer=rho_o)


def film_thickness(line, centre, mid):
    """Distance between the two crossings of the density level `mid` on either side of
    `centre` on the periodic-free profile `line` (0 if line[centre] is below mid)."""
    if line[centre] < mid:
        return 0.0
    left = _crossing(line, centre, -1, mid)
    right = _crossing(line, centre, +1, mid)
    return 0.0 if left is None or right is None else float(right - left)


def flat_film(sim, row=None, mid=None):
    """Film tension and normal stress of a flat liquid film along y (one component, the film
    centred at lx/2): returns dict(h, gamma_f, p_n, p_n_spread, rho_min, rho_max).

    The pressure tensor and the density are averaged over two consecutive steps (the state
    alternates with period two at the last digits), which advances `sim` by two steps.
    gamma_f = sum over the sites of the row of (sigma_xx - sigma_yy); p_n is the mean of
    sigma_xx over the row and p_n_spread its max - min (zero at mechanical equilibrium).  h
    is measured at the density level `mid` (default: half-way between the row's extremes)."""
    row = sim.ly // 2 if row is None else row
    acc_s, acc_r = 0.0, 0.0
    for _ in range(2):
        acc_s = acc_s + sim.stress_field()[:, row, :].cpu().numpy()
        acc_r = acc_r + sim.moments()[0][:, row, :].sum(dim=0).cpu().numpy()
        sim.step(1)
    sig, line = 0.5 * acc_s, 0.5 * acc_r
    lo, hi = float(line.min()), float(line.max())
    level = 0.5 * (lo + hi) if mid is None else mid
    return dict(h=film_thickness(line, sim.lx // 2, level), gamma_f=float((sig[0] - sig[2]).sum()),
                p_n=float(sig[0].mean()), p_n_spread=float(np.ptp(sig[0])), rho_min=lo, rho_max=hi)


def disjoining_from_tension(h, gamma_f):
    """Pi at the thicknesses h (any order, distinct) from the film tensions gamma_f(h) of flat
    films, by eq. (doppiasigma): dPi = dgamma_f / h, integrated from the thickest film, where
    Pi is taken as 0; gamma_f is taken linear between neighbouring thicknesses and 1/h is
    integrated exactly on each interval (lb_disjoining_pressure in the library).  Returns Pi in
    the order of the input."""
    import ctypes
    from . import _binding as B
    h = np.ascontiguousarray(h, dtype=np.float64)
    g = np.ascontiguousarray(gamma_f, dtype=np.float64)
    if h.shape != g.shape or h.ndim != 1 or len(h) < 2:
        raise ValueError("h and gamma_f must be 1-D of the same length >= 2")
    out = np.empty_like(h)
    dp = ctypes.POINTER(ctypes.c_double)
    rc = B.load().lb_disjoining_pressure(h.ctypes.data_as(dp), g.ctypes.data_as(dp), len(h), out.ctypes.data_as(dp))
    if rc != B.LB_OK:
        raise ValueError("thicknesses must be positive, finite and distinct")
    return out
