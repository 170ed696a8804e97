"""Thin-film observables of the disjoining-pressure experiment (section "The case of two
near-interfaces: emergence of the disjoining pressure"): two bubbles pressed against each
other leave a liquid film between them; in mechanical equilibrium the disjoining pressure of
that film equals the capillary pressure between the bulk inside a bubble and the bulk outside.

Every field comes from the GPU (lb_moments for the density along the axis through the film,
lb_stress_field for the pressure tensor); the host only reads a few values and interpolates
the two crossings that bound the film.
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
