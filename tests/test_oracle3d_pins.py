"""Pins of the 3-D CPU oracle (D3Q19, the two belts over the 5x5x5 cube) against what the
mathematics fixes: the isotropy of the derived weights checked by contracting the tensors with
random directions, the shell counts, the equilibrium moments, uniform states, closed forms of
the stencil on sinusoids, the long-wavelength limit that (BULK) needs, Newton's third law,
mass and momentum conservation, the momentum balance of a channel, and the bulk equation of
state across a relaxed flat interface."""

from itertools import product

import numpy as np
import pytest

import lbgen
from oracle import CX3, CY3, CZ3, WL3, Oracle3, Params3
from oracle import diagnostics as dg
from oracle import weights as wt

SHELLS3 = (1, 2, 3, 4, 5, 6, 8)
FILM = dict(g1=(lbgen.FILM_G1, 0.0), g2=(lbgen.FILM_G2, 0.0))
EMUL = dict(g1=lbgen.EMULSION_G1, g2=lbgen.EMULSION_G2, gab=lbgen.EMULSION_GAB, rho0=lbgen.EMULSION_RHO0)


def _cube_links(qmax):
    return [c for c in product(range(-2, 3), repeat=3) if 1 <= c[0] ** 2 + c[1] ** 2 + c[2] ** 2 <= qmax]


def test_shell_counts_and_link_count():
    counts = {q: len(wt.shell_links3(q)) for q in SHELLS3}
    assert counts == {1: 6, 2: 12, 3: 8, 4: 6, 5: 24, 6: 24, 8: 12}
    assert len(_cube_links(4)) == 32 and len(_cube_links(8)) == 92
    o = Oracle3(Params3(5, 5, 5), rho_init=np.ones((1, 5, 5, 5)))
    assert o.nlinks == 92


@pytest.mark.parametrize("name,order", [("w", 6), ("p", 8), ("t", 4)])
def test_weights_isotropic_under_rotation(name, order):
    """An isotropic tensor sum_c W c^(2n) contracted with a unit vector n gives the same value for
    every direction: compare random directions with the x axis for each order up to `order`
    (an independent check of the elimination that produced the weights), and E2 = 1/3."""
    W = {"w": wt.weights3_w, "p": wt.weights3_p, "t": wt.weights3_t}[name]()
    links = [(c, float(W.get(c[0] ** 2 + c[1] ** 2 + c[2] ** 2, 0))) for c in _cube_links(8)]
    cs = np.array([c for c, _ in links], dtype=float)
    ws = np.array([w for _, w in links])
    rng = np.random.default_rng(5)
    dirs = rng.normal(size=(20, 3))
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    for n in range(1, order // 2 + 1):
        ref = (ws * cs[:, 0] ** (2 * n)).sum()
        got = (ws[None, :] * (cs @ dirs.T).T ** (2 * n)).sum(axis=1)
        np.testing.assert_allclose(got, ref, rtol=1e-13)
        assert ref > 0
    assert abs((ws * cs[:, 0] ** 2).sum() - 1.0 / 3.0) < 1e-15
    # the next order up is not isotropic (the order is exactly what was asked for)
    n = order // 2 + 1
    ref = (ws * cs[:, 0] ** (2 * n)).sum()
    got = (ws[None, :] * (cs @ dirs.T).T ** (2 * n)).sum(axis=1)
    assert np.abs(got - ref).max() > 1e-6 * ref


def test_d3q19_tables():
    c = np.stack([CX3, CY3, CZ3], axis=1)
    assert len({tuple(v) for v in c}) == 19
    assert np.allclose(WL3.sum(), 1.0)
    np.testing.assert_allclose((WL3[:, None, None] * c[:, :, None] * c[:, None, :]).sum(0), np.eye(3) / 3, atol=1e-16)
    t = wt.weights3_t()
    assert (float(t[1]), float(t[2])) == (1 / 18, 1 / 36)


def test_equilibrium_moments_with_body_force():
    """tau = 1 relaxes a uniform state to f^eq(rho, u + g) in one step, and streaming leaves a
    uniform state unchanged: the moments of f(t = 1) are rho, rho u', c_s^2 rho delta + rho u' u'."""
    n = 4
    g = (1e-3, -2e-3, 5e-4)
    P = Params3(n, n, n, body=g)
    rng = np.random.default_rng(3)
    f0 = WL3 * 1.1 + 0.004 * rng.uniform(-1, 1, 19)
    f = np.broadcast_to(f0[None, :, None, None, None], (1, 19, n, n, n)).copy()
    o = Oracle3(P, f=f)
    o.step(1)
    f1 = o.get_f()[0, :, 0, 0, 0]
    rho = f0.sum()
    u = np.array([(f0 * CX3).sum(), (f0 * CY3).sum(), (f0 * CZ3).sum()]) / rho + np.array(g)
    c = np.stack([CX3, CY3, CZ3], axis=1)
    np.testing.assert_allclose(f1.sum(), rho, rtol=1e-15)
    np.testing.assert_allclose((f1[:, None] * c).sum(0), rho * u, rtol=1e-13, atol=1e-17)
    pi = (f1[:, None, None] * c[:, :, None] * c[:, None, :]).sum(0)
    np.testing.assert_allclose(pi, rho / 3 * np.eye(3) + rho * np.outer(u, u), rtol=1e-13, atol=1e-17)


def test_uniform_two_component_state_invariant():
    P = Params3(6, 5, 7, ns=2, tau=(0.8, 1.3), **EMUL)
    rho = np.stack([np.full((7, 5, 6), 0.9), np.full((7, 5, 6), 0.4)])
    o = Oracle3(P, rho_init=rho)
    f0 = o.get_f()
    assert np.abs(o.fields()["force"]).max() < 1e-14
    o.step(30)
    np.testing.assert_allclose(o.get_f(), f0, rtol=1e-14, atol=0)


def _force_of_psi(psi, P):
    rho = -P.rho0 * np.log(1.0 - psi / P.psi0)
    o = Oracle3(P, rho_init=np.broadcast_to(rho, (P.ns,) + rho.shape))
    fl = o.fields()
    np.testing.assert_allclose(fl["psi"][0], psi, rtol=1e-14)
    return fl


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_force_closed_form_axis_sinusoid(axis):
    """psi = a + b sin(k s) along one axis s: F_s = -psi 2 b cos(k s) [k_1 sin k + k_2 sin 2k], the
    folded couplings counted by hand from the cube's shells: links with c_s = 1 are one of shell 1,
    four each of shells 2, 3, 5 and eight of shell 6; links with c_s = 2 are one of shell 4 and
    four each of shells 5, 6, 8.  The other two components vanish."""
    n = 20
    P = Params3(n, n if axis == 1 else 3, n if axis == 2 else 3, **FILM)
    shape = (P.lz, P.ly, P.lx)
    kap = 2 * np.pi * 2 / n
    coord = np.indices(shape)[2 - axis]
    a, b = 0.55, 0.15
    psi = a + b * np.sin(kap * coord)
    fl = _force_of_psi(psi, P)
    K = dict(zip(SHELLS3, P.shell_k(0)))
    k1 = K[1] + 4 * K[2] + 4 * K[3] + 4 * K[5] + 8 * K[6]
    k2 = 2 * (K[4] + 4 * K[5] + 4 * K[6] + 4 * K[8])
    ref = -psi * 2 * b * np.cos(kap * coord) * (k1 * np.sin(kap) + k2 * np.sin(2 * kap))
    F = fl["force"][0]
    np.testing.assert_allclose(F[axis], ref, rtol=0, atol=2e-14)
    for d in range(3):
        if d != axis:
            assert np.abs(F[d]).max() < 1e-14


def test_force_long_wavelength_limit():
    """For a slow sinusoid the force tends to -psi grad(psi) (G1 + G2) E2 with E2 = 1/3 for both
    weight sets (what (BULK) needs), along the body diagonal as along an axis."""
    n = 64
    P = Params3(n, n, n, **FILM)
    kap = 2 * np.pi / n
    z, y, x = np.indices((n, n, n))
    s = x + y + z
    a, b = 0.55, 1e-3
    psi = a + b * np.sin(kap * s)
    fl = _force_of_psi(psi, P)
    grad = b * kap * np.cos(kap * s)  # d psi / dx (= dy = dz)
    ref = -psi * grad * (lbgen.FILM_G1 + lbgen.FILM_G2) / 3.0
    F = fl["force"][0]
    for d in range(3):
        err = np.abs(F[d] - ref).max() / np.abs(ref).max()
        assert err < 3 * kap ** 2, err  # O(k^2) corrections


def test_cross_force_closed_form():
    """A-B repulsion with uniform rho_A and rho_B = a + b sin(k x): F_A,x = -G_AB rho_A 2 b cos(kx)
    (t1 + 4 t2) sin k (one axis link and four face diagonals with c_x = 1), plus rho_A g_x."""
    n = 16
    g = (2e-4, -1e-4, 3e-4)
    P = Params3(n, 3, 4, ns=2, gab=0.587, rho0=0.83, body=g)
    kap = 2 * np.pi / n
    x = np.indices((4, 3, n))[2]
    rb = 0.5 + 0.2 * np.sin(kap * x)
    ra = np.full_like(rb, 0.7)
    F = Oracle3(P, rho_init=np.stack([ra, rb])).fields()["force"]
    t1, t2 = P.t
    ref = -0.587 * 0.7 * 2 * 0.2 * np.cos(kap * x) * (t1 + 4 * t2) * np.sin(kap) + 0.7 * g[0]
    np.testing.assert_allclose(F[0, 0], ref, rtol=0, atol=1e-15)
    np.testing.assert_allclose(F[0, 1], 0.7 * g[1], rtol=0, atol=1e-15)
    np.testing.assert_allclose(F[0, 2], 0.7 * g[2], rtol=0, atol=1e-15)


@pytest.mark.parametrize("cross_psi", [0, 1])
def test_pair_forces_cancel(cross_psi):
    P = Params3(10, 9, 8, ns=2, cross_psi=cross_psi, **EMUL)
    rng = np.random.default_rng(11)
    F = Oracle3(P, rho_init=0.2 + rng.random((2, 8, 9, 10))).fields()["force"]
    for d in range(3):
        assert abs(F[:, d].sum()) < 1e-12
    assert np.abs(F).max() > 1e-2


def _emulsion3(lx, ly, lz, seed, walls=False):
    return lbgen.emulsion3d(lx, ly, lz, fraction=0.5, seed=seed, walls=walls, rmin=3, rmax=5)[0]


def test_mass_momentum_two_component_periodic():
    P = Params3(16, 14, 12, ns=2, tau=(0.8, 1.3), **EMUL)
    o = Oracle3(P, rho_init=_emulsion3(16, 14, 12, seed=7))
    rec = o.step(60, record=True)
    for s in range(2):
        assert np.abs(rec[:, s] - rec[0, s]).max() / rec[0, s] < 1e-13
    assert np.abs(rec[:, 2:5] - rec[0, 2:5]).max() / rec[0, :2].sum() < 1e-13


def test_momentum_balance_channel_with_body_force():
    """P_x(t+1) - P_x(t) = g M - A (W_bot + W_top) in every step (A = lx lz the wall area), walls
    with wetting ghost densities; species masses stay exact."""
    lx, ly, lz = 14, 12, 10
    g = 1e-5
    P = Params3(lx, ly, lz, ns=2, walls=1, body=(g, 0.0, 0.0), rho_wall=lbgen.EMULSION_POOR, **EMUL)
    o = Oracle3(P, rho_init=_emulsion3(lx, ly, lz, seed=8, walls=True))
    rec = o.step(60, record=True)
    M = rec[0, 0] + rec[0, 1]
    dP = np.diff(rec[:, 2])
    pred = g * M - lx * lz * (rec[:-1, 5] + rec[:-1, 6])
    assert np.abs(dP - pred).max() < 1e-13 * M
    for s in range(2):
        assert np.abs(rec[:, s] - rec[0, s]).max() / rec[0, s] < 1e-13


@pytest.mark.slow
def test_flat_interface_bulk_equation_of_state():
    """A quasi-one-dimensional liquid slab (film couplings) relaxed to equilibrium: the bulk
    pressure (BULK), c_s^2 rho + (c_s^2 / 2)(G1 + G2) psi^2, is the same in the liquid and the gas,
    the state is at rest, and the slab stays demixed."""
    lx = 96
    x = np.arange(lx)
    prof = 0.28 + 1.11 * 0.5 * (np.tanh((x - 23.5) / 3.0) - np.tanh((x - 71.5) / 3.0))
    P = Params3(lx, 1, 1, **FILM)
    o = Oracle3(P, rho_init=np.broadcast_to(prof, (1, 1, 1, lx)))
    o.step(30000)
    fl = o.fields()
    r = fl["rho"][0, 0, 0]
    rl, rg = r[lx // 2], r[0]
    pl = dg.bulk_pressure(rl, lbgen.FILM_G1 + lbgen.FILM_G2)
    pg = dg.bulk_pressure(rg, lbgen.FILM_G1 + lbgen.FILM_G2)
    assert rl > 1.2 and rg < 0.4
    assert abs(pl - pg) < 1e-9 * abs(pl), (rl, rg, pl, pg)
    assert np.abs(fl["u"]).max() < 1e-6
