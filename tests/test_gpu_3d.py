"""Parity of the 3-D step (D3Q19, include/lb3.h) with the 3-D FP64 oracle, through the C ABI.

Tolerances as in two dimensions: FP64 1e-13 relative on densities, velocities and populations
for t <= 10 (the two sides differ in rounding order: pair-difference force sums, fused
multiply-adds, the rest-population closure), 1e-11 at t = 30; FP32 1e-5.  Lattices are ragged
against the 64-column strips, the ty-row bands and the z-segments; launch shapes give bitwise
identical populations."""

import numpy as np
import pytest

import lbgen

pytestmark = pytest.mark.gpu
U_FLOOR = 1e-2


def case3(lx, ly, lz, ns, walls, seed, tau=(1.0, 1.0), cross_psi=False, g=1e-5):
    if ns == 2:
        rho = lbgen.emulsion3d(lx, ly, lz, fraction=0.5, seed=seed, walls=walls, rmin=3, rmax=5)[0]
        kw = dict(g1=lbgen.EMULSION_G1, g2=lbgen.EMULSION_G2, gab=lbgen.EMULSION_GAB, rho0=lbgen.EMULSION_RHO0,
                  rho_wall=lbgen.EMULSION_POOR if walls else (0.0, 0.0))
    else:
        rng = np.random.default_rng(seed)
        rho = (1.0 + 0.01 * rng.uniform(-1, 1, (1, lz, ly, lx)))
        kw = dict(g1=(lbgen.FILM_G1, 0.0), g2=(lbgen.FILM_G2, 0.0), rho0=1.0, rho_wall=(1.0, 0.0) if walls else (0.0, 0.0))
    kw.update(tau=tau, body=(g if walls else 0.0, 0.0, 0.0), cross_psi=cross_psi)
    return rho, kw


def make_pair(lx, ly, lz, ns, walls, rho, kw, storage="f64", tile=None):
    from oracle import Oracle3, Params3
    from paper_1402_6019_amd import Sim3
    P = Params3(lx, ly, lz, ns=ns, walls=1 if walls else 0, g1=kw["g1"], g2=kw["g2"], gab=kw.get("gab", 0.0),
                body=kw["body"], rho_wall=kw["rho_wall"], tau=kw["tau"], rho0=kw["rho0"],
                cross_psi=1 if kw["cross_psi"] else 0)
    orc = Oracle3(P, rho_init=rho)
    sim = Sim3(lx, ly, lz, rho, n_species=ns, walls=walls, storage=storage, tile=tile, **kw)
    return sim, orc


def compare(sim, orc, tol, pops=True):
    rho, u = (x.cpu().numpy() for x in sim.moments())
    fl = orc.fields()
    e_rho = np.abs(rho - fl["rho"]).max() / np.abs(fl["rho"]).max()
    e_u = np.abs(u - fl["u"]).max() / max(np.abs(fl["u"]).max(), U_FLOOR)
    assert e_rho <= tol, f"rho {e_rho:.3e} at t={orc.time}"
    assert e_u <= tol, f"u {e_u:.3e} at t={orc.time}"
    if pops:
        f = sim.checkpoint().cpu().numpy()
        ref = orc.get_f()
        e_f = np.abs(f - ref).max() / np.abs(ref).max()
        assert e_f <= tol, f"populations {e_f:.3e} at t={orc.time}"
    return e_rho, e_u


@pytest.mark.parametrize("ns,walls,cross_psi", [(1, False, False), (1, True, False), (2, False, False),
                                                (2, True, False), (2, True, True)])
def test_3d_fp64_parity(ns, walls, cross_psi):
    lx, ly, lz = 70, 21, 13
    rho, kw = case3(lx, ly, lz, ns, walls, seed=31, tau=(0.8, 1.3) if ns == 2 else (0.9, 0.9), cross_psi=cross_psi)
    sim, orc = make_pair(lx, ly, lz, ns, walls, rho, kw, tile=(4, 5))
    print(f"3-D {lx}x{ly}x{lz} ns={ns} walls={walls} cross_psi={cross_psi}: tile {sim.get_tile()}", flush=True)
    compare(sim, orc, 1e-13)
    for t, tol in ((1, 1e-13), (10, 1e-13), (30, 1e-11)):
        sim.step(t - sim.time)
        orc.step(t - orc.time)
        e_rho, e_u = compare(sim, orc, tol)
        print(f"  t={t}: rho {e_rho:.2e} u {e_u:.2e}", flush=True)
    sim.close()


@pytest.mark.parametrize("storage,walls", [("f64", True), ("f32", False), ("f32", True)])
def test_3d_tile_shape_invariance_bitwise(storage, walls):
    lx, ly, lz = 70, 21, 13
    rho, kw = case3(lx, ly, lz, 2, walls, seed=32, tau=(0.9, 1.2))
    ref = None
    from paper_1402_6019_amd import Sim3
    tiles = [None, (1, 1), (2, 3), (4, 5), (4, 13), (1, 13)]
    if storage == "f32":  # eight-row workgroups (FP32 only); 21 rows leave a band of five
        tiles += [(8, 4), (8, 13)]
    for tile in tiles:
        sim = Sim3(lx, ly, lz, rho, n_species=2, walls=walls, storage=storage, tile=tile, **kw)
        sim.step(7)
        f = sim.checkpoint().cpu().numpy()
        if ref is None:
            ref = f
        assert np.array_equal(f, ref), tile
        sim.close()


def test_3d_eight_row_tile_is_refused_for_fp64():
    lx, ly, lz = 70, 21, 13
    rho, kw = case3(lx, ly, lz, 2, False, seed=33, tau=(1.0, 1.0))
    from paper_1402_6019_amd import Sim3, LbError
    sim = Sim3(lx, ly, lz, rho, n_species=2, walls=False, storage="f64", **kw)
    with pytest.raises(LbError):
        sim.set_tile(8, 4)
    sim.close()


@pytest.mark.parametrize("walls", [False, True])
def test_3d_fp32_parity(walls):
    lx, ly, lz = 70, 21, 13
    rho, kw = case3(lx, ly, lz, 2, walls, seed=33)
    sim, orc = make_pair(lx, ly, lz, 2, walls, rho, kw, storage="f32")
    for t in (1, 10):
        sim.step(t - sim.time)
        orc.step(t - orc.time)
        e_rho, e_u = compare(sim, orc, 1e-5, pops=False)
        print(f"3-D f32 walls={walls} t={t}: rho {e_rho:.2e} u {e_u:.2e}", flush=True)
    sim.close()


def test_3d_totals_and_conservation():
    """FP64 totals against the oracle's records, and mass and momentum conserved to 1e-12
    relative over 300 steps on a periodic two-species lattice (tau = 1: with tau = (0.8, 1.3) this
    small emulsion's densities dip below zero within 50 steps, in the oracle as on the GPU, and
    the health check reports it)."""
    lx, ly, lz = 40, 24, 20
    rho, kw = case3(lx, ly, lz, 2, False, seed=34, tau=(1.0, 1.0))
    sim, orc = make_pair(lx, ly, lz, 2, False, rho, kw)
    m0, p0, q0 = sim.totals()
    rec = orc.step(1, record=True)[0]
    # the oracle sums the 19,200 site masses one after the other: its rounding error is bounded
    # by (n - 1) 2^-53 ~ 2.1e-12 relative (the device sums in a tree)
    assert m0[0] == pytest.approx(rec[0], rel=3e-12) and m0[1] == pytest.approx(rec[1], rel=3e-12)
    assert q0 == pytest.approx(rec[7], rel=1e-9, abs=1e-15)
    sim.step(300)
    m1, p1, _ = sim.totals()
    for s in range(2):
        assert abs(m1[s] - m0[s]) / m0[s] < 1e-12
    scale = m0[0] + m0[1]
    assert max(abs(a - b) for a, b in zip(p1, p0)) < 1e-12 * scale
    sim.close()


def test_3d_channel_momentum_balance_gpu():
    """With walls and a body force, FP64: P_x grows by g M minus what the walls take, and the
    GPU's totals follow the oracle's after 40 steps."""
    lx, ly, lz = 36, 18, 10
    rho, kw = case3(lx, ly, lz, 2, True, seed=35, g=1e-5)
    sim, orc = make_pair(lx, ly, lz, 2, True, rho, kw)
    sim.step(40)
    orc.step(40)
    m, p, q = sim.totals()
    rec = orc.step(1, record=True)[0]
    assert m[0] == pytest.approx(rec[0], rel=3e-12)  # the oracle's serial sum, as above
    assert p[0] == pytest.approx(rec[2], rel=1e-9, abs=1e-13)
    assert q == pytest.approx(rec[7], rel=1e-9, abs=1e-15)
    sim.close()
