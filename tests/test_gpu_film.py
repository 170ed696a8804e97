"""The thin film between two bubbles pressed together (disjoining-pressure section) on the
GPU: parity with the oracle, the film's survival under the frustrated couplings against its
rupture under a plain attraction of the same G1 + G2, and the film observables over a sweep
of bubble radii."""

import numpy as np
import pytest

import lbgen

pytestmark = pytest.mark.gpu


def geometry(radius, gap=6):
    lx, ly = 2 * radius + 60, 2 * radius + 40
    return lx, ly, ly // 2, lx // 2, int(lx / 2 - gap / 2 - radius / 2)


def make(radius, g1, g2, storage="f64", gap=6):
    from paper_1402_6019_amd import Sim
    lx, ly, _, _, _ = geometry(radius, gap)
    rho = lbgen.facing_bubbles(lx, ly, radius, gap)[None]
    return Sim(lx, ly, rho, n_species=1, storage=storage, g1=(g1, 0.0), g2=(g2, 0.0)), rho


def observe(sim, radius, gap=6):
    from paper_1402_6019_amd.film import film_observables
    lx, ly, yc, xf, xb = geometry(radius, gap)
    return film_observables(sim, yc, xf, xb, (2, 2))


def test_film_parity_with_oracle():
    """FP64 film run against the oracle after 3000 steps: density field, and the film
    observables against the same quantities taken from the oracle's fields."""
    from oracle import Oracle, Params
    from oracle import diagnostics as dg
    R = 16
    lx, ly, yc, xf, xb = geometry(R)
    sim, rho = make(R, lbgen.FILM_G1, lbgen.FILM_G2)
    orc = Oracle(Params(lx=lx, ly=ly, ns=1, g1=(lbgen.FILM_G1, 0.0), g2=(lbgen.FILM_G2, 0.0)), rho_init=rho)
    sim.set_graph(500)
    sim.step(3000)
    orc.step(3000)
    r_gpu = sim.moments()[0].cpu().numpy()
    r_orc = orc.fields()["rho"]
    err = np.abs(r_gpu - r_orc).max() / np.abs(r_orc).max()
    obs = observe(sim, R)
    sxx, _, syy = dg.stress_field(orc)
    p = 0.5 * (sxx + syy)
    pi_ref = p[yc, xb] - p[2, 2]
    print(f"film parity: rho {err:.2e}; h {obs['h']:.4f}; pi_cap {obs['pi_capillary']:.6e} vs {pi_ref:.6e}", flush=True)
    assert err < 1e-11
    assert obs["pi_capillary"] == pytest.approx(pi_ref, rel=1e-9)
    assert obs["h"] > 3.0
    sim.close()


def test_film_survives_frustrated_couplings_and_ruptures_without():
    R = 24
    fr, _ = make(R, lbgen.FILM_G1, lbgen.FILM_G2, storage="f32")
    pl, _ = make(R, lbgen.FILM_G1 + lbgen.FILM_G2, 0.0, storage="f32")
    for s in (fr, pl):
        s.set_graph(1000)
        s.step(20000)
    o_fr, o_pl = observe(fr, R), observe(pl, R)
    print(f"frustrated: {o_fr}\nplain: {o_pl}", flush=True)
    assert o_fr["h"] > 3.0 and o_fr["pi_capillary"] > 0
    assert o_pl["h"] == 0.0
    fr.close()
    pl.close()


def test_film_radius_sweep():
    """Bigger bubbles press with a smaller capillary pressure; the film stays open at
    every radius (FP64, 30000 steps each)."""
    out = []
    for R in (16, 24, 32, 48):
        sim, _ = make(R, lbgen.FILM_G1, lbgen.FILM_G2)
        sim.set_graph(1000)
        sim.step(30000)
        o = observe(sim, R)
        out.append((R, o["h"], o["pi_capillary"], o["pn_film"]))
        print(f"R={R}: h={o['h']:.4f} pi_cap={o['pi_capillary']:.4e} pn_film={o['pn_film']:.4e}", flush=True)
        sim.close()
    pis = [o[2] for o in out]
    assert all(o[1] > 3.0 for o in out)
    assert all(a > b > 0 for a, b in zip(pis, pis[1:]))
