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


def test_flat_film_tension_parity_with_oracle():
    """The film tension and normal stress of a flat film (eq. (doppiasigma)'s input) from the
    GPU's pressure tensor against the same sums over the oracle's Appendix A tensor, FP64,
    after 3000 steps and averaged over the next two."""
    from oracle import Oracle, Params
    from oracle import diagnostics as dg
    from paper_1402_6019_amd import Sim
    from paper_1402_6019_amd.film import film_thickness, flat_film
    lx, ly = 64, 5
    rho = lbgen.flat_film(lx, ly, 5.0)[None]
    sim = Sim(lx, ly, rho, n_species=1, storage="f64", g1=(lbgen.FILM_G1, 0.0), g2=(lbgen.FILM_G2, 0.0))
    orc = Oracle(Params(lx=lx, ly=ly, ns=1, g1=(lbgen.FILM_G1, 0.0), g2=(lbgen.FILM_G2, 0.0)), rho_init=rho)
    sim.step(3000)
    orc.step(3000)
    got = flat_film(sim, mid=0.85)
    sig, line = 0.0, 0.0
    for _ in range(2):
        sxx, _, syy = dg.stress_field(orc)
        sig = sig + 0.5 * np.stack([sxx[ly // 2], syy[ly // 2]])
        line = line + 0.5 * orc.fields()["rho"][0, ly // 2]
        orc.step(1)
    gamma_ref = float((sig[0] - sig[1]).sum())
    print(f"flat film: gamma_f {got['gamma_f']:.12e} vs {gamma_ref:.12e}; p_n {got['p_n']:.12e}; h {got['h']:.4f}",
          flush=True)
    assert got["gamma_f"] == pytest.approx(gamma_ref, rel=1e-11)
    assert got["p_n"] == pytest.approx(float(sig[0].mean()), rel=1e-12)
    assert got["h"] == pytest.approx(film_thickness(line, lx // 2, 0.85), abs=1e-9)
    sim.close()


def test_flat_films_give_a_positive_decaying_disjoining_pressure():
    """Flat films relaxed at the frustrated couplings reach mechanical equilibrium (uniform
    normal stress to rounding), thick films carry the tension of two free interfaces, and
    eq. (doppiasigma) turns the thin films' excess tension into a positive disjoining pressure
    that decreases with the film thickness."""
    from paper_1402_6019_amd import Sim
    from paper_1402_6019_amd.film import disjoining_from_tension, flat_film
    lx, ly = 160, 5
    rows = []
    for h0 in (3.0, 4.0, 5.0, 16.0, 40.0):
        sim = Sim(lx, ly, lbgen.flat_film(lx, ly, h0)[None], n_species=1, storage="f64",
                  g1=(lbgen.FILM_G1, 0.0), g2=(lbgen.FILM_G2, 0.0))
        sim.set_graph(1000)
        sim.step(60000)
        rows.append(flat_film(sim, mid=0.8555))
        sim.close()
    for r in rows:
        print(r, flush=True)
        assert r["p_n_spread"] < 1e-7 * r["p_n"]
    h = np.array([r["h"] for r in rows])
    g = np.array([r["gamma_f"] for r in rows])
    assert np.all(np.diff(h) > 0)
    assert abs(g[3] - g[4]) < 1e-3 * g[4]  # thick films: 2 gamma
    assert np.all(g[:3] > g[4])            # thin films: excess tension
    pi = disjoining_from_tension(h, g)
    print(f"h {h}\nPi {pi}", flush=True)
    assert pi[0] > pi[1] > pi[2] > 0
    assert 1e-4 < pi[0] < 1e-2
