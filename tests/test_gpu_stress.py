"""The site pressure tensor of Appendix A on the GPU (lb_stress_field) against the oracle's
shell-by-shell construction, and the uniform normal stress across a relaxed flat interface."""

import numpy as np
import pytest

import lbgen
from cases import emulsion_case, film_case, make_oracle, make_sim

pytestmark = pytest.mark.gpu


def compare(sim, orc, tol):
    from oracle import diagnostics as dg
    got = sim.stress_field().cpu().numpy()
    ref = np.stack(dg.stress_field(orc))
    scale = np.abs(ref).max()
    err = np.abs(got - ref).max() / scale
    return err


@pytest.mark.parametrize("case,storage,tol", [("film", "f64", 1e-13), ("emulsion", "f64", 1e-13),
                                              ("channel", "f64", 1e-13), ("channel", "f32", 2e-5)])
def test_stress_field_matches_oracle(case, storage, tol):
    if case == "film":
        c = film_case(96, 70)
    elif case == "emulsion":
        c = emulsion_case(70, 40, walls=False, fraction=0.7, seed=50, rmin=4, rmax=8)
    else:
        c = emulsion_case(70, 40, walls=True, fraction=0.7, seed=51, rmin=4, rmax=8, g=2e-5, tau=0.9)
        c["u_wall"] = (-0.02, 0.03)
    c["storage"] = storage
    sim, orc = make_sim(c), make_oracle(c)
    for t in (0, 9, 40):
        sim.step(t - sim.time)
        orc.step(t - orc.time)
        err = compare(sim, orc, tol)
        print(f"{case} {storage} t={t}: stress rel err {err:.2e}", flush=True)
        assert err <= tol
    ref = sim.stress_field().cpu().numpy()
    for tile in ((64, 3), (128, 13), (256, 40)):
        sim.set_tile(*tile)
        assert np.array_equal(sim.stress_field().cpu().numpy(), ref), tile
    import torch
    f32 = sim.stress_field(dtype=torch.float32).cpu().numpy()
    assert np.array_equal(f32, ref.astype(np.float32))  # the same values, rounded once on output
    sim.close()


def test_flat_interface_normal_stress_uniform_on_gpu():
    """A 128 x 5 slab at the single-component couplings relaxed in FP64 on the GPU: the xx
    component, averaged over two consecutive steps, is the same at every site to machine
    precision and equals (BULK) of the liquid density."""
    from oracle import diagnostics as dg
    from paper_1402_6019_amd import Sim
    lx, ly = 128, 5
    x = np.arange(lx)
    prof = 0.28 + (1.39 - 0.28) * 0.5 * (np.tanh((x - 32 + 0.5) / 3.0) - np.tanh((x - 96 + 0.5) / 3.0))
    rho = np.broadcast_to(prof, (1, ly, lx)).copy()
    sim = Sim(lx, ly, rho, n_species=1, storage="f64", g1=(lbgen.FILM_G1, 0.0), g2=(lbgen.FILM_G2, 0.0))
    sim.set_graph(1000)
    sim.step(70000)
    a = sim.stress_field().cpu().numpy()
    sim.step(1)
    b = sim.stress_field().cpu().numpy()
    sxx = 0.5 * (a[0] + b[0])
    print(f"flat interface: sigma_xx mean {sxx.mean():.12e} spread {np.ptp(sxx):.2e}", flush=True)
    assert np.ptp(sxx) / sxx.mean() < 1e-12
    r, _ = sim.moments()
    rl = r.cpu().numpy()[0, 2, 64]
    assert dg.bulk_pressure(rl, lbgen.FILM_G1 + lbgen.FILM_G2) == pytest.approx(sxx.mean(), rel=1e-9)
    sim.close()
