"""lb_profile_noalloc: the profile pass with its block and row sums in the library's static
device scratch instead of a buffer the context allocates.  Called through the C ABI and
compared with lb_profile on the same state (the same kernels, so bit for bit), on two calls in
a row, the second on a smaller lattice; a lattice whose sums exceed the scratch is refused."""

import ctypes

import numpy as np
import pytest

import lbgen

pytestmark = pytest.mark.gpu


def _channel(lx, ly, seed, storage, tile=None):
    from paper_1402_6019_amd import Sim
    rho, _ = lbgen.emulsion(lx, ly, fraction=0.7, seed=seed, walls=True, rmin=5, rmax=10)
    return Sim(lx, ly, rho, n_species=2, walls=True, storage=storage, g1=lbgen.EMULSION_G1, g2=lbgen.EMULSION_G2,
               gab=lbgen.EMULSION_GAB, body=(1e-5, 0.0), rho_wall=lbgen.EMULSION_POOR, rho0=lbgen.EMULSION_RHO0,
               u_wall=(-0.01, 0.02), tile=tile)


def _noalloc(sim):
    torch = sim.torch
    out = torch.full((4 * sim.ly + 1,), float("nan"), dtype=torch.float64, device=sim.device)
    rc = sim._lib.lb_profile_noalloc(sim._h, ctypes.c_void_p(out.data_ptr()))
    return rc, out


def test_profile_noalloc_matches_profile():
    for lx, ly, seed, storage, tile in ((300, 90, 21, "f64", None), (140, 37, 22, "f32", (64, 5))):
        sim = _channel(lx, ly, seed, storage, tile)
        sim.step(15)
        ref = sim.profile().cpu().numpy()
        rc, out = _noalloc(sim)
        assert rc == 0, sim._lib.lb_last_error(sim._h)
        got = out.cpu().numpy()
        print(f"{lx}x{ly} {storage}: max |noalloc - profile| = {np.abs(got - ref).max():.3e}", flush=True)
        assert np.isfinite(got).all()
        assert np.array_equal(got, ref)
        sim.close()


def test_profile_noalloc_refuses_a_lattice_beyond_the_scratch():
    # (4096 / 64 blocks + 1) * 1200 rows * 7 sums = 546,000 doubles > 524,288
    sim = _channel(4096, 1200, 23, "bf16dev", tile=(64, 16))
    rc, _ = _noalloc(sim)
    assert rc == -1
    assert b"static scratch" in sim._lib.lb_last_error(sim._h)
    sim.close()
