"""Planar Couette cell on the GPU: walls sliding along x, the stream-wise averaged velocity
and shear-stress profiles, their time statistics (fluidity, stress correlator), against the
FP64 oracle and the closed forms that pin it."""

import numpy as np
import pytest

import lbgen
from cases import emulsion_case, make_oracle, make_sim, oracle_params, rel_err

pytestmark = pytest.mark.gpu

U_W = (-0.02, 0.03)


def couette_case(lx=70, ly=40, storage="f64", seed=40, tau=1.0):
    c = emulsion_case(lx, ly, walls=True, fraction=0.7, seed=seed, rmin=4, rmax=8, g=0.0, tau=tau)
    c["u_wall"] = U_W
    c["storage"] = storage
    return c


TOL = {"f64": 1e-12, "f32": 1e-5, "bf16dev": 5e-2}


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16dev"])
def test_moving_walls_match_oracle(storage):
    c = couette_case(storage=storage, tau=0.9)
    sim, orc = make_sim(c), make_oracle(c)
    sim.set_reduce_every(1)
    sim.wall_stress(reset=True)
    rec = orc.step(20, record=True)
    sim.step(20)
    rho, u = sim.moments()
    fl = orc.fields()
    e_rho = rel_err(rho.cpu().numpy(), fl["rho"])
    e_u = np.abs(u.cpu().numpy() - fl["u"]).max() / np.abs(fl["u"]).max()
    wb, wt = sim.wall_stress(reset=True)
    e_w = abs(wb - rec[:, 4].mean()) + abs(wt - rec[:, 5].mean())
    print(f"{storage}: rho {e_rho:.2e} u {e_u:.2e} wall stress {e_w:.2e} ({rec[:, 4].mean():.4e}, {rec[:, 5].mean():.4e})",
          flush=True)
    assert e_rho <= TOL[storage] and e_u <= TOL[storage]
    assert e_w <= TOL[storage] * abs(rec[:, 4]).mean()
    sim.close()


def test_moving_walls_tile_invariance_and_batch():
    """Any launch shape, and a batch instance, evolve bitwise like the default shape."""
    from paper_1402_6019_amd import Batch
    c = couette_case(storage="f32", tau=0.9)
    ref = make_sim(c)
    ref.step(15)
    f_ref = ref.checkpoint().cpu().numpy()
    for tile in ((64, 3), (128, 7), (256, 40)):
        sim = make_sim(c, tile=tile)
        sim.step(15)
        assert np.array_equal(sim.checkpoint().cpu().numpy(), f_ref), tile
        sim.close()
    c2 = couette_case(96, 33, storage="f32", seed=41)
    inst = [dict(lx=d["lx"], ly=d["ly"], rho_init=d["rho"], g1=d["g1"], g2=d["g2"], gab=d["gab"], body=d["body"],
                 rho_wall=d["rho_wall"], tau=d["tau"], psi0=d["psi0"], rho0=d["rho0"], rho_ref=d["rho_ref"],
                 u_wall=d["u_wall"]) for d in (c, c2)]
    b = Batch(inst, n_species=2, walls=True, storage="f32")
    b.step(15)
    assert np.array_equal(b.checkpoint(0).cpu().numpy(), f_ref)
    s2 = make_sim(c2)
    s2.step(15)
    assert np.array_equal(b.checkpoint(1).cpu().numpy(), s2.checkpoint().cpu().numpy())
    b.close()
    s2.close()
    ref.close()


def test_couette_closed_form_on_gpu():
    """One component, uniform density equal to the walls': exact linear profile and uniform
    stress rho nu S through every line at steady state (FP64)."""
    from paper_1402_6019_amd import Sim
    lx, ly, tau = 8, 12, 0.8
    ub, ut = -0.01, 0.015
    sim = Sim(lx, ly, np.ones((1, ly, lx)), n_species=1, walls=True, storage="f64", rho_wall=(1.0, 0.0),
              tau=(tau, tau), u_wall=(ub, ut))
    sim.set_graph(1000)
    sim.step(20000)
    prof = sim.profile().cpu().numpy()
    ubar, sigma = prof[:ly], prof[ly:2 * ly + 1]
    np.testing.assert_allclose(prof[2 * ly + 1:3 * ly + 1], 1.0, rtol=1e-12)  # uniform density
    assert np.all(prof[3 * ly + 1:] == 0.0)  # one component
    S = (ut - ub) / ly
    nu = (tau - 0.5) / 3
    y = np.arange(ly)
    assert np.abs(ubar - (ub + S * (y + 0.5))).max() < 1e-12 * abs(ut)
    np.testing.assert_allclose(sigma, nu * S, rtol=1e-10)
    st = sim.profile_stats(sim.profile().reshape(1, -1))
    np.testing.assert_allclose(st["fluidity"].cpu().numpy(), 1.0 / nu, rtol=1e-9)
    sim.close()


@pytest.mark.parametrize("storage,walls", [("f64", True), ("f64", False), ("f32", True)])
def test_profile_matches_oracle(storage, walls):
    """ubar(y) and sigma(k) of the GPU profile pass against the oracle's explicit pair sums,
    at several times; bitwise the same for every launch shape."""
    from oracle import diagnostics as dg
    c = emulsion_case(70, 40, walls=walls, fraction=0.7, seed=42, rmin=4, rmax=8, g=2e-5)
    c["storage"] = storage
    if walls:
        c["u_wall"] = U_W
    sim, orc = make_sim(c), make_oracle(c)
    tol = 1e-11 if storage == "f64" else 2e-4
    for t in (0, 7, 30):
        sim.step(t - sim.time)
        orc.step(t - orc.time)
        prof = sim.profile().cpu().numpy()
        ubar, sigma = dg.shear_profile(orc)
        e_u = np.abs(prof[:c["ly"]] - ubar).max() / max(np.abs(ubar).max(), 1e-3)
        ly = c["ly"]
        e_s = np.abs(prof[ly:2 * ly + 1] - sigma).max() / np.abs(sigma).max()
        rho_rows = orc.fields()["rho"].mean(axis=2)  # [ns, ly]
        e_r = np.abs(prof[2 * ly + 1:].reshape(2, ly) - rho_rows).max() / np.abs(rho_rows).max()
        print(f"{storage} walls={walls} t={t}: ubar {e_u:.2e} sigma {e_s:.2e} rho rows {e_r:.2e} "
              f"(max |sigma| {np.abs(sigma).max():.3e})", flush=True)
        assert e_u <= tol and e_s <= tol and e_r <= tol
    ref = sim.profile().cpu().numpy()
    for tile in ((64, 3), (128, 11), (256, 40)):
        sim.set_tile(*tile)
        assert np.array_equal(sim.profile().cpu().numpy(), ref), tile
    sim.close()


def test_profile_momentum_budget_on_gpu():
    """The GPU stress profile closes the x-momentum balance of every row to FP64 rounding:
    P_row(t+1) - P_row(t) = lx (sigma(y+1) - sigma(y)) + g M_row, with P_row and M_row from
    the GPU's own moments."""
    c = couette_case(storage="f64", tau=0.9)
    c["body"] = (2e-5, 0.0)
    sim = make_sim(c)
    sim.step(25)
    lx = c["lx"]

    def rows():
        rho, u = sim.moments()
        f = sim.checkpoint().cpu().numpy()
        cx = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
        jx = np.einsum("l,sl...->s...", cx, f).sum(axis=(0, 2))
        return jx, rho.cpu().numpy().sum(axis=(0, 2))

    for _ in range(3):
        p0, m0 = rows()
        sigma = sim.profile().cpu().numpy()[c["ly"]:2 * c["ly"] + 1]
        sim.step(1)
        p1, _ = rows()
        pred = lx * (sigma[1:] - sigma[:-1]) + c["body"][0] * m0
        assert np.abs((p1 - p0) - pred).max() < 1e-12 * np.abs(p1 - p0).max()
    sim.close()


def test_profile_stats_match_numpy():
    """Time statistics of GPU profile samples against the same statistics in numpy."""
    c = couette_case(storage="f32", tau=1.0)
    sim = make_sim(c)
    samples = sim.sample_profiles(12, 5)
    ly = c["ly"]
    k0 = ly // 3
    st = sim.profile_stats(samples, k0)
    s = samples.cpu().numpy()
    u, sig = s[:, :ly], s[:, ly:2 * ly + 1]
    np.testing.assert_allclose(st["rho_a"].cpu().numpy(), s[:, 2 * ly + 1:3 * ly + 1].mean(axis=0), rtol=1e-12)
    np.testing.assert_allclose(st["rho_b"].cpu().numpy(), s[:, 3 * ly + 1:].mean(axis=0), rtol=1e-12)
    np.testing.assert_allclose(st["u"].cpu().numpy(), u.mean(axis=0), rtol=1e-12, atol=1e-18)
    np.testing.assert_allclose(st["sigma"].cpu().numpy(), sig.mean(axis=0), rtol=1e-12, atol=1e-18)
    du = np.empty_like(sig)
    du[:, 0] = 2 * (u[:, 0] - U_W[0])
    du[:, ly] = 2 * (U_W[1] - u[:, ly - 1])
    du[:, 1:ly] = u[:, 1:] - u[:, :-1]
    np.testing.assert_allclose(st["fluidity"].cpu().numpy(), (du / sig).mean(axis=0), rtol=1e-10)
    d = sig - sig.mean(axis=0)
    corr = (d * d[:, [k0]]).mean(axis=0) / (d[:, k0] ** 2).mean()
    np.testing.assert_allclose(st["corr"].cpu().numpy(), corr, rtol=1e-9, atol=1e-12)
    assert st["corr"][k0].item() == pytest.approx(1.0, rel=1e-12)
    from paper_1402_6019_amd import LbError
    with pytest.raises(LbError):
        sim.profile_stats(samples, ly + 1)
    with pytest.raises(ValueError):
        sim.profile_stats(samples[:, :-1])
    sim.close()


def test_adjoint_with_moving_walls_matches_oracle_complex_step():
    """The adjoint's loss carries the moving walls' momentum; its gradient is unchanged in
    form (the wall term does not depend on the state)."""
    from oracle import cs_grad
    c = couette_case(40, 24, storage="f64", seed=43)
    c["body"] = (2e-5, 0.0)
    T, lw = 40, (1.0, 0.3)
    sim = make_sim(c)
    loss, g7 = sim.adjoint(T, lw, every=7)
    P = oracle_params(c)
    f0 = make_oracle(c).get_f()
    ref = [cs_grad(P, f0, T, lw, k) for k in range(4)]
    g4 = np.array([g7[0] + g7[1], g7[2] + g7[3], g7[4], g7[5]])
    d_o = np.array([d for _, d in ref])
    print(f"moving walls: loss {loss:.12e} vs {ref[0][0]:.12e}; grad {g4} vs {d_o}", flush=True)
    assert loss == pytest.approx(ref[0][0], rel=1e-10)
    np.testing.assert_allclose(g4, d_o, rtol=1e-8, atol=1e-12 * np.abs(d_o).max())
    sim.close()
