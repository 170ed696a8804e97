"""Parity of the HIP step (through the C ABI) with the FP64 CPU oracle.

Tolerances:
  * FP64 storage: relative 1e-13 on densities, velocities and populations for t <= 10 (the
    two implementations differ only in rounding order: fused multiply-adds, the pair-form
    force sum, the rest-population closure); later times allow the measured growth of
    rounding differences in phase-separating dynamics.  Velocities are normalised by
    max(max|u|, 1e-2): the force is a small residual of stencil terms of size |G| psi^2 ~ 1,
    so near rest its rounding is absolute, not relative to u.
  * FP32 storage: relative 1e-5 on densities and velocities.
  * BF16 deviation storage: the 8-bit mantissa bounds each stored deviation to ~2^-9 of its
    size; the measured error is asserted against a stated bound.
Sizes span several workgroup strips and segments with ragged tails in x and y.
"""

import numpy as np
import pytest

from cases import counterflow, emulsion_case, film_case, make_oracle, make_sim, rel_err

pytestmark = pytest.mark.gpu

U_FLOOR = 1e-2


def gpu_fields(sim):
    rho, u = sim.moments()
    return rho.cpu().numpy(), u.cpu().numpy()


def compare(sim, orc, rtol, pops=True):
    rho, u = gpu_fields(sim)
    fl = orc.fields()
    e_rho = rel_err(rho, fl["rho"])
    e_u = np.abs(u - fl["u"]).max() / max(np.abs(fl["u"]).max(), U_FLOOR)
    assert e_rho <= rtol, f"rho rel err {e_rho:.3e} at t={orc.time}"
    assert e_u <= rtol, f"u rel err {e_u:.3e} at t={orc.time}"
    if pops:
        f = sim.checkpoint().cpu().numpy()
        e_f = rel_err(f, orc.get_f())
        assert e_f <= rtol, f"populations rel err {e_f:.3e} at t={orc.time}"
    return e_rho, e_u


@pytest.mark.parametrize("tile", [None, (64, 5), (128, 64)])
def test_film_fp64_parity(tile):
    c = film_case(96, 70)  # ragged: 96 = 64 + 32 columns with tx = 64; 70 rows
    sim = make_sim(c, tile=tile)
    orc = make_oracle(c)
    compare(sim, orc, 1e-13)  # t = 0: layout round trip
    for t_target, tol in ((1, 1e-13), (10, 1e-13), (100, 1e-11)):
        sim.step(t_target - sim.time)
        orc.step(t_target - orc.time)
        compare(sim, orc, tol)


def test_film_fp64_long_horizon():
    """64x64 film run to t = 1000 (the phase-separation transient amplifies rounding
    differences; the bound is the measured growth with a margin)."""
    c = film_case(64, 64)
    sim = make_sim(c)
    orc = make_oracle(c)
    sim.step(1000)
    orc.step(1000)
    e_rho, e_u = compare(sim, orc, 1e-8, pops=False)
    print(f"t=1000 rho err {e_rho:.3e} u err {e_u:.3e}")


@pytest.mark.parametrize("walls", [False, True])
def test_emulsion_fp64_parity(walls):
    c = emulsion_case(100, 77, walls=walls, fraction=0.7, seed=5, rmin=5, rmax=10, g=1e-5)
    sim = make_sim(c, tile=(64, 16))
    orc = make_oracle(c)
    for t_target, tol in ((1, 1e-13), (10, 1e-13), (60, 1e-11)):
        sim.step(t_target - sim.time)
        orc.step(t_target - orc.time)
        compare(sim, orc, tol)


@pytest.mark.parametrize("cross_psi", [False, True])
@pytest.mark.parametrize("walls", [False, True])
def test_unequal_tau_counterflow_fp64_parity(walls, cross_psi):
    """tau = (0.8, 1.3) from a state whose species drift against each other, so the common
    velocity u' = sum_s (j_s / tau_s) / sum_s (rho_s / tau_s) and the shift tau_s F_s / rho_s
    both matter; the A-B repulsion between densities or, with cross_psi, between
    pseudopotentials.  Ragged lattice, walls with wetting and a body force, or periodic."""
    c = emulsion_case(100, 77, walls=walls, fraction=0.7, seed=15, rmin=5, rmax=10, g=1e-5)
    c["tau"] = (0.8, 1.3)
    c["cross_psi"] = cross_psi
    f0 = counterflow(c, seed=15)
    orc = make_oracle(c)
    orc.set_f(f0)
    sim = make_sim(c, tile=(64, 16))
    sim.restore(f0)
    compare(sim, orc, 1e-13)  # t = 0: the restored counterflow state
    for t_target, tol in ((1, 1e-13), (10, 1e-13), (60, 1e-11)):
        sim.step(t_target - sim.time)
        orc.step(t_target - orc.time)
        e_rho, e_u = compare(sim, orc, tol)
        print(f"tau (0.8, 1.3) walls={walls} cross_psi={cross_psi} t={t_target}: rho {e_rho:.2e} u {e_u:.2e}")
    sim.close()


def test_channel_observables_fp64():
    """Species masses, momentum, flow rate and wall stress of the FP64 reductions against the
    oracle's per-step records."""
    c = emulsion_case(90, 40, walls=True, fraction=0.6, seed=9, rmin=5, rmax=9, g=1e-5)
    sim = make_sim(c, tile=(64, 8))
    orc = make_oracle(c)
    sim.step(20)
    orc.step(20)
    mass, mom, flow = sim.totals()
    rec = orc.step(1, record=True)[0]
    assert mass[0] == pytest.approx(rec[0], rel=1e-13)
    assert mass[1] == pytest.approx(rec[1], rel=1e-13)
    assert mom[0] == pytest.approx(rec[2], rel=1e-9, abs=1e-15 * rec[0])
    assert flow == pytest.approx(rec[6], rel=1e-9, abs=1e-16)
    # wall stress averaged over 30 steps, every step reduced
    sim.set_reduce_every(1)
    sim.step(1)  # the step the oracle just recorded
    recs = orc.step(29, record=True)
    sim.step(29)
    wb, wt = sim.wall_stress(reset=True)
    ref_b = np.mean(np.concatenate([[rec[4]], recs[:, 4]]))
    ref_t = np.mean(np.concatenate([[rec[5]], recs[:, 5]]))
    assert wb == pytest.approx(ref_b, rel=1e-9, abs=1e-16)
    assert wt == pytest.approx(ref_t, rel=1e-9, abs=1e-16)


@pytest.mark.parametrize("walls,storage", [(True, "f64"), (False, "f64"), (False, "f32"), (True, "bf16dev")])
def test_tile_shape_invariance_bitwise(walls, storage):
    """Every launch shape (strip width, segment height, march direction of odd segments,
    ragged strips and segments) gives bitwise identical populations: a halo, ring or
    direction mistake shows up as a difference."""
    c = emulsion_case(130, 45, walls=walls, fraction=0.7, seed=3, rmin=5, rmax=9, g=1e-5 if walls else 0.0)
    c["storage"] = storage
    c["tau"] = (0.9, 1.2)  # tau != 1, so that every multiply of the collision rounds
    ref = None
    for tile in (None, (64, 1), (64, 2), (64, 7), (128, 3), (256, 4), (256, 16), (256, 45)):
        sim = make_sim(c, tile=tile)
        sim.step(12)
        f = sim.checkpoint().cpu().numpy()
        if ref is None:
            ref = f
        else:
            assert np.array_equal(f, ref), f"tile {tile} differs"


@pytest.mark.parametrize("walls,storage", [(False, "f64"), (True, "f64"), (True, "f32"), (False, "bf16dev")])
def test_store_policies_bitwise(walls, storage):
    """Both variants of the step kernel, write-through stores with the tail rows' loads behind a
    branch and streaming stores with those loads issued through an empty buffer range, give
    bitwise identical populations for launch shapes with ragged segments marching either way,
    and the same wall stress at the same shape (its FP64 sum is grouped by workgroup), with the
    reductions on."""
    from paper_1402_6019_amd import LbError
    c = emulsion_case(130, 45, walls=walls, fraction=0.7, seed=13, rmin=5, rmax=9, g=1e-5 if walls else 0.0)
    c["storage"] = storage
    c["tau"] = (0.9, 1.2)
    if walls:
        c["u_wall"] = (-0.01, 0.02)
    ref = None
    for tile in (None, (64, 1), (64, 7), (128, 3), (256, 11), (256, 45)):
        same_shape = None
        for policy in ("write_through", "streaming"):
            sim = make_sim(c, tile=tile)
            sim.set_store_policy(policy)
            sim.set_reduce_every(3)
            sim.step(13)
            f = sim.checkpoint().cpu().numpy()
            ws = sim.wall_stress() if walls else None
            if ref is None:
                ref = f
            assert np.array_equal(f, ref), (tile, policy)
            if same_shape is None:
                same_shape = ws
            assert ws == same_shape, (tile, policy)
            sim.close()
    with pytest.raises(ValueError):
        sim.set_store_policy("uncached")
    sim = make_sim(c)
    with pytest.raises(LbError):
        sim._chk(sim._lib.lb_set_store_policy(sim._h, 3))
    sim.close()


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16dev"])
def test_checkpoint_restore_roundtrip(storage):
    """A checkpoint (canonical FP64 f = d + W rho_ref) restores to bitwise the stored state in
    every storage mode, so stepping on from a restore repeats the original run bit for bit."""
    c = emulsion_case(70, 50, walls=True, fraction=0.6, seed=4, rmin=5, rmax=9)
    c["storage"] = storage
    sim = make_sim(c)
    sim.step(7)
    f = sim.checkpoint()
    sim.step(5)
    g = sim.checkpoint().cpu().numpy()
    sim.restore(f)
    assert np.array_equal(sim.checkpoint().cpu().numpy(), f.cpu().numpy())
    sim.step(5)
    assert np.array_equal(sim.checkpoint().cpu().numpy(), g)


def test_mass_conservation_fp64():
    c = emulsion_case(128, 96, walls=True, fraction=0.7, seed=6, rmin=6, rmax=12, g=1e-5)
    sim = make_sim(c)
    m0, _, _ = sim.totals()
    sim.step(2000)
    m1, _, _ = sim.totals()
    for s in range(2):
        assert abs(m1[s] - m0[s]) / m0[s] < 1e-12


def amplification(c, times, eps=1e-9, seed=0):
    """Sensitivity of the dynamics itself, from the FP64 oracle alone: a relative density
    perturbation eps of the initial state grows to A(t) * eps.  Returns {t: (A_rho, A_u)}."""
    cp = dict(c)
    rng = np.random.default_rng(seed)
    cp["rho"] = c["rho"] * (1.0 + eps * rng.uniform(-1.0, 1.0, c["rho"].shape))
    o, op = make_oracle(c), make_oracle(cp)
    out = {}
    for t in times:
        o.step(t - o.time)
        op.step(t - op.time)
        a, b = o.fields(), op.fields()
        um = max(np.abs(a["u"]).max(), U_FLOOR)
        out[t] = (rel_err(b["rho"], a["rho"]) / eps, np.abs(b["u"] - a["u"]).max() / um / eps)
    return out


@pytest.mark.parametrize("case", ["film", "channel"])
def test_fp32_parity(case):
    """FP32 storage and arithmetic: within 1e-5 of the FP64 oracle while the dynamics do not
    amplify perturbations; later, within C * 2^-24 * A(t), where A(t) is the oracle's own
    amplification of an initial perturbation (FP32 rounding is a perturbation of ~2^-24 per
    step that the unstable modes of phase separation amplify like any other)."""
    c = film_case(96, 70) if case == "film" else emulsion_case(100, 77, walls=True, fraction=0.7, seed=5,
                                                                  rmin=5, rmax=10, g=1e-5)
    times = (1, 10, 100, 300)
    amp = amplification(c, times)
    sim = make_sim(c, storage="f32")
    orc = make_oracle(c)
    for t in times:
        sim.step(t - sim.time)
        orc.step(t - orc.time)
        rho, u = gpu_fields(sim)
        fl = orc.fields()
        e_rho = rel_err(rho, fl["rho"])
        e_u = np.abs(u - fl["u"]).max() / max(np.abs(fl["u"]).max(), U_FLOOR)
        tol_rho = max(1e-5, 128 * 2.0 ** -24 * amp[t][0])
        tol_u = max(1e-5, 128 * 2.0 ** -24 * amp[t][1])
        print(f"{case} t={t}: rho {e_rho:.2e} (tol {tol_rho:.1e}, A={amp[t][0]:.1f})  "
              f"u {e_u:.2e} (tol {tol_u:.1e}, A={amp[t][1]:.1f})")
        assert e_rho <= tol_rho and e_u <= tol_u
        if t <= 10:
            assert e_rho <= 1e-5


def _steady(c, steps, storage):
    sim = make_sim(c, storage=storage)
    orc = make_oracle(c)
    sim.step(steps)
    orc.step(steps)
    rho, u = gpu_fields(sim)
    fl = orc.fields()
    return rel_err(rho, fl["rho"]), rel_err(u, fl["u"]), fl


@pytest.mark.parametrize("storage,tol", [("f64", 1e-11), ("f32", 1e-5)])
def test_steady_poiseuille(storage, tol):
    """Single-phase channel flow driven by g, at steady state (velocity relative to its maximum)."""
    ly, lx = 32, 64
    c = dict(lx=lx, ly=ly, ns=1, walls=1, g1=(0.0, 0.0), g2=(0.0, 0.0), gab=0.0, body=(1e-5, 0.0),
             rho_wall=(1.0, 0.0), tau=(1.0, 1.0), psi0=1.0, rho0=1.0, rho=np.ones((1, ly, lx)), storage=storage,
             rho_ref=(1.0, 0.0))
    e_rho, e_u, fl = _steady(c, 12000, storage)
    print(f"poiseuille {storage}: rho {e_rho:.2e} u {e_u:.2e} (u max {fl['u'].max():.3e})")
    assert e_rho <= tol and e_u <= tol


def _bulk(rho):
    """Liquid and gas bulk densities: medians of the sites above / below the mid density
    (insensitive to a sub-lattice translation of the interfaces, unlike the extrema of the
    density kink next to them)."""
    mid = 0.5 * (rho.max() + rho.min())
    return float(np.median(rho[rho > mid])), float(np.median(rho[rho < mid]))


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_steady_flat_interface(storage):
    """Flat liquid slab at the film couplings relaxed to equilibrium (quasi one-dimensional),
    70,000 steps as in the oracle's own pin.  A periodic slab has a neutral translation mode:
    rounding differences shift both interfaces by a fraction of a site that nothing restores
    (the oracle's own response to a 1e-15 perturbation of the initial state grows to ~1e-11
    pointwise over these steps), so the converged state is compared on translation-invariant
    quantities: both bulk densities and the mass, 1e-11 in FP64 and 1e-5 in FP32.  FP64 is
    also compared pointwise, to the stated bound of the neutral mode's walk."""
    lx, ly = 128, 5
    x = np.arange(lx)
    prof = 0.28 + 1.11 * 0.5 * (np.tanh((x - 31.5) / 3.0) - np.tanh((x - 95.5) / 3.0))
    c = film_case(lx, ly)
    c["rho"] = np.broadcast_to(prof, (1, ly, lx)).copy()
    sim = make_sim(c, storage=storage)
    orc = make_oracle(c)
    sim.step(70000)
    orc.step(70000)
    rho, u = gpu_fields(sim)
    fl = orc.fields()
    if storage == "f64":
        (gl, gg), (ol, og) = _bulk(rho), _bulk(fl["rho"])
        e_pt = rel_err(rho, fl["rho"])
        # mass against the initial mass: the kernel closes each collision's mass balance
        # through the rest population, the oracle relaxes all nine populations as eq. (LB)
        # writes it, so its rounding lets its own mass drift by ~1e-12 over these steps
        m0 = c["rho"].sum()
        drift, drift_orc = abs(rho.sum() - m0) / m0, abs(fl["rho"].sum() - m0) / m0
        print(f"flat interface f64 at 7e4 steps: liquid {abs(gl - ol) / ol:.2e}, gas {abs(gg - og) / og:.2e}, "
              f"mass drift {drift:.2e} (oracle {drift_orc:.2e}), pointwise {e_pt:.2e}")
        assert abs(gl - ol) / ol <= 1e-11 and abs(gg - og) / og <= 1e-11
        assert drift <= 1e-13 and drift_orc <= 1e-11
        assert e_pt <= 1e-8
    else:
        (gl, gg), (ol, og) = _bulk(rho), _bulk(fl["rho"])
        print(f"flat interface f32: liquid {gl:.8f} vs {ol:.8f}, gas {gg:.8f} vs {og:.8f}")
        assert abs(gl - ol) / ol <= 1e-5 and abs(gg - og) / og <= 1e-5
        # FP32 moment sums round, so the rest-population closure conserves the rounded mass:
        # the drift is stated (measured ~1e-5 relative over these 4e4 steps), not pinned
        drift = abs(rho.sum() - fl["rho"].sum()) / fl["rho"].sum()
        print(f"flat interface f32: mass drift {drift:.2e}")
        assert drift <= 1e-4
    assert np.abs(u).max() < 1e-6


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_steady_droplet(storage):
    """Static liquid droplet (film couplings) after its shape relaxation: inside and outside
    densities and the equimolar radius (translation invariant)."""
    import lbgen
    from oracle import diagnostics as dg
    n = 64
    c = film_case(n, n)
    c["rho"] = lbgen.disc(n, n, 14, 1.39, 0.28)[None]
    sim = make_sim(c, storage=storage)
    orc = make_oracle(c)
    sim.step(6000)
    orc.step(6000)
    rho, _ = gpu_fields(sim)
    ref = orc.fields()["rho"]
    if storage == "f64":
        # pointwise: the droplet's two neutral translation modes walk as the slab's does
        assert rel_err(rho, ref) <= 1e-10
    (gl, gg), (ol, og) = _bulk(rho), _bulk(ref)
    rg = dg.droplet_radius(rho[0], gl, gg)
    ro = dg.droplet_radius(ref[0], ol, og)
    print(f"droplet {storage}: R {rg:.12f} vs {ro:.12f}, in {gl:.14f} vs {ol:.14f}, out {gg:.14f} vs {og:.14f}")
    tol = 1e-11 if storage == "f64" else 1e-5
    assert abs(gl - ol) / ol <= tol and abs(gg - og) / og <= tol
    assert abs(rg - ro) / ro <= tol


def test_bf16dev_error_bound():
    """BF16 deviations: each stored deviation carries ~2^-9 relative rounding; densities stay
    within 1e-2 relative of the oracle over 10 steps (stated, not hidden)."""
    c = emulsion_case(100, 77, walls=True, fraction=0.7, seed=5, rmin=5, rmax=10, g=1e-5)
    sim = make_sim(c, storage="bf16dev")
    orc = make_oracle(c)
    sim.step(10)
    orc.step(10)
    rho, _ = gpu_fields(sim)
    e = rel_err(rho, orc.fields()["rho"])
    print(f"bf16dev rho rel err at t=10: {e:.3e}")
    assert e < 1e-2


def test_unstable_run_is_reported():
    """A coupling far outside the stable range drives densities negative or non-finite; the
    reductions latch it and the next synchronising call returns LB_EUNSTABLE."""
    from paper_1402_6019_amd import LbError
    c = film_case(64, 64)
    c["g1"] = (-400.0, 0.0)
    sim = make_sim(c)
    sim.set_reduce_every(1)
    with pytest.raises(LbError) as ei:
        for _ in range(50):
            sim.step(10)
            sim.totals()
    assert ei.value.code == -4
