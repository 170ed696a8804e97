"""Two time steps per launch (lb_set_two_step): the intermediate post-collision populations
stay on chip, and the per-site arithmetic and the rounding of the intermediate to the storage
format are those of two single steps, so the populations must be bitwise those of the
single-step kernel: ragged strips (54 columns) and segments, walls sliding or at rest, one and
two species, FP32 and BF16 (rounded to nearest and stochastically), odd step counts (a pair
launch plus one single step), graph replay, and a lattice narrower than one 64-lane window."""

import numpy as np
import pytest

from cases import emulsion_case, film_case, make_sim

pytestmark = pytest.mark.gpu


def run(c, steps, two_step=None, rows=0, graph=0, rounding=None, tile=None):
    sim = make_sim(c, tile=tile)
    if rounding:
        sim.set_rounding(rounding)
    sim.set_two_step(bool(two_step), rows)
    if graph:
        sim.set_graph(graph)
    sim.step(steps)
    f = sim.checkpoint().cpu().numpy()
    t = sim.time
    sim.close()
    return f, t


@pytest.mark.parametrize("storage,walls,rounding", [("f32", False, None), ("f32", True, None),
                                                    ("bf16dev", True, None), ("bf16dev", False, "stochastic"),
                                                    ("bf16dev", True, "stochastic")])
def test_two_step_bitwise_two_species(storage, walls, rounding):
    c = emulsion_case(130, 45, walls=walls, fraction=0.7, seed=41, rmin=5, rmax=9, g=1e-5 if walls else 0.0)
    c["storage"] = storage
    c["tau"] = (0.9, 1.2)
    if walls:
        c["u_wall"] = (-0.01, 0.02)
    for steps in (14, 13):
        ref, _ = run(c, steps, rounding=rounding)
        for rows in (0, 1, 3, 7, 45):
            f, t = run(c, steps, two_step=True, rows=rows, rounding=rounding)
            assert t == steps
            assert np.array_equal(f, ref), (steps, rows)
    ref, _ = run(c, 24, rounding=rounding)
    f, _ = run(c, 24, two_step=True, graph=6, rounding=rounding)
    assert np.array_equal(f, ref), "graph replay"
    f, _ = run(c, 24, two_step=True, graph=8, rounding=rounding)
    assert np.array_equal(f, ref), "graph replay, even number of launches"


@pytest.mark.parametrize("lx,ly,walls", [(96, 70, False), (40, 33, False), (61, 20, True)])
def test_two_step_bitwise_one_species(lx, ly, walls):
    c = film_case(lx, ly, storage="f32", tau=0.8)
    if walls:
        c["walls"] = 1
        c["rho_wall"] = (1.0, 0.0)
        c["body"] = (1e-5, 0.0)
    ref, _ = run(c, 20)
    for rows in (0, 2, 11):
        f, _ = run(c, 20, two_step=True, rows=rows)
        assert np.array_equal(f, ref), rows


def test_two_step_bitwise_full_size_emulsion():
    """The 1024^2 headline lattice, FP32 and BF16, ten steps, default segments."""
    import bench
    from paper_1402_6019_amd import Sim
    rho, _, kw = bench.workload()
    for storage in ("f32", "bf16dev"):
        out = []
        for two in (False, True):
            sim = Sim(1024, 1024, rho, storage=storage, **kw)
            sim.set_two_step(two)
            sim.step(10)
            out.append(sim.checkpoint().cpu().numpy())
            sim.close()
        assert np.array_equal(out[0], out[1]), storage


@pytest.mark.parametrize("walls", [True, False])
def test_two_step_bitwise_fp64(walls):
    """FP64 runs the same march at one wave per SIMD (its register FIFOs in the accumulation
    registers), the intermediate kept exactly."""
    c = emulsion_case(130, 45, walls=walls, fraction=0.7, seed=43, rmin=5, rmax=9, g=1e-5 if walls else 0.0)
    c["storage"] = "f64"
    c["tau"] = (0.9, 1.2)
    if walls:
        c["u_wall"] = (-0.01, 0.02)
    for steps in (14, 13):
        ref, _ = run(c, steps)
        for rows in (0, 1, 7, 45):
            f, t = run(c, steps, two_step=True, rows=rows)
            assert t == steps
            assert np.array_equal(f, ref), (steps, rows)
    ref, _ = run(c, 24)
    f, _ = run(c, 24, two_step=True, graph=8)
    assert np.array_equal(f, ref), "graph replay"
    c1 = film_case(61, 20, storage="f64", tau=0.8)
    ref, _ = run(c1, 11)
    f, _ = run(c1, 11, two_step=True, rows=3)
    assert np.array_equal(f, ref), "one species"


def test_two_step_auto_picks_pairs_beyond_the_cache():
    """The default (auto) pairs the steps of an FP32 lattice whose buffers exceed the Infinity
    Cache and leaves smaller ones alone; either way the populations equal those of forced single
    steps."""
    import lbgen
    from paper_1402_6019_amd import Sim
    lx, ly = 4096, 512  # 2 x 151 MB in FP32
    rho, _ = lbgen.emulsion(lx, ly, fraction=0.85, seed=3, walls=True)
    kw = dict(n_species=2, walls=True, g1=lbgen.EMULSION_G1, g2=lbgen.EMULSION_G2, gab=lbgen.EMULSION_GAB,
              body=(1e-6, 0.0), rho_wall=lbgen.EMULSION_POOR, rho0=lbgen.EMULSION_RHO0,
              rho_ref=(float(rho[0].mean()), float(rho[1].mean())))
    out = {}
    for mode in ("auto", False):
        sim = Sim(lx, ly, rho, storage="f32", **kw)
        sim.set_two_step(mode)
        assert sim.two_step_active == (mode == "auto")
        sim.step(6)
        out[mode] = sim.checkpoint().cpu().numpy()
        sim.close()
    assert np.array_equal(out["auto"], out[False])
    # a reducing context steps one launch at a time
    sim = Sim(lx, ly, rho, storage="f32", **kw)
    sim.set_reduce_every(1)
    assert not sim.two_step_active
    sim.close()


@pytest.mark.parametrize("walls,storage,pairs", [(False, "f64", True), (True, "f64", False), (False, "f32", False)])
def test_two_step_auto_rule_at_1024(walls, storage, pairs):
    """At 1024^2, auto pairs the steps of the periodic FP64 lattice (2 x 151 MB) and of no walled
    FP64 one, nor of the cache-resident FP32 lattice; the populations equal forced single steps."""
    import lbgen
    from paper_1402_6019_amd import Sim
    lx = ly = 1024
    rho, _ = lbgen.emulsion(lx, ly, fraction=0.8, seed=2, walls=walls)
    kw = dict(n_species=2, walls=walls, g1=lbgen.EMULSION_G1, g2=lbgen.EMULSION_G2, gab=lbgen.EMULSION_GAB,
              rho_wall=lbgen.EMULSION_POOR, rho0=lbgen.EMULSION_RHO0,
              rho_ref=(float(rho[0].mean()), float(rho[1].mean())))
    out = {}
    for mode in ("auto", False):
        sim = Sim(lx, ly, rho, storage=storage, **kw)
        sim.set_two_step(mode)
        assert sim.two_step_active == (pairs and mode == "auto")
        sim.step(5)
        out[mode] = sim.checkpoint().cpu().numpy()
        sim.close()
    assert np.array_equal(out["auto"], out[False])
