"""Batched persistent launches, HIP graph replay and the autotuner, on the GPU.

A batch instance must evolve exactly as the same lattice in its own context (same kernel
body, same per-site arithmetic): checked bitwise, for tile shapes and persistent grids that
give many rounds, ragged strips and segments, and both march directions.  One instance is
also checked against the FP64 oracle.  Graph replays are checked against individual launches
on every replay, with eager work between the replays.
"""

import numpy as np
import pytest

import lbgen
from cases import emulsion_case, make_oracle, make_sim, rel_err

pytestmark = pytest.mark.gpu

SHAPES = [(70, 40), (130, 33), (256, 20), (64, 64), (300, 17)]


def batch_cases(storage, walls=True):
    cases = []
    for i, (lx, ly) in enumerate(SHAPES):
        c = emulsion_case(lx, ly, walls=walls, fraction=0.7, seed=20 + i, rmin=4, rmax=8, g=1e-5 * (1 + 0.3 * i))
        # per-instance couplings and relaxation times
        c["g1"] = tuple(v * (1.0 + 0.03 * i) for v in c["g1"])
        c["g2"] = tuple(v * (1.0 + 0.02 * i) for v in c["g2"])
        c["gab"] = c["gab"] * (1.0 - 0.05 * i)
        c["tau"] = (1.0 + 0.05 * i, 1.0 + 0.05 * i)
        c["storage"] = storage
        cases.append(c)
    return cases


def make_batch(cases, storage):
    from paper_1402_6019_amd import Batch
    inst = [dict(lx=c["lx"], ly=c["ly"], rho_init=c["rho"], g1=c["g1"], g2=c["g2"], gab=c["gab"], body=c["body"],
                 rho_wall=c["rho_wall"], tau=c["tau"], psi0=c["psi0"], rho0=c["rho0"], rho_ref=c["rho_ref"],
                 u_wall=c.get("u_wall", (0.0, 0.0)))
            for c in cases]
    return Batch(inst, n_species=2, walls=bool(cases[0]["walls"]), storage=storage)


@pytest.mark.parametrize("storage,walls,tile", [("f64", True, None), ("f64", True, (64, 3, 7)),
                                                ("f32", False, (128, 5, 0)), ("bf16dev", True, (256, 8, 40))])
def test_batch_instances_match_single_contexts_bitwise(storage, walls, tile):
    cases = batch_cases(storage, walls)
    b = make_batch(cases, storage)
    if tile is not None:
        b.set_tile(*tile)
    print("batch tile", b.get_tile(), flush=True)
    b.step(13)
    for i, c in enumerate(cases):
        sim = make_sim(c)
        sim.step(13)
        ref = sim.checkpoint().cpu().numpy()
        got = b.checkpoint(i).cpu().numpy()
        assert np.array_equal(got, ref), f"instance {i} differs"
        r_b, u_b = b.moments(i)
        r_s, u_s = sim.moments()
        assert np.array_equal(r_b.cpu().numpy(), r_s.cpu().numpy())
        assert np.array_equal(u_b.cpu().numpy(), u_s.cpu().numpy())
        sim.close()
    b.close()


def test_batch_instance_against_oracle():
    cases = batch_cases("f64", True)
    b = make_batch(cases, "f64")
    b.step(20)
    for i in (0, 3):
        orc = make_oracle(cases[i])
        orc.step(20)
        fl = orc.fields()
        rho, u = b.moments(i)
        assert rel_err(rho.cpu().numpy(), fl["rho"]) < 1e-12
        assert np.abs(u.cpu().numpy() - fl["u"]).max() / max(np.abs(fl["u"]).max(), 1e-2) < 1e-11
    b.close()


def test_batch_totals_and_wall_stress_match_single_contexts():
    cases = batch_cases("f64", True)
    b = make_batch(cases, "f64")
    b.set_reduce_every(1)
    b.step(9)
    tot = b.totals()
    ws = b.wall_stress(reset=True)
    for i, c in enumerate(cases):
        sim = make_sim(c)
        sim.set_reduce_every(1)
        sim.step(9)
        (m0, m1), (px, py), q = sim.totals()
        w = sim.wall_stress(reset=True)
        np.testing.assert_allclose(tot[i], [m0, m1, px, py, q], rtol=1e-12, atol=1e-15 * m0)
        np.testing.assert_allclose(ws[i], w, rtol=1e-12, atol=1e-18)
        sim.close()
    b.close()


def test_batch_profiles_and_stress_fields_match_single_contexts():
    """Per-instance profiles and pressure tensors of a batch equal those of the same lattices
    in their own contexts, bit for bit (sliding walls on two instances)."""
    cases = batch_cases("f64", True)
    cases[1]["u_wall"] = (-0.01, 0.02)
    cases[3]["u_wall"] = (0.015, -0.005)
    b = make_batch(cases, "f64")
    b.step(11)
    for i, c in enumerate(cases):
        sim = make_sim(c)
        sim.step(11)
        assert np.array_equal(b.profile(i).cpu().numpy(), sim.profile().cpu().numpy()), i
        assert np.array_equal(b.stress_field(i).cpu().numpy(), sim.stress_field().cpu().numpy()), i
        sim.close()
    b.close()


def test_batch_graph_replays_match_individual_launches():
    cases = batch_cases("f32", True)
    ref = make_batch(cases, "f32")
    g = make_batch(cases, "f32")
    g.set_graph(4)
    for r in range(3):
        # 4 steps: one graph replay; then 3 eager steps that flip the parity, so the next
        # replay uses the other captured graph
        g.step(4)
        ref.step(4)
        for i in range(len(cases)):
            assert np.array_equal(g.checkpoint(i).cpu().numpy(), ref.checkpoint(i).cpu().numpy()), (r, i)
        g.step(3)
        ref.step(3)
        tot_g, tot_r = g.totals(), ref.totals()
        assert np.array_equal(tot_g, tot_r)
    assert g.time == ref.time == 21
    g.close()
    ref.close()


def test_single_context_graph_replay_matches_individual_launches():
    c = emulsion_case(200, 90, walls=True, fraction=0.7, seed=31, rmin=5, rmax=9, g=1e-5)
    c["storage"] = "f32"
    a, g = make_sim(c), make_sim(c)
    g.set_graph(6)
    for r in range(3):
        g.step(6)
        a.step(6)
        assert np.array_equal(g.checkpoint().cpu().numpy(), a.checkpoint().cpu().numpy()), r
        g.step(1)
        a.step(1)
    assert np.array_equal(g.checkpoint().cpu().numpy(), a.checkpoint().cpu().numpy())
    a.close()
    g.close()


def test_autotune_leaves_state_unchanged_and_picks_a_valid_shape():
    c = emulsion_case(300, 120, walls=False, fraction=0.7, seed=32, rmin=5, rmax=9)
    c["storage"] = "f32"
    sim, ref = make_sim(c), make_sim(c)
    sim.step(5)
    ref.step(5)
    before = sim.checkpoint().cpu().numpy()
    (tx, sy), ms = sim.autotune(trial_steps=3)
    print(f"autotune single: tile ({tx}, {sy}) {ms * 1e3:.1f} us/step", flush=True)
    assert tx in (64, 128, 256) and 1 <= sy <= 120 and ms > 0
    assert np.array_equal(sim.checkpoint().cpu().numpy(), before)
    sim.step(4)
    ref.step(4)
    assert np.array_equal(sim.checkpoint().cpu().numpy(), ref.checkpoint().cpu().numpy())
    sim.close()
    ref.close()

    cases = batch_cases("f32", True)
    b, bref = make_batch(cases, "f32"), make_batch(cases, "f32")
    b.step(3)
    bref.step(3)
    (tx, sy, grid), ms = b.autotune(trial_steps=2)
    print(f"autotune batch: tile ({tx}, {sy}) grid {grid} {ms * 1e3:.1f} us/step", flush=True)
    b.step(3)
    bref.step(3)
    for i in range(len(cases)):
        assert np.array_equal(b.checkpoint(i).cpu().numpy(), bref.checkpoint(i).cpu().numpy())
    b.close()
    bref.close()


def test_batch_sweep_specs_run():
    """A few instances drawn like the uneven sweep (sizes, couplings and body force from the
    seed) run in one batch, conserve mass per instance in FP64 reductions."""
    specs = lbgen.batch_specs(n=6, seed=4, ly_range=(64, 160), lx_range=(256, 640))
    inst = []
    for sp in specs:
        rho, _ = lbgen.emulsion(sp["lx"], sp["ly"], fraction=0.8, seed=sp["seed"], walls=True, rmin=6, rmax=14)
        inst.append(dict(lx=sp["lx"], ly=sp["ly"], rho_init=rho, g1=sp["g1"], g2=sp["g2"], gab=sp["gab"],
                         body=sp["body"], rho_wall=lbgen.EMULSION_POOR, tau=(1.0, 1.0), psi0=1.0,
                         rho0=lbgen.EMULSION_RHO0))
    from paper_1402_6019_amd import Batch
    b = Batch(inst, n_species=2, walls=True, storage="f32")
    t0 = b.totals()
    b.set_graph(10)
    b.step(50)
    t1 = b.totals()
    drift = np.abs(t1[:, :2] - t0[:, :2]) / t0[:, :2]
    print("FP32 mass drift per instance over 50 steps:", drift.max(), flush=True)
    assert drift.max() < 1e-5
    b.close()
