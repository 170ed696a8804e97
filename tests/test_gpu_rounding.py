"""Stochastic rounding of BF16 population stores (lb_set_rounding): bitwise reproducible for
every launch shape and under graph replay, and unbiased enough to carry a body force whose
increments are far below one BF16 step, which round-to-nearest loses."""

import hashlib

import numpy as np
import pytest

import lbgen

pytestmark = pytest.mark.gpu


def channel(lx, ly, seed=3, g=1e-6):
    rho, _ = lbgen.emulsion(lx, ly, fraction=0.85, seed=seed, walls=True, rmin=6, rmax=14)
    kw = dict(n_species=2, walls=True, g1=lbgen.EMULSION_G1, g2=lbgen.EMULSION_G2, gab=lbgen.EMULSION_GAB,
              body=(g, 0.0), rho_wall=lbgen.EMULSION_POOR, tau=(1.0, 1.0), psi0=1.0, rho0=lbgen.EMULSION_RHO0,
              rho_ref=(float(rho[0].mean()), float(rho[1].mean())))
    return rho, kw


def test_stochastic_rounding_is_reproducible():
    """Ragged strips and segments marching either way, and graph replay, give the same bits;
    the result differs from round-to-nearest."""
    from paper_1402_6019_amd import Sim
    rho, kw = channel(130, 45)
    ref = None
    for tile, graph in ((None, 0), ((64, 3), 0), ((128, 7), 0), ((256, 45), 0), (None, 10)):
        sim = Sim(130, 45, rho, storage="bf16dev", tile=tile, **kw)
        sim.set_rounding("stochastic")
        if graph:
            sim.set_graph(graph)
        sim.step(37)
        f = sim.checkpoint().cpu().numpy()
        print(tile, graph, hashlib.sha1(f.tobytes()).hexdigest()[:10], flush=True)
        if ref is None:
            ref = f
        assert np.array_equal(f, ref), (tile, graph)
        sim.close()
    sim = Sim(130, 45, rho, storage="bf16dev", **kw)
    sim.step(37)
    assert not np.array_equal(sim.checkpoint().cpu().numpy(), ref)
    sim.close()


def test_stochastic_rounding_carries_a_weak_body_force():
    """512 x 128 channel at g = 1e-6 for 20,000 steps, profiles averaged over the second half:
    round-to-nearest BF16 loses most of the flow, stochastic rounding keeps the flow rate and
    wall stress within a few percent of FP64."""
    from paper_1402_6019_amd import Sim
    rho, kw = channel(512, 128)
    out = {}
    for name, storage, rounding in (("f64", "f64", None), ("nearest", "bf16dev", None),
                                    ("stochastic", "bf16dev", "stochastic")):
        sim = Sim(512, 128, rho, storage=storage, **kw)
        if rounding:
            sim.set_rounding(rounding)
        sim.set_graph(100)
        sim.step(10000)
        st = sim.profile_stats(sim.sample_profiles(100, 100))
        u, sig = st["u"].cpu().numpy(), st["sigma"].cpu().numpy()
        out[name] = (u.sum(), sig[0], -sig[-1])
        print(name, out[name], flush=True)
        sim.close()
    q, wb, wt = out["f64"]
    assert abs(out["nearest"][0] / q - 1) > 0.5
    assert abs(out["stochastic"][0] / q - 1) < 0.05
    assert abs(out["stochastic"][1] / wb - 1) < 0.05 and abs(out["stochastic"][2] / wt - 1) < 0.05


def test_rounding_arguments():
    from paper_1402_6019_amd import LbError, Sim
    rho, kw = channel(64, 32)
    sim = Sim(64, 32, rho, storage="f32", **kw)
    with pytest.raises(LbError):
        sim.set_rounding("stochastic")  # FP32 storage
    sim.set_rounding("nearest")
    with pytest.raises(ValueError):
        sim.set_rounding("truncate")
    sim.close()
    sim = Sim(64, 32, rho, storage="bf16dev", **kw)
    sim.set_rounding("stochastic")
    with pytest.raises(LbError):
        sim.adjoint(10, (1.0, 0.0), every=5)  # the adjoint recomputes states
    sim.set_rounding("nearest")
    sim.close()


def test_batch_stochastic_rounding_matches_single_contexts():
    """A batch's instance rounds with the same bits as a single context of that lattice, over
    graph-replayed and individual steps."""
    from paper_1402_6019_amd import Batch, Sim
    cases = [channel(130, 45, seed=5), channel(96, 33, seed=6)]
    dims = [(130, 45), (96, 33)]
    inst = []
    for (rho, kw), (lx, ly) in zip(cases, dims):
        inst.append(dict(lx=lx, ly=ly, rho_init=rho, g1=kw["g1"], g2=kw["g2"], gab=kw["gab"], body=kw["body"],
                         rho_wall=kw["rho_wall"], tau=kw["tau"], psi0=kw["psi0"], rho0=kw["rho0"],
                         rho_ref=kw["rho_ref"]))
    b = Batch(inst, n_species=2, walls=True, storage="bf16dev")
    b.set_rounding("stochastic")
    b.set_graph(10)
    b.step(23)
    for i, ((rho, kw), (lx, ly)) in enumerate(zip(cases, dims)):
        sim = Sim(lx, ly, rho, storage="bf16dev", **kw)
        sim.set_rounding("stochastic")
        sim.step(23)
        assert np.array_equal(b.checkpoint(i).cpu().numpy(), sim.checkpoint().cpu().numpy()), i
        sim.close()
    b.close()
    b = Batch(inst, n_species=2, walls=True, storage="f32")
    from paper_1402_6019_amd import LbError
    with pytest.raises(LbError):
        b.set_rounding("stochastic")
    b.close()


def test_stochastic_rounding_resumes_bitwise_in_a_new_context():
    """A run checkpointed at step 7 and resumed in a new context with lb_set_time(7) continues
    bit for bit as the first context does after restoring the same checkpoint (the rounding bits
    of step t are seeded by t); without the step count the resumed run rounds differently."""
    from paper_1402_6019_amd import Sim
    rho, kw = channel(130, 45)
    first = Sim(130, 45, rho, storage="bf16dev", tile=(64, 7), **kw)
    first.set_rounding("stochastic")
    first.step(7)
    ck = first.checkpoint().clone()
    first.restore(ck)  # the same canonical round trip the resumed context takes
    first.step(9)
    ref = first.checkpoint().cpu().numpy()
    assert first.time == 16
    first.close()
    for set_time in (True, False):
        sim = Sim(130, 45, rho, storage="bf16dev", **kw)
        sim.set_rounding("stochastic")
        sim.restore(ck)
        if set_time:
            sim.set_time(7)
        sim.step(9)
        f = sim.checkpoint().cpu().numpy()
        assert np.array_equal(f, ref) == set_time, set_time
        sim.close()
    with pytest.raises(Exception):
        Sim(130, 45, rho, storage="bf16dev", **kw).set_time(-1)
