"""Parity at the benchmark workloads' full sizes, in the launch configuration bench.py times
(default tile shapes; for the batch, the tile and grid the autotuner picks): short horizons
the FP64 oracle computes in seconds on the whole lattice."""

import numpy as np
import pytest

import lbgen

pytestmark = pytest.mark.gpu


def rel_fields(rho, u, ref):
    return (float(np.abs(rho - ref["rho"]).max() / np.abs(ref["rho"]).max()),
            float(np.abs(u - ref["u"]).max() / np.abs(ref["u"]).max()))


def run_pair(lx, ly, rho, kw, storage, steps):
    from oracle import Oracle, Params
    from paper_1402_6019_amd import Sim
    P = Params(lx=lx, ly=ly, ns=2, walls=1 if kw["walls"] else 0, g1=kw["g1"], g2=kw["g2"], gab=kw["gab"],
               body=kw["body"], rho_wall=kw.get("rho_wall", (0.0, 0.0)), tau=kw["tau"], psi0=kw["psi0"],
               rho0=kw["rho0"])
    orc = Oracle(P, rho_init=rho)
    orc.step(steps)
    sim = Sim(lx, ly, rho, storage=storage, **kw)
    print(f"{lx}x{ly} {storage}: tile {sim.get_tile()}", flush=True)
    sim.step(steps)
    r, u = sim.moments()
    out = rel_fields(r.cpu().numpy(), u.cpu().numpy(), orc.fields())
    sim.close()
    return out


TOL = {"f64": (1e-12, 1e-11), "f32": (1e-5, 1e-5), "bf16dev": (1e-2, 5e-2)}


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16dev"])
def test_emulsion_1024_full_size(storage):
    """Two-component emulsion, 1024 x 1024 periodic, volume fraction 0.8 (the headline
    workload), 10 steps; FP64 advances them two per launch (its default for this lattice)."""
    import bench
    rho, _, kw = bench.workload()
    kw = dict(kw, walls=False)
    e_rho, e_u = run_pair(1024, 1024, rho, kw, storage, 10)
    print(f"emulsion 1024 {storage}: rho {e_rho:.2e} u {e_u:.2e}", flush=True)
    assert e_rho <= TOL[storage][0] and e_u <= TOL[storage][1]


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16dev"])
def test_channel_4096x512_full_size(storage):
    """Confined emulsion channel 4096 x 512 (walls, wetting, g = 1e-6, fraction 0.85), 6 steps,
    in the default launch shape and store policy: the FP64 and FP32 buffers exceed the Infinity
    Cache, so FP64 runs the streaming-store single step and FP32 two steps per launch."""
    lx, ly = 4096, 512
    rho, _ = lbgen.emulsion(lx, ly, fraction=0.85, seed=3, walls=True)
    kw = dict(n_species=2, walls=True, g1=lbgen.EMULSION_G1, g2=lbgen.EMULSION_G2, gab=lbgen.EMULSION_GAB,
              body=(1e-6, 0.0), rho_wall=lbgen.EMULSION_POOR, tau=(1.0, 1.0), psi0=1.0, rho0=lbgen.EMULSION_RHO0,
              rho_ref=(float(rho[0].mean()), float(rho[1].mean())))
    e_rho, e_u = run_pair(lx, ly, rho, kw, storage, 6)
    print(f"channel 4096x512 {storage}: rho {e_rho:.2e} u {e_u:.2e}", flush=True)
    assert e_rho <= TOL[storage][0] and e_u <= TOL[storage][1]


def test_couette_1040_full_size():
    """The Couette cell at the paper's 1040 x 1040 domain in the launch shape bench.py times
    (the autotuner's 128 x 10): FP32 fields and profile against the oracle after 6 steps."""
    from oracle import Oracle, Params
    from oracle import diagnostics as dg
    from paper_1402_6019_amd import Sim
    L = 1040
    rho, _ = lbgen.emulsion(L, L, fraction=0.8, seed=6, walls=True)
    kw = dict(g1=lbgen.EMULSION_G1, g2=lbgen.EMULSION_G2, gab=lbgen.EMULSION_GAB, rho_wall=lbgen.EMULSION_POOR,
              rho0=lbgen.EMULSION_RHO0, u_wall=(-0.01, 0.01))
    sim = Sim(L, L, rho, n_species=2, walls=True, storage="f32", tile=(128, 10), **kw)
    orc = Oracle(Params(lx=L, ly=L, ns=2, walls=1, **kw), rho_init=rho)
    sim.step(6)
    orc.step(6)
    r, u = sim.moments()
    e_rho, e_u = rel_fields(r.cpu().numpy(), u.cpu().numpy(), orc.fields())
    prof = sim.profile().cpu().numpy()
    ubar, sigma = dg.shear_profile(orc)
    e_ub = np.abs(prof[:L] - ubar).max() / np.abs(ubar).max()
    e_s = np.abs(prof[L:2 * L + 1] - sigma).max() / np.abs(sigma).max()
    print(f"couette 1040 f32: rho {e_rho:.2e} u {e_u:.2e} ubar {e_ub:.2e} sigma {e_s:.2e}", flush=True)
    assert e_rho <= 1e-5 and e_u <= 1e-5 and e_ub <= 1e-5 and e_s <= 1e-4
    sim.close()


def test_batched_sweep_full_size():
    """The 64-instance uneven sweep (seed 4) in FP32 with the autotuned shape; the three
    smallest instances against the oracle after 5 steps."""
    from oracle import Oracle, Params
    from paper_1402_6019_amd import Batch
    specs = lbgen.batch_specs(n=64, seed=4)
    inst = []
    for sp in specs:
        rho, _ = lbgen.emulsion(sp["lx"], sp["ly"], fraction=0.8, seed=sp["seed"], walls=True)
        inst.append(dict(lx=sp["lx"], ly=sp["ly"], rho_init=rho, g1=sp["g1"], g2=sp["g2"], gab=sp["gab"],
                         body=sp["body"], rho_wall=lbgen.EMULSION_POOR, tau=(1.0, 1.0), psi0=1.0,
                         rho0=lbgen.EMULSION_RHO0))
    b = Batch(inst, n_species=2, walls=True, storage="f32")
    shape, ms = b.autotune(trial_steps=3)
    print(f"sweep: autotuned {shape}, {ms:.3f} ms/step", flush=True)
    b.set_graph(2)
    b.step(5)
    order = np.argsort([sp["lx"] * sp["ly"] for sp in specs])[:3]
    for i in order:
        sp, it = specs[i], inst[i]
        P = Params(lx=sp["lx"], ly=sp["ly"], ns=2, walls=1, g1=sp["g1"], g2=sp["g2"], gab=sp["gab"], body=sp["body"],
                   rho_wall=lbgen.EMULSION_POOR, rho0=lbgen.EMULSION_RHO0)
        orc = Oracle(P, rho_init=it["rho_init"])
        orc.step(5)
        r, u = b.moments(int(i))
        e_rho, e_u = rel_fields(r.cpu().numpy(), u.cpu().numpy(), orc.fields())
        print(f"instance {i} ({sp['lx']}x{sp['ly']}): rho {e_rho:.2e} u {e_u:.2e}", flush=True)
        assert e_rho <= 1e-5 and e_u <= 1e-5
    b.close()
