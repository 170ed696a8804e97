"""Benchmark of the fused two-belt lattice Boltzmann step on one MI355X.

Workload: two-component D2Q9 emulsion, 1024 x 1024 periodic, seeded polydisperse A droplets
(radii U(8, 24), volume fraction 0.8) in B, emulsion couplings (G_AA = -9.0/8.1,
G_BB = -8.0/7.1, G_AB = 0.587, psi = 1 - exp(-rho/0.83), tau = 1).  One step = one launch
of the fused kernel over the whole lattice (pull streaming, two-belt force, collision).

The headline value is the FP32-storage throughput in MLUPS (million lattice-site updates per
second, a two-component site counting once), with the FP64 path, the BF16-deviation path and
the FP32/BF16 error against the FP64 CPU oracle reported beside it.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--core]
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
LX, LY = 1024, 1024
BYTES_PER_VALUE = {"f64": 8, "f32": 4, "bf16dev": 2}


def kernel_source_hash():
    h = hashlib.sha256()
    # the step kernels' own source (lb_kernels.hip holds only their dispatch and the layout
    # and reduction kernels)
    for f in ("lb_step.hpp", "lb_step2.hpp", "lb_step_f64.hip", "lb_step_f32.hip", "lb_step_bf16.hip",
              "lb_internal.hpp", "lb_tables.hpp"):
        with open(os.path.join(ROOT, "paper_1402_6019_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def workload():
    import lbgen
    rho, info = lbgen.emulsion(LX, LY, fraction=0.8, seed=2)
    kw = dict(n_species=2, walls=False, g1=lbgen.EMULSION_G1, g2=lbgen.EMULSION_G2, gab=lbgen.EMULSION_GAB,
              body=(0.0, 0.0), tau=(1.0, 1.0), psi0=1.0, rho0=lbgen.EMULSION_RHO0,
              rho_ref=(float(rho[0].mean()), float(rho[1].mean())))
    return rho, info, kw


# whether the last time_storage run of (storage, shape) advanced its steps two per launch
PAIRS_SEEN = {}


def time_storage(storage, rho, kw, steps, warmup, tile=None, shape=(LX, LY), rounding=None):
    """Average duration of one step (= one fused-kernel launch) over `steps` launches, timed
    with HIP events recorded on the stream the kernels run on."""
    import torch
    from paper_1402_6019_amd import Sim
    sim = Sim(shape[0], shape[1], rho, storage=storage, tile=tile, **kw)
    if rounding:
        sim.set_rounding(rounding)
    sim.step(warmup)
    torch.cuda.synchronize()
    stream = sim.stream
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(stream)
    sim.step(steps)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(stop) / steps
    tile_used = sim.get_tile()
    PAIRS_SEEN[(storage, tuple(shape))] = sim.two_step_active
    sim.close()
    return ms, wall, tile_used


def headline_median(rho, kw, tile=None, repeats=5, steps=1000, graph=100):
    """The headline FP32 step timed the way a production loop runs it: plain steps replayed
    from captured HIP graphs of `graph` steps, `repeats` timings of `steps` steps each after a
    50-step warm-up; the median and every repeat, in ms per step."""
    import torch
    from paper_1402_6019_amd import Sim
    sim = Sim(LX, LY, rho, storage="f32", tile=tile, **kw)
    sim.set_graph(graph)
    sim.step(50 + graph)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    reps = []
    for _ in range(repeats):
        start.record(sim.stream)
        sim.step(steps)
        stop.record(sim.stream)
        torch.cuda.synchronize()
        reps.append(start.elapsed_time(stop) / steps)
    sim.close()
    med = sorted(reps)[len(reps) // 2]
    return {"ms_per_step": med, "mlups": LX * LY / (med * 1e-3) / 1e6,
            "frac": 144 * LX * LY / (med * 1e-3) / 1e9 / HBM_PEAK_GBS, "repeats_ms": reps, "graph_steps": graph,
            "steps_per_repeat": steps}


def gpu_warmup(rho, kw, seconds=1.0):
    """Untimed FP64 steps on the headline lattice until `seconds` of GPU work have run: the
    first timing in a fresh process otherwise reads 3-5% slow while the clocks ramp up."""
    import torch
    from paper_1402_6019_amd import Sim
    sim = Sim(LX, LY, rho, storage="f64", **kw)
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        sim.step(500)
        torch.cuda.synchronize()
    sim.close()


def channel_profiles(rho, kw, lx, ly, samples=20, every=100):
    """The channel's time-averaged outputs (velocity and density profiles, wall stress) from
    profile samples taken every `every` steps (FP32): a short average, to show the outputs
    and the cost of the profile pass at this size, not a converged flow."""
    import torch
    from paper_1402_6019_amd import Sim
    sim = Sim(lx, ly, rho, storage="f32", **kw)
    sim.set_graph(every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    smp = sim.sample_profiles(samples, every)
    st = sim.profile_stats(smp)
    torch.cuda.synchronize()
    seconds = time.perf_counter() - t0
    u, sig, ra, rb = (st[k].cpu().numpy() for k in ("u", "sigma", "rho_a", "rho_b"))
    sim.close()
    return {"steps": samples * every, "samples": samples, "seconds": seconds,
            "wall_stress_bot_top": [float(sig[0]), float(-sig[-1])], "u_centre": float(u[ly // 2]),
            "u_max": float(u.max()), "rho_a_centre": float(ra[ly // 2]), "rho_b_wall_rows": [float(rb[0]), float(rb[-1])]}


def channel_beyond_cache(steps):
    """Confined emulsion channel 4096 x 512 (walls, wetting, g = 1e-6, volume fraction 0.85):
    its FP32 ping-pong footprint (302 MB) exceeds the 256 MB Infinity Cache, so this rate is
    HBM-served, unlike the 1024^2 FP32 headline (151 MB)."""
    import lbgen
    lx, ly = 4096, 512
    rho, info = lbgen.emulsion(lx, ly, fraction=0.85, seed=3, walls=True)
    kw = dict(n_species=2, walls=True, g1=lbgen.EMULSION_G1, g2=lbgen.EMULSION_G2, gab=lbgen.EMULSION_GAB,
              body=(1e-6, 0.0), rho_wall=lbgen.EMULSION_POOR, tau=(1.0, 1.0), psi0=1.0, rho0=lbgen.EMULSION_RHO0,
              rho_ref=(float(rho[0].mean()), float(rho[1].mean())))
    out = {"workload": f"confined emulsion channel {lx}x{ly}, walls + wetting, g = 1e-6, volume fraction 0.85, seed 3"}
    out["profiles_f32"] = channel_profiles(rho, kw, lx, ly)
    out["copy_ceiling_f32_footprint"] = stream_copy(9 * 2 * 4 * lx * ly, 100)  # one FP32 population buffer
    # the kernel each mode runs at this footprint by default: FP32 two steps per launch, FP64
    # single steps with streaming stores (both beyond the Infinity Cache), BF16 (2 x 75.5 MB,
    # inside it) single steps with write-through stores
    kernels = {"f32": "step2_kernel<F32, 2 species, channel>: two steps per launch, write-through stores",
               "bf16dev": "step_kernel<BF16 deviations, 2 species, channel>, write-through stores",
               "f64": "step_kernel<F64, 2 species, channel>, streaming stores"}
    for storage in ("f32", "bf16dev", "f64"):
        ms, wall, tile = time_storage(storage, rho, kw, steps, max(10, steps // 10), shape=(lx, ly))
        bpl = 2 * 9 * 2 * BYTES_PER_VALUE[storage]
        gbs = bpl * lx * ly / (ms * 1e-3) / 1e9
        out[storage] = {"ms_per_step": ms, "mlups": lx * ly / (ms * 1e-3) / 1e6, "gbs": gbs, "frac": gbs / HBM_PEAK_GBS,
                        "footprint_mb": 2 * bpl / 2 * lx * ly / 1e6, "tile": list(tile), "kernel": kernels[storage]}
    return out


def channel_long_run(steps=50000, average_last=25000, every=100):
    """The confined channel 4096 x 512 run for `steps` steps in each storage mode from the same
    initial state, with the velocity, density and shear-stress profiles averaged over the last
    `average_last` steps (a profile every `every` steps); FP32 and BF16 (rounded to nearest, and
    stochastically) are compared with FP64, whose step matches the FP64 oracle to 1e-12.  The
    emulsion flow is chaotic, so the differences are those of time averages over decorrelated
    trajectories."""
    import numpy as np
    import torch
    import lbgen
    from paper_1402_6019_amd import Sim
    lx, ly = 4096, 512
    rho, info = lbgen.emulsion(lx, ly, fraction=0.85, seed=3, walls=True)
    kw = dict(n_species=2, walls=True, g1=lbgen.EMULSION_G1, g2=lbgen.EMULSION_G2, gab=lbgen.EMULSION_GAB,
              body=(1e-6, 0.0), rho_wall=lbgen.EMULSION_POOR, tau=(1.0, 1.0), psi0=1.0, rho0=lbgen.EMULSION_RHO0,
              rho_ref=(float(rho[0].mean()), float(rho[1].mean())))
    avg = {}
    for name, storage, rounding in (("f64", "f64", None), ("f32", "f32", None), ("bf16dev", "bf16dev", None),
                                    ("bf16dev_stochastic", "bf16dev", "stochastic")):
        t0 = time.perf_counter()
        sim = Sim(lx, ly, rho, storage=storage, **kw)
        if rounding:
            sim.set_rounding(rounding)
        m0, p0, _ = sim.totals()
        sim.set_graph(every)
        sim.step(steps - average_last)
        st = sim.profile_stats(sim.sample_profiles(average_last // every, every))
        torch.cuda.synchronize()
        u, sig, ra = (st[k].cpu().numpy() for k in ("u", "sigma", "rho_a"))
        m1, p1, _ = sim.totals()
        avg[name] = {"u": u, "sigma": sig, "rho_a": ra, "seconds": time.perf_counter() - t0,
                     "drift": conservation_drift(m0, m1, p0, p1, walls=True)}
        sim.close()
    ref = avg["f64"]
    out = {"workload": f"confined emulsion channel {lx}x{ly}, fraction 0.85, seed 3, g = 1e-6, {steps} steps, "
                       f"profiles averaged over the last {average_last} (every {every})",
           "f64": {"flow_rate": float(ref["u"].sum()), "u_max": float(ref["u"].max()),
                   "wall_stress_bot_top": [float(ref["sigma"][0]), float(-ref["sigma"][-1])],
                   "seconds": ref["seconds"], "drift": ref["drift"]}}
    for name in ("f32", "bf16dev", "bf16dev_stochastic"):
        a = avg[name]
        out[name] = {
            "u_rel_err": float(np.abs(a["u"] - ref["u"]).max() / np.abs(ref["u"]).max()),
            "rho_a_rel_err": float(np.abs(a["rho_a"] - ref["rho_a"]).max() / np.abs(ref["rho_a"]).max()),
            "flow_rate_rel_err": float(abs(a["u"].sum() - ref["u"].sum()) / abs(ref["u"].sum())),
            "wall_stress_rel_err": [float(abs(a["sigma"][0] - ref["sigma"][0]) / abs(ref["sigma"][0])),
                                    float(abs(a["sigma"][-1] - ref["sigma"][-1]) / abs(ref["sigma"][-1]))],
            "seconds": a["seconds"], "drift": a["drift"]}
    return out


def conservation_drift(m0, m1, p0, p1, walls):
    """Relative change of each species' mass (FP64 totals) and, on periodic lattices without a
    body force, of the total momentum relative to the total mass (momentum per unit mass).  The
    walls of a channel exchange momentum with the fluid in both directions, so there only the
    masses are invariants."""
    M = m0[0] + m0[1]
    out = {"mass_rel": [abs(m1[s] - m0[s]) / m0[s] if m0[s] else 0.0 for s in range(2)]}
    if not walls:
        out["momentum_per_mass"] = max(abs(a - b) for a, b in zip(p1, p0)) / M
    return out


def long_run_1024(steps=20000):
    """The 1024^2 emulsion (the headline workload) run for `steps` steps in FP64 and FP32 from
    the same state: time, and the drift of each species' mass and of the total momentum
    (periodic, no body force: both are conserved), from the FP64 reductions."""
    import torch
    from paper_1402_6019_amd import Sim
    rho, _, kw = workload()
    out = {"workload": f"emulsion 1024x1024 periodic, fraction 0.8, seed 2, {steps} steps"}
    for storage in ("f64", "f32"):
        sim = Sim(LX, LY, rho, storage=storage, **kw)
        m0, p0, _ = sim.totals()
        sim.set_graph(100)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        m1, p1, _ = sim.totals()
        sim.close()
        out[storage] = {"seconds": dt, "mlups": LX * LY * steps / dt / 1e6,
                        "drift": conservation_drift(m0, m1, p0, p1, walls=False)}
    return out


def single_component_64(steps=1000):
    """Config 1: one component, 64 x 64 periodic, film couplings (G1 = -20.4, G2 = 16), tau = 1,
    rho = 1 + 0.01 U(-1, 1) (seed 1), FP64, 1000 steps: the GPU's time (launch-bound at this
    size; no roofline claim) against the FP64 oracle on one host thread and on all of them, the
    same run; and the GPU's fields against the oracle's at the end."""
    import numpy as np
    import torch
    import lbgen
    import oracle
    from oracle import Oracle, Params
    from paper_1402_6019_amd import Sim
    n = 64
    rho = lbgen.uniform_noise(n, n, 1.0, 0.01, seed=1)[None]
    kw = dict(n_species=1, walls=False, g1=(lbgen.FILM_G1, 0.0), g2=(lbgen.FILM_G2, 0.0), tau=(1.0, 1.0), psi0=1.0,
              rho0=1.0)
    sim = Sim(n, n, rho, storage="f64", **kw)
    sim.set_graph(100)
    sim.step(100)
    torch.cuda.synchronize()
    sim.restore(torch.as_tensor(np.broadcast_to(np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)[None, :, None, None]
                                                * rho[:, None], (1, 9, n, n)).copy()))
    sim.set_time(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    r_gpu = sim.moments()[0].cpu().numpy()
    m1, p1, _ = sim.totals()
    sim.close()
    P = Params(lx=n, ly=n, ns=1, g1=kw["g1"], g2=kw["g2"], tau=kw["tau"], psi0=1.0, rho0=1.0)
    threads = oracle.get_threads()
    res = {}
    for nt in (1, threads):
        oracle.set_threads(nt)
        o = Oracle(P, rho_init=rho)
        t0 = time.perf_counter()
        o.step(steps)
        res[nt] = (time.perf_counter() - t0, o.fields()["rho"])
    oracle.set_threads(threads)
    ref = res[threads][1]
    return {"workload": f"one component, {n}x{n} periodic, film couplings, tau = 1, seed 1, {steps} steps, FP64",
            "gpu_seconds": dt, "gpu_mlups": n * n * steps / dt / 1e6,
            "oracle_1_thread_seconds": res[1][0], "oracle_1_thread_mlups": n * n * steps / res[1][0] / 1e6,
            "oracle_all_threads_seconds": res[threads][0], "oracle_threads": threads,
            "oracle_all_threads_mlups": n * n * steps / res[threads][0] / 1e6,
            "rho_rel_err_vs_oracle": float(np.abs(r_gpu - ref).max() / np.abs(ref).max()),
            "mass_rel_drift": abs(m1[0] - float(rho.sum())) / float(rho.sum())}


def three_d(steps):
    """The 3-D extension (include/lb3.h): two-component emulsion, 256^3 periodic (a seeded 128^3
    periodic emulsion, radii U(6, 12), volume fraction 0.5, tiled 2 x 2 x 2), emulsion couplings,
    D3Q19 with the two-belt cube stencil; FP32 and FP64 steps timed with HIP events on the
    context's stream; algorithmic bytes per lattice update 2 * 19 * 2 values; mass and momentum
    drift over the timed steps."""
    import numpy as np
    import torch
    import lbgen
    from paper_1402_6019_amd import Sim3
    n = 256
    rho = np.tile(lbgen.emulsion3d(128, 128, 128, fraction=0.5, seed=7, rmin=6.0, rmax=12.0)[0], (1, 2, 2, 2))
    kw = dict(n_species=2, walls=False, g1=lbgen.EMULSION_G1, g2=lbgen.EMULSION_G2, gab=lbgen.EMULSION_GAB,
              tau=(1.0, 1.0), psi0=1.0, rho0=lbgen.EMULSION_RHO0,
              rho_ref=(float(rho[0].mean()), float(rho[1].mean())))
    out = {"workload": f"3-D two-component emulsion {n}^3 periodic, fraction 0.5, seed 7 (128^3 tiled 2x2x2)"}
    sites = n ** 3
    for storage, bpv in (("f32", 4), ("f64", 8)):
        sim = Sim3(n, n, n, rho, storage=storage, **kw)
        sim.step(5)
        m0, p0, _ = sim.totals()
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        start.record(sim.stream)
        sim.step(steps)
        stop.record(sim.stream)
        torch.cuda.synchronize()
        ms = start.elapsed_time(stop) / steps
        m1, p1, _ = sim.totals()
        tile = sim.get_tile()
        sim.close()
        bpl = 2 * 19 * 2 * bpv
        gbs = bpl * sites / (ms * 1e-3) / 1e9
        out[storage] = {"ms_per_step": ms, "mlups": sites / (ms * 1e-3) / 1e6, "bytes_per_lu": bpl,
                        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                     "frac": gbs / HBM_PEAK_GBS},
                        "tile_ty_sz": list(tile), "footprint_mb": 2 * bpl / 2 * sites / 1e6,
                        "drift": conservation_drift(m0, m1, p0, p1, walls=False)}
    return out


def batched_sweep(steps, n=64):
    """Uneven sweep of n independent confined emulsion channels (Ly ~ U{64..512},
    Lx ~ U{256..2048}, per-instance couplings and body force drawn from seed 4, volume
    fraction 0.8), FP32, all stepped by one persistent launch per step, replayed from a
    captured HIP graph; tile shape and grid from the autotuner."""
    import torch
    import lbgen
    from paper_1402_6019_amd import Batch
    specs = lbgen.batch_specs(n=n, seed=4)
    inst = []
    for sp in specs:
        rho, _ = lbgen.emulsion(sp["lx"], sp["ly"], fraction=0.8, seed=sp["seed"], walls=True)
        inst.append(dict(lx=sp["lx"], ly=sp["ly"], rho_init=rho, g1=sp["g1"], g2=sp["g2"], gab=sp["gab"],
                         body=sp["body"], rho_wall=lbgen.EMULSION_POOR, tau=(1.0, 1.0), psi0=1.0,
                         rho0=lbgen.EMULSION_RHO0))
    sites = sum(sp["lx"] * sp["ly"] for sp in specs)
    b = Batch(inst, n_species=2, walls=True, storage="f32")
    default_tile = b.get_tile()
    (tx, sy, grid), tuned_ms = b.autotune(trial_steps=5)
    graph = 20
    b.set_graph(graph)
    steps = max(graph, steps // graph * graph)
    b.step(2 * graph)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(b.stream)
    b.step(steps)
    stop.record(b.stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / steps
    b.set_graph(0)
    start.record(b.stream)
    b.step(steps)
    stop.record(b.stream)
    torch.cuda.synchronize()
    ms_eager = start.elapsed_time(stop) / steps
    # the persistent grid (as many workgroups as are resident at two waves per SIMD, each
    # taking tiles in rounds) at the tuned strip width and a few segment heights, graph-replayed
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    persistent = {}
    for sy_p in sorted({sy, 8, 16, 24}):
        b.set_tile(tx, sy_p, 2 * 4 * n_cu * 64 // tx)
        b.set_graph(graph)
        b.step(2 * graph)
        torch.cuda.synchronize()
        start.record(b.stream)
        b.step(steps)
        stop.record(b.stream)
        torch.cuda.synchronize()
        persistent[sy_p] = start.elapsed_time(stop) / steps
    b.set_tile(tx, sy, grid)
    # the sweep's horizon: 10,000 graph-replayed steps in all, then every instance's health
    # and FP64 species masses against the initial ones
    tot0 = b.totals()
    b.set_graph(graph)
    horizon = 10000
    b.step(max(0, horizon - b.time))
    tot1 = b.totals()  # raises on a latched non-finite or non-positive density
    import numpy as np
    mass_drift = float(np.max(np.abs(tot1[:, :2] - tot0[:, :2]) / tot0[:, :2]))
    steps_done = b.time
    b.close()
    gbs = 144 * sites / (ms * 1e-3) / 1e9
    return {"workload": f"{n} confined emulsion channels, Ly U{{64..512}}, Lx U{{256..2048}}, per-instance "
                        f"couplings and body force, seed 4, FP32", "sites": sites,
            "ms_per_step": ms, "ms_per_step_eager": ms_eager, "mlups": sites / (ms * 1e-3) / 1e6, "gbs": gbs,
            "frac": gbs / HBM_PEAK_GBS, "graph_steps": graph, "tile": [tx, sy], "grid": grid,
            "persistent_grid": {"workgroups": 2 * 4 * n_cu * 64 // tx,
                                "ms_per_step_by_sy": {str(k): v for k, v in persistent.items()},
                                "best_over_tuned": min(persistent.values()) / ms},
            "default_tile": list(default_tile), "autotune_best_ms": tuned_ms,
            "footprint_mb": 144 * sites / 1e6, "steps_total": steps_done, "all_instances_healthy": True,
            "max_species_mass_drift_fp32": mass_drift}


def auxiliary_passes(rho, kw, reps=200):
    """Cost of the passes around the plain step on the 1024^2 emulsion, FP32: the step with
    the FP64 reductions in its epilogue (mass, momentum, wall stress, flow rate, health), the
    moments output, the profile pass and the site pressure tensor; each timed over `reps`
    launches with HIP events on the library's stream (the steps as one lb_step call)."""
    import torch
    from paper_1402_6019_amd import Sim
    sim = Sim(LX, LY, rho, storage="f32", **kw)
    sim.step(50)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        start.record(sim.stream)
        for _ in range(reps):
            fn()
        stop.record(sim.stream)
        torch.cuda.synchronize()
        return start.elapsed_time(stop) / reps

    def timed_steps():
        sim.step(reps)
        torch.cuda.synchronize()
        start.record(sim.stream)
        sim.step(reps)
        stop.record(sim.stream)
        torch.cuda.synchronize()
        return start.elapsed_time(stop) / reps

    out = {}
    out["step_ms"] = timed_steps()
    sim.set_reduce_every(1)
    out["step_with_reductions_ms"] = timed_steps()
    sim.set_reduce_every(100)
    out["step_with_reductions_every_100_ms"] = timed_steps()
    sim.set_reduce_every(0)
    rho_o = torch.empty((2, LY, LX), dtype=torch.float32, device="cuda")
    u_o = torch.empty((2, LY, LX), dtype=torch.float32, device="cuda")
    import ctypes
    from paper_1402_6019_amd import _binding as B
    out["moments_f32_ms"] = timed(lambda: sim._lib.lb_moments(sim._h, ctypes.c_void_p(rho_o.data_ptr()),
                                                               ctypes.c_void_p(u_o.data_ptr()), B.LB_OUT_F32))
    prof = torch.empty(4 * LY + 1, dtype=torch.float64, device="cuda")
    out["profile_ms"] = timed(lambda: sim.profile(prof))
    sig = torch.empty((3, LY, LX), dtype=torch.float32, device="cuda")
    out["stress_field_f32_ms"] = timed(lambda: sim._lib.lb_stress_field(sim._h, ctypes.c_void_p(sig.data_ptr()),
                                                                         B.LB_OUT_F32))
    sim.close()
    read = 9 * 2 * 4 * LX * LY
    out["reduction_overhead"] = out["step_with_reductions_ms"] / out["step_ms"] - 1.0
    out["moments_gbs"] = (read + 4 * 4 * LX * LY) / (out["moments_f32_ms"] * 1e-3) / 1e9
    out["stress_field_gbs"] = (read + 3 * 4 * LX * LY) / (out["stress_field_f32_ms"] * 1e-3) / 1e9
    out["note"] = "moments and stress field: reads of the state plus their own FP32 outputs, per launch"
    return out


def couette_cell(steps, sample_every=100):
    """Planar Couette cell of the emulsion section at its 1040 x 1040 domain: confined
    emulsion (volume fraction 0.8, seed 6), walls wetted by B sliding with -U_w and +U_w
    (U_w = 0.01), FP32.  Times the plain step, the profile pass (lb_profile: a step's read of
    the state without the store, plus a small second pass) and a run that takes a profile
    every `sample_every` steps followed by the statistics pass.  The launch shape is the
    autotuner's (1040 columns do not fill whole 256-wide strips)."""
    import torch
    import lbgen
    from paper_1402_6019_amd import Sim
    lx = ly = 1040
    uw = 0.01
    rho, info = lbgen.emulsion(lx, ly, fraction=0.8, seed=6, walls=True)
    sim = Sim(lx, ly, rho, n_species=2, walls=True, storage="f32", g1=lbgen.EMULSION_G1, g2=lbgen.EMULSION_G2,
              gab=lbgen.EMULSION_GAB, rho_wall=lbgen.EMULSION_POOR, tau=(1.0, 1.0), psi0=1.0,
              rho0=lbgen.EMULSION_RHO0, u_wall=(-uw, uw))
    sim.step(200)
    default_tile = sim.get_tile()
    tile, _ = sim.autotune(trial_steps=20)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)

    def timed(fn, reps):
        start.record(sim.stream)
        for _ in range(reps):
            fn()
        stop.record(sim.stream)
        torch.cuda.synchronize()
        return start.elapsed_time(stop) / reps

    ms_step = timed(lambda: sim.step(1), steps)
    nprof = 50
    buf = torch.empty((nprof, 4 * ly + 1), dtype=torch.float64, device="cuda")
    it = iter(range(nprof))
    ms_prof = timed(lambda: sim.profile(buf[next(it)]), nprof)
    nsamp = max(2, steps // sample_every)
    start.record(sim.stream)
    samples = sim.sample_profiles(nsamp, sample_every)
    st = sim.profile_stats(samples)
    stop.record(sim.stream)
    torch.cuda.synchronize()
    ms_run = start.elapsed_time(stop) / (nsamp * sample_every)
    sig = st["sigma"].cpu().numpy()

    # two steps per launch (lb_set_two_step), timed over whole runs of steps
    def bulk(s, n):
        s.step(20)
        start.record(s.stream)
        s.step(n)
        stop.record(s.stream)
        torch.cuda.synchronize()
        return start.elapsed_time(stop) / n

    sim.set_two_step(True)
    ms_two = bulk(sim, steps)
    sim.close()
    # the same cell at 1024 x 1024 (whole 128- and 256-wide strips, whole 8-row segments) for
    # the cost per site of the ragged width
    rho_r, _ = lbgen.emulsion(1024, 1024, fraction=0.8, seed=6, walls=True)
    ref = Sim(1024, 1024, rho_r, n_species=2, walls=True, storage="f32", g1=lbgen.EMULSION_G1, g2=lbgen.EMULSION_G2,
              gab=lbgen.EMULSION_GAB, rho_wall=lbgen.EMULSION_POOR, tau=(1.0, 1.0), psi0=1.0,
              rho0=lbgen.EMULSION_RHO0, u_wall=(-uw, uw))
    ref.step(50)
    ref.autotune(trial_steps=20)
    ref_single = bulk(ref, steps)
    ref.set_two_step(True)
    ref_two = bulk(ref, steps)
    ref.close()
    ps = lambda ms, n: ms * 1e9 / (n * n)
    read_bytes = 9 * 2 * 4 * lx * ly
    return {"workload": f"Couette cell {lx}x{ly}, confined emulsion, volume fraction 0.8, seed 6, walls +-{uw}, FP32",
            "mass_fraction": info["mass_fraction"], "tile": list(tile), "default_tile": list(default_tile),
            "ms_per_step": ms_step, "mlups": lx * ly / (ms_step * 1e-3) / 1e6,
            "gbs": 144 * lx * ly / (ms_step * 1e-3) / 1e9,
            "ms_per_step_two_step": ms_two, "gbs_two_step": 144 * lx * ly / (ms_two * 1e-3) / 1e9,
            "ms_per_profile": ms_prof, "profile_read_gbs": read_bytes / (ms_prof * 1e-3) / 1e9,
            "profile_every": sample_every, "ms_per_step_with_profiles": ms_run,
            "profile_overhead": ms_run / ms_step - 1.0, "samples": nsamp,
            "mean_wall_stress": [float(sig[0]), float(-sig[-1])],
            "ragged_width": {"note": "ps per site of the 1040^2 cell against the same cell at 1024^2 (autotuned tile, "
                                     "whole runs of steps), single steps and two steps per launch",
                             "ps_per_site_1040": {"single": ps(ms_step, lx), "two_step": ps(ms_two, lx)},
                             "ps_per_site_1024": {"single": ps(ref_single, 1024), "two_step": ps(ref_two, 1024)},
                             "best_1040_over_best_1024": min(ps(ms_step, lx), ps(ms_two, lx)) /
                                                         min(ps(ref_single, 1024), ps(ref_two, 1024))}}


def couette_study(u_wall=0.01, fraction=0.8, warm=200000, samples=1500, every=200):
    """The fluidity profile of the Couette cell (emulsion section, eq. (predict)) at the
    paper's 1040 x 1040 domain: confined emulsion (volume fraction `fraction`, seed 6), walls
    sliding with -+u_wall, FP32, `warm` steps to forget the start, then a profile every `every`
    steps; time-averaged velocity, stress and local fluidity, and the cooperative-length fit
    (fluidity averaged over bins of 13 lines).  Not part of the default run."""
    import numpy as np
    import torch
    import lbgen
    from paper_1402_6019_amd import Sim, fit_cooperative_length
    L = 1040
    rho, info = lbgen.emulsion(L, L, fraction=fraction, seed=6, walls=True)
    sim = Sim(L, L, rho, n_species=2, walls=True, storage="f32", g1=lbgen.EMULSION_G1, g2=lbgen.EMULSION_G2,
              gab=lbgen.EMULSION_GAB, rho_wall=lbgen.EMULSION_POOR, rho0=lbgen.EMULSION_RHO0,
              u_wall=(-u_wall, u_wall))
    tile, _ = sim.autotune(10)
    sim.set_graph(every)
    t0 = time.perf_counter()
    sim.step(warm)
    smp = sim.sample_profiles(samples, every)
    st = sim.profile_stats(smp)
    torch.cuda.synchronize()
    seconds = time.perf_counter() - t0
    u, sig, fl = (st[k].cpu().numpy() for k in ("u", "sigma", "fluidity"))
    sim.close()
    z = np.arange(1, L, dtype=float)
    f = fl[1:-1]
    nb = len(f) // 13 * 13
    fit = fit_cooperative_length(z[:nb].reshape(-1, 13).mean(axis=1), f[:nb].reshape(-1, 13).mean(axis=1), float(L),
                                 (1.0, 5.0 * L))
    return {"workload": f"Couette cell {L}x{L}, confined emulsion, volume fraction {fraction}, seed 6, walls -+{u_wall}, "
                        f"FP32, {warm} + {samples} x {every} steps", "mass_fraction": info["mass_fraction"],
            "tile": list(tile), "seconds": seconds, "steps": warm + samples * every,
            "mean_shear_rate": 2 * u_wall / L, "sigma_mean": float(sig.mean()), "sigma_spread": float(np.ptp(sig)),
            "fluidity_at": {str(k): float(f[k - 1]) for k in (1, 5, 20, 50, 100, 200, 520)},
            "apparent_fluidity": float(2 * u_wall / L / sig.mean()), "fit": fit}


def film_sweep(radii=(16, 24, 32, 48, 64), steps=30000):
    """Disjoining pressure of the thin film between two gas bubbles pressed together
    (single component, G1 = -20.4, G2 = 16, FP64): for each bubble radius, the film thickness
    h on the axis and the capillary pressure between the bubble and outer bulk, which equals
    the film's disjoining pressure at equilibrium; `steps` graph-replayed steps per radius."""
    import torch
    import lbgen
    from paper_1402_6019_amd import Sim
    from paper_1402_6019_amd.film import film_observables
    gap = 6
    rows = []
    t0 = time.perf_counter()
    for R in radii:
        lx, ly = 2 * R + 60, 2 * R + 40
        sim = Sim(lx, ly, lbgen.facing_bubbles(lx, ly, R, gap)[None], n_species=1, storage="f64",
                  g1=(lbgen.FILM_G1, 0.0), g2=(lbgen.FILM_G2, 0.0))
        sim.set_graph(1000)
        sim.step(steps)
        o = film_observables(sim, ly // 2, lx // 2, int(lx / 2 - gap / 2 - R / 2), (2, 2))
        torch.cuda.synchronize()
        rows.append({"radius": R, "h": o["h"], "pi": o["pi_capillary"], "pn_film": o["pn_film"]})
        sim.close()
    import numpy as np
    theory = flat_film_theory()
    th, tp = np.array(theory["h"]), np.array(theory["pi"])
    order = np.argsort(th)
    for r in rows:
        r["pi_flat_film_theory"] = float(np.interp(r["h"], th[order], tp[order])) if r["h"] > 0 else None
    return {"workload": f"two facing half-disc bubbles, gap {gap}, G1 = -20.4, G2 = 16, FP64, {steps} steps each",
            "points": rows, "theory": theory, "seconds": time.perf_counter() - t0}


def flat_film_theory(thicknesses=(3.0, 3.5, 4.0, 4.5, 5.0, 5.5, 6.0, 6.5, 7.0, 8.0, 9.0, 10.0, 12.0, 16.0, 24.0, 40.0),
                     steps=60000, lx=160, ly=5):
    """The theoretical disjoining pressure of eq. (doppiasigma): flat films of several
    thicknesses relaxed at the same couplings (FP64), their film tension gamma_f(h) from the
    site pressure tensor, and Pi(h) = -int_h^inf gamma_f'/h' dh' (Pi = 0 at the thickest).
    The film thickness is measured at the density half-way between the bulk liquid and gas
    of the thickest film."""
    import lbgen
    from paper_1402_6019_amd import Sim
    from paper_1402_6019_amd.film import disjoining_from_tension, flat_film
    t0 = time.perf_counter()
    sims = []
    for h0 in thicknesses:
        sim = Sim(lx, ly, lbgen.flat_film(lx, ly, h0)[None], n_species=1, storage="f64",
                  g1=(lbgen.FILM_G1, 0.0), g2=(lbgen.FILM_G2, 0.0))
        sim.set_graph(1000)
        sim.step(steps)
        sims.append(sim)
    thick = flat_film(sims[-1])
    mid = 0.5 * (thick["rho_min"] + thick["rho_max"])
    rows = [flat_film(s, mid=mid) for s in sims]
    for s in sims:
        s.close()
    h = [r["h"] for r in rows]
    g = [r["gamma_f"] for r in rows]
    pi = disjoining_from_tension(h, g)
    return {"workload": f"flat films {lx}x{ly}, initial thickness {thicknesses[0]}..{thicknesses[-1]}, {steps} steps each, FP64",
            "h": h, "gamma_f": g, "pi": [float(p) for p in pi], "max_p_n_spread": max(r["p_n_spread"] for r in rows),
            "two_gamma": g[-1], "seconds": time.perf_counter() - t0}


def adjoint_channel(T=4000, prerelax=2000, check_fd=True):
    """Gradient of L = <(W_bot + W_top)/2> + <Q> over T steps with respect to (G1, G2, G_AB,
    g_x) on a 512 x 256 confined emulsion channel (G1, G2 shared by both species), after an
    FP64 pre-relaxation that is not differentiated: FP32 forward and reverse sweep with
    sqrt(T) FP64 checkpoints.  Checked against central differences (relative step 1e-4) of
    the FP64 forward path's own reductions."""
    import numpy as np
    import torch
    import lbgen
    from paper_1402_6019_amd import Sim
    lx, ly = 512, 256
    rho, _ = lbgen.emulsion(lx, ly, fraction=0.8, seed=5, walls=True)
    base = dict(n_species=2, walls=True, g1=(-9.0, -9.0), g2=(8.1, 8.1), gab=lbgen.EMULSION_GAB, body=(1e-6, 0.0),
                rho_wall=lbgen.EMULSION_POOR, tau=(1.0, 1.0), psi0=1.0, rho0=lbgen.EMULSION_RHO0)
    pre = Sim(lx, ly, rho, storage="f64", **base)
    pre.step(prerelax)
    f0 = pre.checkpoint().clone()
    pre.close()
    lw = (1.0, 1.0)
    sim = Sim(lx, ly, rho, storage="f32", **base)
    # one untimed call first: the workspace's first allocation is not part of a call's cost
    sim.restore(f0)
    sim.adjoint(T, lw, fp64_reverse=True)
    sim.restore(f0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss, g7 = sim.adjoint(T, lw, fp64_reverse=True)
    t_adj = time.perf_counter() - t0
    sim.restore(f0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss_all, g7_all = sim.adjoint(T, lw, every=1, fp64_reverse=True)
    t_adj_all = time.perf_counter() - t0
    ws_ckpt = sim._lib.lb_adjoint_workspace_bytes(sim._h, T, 0, 1)
    ws_all = sim._lib.lb_adjoint_workspace_bytes(sim._h, T, 1, 1)
    sim.restore(f0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss32, g7_32 = sim.adjoint(T, lw, fp64_reverse=False)
    t_adj32 = time.perf_counter() - t0
    sim.restore(f0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(T)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    sim.close()
    grad = [g7[0] + g7[1], g7[2] + g7[3], g7[4], g7[5]]
    grad32 = [g7_32[0] + g7_32[1], g7_32[2] + g7_32[3], g7_32[4], g7_32[5]]
    keys = ("G1", "G2", "G_AB", "g_x")
    out = {"workload": f"confined emulsion channel {lx}x{ly}, G1 = -9.0, G2 = 8.1 both species, g = 1e-6, "
                       f"fraction 0.8, seed 5, {prerelax} FP64 steps of pre-relaxation, then T = {T}",
           "storage": "FP32 forward (and recompute), FP64 checkpoints every ceil(sqrt(T)) steps, reverse sweep in "
                      "FP64 (grad) and in FP32 (grad_fp32_reverse)",
           "loss": loss, "grad": dict(zip(keys, grad)), "grad_fp32_reverse": dict(zip(keys, grad32)),
           "seconds_adjoint": t_adj, "seconds_adjoint_fp32_reverse": t_adj32, "seconds_forward_only": t_fwd,
           "adjoint_over_forward": t_adj / t_fwd, "workspace_gb": ws_ckpt / 1e9,
           "every_state_kept": {"note": "every = 1: the forward pass keeps what the reverse step reads of every "
                                        "state, nothing is recomputed; same FP64 reverse sweep",
                                "seconds_adjoint": t_adj_all, "adjoint_over_forward": t_adj_all / t_fwd,
                                "workspace_gb": ws_all / 1e9,
                                "grad_bitwise_equal_to_checkpointed": bool(loss_all == loss and (g7_all == g7).all())}}
    if check_fd:
        def fwd_loss(**kw):
            p = dict(base, **kw)
            sm = Sim(lx, ly, rho, storage="f64", **p)
            sm.restore(f0)
            sm.set_reduce_every(1)
            sm.wall_stress(reset=True)
            q = 0.0
            for _ in range(T):
                q += sm.totals()[2]
                sm.step(1)
            wb, wt = sm.wall_stress(reset=True)
            sm.close()
            return lw[0] * 0.5 * (wb + wt) + lw[1] * q / T
        names = ("g1", "g2", "gab", "body")
        vals = (-9.0, 8.1, lbgen.EMULSION_GAB, 1e-6)
        fd = []
        for name, v in zip(names, vals):
            h = 1e-4 * abs(v)
            def kw(x):
                return {name: (x, x)} if name in ("g1", "g2") else ({name: x} if name == "gab" else {name: (x, 0.0)})
            fd.append((fwd_loss(**kw(v + h)) - fwd_loss(**kw(v - h))) / (2 * h))
        out["fd_central_h1e-4"] = dict(zip(("G1", "G2", "G_AB", "g_x"), fd))
        out["rel_err_vs_fd"] = dict(zip(keys, [abs(a - b) / abs(b) for a, b in zip(grad, fd)]))
        out["rel_err_vs_fd_fp32_reverse"] = dict(zip(keys, [abs(a - b) / abs(b) for a, b in zip(grad32, fd)]))
        out["loss_fp64_forward"] = fwd_loss()
    return out


def copy_reference(nbytes, steps):
    """Plain device-to-device copy of one population buffer (torch's copy kernel), timed the
    same way: the practical streaming ceiling at this footprint, and the known-size kernel that
    scales the HBM byte counters."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(10):
        b.copy_(a)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(steps):
        b.copy_(a)
    stop.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / steps
    out = {"bytes_per_launch": 2 * nbytes, "ms": ms, "gbs": 2 * nbytes / (ms * 1e-3) / 1e9,
           "kernel": "torch copy_ (float32, contiguous)"}
    out.update(stream_copy(nbytes, steps))
    return out


def stream_copy(nbytes, steps):
    """The library's streaming copy (16-byte accesses, plain and non-temporal) of one buffer of
    nbytes into another, timed with HIP events: the bandwidth a stencil-free pass reaches."""
    import ctypes
    import torch
    from paper_1402_6019_amd import _binding as B
    lib = B.load()
    n = nbytes // 16 * 16
    a = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream()
    res = {}
    for nt in (0, 1):
        def run():
            B.check(lib.lb_stream_copy(ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(a.data_ptr()), n, nt,
                                       ctypes.c_void_p(stream.cuda_stream)))
        for _ in range(5):
            run()
        torch.cuda.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        start.record(stream)
        for _ in range(steps):
            run()
        stop.record(stream)
        torch.cuda.synchronize()
        ms = start.elapsed_time(stop) / steps
        res["stream_copy_nt_gbs" if nt else "stream_copy_gbs"] = 2 * n / (ms * 1e-3) / 1e9
    return res


def rel_errors(r, u, ref):
    """Max-norm errors of rho and u relative to the max-norm of the oracle's fields."""
    import numpy as np
    return {"rho": float(np.abs(r - ref["rho"]).max() / np.abs(ref["rho"]).max()),
            "u": float(np.abs(u - ref["u"]).max() / np.abs(ref["u"]).max())}


def emulsion_errors(rho, kw, ref_by_t):
    """rho and u of each GPU storage mode against the oracle at the checkpoint times (the
    emulsion coarsens, so a rounding difference grows with time like any perturbation)."""
    from paper_1402_6019_amd import Sim
    out = {}
    for storage in ("f64", "f32", "bf16dev"):
        sim = Sim(LX, LY, rho, storage=storage, **kw)
        out[storage] = {}
        for t in sorted(ref_by_t):
            sim.step(t - sim.time)
            r, u = sim.moments()
            out[storage][str(t)] = rel_errors(r.cpu().numpy(), u.cpu().numpy(), ref_by_t[t])
        sim.close()
    return out


CHANNEL_ERR = dict(lx=256, ly=128, steps=300, window=200)


def channel_err_case():
    """Confined emulsion in a 256 x 128 channel (walls, wetting, body force 1e-5)."""
    import lbgen
    rho, _ = lbgen.emulsion(CHANNEL_ERR["lx"], CHANNEL_ERR["ly"], fraction=0.85, seed=4, walls=True, rmin=6, rmax=14)
    kw = dict(n_species=2, walls=True, g1=lbgen.EMULSION_G1, g2=lbgen.EMULSION_G2, gab=lbgen.EMULSION_GAB,
              body=(1e-5, 0.0), rho_wall=lbgen.EMULSION_POOR, tau=(1.0, 1.0), psi0=1.0, rho0=lbgen.EMULSION_RHO0)
    return rho, kw


def channel_errors(oracle_ref):
    """The channel of channel_err_case: rho, u after `steps` steps and the wall stress averaged
    over the last `window` steps, each GPU storage mode against the oracle's (computed in the
    CPU baseline leg)."""
    import numpy as np
    from paper_1402_6019_amd import Sim
    lx, ly, steps, window = (CHANNEL_ERR[k] for k in ("lx", "ly", "steps", "window"))
    rho, kw = channel_err_case()
    ref, ref_w = oracle_ref
    out = {"workload": f"confined emulsion {lx}x{ly}, walls + wetting, g = 1e-5, fraction 0.85, seed 4",
           "steps": steps, "stress_window": window}
    for storage in ("f64", "f32", "bf16dev"):
        sim = Sim(lx, ly, rho, storage=storage, rho_ref=(float(rho[0].mean()), float(rho[1].mean())), **kw)
        sim.step(steps - window)
        sim.set_reduce_every(1)
        sim.wall_stress(reset=True)
        sim.step(window)
        w = np.array(sim.wall_stress(reset=True))
        r, u = sim.moments()
        e = rel_errors(r.cpu().numpy(), u.cpu().numpy(), ref)
        e["wall_stress"] = float(np.abs(w - ref_w).max() / np.abs(ref_w).max())
        out[storage] = e
        sim.close()
    return out


def cpu_baseline(rho, kw, budget_s=15.0):
    """The FP64 CPU oracle, as it stands, on the same lattice for a bounded number of steps; its
    fields at a few times, and the oracle's run of the small channel, are the references of the
    GPU errors.  Every use of the oracle in this script is in this leg."""
    import numpy as np
    import oracle
    from oracle import Oracle, Params
    P = Params(lx=LX, ly=LY, ns=2, walls=0, g1=kw["g1"], g2=kw["g2"], gab=kw["gab"], body=kw["body"],
               tau=kw["tau"], psi0=kw["psi0"], rho0=kw["rho0"])
    orc = Oracle(P, rho_init=rho)
    refs = {}
    t0 = time.perf_counter()
    orc.step(10)
    per = (time.perf_counter() - t0) / 10
    refs[10] = orc.fields()
    orc.step(90)
    refs[100] = orc.fields()
    n = max(2, int(budget_s / per))
    t0 = time.perf_counter()
    orc.step(n)
    dt = time.perf_counter() - t0
    refs[100 + n] = orc.fields()
    # the same binary on one thread, for a few steps of the same lattice
    threads = oracle.get_threads()
    oracle.set_threads(1)
    t1 = time.perf_counter()
    orc.step(3)
    dt1 = time.perf_counter() - t1
    oracle.set_threads(threads)
    # the small channel's reference
    crho, ckw = channel_err_case()
    cP = Params(lx=CHANNEL_ERR["lx"], ly=CHANNEL_ERR["ly"], ns=2, walls=1, g1=ckw["g1"], g2=ckw["g2"], gab=ckw["gab"],
                body=ckw["body"], rho_wall=ckw["rho_wall"], tau=ckw["tau"], psi0=ckw["psi0"], rho0=ckw["rho0"])
    corc = Oracle(cP, rho_init=crho)
    corc.step(CHANNEL_ERR["steps"] - CHANNEL_ERR["window"])
    recs = corc.step(CHANNEL_ERR["window"], record=True)
    chan_ref = (corc.fields(), np.array([recs[:, 4].mean(), recs[:, 5].mean()]))
    return {
        "value": LX * LY * n / dt / 1e6,
        "unit": "MLUPS",
        "cores": threads,
        "cpu_model": cpu_model(),
        "kind": "oracle",
        "sample": f"{n} steps (steps 100..{100 + n}) of the same 1024x1024 two-component lattice from the "
                  f"same initial state ({dt:.1f} s, FP64, OpenMP over rows)",
        "one_thread_mlups": LX * LY * 3 / dt1 / 1e6,
    }, refs, chan_ref


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo) and its logical CPU count."""
    name = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{name} ({os.cpu_count()} logical CPUs)"


def leg(name, fn, *args, **kwargs):
    """Run one benchmark leg, with a progress line on stderr before and after it."""
    print(f"[bench] {name} ...", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    r = fn(*args, **kwargs)
    print(f"[bench] {name} done in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    return r


def traffic_from_profile(kernel_hash, storage, tile):
    """HBM bytes per launch (FETCH_SIZE and WRITE_SIZE, each scaled by what the counter reads
    for a copy of known size) from the committed rocprofv3 counter summary, if it was taken
    on the current kernel source and at the launch shape timed here; otherwise None."""
    path = os.path.join(ROOT, "profiles", "step_kernel_traffic_emulsion1024.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_source_hash") != kernel_hash or storage not in d.get("storage", {}):
        return None
    rec = d["storage"][storage]
    if list(rec.get("tile", [])) != list(tile):
        return None
    return rec.get("hbm_bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline and error check")
    ap.add_argument("--tile", type=str, default=None, help="tx,sy launch shape")
    ap.add_argument("--core", action="store_true",
                    help="headline lattice and copy only (skip the channel, batched and adjoint legs)")
    ap.add_argument("--channel-only", action="store_true",
                    help="run only the 4096 x 512 channel leg (served by HBM) and print it")
    ap.add_argument("--three-d-only", action="store_true",
                    help="run only the 3-D leg (256^3 emulsion, FP32 and FP64) and print it")
    ap.add_argument("--couette-study", action="store_true",
                    help="run only the Couette-cell fluidity study (half a million steps at 1040^2) and print it")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); sharding over several GPUs is "
              f"described, not implemented", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.couette_study:
        print(json.dumps(couette_study()), flush=True)
        return
    if args.channel_only:
        print(json.dumps(channel_beyond_cache(args.steps)), flush=True)
        return
    if args.three_d_only:
        print(json.dumps(three_d(max(5, args.steps // 40))), flush=True)
        return
    tile = tuple(int(v) for v in args.tile.split(",")) if args.tile else None

    rho, info, kw = workload()
    nsite = LX * LY
    gpu_warmup(rho, kw)
    res = {}
    for storage in ("f64", "f32", "bf16dev"):
        ms, wall, tile_used = time_storage(storage, rho, kw, args.steps, args.warmup, tile)
        algo = 2 * 9 * 2 * BYTES_PER_VALUE[storage] * nsite
        res[storage] = {"ms_per_step": ms, "mlups": nsite / (ms * 1e-3) / 1e6, "gbs": algo / (ms * 1e-3) / 1e9,
                        "algo_bytes_per_launch": algo, "wall_s": wall, "tile": list(tile_used)}

    ms_sr, _, tile_sr = time_storage("bf16dev", rho, kw, args.steps, args.warmup, tile, rounding="stochastic")
    bf16_sr = {"mlups": nsite / (ms_sr * 1e-3) / 1e6, "ms_per_step": ms_sr, "tile": list(tile_sr),
               "note": "BF16 deviations with stochastic rounding of the stores (unbiased; see channel_50k_averages)"}

    khash = kernel_source_hash()
    head = res["f32"]
    copy = copy_reference(head["algo_bytes_per_launch"] // 2, min(args.steps, 500))
    roof = {"bound": "hbm", "achieved": head["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": head["gbs"] / HBM_PEAK_GBS,
            "traffic": traffic_from_profile(khash, "f32", head["tile"]),
            "kernel": "step_kernel<F32, 2 species, periodic>", "bytes_per_lu": 144,
            "copy_ceiling_gbs": copy["gbs"], "frac_of_copy": head["gbs"] / copy["gbs"],
            "stream_copy_gbs": max(copy["stream_copy_gbs"], copy["stream_copy_nt_gbs"]),
            "frac_of_stream_copy": head["gbs"] / max(copy["stream_copy_gbs"], copy["stream_copy_nt_gbs"]),
            "served_by": "infinity_cache",
            "note": "footprint 2 x 75.5 MB fits in the 256 MB Infinity Cache, so this rate is served by that "
                    "cache, not by HBM; hbm_served gives the same kernel on the 4096 x 512 channel, whose "
                    "302 MB footprint exceeds it"}
    beyond = None if args.core else leg("beyond_infinity_cache", channel_beyond_cache, max(50, args.steps // 4))
    if beyond is not None:
        ch = beyond["f32"]
        roof["hbm_served"] = {"workload": beyond["workload"], "achieved": ch["gbs"], "peak": HBM_PEAK_GBS,
                              "unit": "GB/s", "frac": ch["frac"], "mlups": ch["mlups"],
                              "footprint_mb": ch["footprint_mb"],
                              "kernel": ch["kernel"]}

    out = {
        # value: FP32 MLUPS; % of HBM peak in roofline.frac; FP64 (and BF16) beside it; the
        # errors against the FP64 oracle in error_vs_oracle
        "metric": "MLUPS + % HBM peak, 2-component D2Q9 two-belt step, FP32 vs FP64 at stated err",
        "value": head["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "emulsion 1024x1024 periodic, 2 species, volume fraction 0.8, seed 2",
                   "lx": LX, "ly": LY, "n_species": 2, "parallelism": "single GPU",
                   "mass_fraction": info["mass_fraction"]},
        "roofline": roof,
        "fp64": {"mlups": res["f64"]["mlups"], "ms_per_step": res["f64"]["ms_per_step"],
                 "kernel": ("step2_kernel<F64, 2 species, periodic>: two steps per launch, write-through stores"
                            if PAIRS_SEEN.get(("f64", (LX, LY))) else
                            "step_kernel<F64, 2 species, periodic>, streaming stores"),
                 "roofline": {"bound": "hbm", "achieved": res["f64"]["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": res["f64"]["gbs"] / HBM_PEAK_GBS, "bytes_per_lu": 288,
                              "steps_per_launch": 2 if PAIRS_SEEN.get(("f64", (LX, LY))) else 1,
                              "traffic": traffic_from_profile(khash, "f64", res["f64"]["tile"])}},
        "bf16dev": {"mlups": res["bf16dev"]["mlups"], "ms_per_step": res["bf16dev"]["ms_per_step"],
                    "roofline": {"bound": "hbm", "achieved": res["bf16dev"]["gbs"], "peak": HBM_PEAK_GBS,
                                 "unit": "GB/s", "frac": res["bf16dev"]["gbs"] / HBM_PEAK_GBS, "bytes_per_lu": 72,
                                 "traffic": traffic_from_profile(khash, "bf16dev", res["bf16dev"]["tile"])}},
        "bf16dev_stochastic": bf16_sr,
        "f32_graph_replay_median_of_5": headline_median(rho, kw, tile),
        "speedup_vs_fp64": {"f32": res["f64"]["ms_per_step"] / res["f32"]["ms_per_step"],
                            "bf16dev": res["f64"]["ms_per_step"] / res["bf16dev"]["ms_per_step"]},
        "tiles": {k: v["tile"] for k, v in res.items()},
        "copy_reference": copy,
        "beyond_infinity_cache": beyond,
        "long_run_1024_20k": None if args.core else leg("long_run_1024_20k", long_run_1024),
        "config1_single_component_64": None if args.core or args.no_cpu else leg("config1", single_component_64),
        "three_d": None if args.core else leg("three_d", three_d, max(20, args.steps // 40)),
        "channel_50k_averages": None if args.core else leg("channel_50k", channel_long_run),
        "batched_sweep": None if args.core else leg("batched_sweep", batched_sweep, max(100, args.steps // 10)),
        "couette_cell": None if args.core else leg("couette_cell", couette_cell, max(200, args.steps // 2)),
        "auxiliary_passes": None if args.core else leg("auxiliary_passes", auxiliary_passes, rho, kw),
        "film_sweep": None if args.core else leg("film_sweep", film_sweep),
        "adjoint": None if args.core else leg("adjoint", adjoint_channel, check_fd=not args.no_cpu),
        "kernel_source_hash": khash,
    }
    if not args.no_cpu:
        base, refs, chan_ref = leg("cpu_baseline", cpu_baseline, rho, kw)
        out["cpu_baseline"] = base
        out["error_vs_oracle"] = {"emulsion_1024_by_step": emulsion_errors(rho, kw, refs),
                                  "channel_256x128": channel_errors(chan_ref)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
