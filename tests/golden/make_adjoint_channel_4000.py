"""Writes adjoint_channel_512x256_T4000.json: the oracle's complex-step gradient of the
channel loss over the full horizon of the adjoint benchmark, from the oracle alone.

Workload: two-component confined emulsion, 512 x 256, walls with the wetting ghost densities,
G1 = -9.0 and G2 = 8.1 for both species, G_AB = 0.587, g = 1e-6, rho0 = 0.83, volume fraction
0.8 (seed 5); 2000 FP64 steps of pre-relaxation (not differentiated), then T = 4000 steps of
L = <(W_bot + W_top) / 2> + <Q> (section "Numerical simulations of confined pressure-driven
flows": wall stress and flow rate).  Gradient with respect to (G1, G2, G_AB, g_x) by the complex
step (h = 1e-30) through the oracle's step, which is analytic in the couplings.

Run: python tests/golden/make_adjoint_channel_4000.py  (about half an hour on 8 cores)."""

import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import lbgen  # noqa: E402
import oracle  # noqa: E402
from oracle import Oracle, Params, cs_grad  # noqa: E402

LX, LY, PRERELAX, T = 512, 256, 2000, 4000
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint_channel_512x256_T4000.json")


def params():
    return Params(lx=LX, ly=LY, ns=2, walls=1, g1=(-9.0, -9.0), g2=(8.1, 8.1), gab=lbgen.EMULSION_GAB,
                  body=(1e-6, 0.0), rho_wall=lbgen.EMULSION_POOR, tau=(1.0, 1.0), psi0=1.0,
                  rho0=lbgen.EMULSION_RHO0)


def prerelaxed_state():
    """The oracle's state after the pre-relaxation (deterministic for any thread count)."""
    rho, _ = lbgen.emulsion(LX, LY, fraction=0.8, seed=5, walls=True)
    o = Oracle(params(), rho_init=rho)
    o.step(PRERELAX)
    return o.get_f()


def state_digest(f):
    return hashlib.sha256(np.ascontiguousarray(f, dtype=np.float64).tobytes()).hexdigest()[:16]


def main():
    oracle.set_threads(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
    t0 = time.time()
    f0 = prerelaxed_state()
    out = {"workload": __doc__.split("\n\n")[1].replace("\n", " "), "lx": LX, "ly": LY, "prerelax": PRERELAX,
           "T": T, "loss_weights": [1.0, 1.0], "h": 1e-30, "prerelaxed_state_sha256_16": state_digest(f0),
           "prerelaxed_mass": [float(f0[0].sum()), float(f0[1].sum())], "params": ["G1", "G2", "G_AB", "g_x"]}
    grads, losses = [], []
    for k in range(4):
        loss, d = cs_grad(params(), f0, T, (1.0, 1.0), k, h=1e-30)
        grads.append(d)
        losses.append(loss)
        print(f"param {k}: dL = {d:.17g} (loss {loss:.17g}), {time.time() - t0:.0f} s", flush=True)
    out["loss"] = losses[0]
    out["grad"] = grads
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
