"""Shared test cases: one description feeds both the HIP path (through the C ABI binding)
and the CPU oracle, with the same seeded inputs from lbgen."""

import numpy as np

import lbgen


def film_case(lx=64, ly=64, seed=1, storage="f64", tau=1.0):
    """Single component, film couplings, noise around rho = 1 (periodic)."""
    rho = lbgen.uniform_noise(lx, ly, 1.0, 0.01, seed=seed)[None]
    return dict(lx=lx, ly=ly, ns=1, walls=0, g1=(lbgen.FILM_G1, 0.0), g2=(lbgen.FILM_G2, 0.0), gab=0.0,
                body=(0.0, 0.0), rho_wall=(0.0, 0.0), tau=(tau, tau), psi0=1.0, rho0=1.0, rho=rho,
                storage=storage, rho_ref=(1.0, 0.0))


def emulsion_case(lx, ly, walls=False, fraction=0.8, seed=2, storage="f64", g=1e-6, rmin=8.0, rmax=24.0,
                  tau=1.0):
    rho, _ = lbgen.emulsion(lx, ly, fraction=fraction, seed=seed, walls=walls, rmin=rmin, rmax=rmax)
    return dict(lx=lx, ly=ly, ns=2, walls=1 if walls else 0, g1=lbgen.EMULSION_G1, g2=lbgen.EMULSION_G2,
                gab=lbgen.EMULSION_GAB, body=(g if walls else 0.0, 0.0),
                rho_wall=lbgen.EMULSION_POOR if walls else (0.0, 0.0), tau=(tau, tau), psi0=1.0,
                rho0=lbgen.EMULSION_RHO0, rho=rho, storage=storage,
                rho_ref=(float(rho[0].mean()), float(rho[1].mean())))


def oracle_params(c):
    from oracle import Params
    return Params(lx=c["lx"], ly=c["ly"], ns=c["ns"], walls=c["walls"], g1=c["g1"], g2=c["g2"], gab=c["gab"],
                  body=c["body"], rho_wall=c["rho_wall"], tau=c["tau"], psi0=c["psi0"], rho0=c["rho0"],
                  u_wall=c.get("u_wall", (0.0, 0.0)), cross_psi=1 if c.get("cross_psi") else 0)


def make_oracle(c):
    from oracle import Oracle
    return Oracle(oracle_params(c), rho_init=c["rho"])


def make_sim(c, tile=None, storage=None):
    from paper_1402_6019_amd import Sim
    return Sim(c["lx"], c["ly"], c["rho"], n_species=c["ns"], walls=bool(c["walls"]),
               storage=storage or c["storage"], g1=c["g1"], g2=c["g2"], gab=c["gab"], body=c["body"],
               rho_wall=c["rho_wall"], tau=c["tau"], psi0=c["psi0"], rho0=c["rho0"], rho_ref=c["rho_ref"],
               tile=tile, u_wall=c.get("u_wall", (0.0, 0.0)), cross_psi=bool(c.get("cross_psi", False)))


def counterflow(c, seed, u_amp=0.04):
    """Canonical FP64 pre-collision populations [ns][9][ly][lx] of the case's densities with the
    species drifting against each other: W_l rho_s (1 + 3 c_l . u_s), u_B = -u_A, u_A random per
    site with amplitude u_amp (a seeded input; both sides start from it)."""
    cx = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])[:, None, None]
    cy = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])[:, None, None]
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)[:, None, None]
    rng = np.random.default_rng(seed)
    u = u_amp * rng.uniform(-1.0, 1.0, (2, c["ly"], c["lx"]))
    rho = c["rho"]
    f = np.empty((c["ns"], 9, c["ly"], c["lx"]))
    for s in range(c["ns"]):
        sign = 1.0 if s == 0 else -1.0
        f[s] = w * rho[s] * (1.0 + 3.0 * sign * (cx * u[0] + cy * u[1]))
    return f


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
