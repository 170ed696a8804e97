"""CPU-side checks of the C ABI library: it loads, exports every symbol that include/lb.h
declares, its default weights equal the oracle's independently derived isotropic sets, and
lb_init rejects invalid input before touching the device."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def B():
    from paper_1402_6019_amd import _binding
    return _binding


def header_functions():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not h.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(lb_[a-z_0-9]+)\s*\(", text, flags=re.M)
    return names


def test_library_exports_every_declared_symbol(B):
    lib = B.load()
    names = header_functions()
    assert "lb_init" in names and "lb_step" in names and "lb_moments" in names and "lb_wall_stress" in names
    for n in names:
        assert hasattr(lib, n), n
        assert n in B.SIGNATURES, f"binding misses {n}"


def test_default_weights_match_oracle_derivation(B):
    from oracle import weights as wt
    c = B.default_couplings()
    np.testing.assert_array_equal(list(c.w), wt.as_float_list(wt.weights_w()))
    np.testing.assert_array_equal(list(c.p), wt.as_float_list(wt.weights_p()))
    t = wt.weights_t()
    np.testing.assert_array_equal(list(c.t), [float(t[1]), float(t[2])])


def test_3d_default_weights_match_oracle_derivation(B):
    """The 3-D library's default weights equal the oracle's sets, derived from the 3-D isotropy
    conditions by exact rational elimination (w sixth order, p eighth order, t the D3Q19 set)."""
    from oracle import weights as wt
    c = B.Lb3Couplings()
    assert B.load().lb3_default_couplings(ctypes.byref(c)) == 0
    np.testing.assert_array_equal(list(c.w), wt.as_float_list3(wt.weights3_w()))
    np.testing.assert_array_equal(list(c.p), wt.as_float_list3(wt.weights3_p()))
    t = wt.weights3_t()
    np.testing.assert_array_equal(list(c.t), [float(t[1]), float(t[2])])


def test_3d_pop_bytes_and_host_validation(B):
    lib = B.load()
    for lx, ly, lz, ns, st, es in ((5, 5, 5, 1, 0, 8), (70, 21, 13, 2, 1, 4), (256, 256, 256, 2, 0, 8)):
        lat = B.Lb3Lattice(lx, ly, lz, ns, 0, st)
        pitch = (lx + 63) // 64 * 64
        assert lib.lb3_pop_bytes(ctypes.byref(lat)) == lz * ly * 19 * pitch * ns * es
    assert lib.lb3_pop_bytes(ctypes.byref(B.Lb3Lattice(5, 5, 4, 1, 0, 0))) == 0
    assert lib.lb3_pop_bytes(ctypes.byref(B.Lb3Lattice(8, 8, 8, 1, 0, 2))) == 0  # no BF16 in 3-D
    cpl = B.Lb3Couplings()
    lib.lb3_default_couplings(ctypes.byref(cpl))
    pp = B.LbPsiParams(1.0, 1.0, (ctypes.c_double * 2)(0.0, 0.0))
    rho = np.ones((1, 8, 8, 8))
    h = ctypes.c_void_p()
    bad_tau = (ctypes.c_double * 2)(0.5, 1.0)
    rc = lib.lb3_init(ctypes.byref(h), ctypes.byref(B.Lb3Lattice(8, 8, 8, 1, 0, 0)), ctypes.byref(cpl), bad_tau,
                      ctypes.byref(pp), rho.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.c_void_p(16),
                      ctypes.c_void_p(32), 1 << 40, None)
    assert rc == B.LB_EINVAL and b"tau" in lib.lb3_last_error(None)
    rho[0, 3, 3, 3] = -1.0
    rc = lib.lb3_init(ctypes.byref(h), ctypes.byref(B.Lb3Lattice(8, 8, 8, 1, 0, 0)), ctypes.byref(cpl),
                      (ctypes.c_double * 2)(1.0, 1.0), ctypes.byref(pp),
                      rho.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.c_void_p(16), ctypes.c_void_p(32),
                      1 << 40, None)
    assert rc == B.LB_EINVAL and b"rho_init" in lib.lb3_last_error(None)


@pytest.mark.parametrize("storage,es", [(0, 8), (1, 4), (2, 2)])
def test_pop_bytes(B, storage, es):
    for lx, ly, ns in ((5, 5, 1), (64, 7, 2), (1000, 33, 2)):
        lat = B.LbLattice(lx, ly, ns, 0, storage)
        pitch = (lx + 255) // 256 * 256
        assert B.pop_bytes(lat) == ns * 9 * ly * pitch * es
    assert B.pop_bytes(B.LbLattice(4, 10, 1, 0, storage)) == 0
    assert B.pop_bytes(B.LbLattice(10, 10, 3, 0, storage)) == 0


def _init(B, lat, tau=(1.0, 1.0), rho=None, nbytes=None, psi=(1.0, 1.0), u_wall=(0.0, 0.0)):
    lib = B.load()
    cpl = B.default_couplings()
    cpl.wall_velocity[:] = u_wall
    t = (ctypes.c_double * 2)(*tau)
    pp = B.LbPsiParams(psi[0], psi[1], (ctypes.c_double * 2)(0.0, 0.0))
    if rho is None:
        rho = np.ones((max(lat.n_species, 1), max(lat.ly, 1), max(lat.lx, 1)))
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    h = ctypes.c_void_p()
    rc = lib.lb_init(ctypes.byref(h), ctypes.byref(lat), ctypes.byref(cpl), t, ctypes.byref(pp),
                     rho.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.c_void_p(16), ctypes.c_void_p(32),
                     nbytes if nbytes is not None else (1 << 40), None)
    return rc, lib.lb_last_error(None).decode()


def test_init_rejects_invalid_arguments_on_host(B):
    ok = B.LbLattice(16, 16, 1, 0, 0)
    assert _init(B, ok, tau=(0.5, 1.0))[0] == B.LB_EINVAL
    assert "tau" in _init(B, ok, tau=(0.5, 1.0))[1]
    assert _init(B, B.LbLattice(4, 16, 1, 0, 0))[0] == B.LB_EINVAL
    assert _init(B, B.LbLattice(16, 16, 3, 0, 0))[0] == B.LB_EINVAL
    assert _init(B, B.LbLattice(16, 16, 1, 2, 0))[0] == B.LB_EINVAL
    assert _init(B, B.LbLattice(16, 16, 1, 0, 7))[0] == B.LB_EINVAL
    assert _init(B, B.LbLattice(16, 70000, 1, 0, 0))[0] == B.LB_EINVAL
    bad = np.ones((1, 16, 16))
    bad[0, 3, 4] = 0.0
    assert _init(B, ok, rho=bad)[0] == B.LB_EINVAL
    bad[0, 3, 4] = np.nan
    assert _init(B, ok, rho=bad)[0] == B.LB_EINVAL
    assert _init(B, ok, psi=(1.0, 0.0))[0] == B.LB_EINVAL
    assert _init(B, ok, nbytes=100)[0] == B.LB_ENOMEM
    # sliding walls need walls
    rc, msg = _init(B, ok, u_wall=(0.0, 0.01))
    assert rc == B.LB_EINVAL and "wall_velocity" in msg
    assert _init(B, B.LbLattice(16, 16, 1, 1, 0), u_wall=(np.inf, 0.0))[0] == B.LB_EINVAL


def test_product_package_does_not_reach_the_oracle():
    """The product package imports nothing from oracle/ (and fails loudly without its library)."""
    pkg = os.path.join(ROOT, "paper_1402_6019_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".hpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text and "lb_oracle" not in text, f


def _batch_init(B, lats, tau=None, rho=None, nbytes=1 << 40):
    lib = B.load()
    n = len(lats)
    L = (B.LbLattice * n)(*lats)
    C = (B.LbCouplings * n)(*[B.default_couplings() for _ in range(n)])
    P = (B.LbPsiParams * n)(*[B.LbPsiParams(1.0, 1.0, (ctypes.c_double * 2)(0.0, 0.0)) for _ in range(n)])
    T = (ctypes.c_double * (2 * n))(*(tau or [1.0] * (2 * n)))
    arrs = rho or [np.ones((max(l.n_species, 1), max(l.ly, 1), max(l.lx, 1))) for l in lats]
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in arrs]
    ptrs = (ctypes.POINTER(ctypes.c_double) * n)(*[a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for a in arrs])
    h = ctypes.c_void_p()
    rc = lib.lb_batch_init(ctypes.byref(h), n, L, C, T, P, ptrs, ctypes.c_void_p(16), ctypes.c_void_p(32), nbytes, None)
    return rc, lib.lb_batch_last_error(None).decode()


def test_batch_init_rejects_invalid_arguments_on_host(B):
    a = B.LbLattice(16, 16, 2, 1, 1)
    assert _batch_init(B, [a, B.LbLattice(20, 12, 2, 0, 1)])[0] == B.LB_EINVAL  # walls differ
    assert "share" in _batch_init(B, [a, B.LbLattice(20, 12, 2, 1, 0)])[1]      # storage differs
    assert _batch_init(B, [a, B.LbLattice(20, 12, 1, 1, 1)])[0] == B.LB_EINVAL  # species differ
    rc, msg = _batch_init(B, [a, B.LbLattice(4, 12, 2, 1, 1)])
    assert rc == B.LB_EINVAL and "instance 1" in msg
    assert _batch_init(B, [a, a], tau=[1.0, 1.0, 0.4, 1.0])[0] == B.LB_EINVAL
    bad = np.ones((2, 16, 16))
    bad[1, 2, 3] = -1.0
    assert _batch_init(B, [a, a], rho=[np.ones((2, 16, 16)), bad])[0] == B.LB_EINVAL
    assert _batch_init(B, [a, a], nbytes=1000)[0] == B.LB_ENOMEM


def test_batch_pop_bytes_is_the_aligned_sum(B):
    lib = B.load()
    lats = [B.LbLattice(300, 17, 2, 1, 1), B.LbLattice(70, 40, 2, 1, 1), B.LbLattice(64, 64, 2, 1, 1)]
    arr = (B.LbLattice * 3)(*lats)
    total = sum((B.pop_bytes(l) + 255) // 256 * 256 for l in lats)
    assert lib.lb_batch_pop_bytes(3, arr) == total
    assert lib.lb_batch_pop_bytes(0, arr) == 0


def test_null_contexts_fail_cleanly(B):
    lib = B.load()
    assert lib.lb_step(None, 1) == B.LB_EINVAL
    assert lib.lb_batch_step(None, 1) == B.LB_EINVAL
    assert lib.lb_set_couplings(None, None) == B.LB_EINVAL
    assert lib.lb_adjoint_workspace_bytes(None, 10, 0, 0) == 0
    assert lib.lb_time(None) == -1
    assert lib.lb_batch_time(None) == -1
    assert lib.lb_two_step_active(None) == -1
    assert lib.lb_set_two_step(None, 1, 0) == B.LB_EINVAL


def test_cooperative_length_fit_recovers_the_prediction(B):
    """The host fit of eq. (predict): exact profiles give back (zeta, f_b, f_w); on noisy
    data it agrees with scipy's general least squares started from the truth."""
    from scipy.optimize import curve_fit
    from paper_1402_6019_amd import fit_cooperative_length
    H = 120.0
    z = np.arange(1.0, H)

    def model(z, zeta, fb, fw):
        return fb + (fw - fb) * np.cosh((z - H / 2) / zeta) / np.cosh(H / (2 * zeta))

    for zeta, fb, fw in ((18.0, 0.05, 0.9), (68.0, 0.3, 1.1), (4.0, 1e-3, 0.2)):
        r = fit_cooperative_length(z, model(z, zeta, fb, fw), H)
        assert r["zeta"] == pytest.approx(zeta, rel=1e-7)
        assert r["f_b"] == pytest.approx(fb, rel=1e-6, abs=1e-9)
        assert r["f_w"] == pytest.approx(fw, rel=1e-6)
        assert r["rms"] < 1e-9
    rng = np.random.default_rng(3)
    f = model(z, 25.0, 0.1, 0.8) + 0.01 * rng.standard_normal(z.size)
    r = fit_cooperative_length(z, f, H)
    (zs, fbs, fws), _ = curve_fit(model, z, f, p0=(25.0, 0.1, 0.8))
    assert r["zeta"] == pytest.approx(zs, rel=1e-5)
    assert r["f_b"] == pytest.approx(fbs, rel=1e-5)
    assert r["f_w"] == pytest.approx(fws, rel=1e-5)
    lib = B.load()
    dp = ctypes.POINTER(ctypes.c_double)
    out = (ctypes.c_double * 4)()
    zz = np.array([0.0, 1.0, 200.0])  # outside [0, H]
    assert lib.lb_fit_cooperative_length(zz.ctypes.data_as(dp), zz.ctypes.data_as(dp), 3, H, 1.0, 10.0, out) == B.LB_EINVAL
    assert lib.lb_fit_cooperative_length(z.ctypes.data_as(dp), f.ctypes.data_as(dp), 2, H, 1.0, 10.0, out) == B.LB_EINVAL


def test_disjoining_pressure_from_film_tension():
    """Eq. (doppiasigma) inverted on the host: for Pi(h) = A exp(-h / l), the film tension is
    gamma_f(h) = 2 gamma + A (l + h) exp(-h / l) (from (doppiasigma) with Pi(inf) = 0), and the
    routine recovers Pi from gamma_f sampled on a grid, in any order; a dropped 1/h weight or
    a sign error fails."""
    from paper_1402_6019_amd.film import disjoining_from_tension, film_thickness
    A, lam, two_gamma = 1e-3, 2.0, 0.0175
    h = np.linspace(2.0, 60.0, 581)
    g = two_gamma + A * (lam + h) * np.exp(-h / lam)
    exact = A * (np.exp(-h / lam) - np.exp(-h[-1] / lam))  # Pi taken 0 at the thickest film
    pi = disjoining_from_tension(h, g)
    assert np.abs(pi - exact).max() < 2e-3 * A
    perm = np.random.default_rng(0).permutation(h.size)
    assert np.array_equal(disjoining_from_tension(h[perm], g[perm]), pi[perm])
    # a constant tension (two independent interfaces) carries no disjoining pressure
    assert np.all(disjoining_from_tension(h, np.full_like(h, two_gamma)) == 0.0)
    with pytest.raises(ValueError):
        disjoining_from_tension([3.0, 3.0], [1.0, 2.0])
    # thickness between the two crossings of a level, linearly interpolated
    line = np.array([0.2, 0.2, 0.6, 1.4, 1.4, 1.0, 0.2, 0.2])
    assert film_thickness(line, 3, 0.8) == pytest.approx((5 + 0.2 / 0.8) - (2 + 0.2 / 0.8))
    assert film_thickness(line, 0, 0.8) == 0.0
