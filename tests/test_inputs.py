"""The seeded input generators (CPU): the emulsion packing hits its volume fraction, is
reproducible from its seed, keeps the wall rows in the continuous phase and separates
droplets by films; the film geometries are symmetric."""

import numpy as np
import pytest

import lbgen


@pytest.mark.parametrize("walls", [False, True])
def test_emulsion_fraction_seed_and_phases(walls):
    rho, info = lbgen.emulsion(256, 192, fraction=0.8, seed=11, walls=walls)
    rich, poor = np.asarray(lbgen.EMULSION_RICH, dtype=float), np.asarray(lbgen.EMULSION_POOR, dtype=float)
    a_rich = rho[0] == rich[0]
    assert np.all(a_rich == (rho[1] == rich[1]))
    assert np.all(a_rich | (rho[0] == poor[0]))
    assert abs(info["volume_fraction"] - 0.8) <= 2.0 / rho[0].size
    assert info["volume_fraction"] == pytest.approx(a_rich.mean())
    again, _ = lbgen.emulsion(256, 192, fraction=0.8, seed=11, walls=walls)
    other, _ = lbgen.emulsion(256, 192, fraction=0.8, seed=12, walls=walls)
    assert np.array_equal(rho, again) and not np.array_equal(rho, other)
    if walls:
        assert not a_rich[0].any() and not a_rich[-1].any()
    # droplets are separated by films: the A-rich set has several connected parts
    from scipy.ndimage import label
    _, n = label(a_rich, structure=np.ones((3, 3)))
    assert n >= 0.5 * info["n_drops"]


def test_emulsion_saturates_at_the_densest_packing():
    """Small droplets with films of two sites cannot cover 80%: the generator returns its
    densest packing and says so."""
    rho, info = lbgen.emulsion(160, 96, fraction=0.8, seed=11, rmin=5, rmax=12)
    assert info["volume_fraction"] < 0.8
    assert info["volume_fraction"] == pytest.approx((rho[0] == rho[0].max()).mean())


def test_film_geometries_are_mirror_symmetric():
    b = lbgen.facing_bubbles(100, 80, 16, 6)
    np.testing.assert_allclose(b, b[:, ::-1], atol=1e-12)
    np.testing.assert_allclose(b, b[::-1, :], atol=1e-12)
    assert b[40, 50] > 1.3 and b[40, 40] < 0.3  # liquid film at the centre, gas in a bubble
    f = lbgen.flat_film(64, 5, 8.0)  # centred at x = 32
    np.testing.assert_allclose(f[:, 1:], f[:, 1:][:, ::-1], atol=1e-12)
    assert f[0, 32] > 1.3 and f[0, 0] < 0.3
    assert np.ptp(f, axis=0).max() == 0.0
