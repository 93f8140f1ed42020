"""Pins of the oracle read-outs (oracle/measure.py) on fields whose answer is
known in closed form.  CPU only."""
import math

import numpy as np
import pytest

from oracle import hostmap as hm
from oracle import measure


def tanh_slab(n, lo, hi, c1, delta):
    """Periodic profile: lo outside, hi between c1 and c1 + n/2, tanh layers
    of half-width delta (both layers far from the domain edges)."""
    y = np.arange(n, dtype=np.float64)
    s = np.tanh((y - c1) / delta) - np.tanh((y - c1 - n / 2) / delta) - 1.0
    return 0.5 * (lo + hi) + 0.5 * (hi - lo) * s


def test_interface_width_of_tanh_layer():
    """5%-95% thickness of tanh((y - y0)/delta): the levels sit at
    tanh = -0.9 and +0.9, so W = 2 delta atanh(0.9)."""
    delta = 12.0
    prof = tanh_slab(512, 0.1, 0.9, 128.3, delta)
    exact = 2 * delta * math.atanh(0.9)
    assert measure.interface_width(prof, 0.1, 0.9) == pytest.approx(exact, rel=2e-3)


def test_level_crossings_of_a_sawtooth():
    """A periodic sawtooth crosses a level on its ramp and on the wrap from
    its last node back to the first, at the interpolated positions; a node
    exactly on the level counts once."""
    p = np.arange(10.0)
    np.testing.assert_allclose(measure.level_crossings(p, 3.25), [3.25, 9 + 5.75 / 9])
    np.testing.assert_allclose(measure.level_crossings(p, 3.0), [3.0, 9 + 6 / 9])


@pytest.mark.parametrize("R", [40.0, 40.3])
def test_droplet_radius_of_a_tanh_disc(R):
    """The mid-level contour of rho_g + (rho_l - rho_g)(1 - tanh((r - R)/d))/2
    is the circle r = R (R = 40 puts a node exactly on the level)."""
    n, d = 256, 3.0
    y, x = np.mgrid[0:n, 0:n]
    r = np.hypot(x - n // 2, y - n // 2)
    rho = 0.1 + 0.8 * 0.5 * (1 - np.tanh((r - R) / d))
    assert measure.droplet_radius(rho, (n // 2, n // 2), 0.1, 0.9) == pytest.approx(R, abs=0.02)


def test_laplace_sigma_is_pressure_jump_times_radius():
    """laplace_sigma returns (p_EOS(centre) - p_EOS(far corner)) R with the CS
    pressure of the run's coefficients."""
    co = hm.derive(hm.Params(tr=0.7, width=10.0))
    n, R, d = 200, 30.0, 2.0
    y, x = np.mgrid[0:n, 0:n]
    r = np.hypot(x - n // 2, y - n // 2)
    lo, hi = co.rho_g * 1.01, co.rho_l * 1.002
    rho = lo + (hi - lo) * 0.5 * (1 - np.tanh((r - R) / d))
    sigma, radius, dp = measure.laplace_sigma(rho, (n // 2, n // 2), co)

    def p(v):  # CS pressure of main Eq. 20 with K' = K_EOS
        w = co.b * v / 4
        return co.Kp * (v * co.RT * (1 + w + w * w - w ** 3) / (1 - w) ** 3 - co.a * v * v)

    exact_dp = p(rho[n // 2, n // 2]) - p(rho[0, 0])
    assert dp == pytest.approx(exact_dp, rel=1e-12)
    assert radius == pytest.approx(R, abs=0.02)
    assert sigma == pytest.approx(exact_dp * radius, rel=1e-12)


@pytest.mark.parametrize("wavelength", [16, 32, 64])
def test_domain_length_of_a_single_mode(wavelength):
    """One Fourier mode of wavelength lambda has L = 2 pi / |k| = lambda."""
    n = 128
    x = np.arange(n)[None, :] + 0 * np.arange(n)[:, None]
    rho = 0.3 + 0.05 * np.cos(2 * np.pi * x / wavelength)
    assert measure.domain_length(rho) == pytest.approx(wavelength, rel=1e-12)


def test_totals_of_a_single_population():
    """Mass and momentum of a state holding only population 5 (+x+y)."""
    f = np.zeros((9, 4, 6))
    f[5] = 0.25
    mass, jx, jy = measure.totals(f)
    assert (mass, jx, jy) == pytest.approx((6.0, 6.0, 6.0))
