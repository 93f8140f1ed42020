"""Pins of the oracle host map against what the paper prints and what the
mathematics fixes.  CPU only."""
import numpy as np
import pytest
from scipy import integrate, optimize

from oracle import hostmap as hm

TRS = [0.9, 0.8, 0.7, 0.6, 0.5]
# Analytical proportionality constants printed in the supplement (Sec. V):
# W / K_INT and sigma / K_INT at K_EOS = 1, a = 1, b = 4, R = 1.
PRINTED_CW = [6.3711, 4.3574, 3.4423, 2.8875, 2.5052]
PRINTED_CSIGMA = [0.003146, 0.009081, 0.01710, 0.02716, 0.03954]
# One unit of the last printed digit of each value.
CW_DIGIT = 1e-4
CSIGMA_DIGIT = [1e-6, 1e-6, 1e-5, 1e-5, 1e-5]


def cstep(fn, x, h=1e-30):
    """Exact first derivative by the complex-step method."""
    return np.imag(fn(x + 1j * h)) / h


def test_critical_point_matches_printed_constants():
    """The CS EOS with a, b from the printed constants has its critical point
    (dp/drho = d2p/drho2 = 0) at the T_c those constants imply."""
    a, b, R = 1.0, 4.0, 1.0

    def conditions(z):
        rho, T = z
        d1 = lambda r: cstep(lambda q: hm.cs_pressure(q, R * T, a, b), r)
        d2 = (d1(rho + 1e-6) - d1(rho - 1e-6)) / 2e-6
        return [d1(rho), d2]

    rho_c, t_c = optimize.fsolve(conditions, [0.13, 0.094], xtol=1e-14)
    assert t_c == pytest.approx(hm.critical_temperature(a, b, R), rel=1e-5)
    assert hm.cs_pressure(rho_c, R * t_c, a, b) == pytest.approx(hm.critical_pressure(a, b, R), rel=1e-4)
    assert t_c == pytest.approx(0.0943287, rel=2e-6)


def test_free_energy_derivatives():
    """p = rho psi' - psi (main Eq. 19), mu = psi', and the closed-form slopes."""
    rt = 0.7 * hm.critical_temperature(1.0, 4.0, 1.0)
    rho = np.linspace(0.002, 0.6, 57)
    psi = lambda r: hm.cs_free_energy(r, rt, 1.0, 4.0)
    mu = hm.cs_chemical_potential(rho, rt, 1.0, 4.0)
    np.testing.assert_allclose(cstep(psi, rho), mu, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(rho * mu - psi(rho), hm.cs_pressure(rho, rt, 1.0, 4.0), rtol=1e-11, atol=1e-15)
    np.testing.assert_allclose(cstep(lambda r: hm.cs_pressure(r, rt, 1.0, 4.0), rho),
                               hm.cs_pressure_slope(rho, rt, 1.0, 4.0), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(cstep(lambda r: hm.cs_pressure(r, rt, 1.0, 4.0) + r * r, rho),
                               hm.cs_repulsive_slope(rho, rt, 4.0), rtol=1e-12)


@pytest.mark.parametrize("tr", TRS)
def test_maxwell_equal_area(tr):
    """Equal pressure, equal chemical potential, and the equal-area rule in the
    specific-volume plane, int (p - p0) d(1/rho) = 0, by independent quadrature."""
    rt = tr * hm.critical_temperature(1.0, 4.0, 1.0)
    rg, rl, p0 = hm.maxwell(tr)
    assert hm.cs_pressure(rg, rt, 1, 4) == pytest.approx(p0, rel=1e-12)
    assert hm.cs_pressure(rl, rt, 1, 4) == pytest.approx(p0, rel=1e-12)
    assert hm.cs_chemical_potential(rg, rt, 1, 4) == pytest.approx(hm.cs_chemical_potential(rl, rt, 1, 4), rel=1e-12)
    area, _ = integrate.quad(lambda v: hm.cs_pressure(1.0 / v, rt, 1, 4) - p0, 1.0 / rl, 1.0 / rg,
                             limit=500, epsabs=1e-15, epsrel=1e-12)
    assert abs(area) < 1e-9 * p0 * (1.0 / rg - 1.0 / rl)
    assert 0 < rg < rl < 1.0


@pytest.mark.parametrize("i,tr", list(enumerate(TRS)))
def test_interface_constants_printed(i, tr):
    """C_sigma rounds to the printed analytical value (within half a unit of
    its last digit); C_W is within one unit of its last printed digit."""
    c_sigma, c_w = hm.interface_constants(tr)
    assert abs(c_w - PRINTED_CW[i]) <= 1.0 * CW_DIGIT
    assert abs(c_sigma - PRINTED_CSIGMA[i]) <= 0.5 * CSIGMA_DIGIT[i]


def test_k_int_printed():
    """W = 10 at T_r = 0.8 is K_INT = 2.2949 (supplement Sec. V)."""
    co = hm.derive(hm.Params(tr=0.8, width=10.0))
    assert co.k_int == pytest.approx(2.2949, abs=6e-5)


def test_sigma_keos_slopes():
    """sigma / K_EOS slopes of supplement Fig. 4 (W = 20, 30 at T_r = 0.5):
    the analytical slope C_sigma K_INT = C_sigma W / C_W lies within 1.5% of
    the simulated slopes the paper prints."""
    printed = [0.009879, 0.04174, 0.09959, 0.1887, 0.4758]
    for tr, w, s in zip(TRS, [20, 20, 20, 20, 30], printed):
        c_sigma, c_w = hm.interface_constants(tr)
        assert c_sigma * w / c_w == pytest.approx(s, rel=0.015)


def test_flat_profile_thickness_consistency():
    """The thickness integral equals the distance between the 5% and 95%
    levels of the planar profile obtained by integrating
    d rho / dz = sqrt(2 dOmega / kappa) as an ODE."""
    tr = 0.8
    rt = tr * hm.critical_temperature(1, 4, 1)
    rg, rl, p0 = hm.maxwell(tr)
    mu0 = hm.cs_chemical_potential(rg, rt, 1, 4)
    kappa = 0.5
    dom = lambda r: hm.cs_free_energy(r, rt, 1, 4) - mu0 * r + p0
    mid = 0.5 * (rg + rl)
    sol = integrate.solve_ivp(lambda z, r: [np.sqrt(max(2 * dom(r[0]) / kappa, 0.0))],
                              [0, 20], [mid], rtol=1e-11, atol=1e-14, dense_output=True)
    solb = integrate.solve_ivp(lambda z, r: [-np.sqrt(max(2 * dom(r[0]) / kappa, 0.0))],
                               [0, 20], [mid], rtol=1e-11, atol=1e-14, dense_output=True)
    r95 = 0.05 * rg + 0.95 * rl
    r5 = 0.95 * rg + 0.05 * rl
    z95 = optimize.brentq(lambda z: sol.sol(z)[0] - r95, 0, 20)
    z5 = optimize.brentq(lambda z: solb.sol(z)[0] - r5, 0, 20)
    _, c_w = hm.interface_constants(tr)
    assert z95 + z5 == pytest.approx(c_w, rel=1e-6)


@pytest.mark.parametrize("varpi", [1 / 6, 0.1, 0.25, 0.45, 0.7])
def test_coefficient_constraints(varpi):
    """alpha2, beta2, k, h, b satisfy the three constraint systems of the
    supplement (Eqs. 24, 27, 30) with alpha1 = -1, beta1 = 1."""
    a1, b1 = -1.0, 1.0
    a2, b2, k, h, b = hm.model_coefficients(varpi)
    assert 2 * a1 + k * a2 + k == pytest.approx(-2 * varpi, abs=1e-14)
    assert h * ((a2 - 4) * b1 - (a1 + 2) * b2) / (3 * b1) == pytest.approx(-2 * varpi, abs=1e-13)
    assert (h * (3 * b1 + b2) - 6 * b1 * (1 - k)) / b1 == pytest.approx(0.0, abs=1e-13)
    assert 2 * b1 + k * b2 == pytest.approx(0.0, abs=1e-14)
    assert b * ((a2 - 4) * b1 - (a1 + 2) * b2) / b1 == pytest.approx(-1.0, abs=1e-13)
    assert ((6 * b - 2) * b1 + 2 * b * b2) / b1 == pytest.approx(0.0, abs=1e-13)
    assert ((3 * b - 1) * b1 + b * b2) / b1 == pytest.approx(0.0, abs=1e-13)


def test_coefficients_paper_setting():
    """varpi = 1/6 (supplement Sec. V): alpha2 = 1, beta2 = -12/5, k = 5/6,
    h = b = 5/3; varpi = 1/3 makes h and b singular (main text)."""
    a2, b2, k, h, b = hm.model_coefficients(1 / 6)
    assert (a2, b2, k, h, b) == pytest.approx((1.0, -2.4, 5 / 6, 5 / 3, 5 / 3), rel=1e-14)
    with pytest.raises(ZeroDivisionError):
        hm.model_coefficients(1 / 3)
    with pytest.raises(ZeroDivisionError):
        hm.model_coefficients(1.0)


@pytest.mark.parametrize("s_p", [0.6, 1.0, 1.5, 1.9])
def test_relaxation_constraint(s_p):
    """tau_p tau_q = (k + 1) tau_e tau_q = 1/12 (main Eq. 16)."""
    varpi = 1 / 6
    s_q, s_e = hm.relaxation_rates(s_p, varpi)
    tau = lambda s: 1 / s - 0.5
    k = 1 - varpi
    assert tau(s_p) * tau(s_q) == pytest.approx(1 / 12, rel=1e-13)
    assert (k + 1) * tau(s_e) * tau(s_q) == pytest.approx(1 / 12, rel=1e-13)
    if s_p == 1.0:
        assert s_q == pytest.approx(1.5, rel=1e-14)
        assert s_e == pytest.approx(22 / 17, rel=1e-14)


def test_sigma_paper_makes_lattice_speed_one():
    """At sigma_paper the sound-speed rule (main Eq. 22) gives c = sqrt(3) c_s = 1:
    3 K_INT^2 K_EOS RT (rho phi)'(rho_l) = 1, and K_EOS drops out of G'^2."""
    for tr in (0.8, 0.7, 0.6):
        co = hm.derive(hm.Params(tr=tr, width=10.0))
        c2 = 3 * co.k_int ** 2 * co.k_eos * hm.cs_repulsive_slope(co.rho_l, co.RT, co.b)
        assert c2 == pytest.approx(1.0, rel=1e-12)
        assert co.G2 == pytest.approx(2 * co.a / (3 * hm.cs_repulsive_slope(co.rho_l, co.RT, co.b)), rel=1e-12)


def test_sigma_width_scaling():
    """sigma = C_sigma K_INT K_EOS and W = C_W K_INT (main Eq. 23): the map
    inverts exactly for any prescribed pair."""
    for sigma, width in [(1e-3, 8.0), (5e-3, 15.0), (2e-2, 30.0)]:
        co = hm.derive(hm.Params(tr=0.7, width=width, sigma=sigma))
        assert co.c_sigma * co.k_int * co.k_eos == pytest.approx(sigma, rel=1e-14)
        assert co.c_w * co.k_int == pytest.approx(width, rel=1e-14)
        assert co.G2 == pytest.approx(2 * co.k_int ** 2 * co.k_eos * co.a, rel=1e-14)
