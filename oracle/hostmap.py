"""Oracle host map: equation of state, coexistence, interface constants and
the lattice coefficients of the self-tuning-EOS model.  FP64, scipy-based.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Units: lattice units with dx = dt = 1 and c = 1, so c_s^2 = 1/3.  The
surface tension sigma and the thickness W are prescribed in these units;
K_INT = W / C_W and K_EOS = sigma / (C_sigma K_INT) follow from the
proportionalities of main Eq. 23, whose constants C_W, C_sigma are the
flat-interface thickness and tension at K_EOS = K_INT = 1.  The paper's own
sound-speed rule (main Eq. 22) is one particular sigma, returned by
``sigma_paper``; at that sigma this map reproduces the paper's scheme.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy import integrate, optimize

# Carnahan-Starling constants as printed with main Eq. 20:
#   a = 0.496388 R^2 Tc^2 / pc,  b = 0.187295 R Tc / pc.
CS_A_COEF = 0.496388
CS_B_COEF = 0.187295


# --------------------------------------------------------------------------
# Carnahan-Starling EOS (main Eq. 20) and its bulk free energy (main Eq. 19)
# --------------------------------------------------------------------------
def critical_temperature(a: float, b: float, r_gas: float) -> float:
    """T_c from the two printed relations of main Eq. 20 (ratio a/b)."""
    return CS_B_COEF / CS_A_COEF * a / (b * r_gas)


def critical_pressure(a: float, b: float, r_gas: float) -> float:
    """p_c from b = 0.187295 R T_c / p_c (main Eq. 20)."""
    return CS_B_COEF * r_gas * critical_temperature(a, b, r_gas) / b


def cs_pressure(rho, rt, a, b, k_eos=1.0):
    """p_EOS = K_EOS [rho R T (1+v+v^2-v^3)/(1-v)^3 - a rho^2], v = b rho / 4."""
    v = b * rho / 4.0
    return k_eos * (rho * rt * (1.0 + v + v * v - v ** 3) / (1.0 - v) ** 3 - a * rho * rho)


def cs_free_energy(rho, rt, a, b):
    """Bulk free-energy density psi_b of the CS EOS at K_EOS = 1.

    psi_b = rho R T [ln rho - 1 + (4v - 3v^2)/(1-v)^2] - a rho^2; it satisfies
    p_EOS = rho psi_b' - psi_b (main Eq. 19), which the tests check.
    """
    v = b * rho / 4.0
    return rho * rt * (np.log(rho) - 1.0 + (4.0 * v - 3.0 * v * v) / (1.0 - v) ** 2) - a * rho * rho


def cs_chemical_potential(rho, rt, a, b):
    """mu = d psi_b / d rho at K_EOS = 1."""
    v = b * rho / 4.0
    return (rt * (np.log(rho) + (4.0 * v - 3.0 * v * v) / (1.0 - v) ** 2
                  + (4.0 * v - 2.0 * v * v) / (1.0 - v) ** 3) - 2.0 * a * rho)


def cs_repulsive_slope(rho, rt, b):
    """R T d(rho phi)/d rho: slope of the repulsive part of the CS pressure.

    This is d(p_EOS + K_EOS a rho^2)/d rho at K_EOS = 1, the quantity inside
    the square root of the sound-speed rule (main Eq. 22).
    """
    v = b * rho / 4.0
    return rt * (1.0 + 4.0 * v + 4.0 * v * v - 4.0 * v ** 3 + v ** 4) / (1.0 - v) ** 4


def cs_pressure_slope(rho, rt, a, b, k_eos=1.0):
    """d p_EOS / d rho."""
    return k_eos * (cs_repulsive_slope(rho, rt, b) - 2.0 * a * rho)


# --------------------------------------------------------------------------
# Maxwell construction (main Eq. 19 and the text after it)
# --------------------------------------------------------------------------
def spinodal_densities(rt, a, b):
    """The two zeros of dp/drho below the packing limit rho = 4/b."""
    grid = np.linspace(1e-6, 4.0 / b * (1 - 1e-6), 200001)
    s = cs_pressure_slope(grid, rt, a, b)
    idx = np.nonzero(np.sign(s[:-1]) != np.sign(s[1:]))[0]
    if len(idx) != 2:
        raise ValueError("temperature is not below the critical temperature")
    f = lambda r: cs_pressure_slope(r, rt, a, b)
    r1 = optimize.brentq(f, grid[idx[0]], grid[idx[0] + 1], xtol=1e-16, rtol=1e-15)
    r2 = optimize.brentq(f, grid[idx[1]], grid[idx[1] + 1], xtol=1e-16, rtol=1e-15)
    return r1, r2


def maxwell(tr, a=1.0, b=4.0, r_gas=1.0):
    """Coexistence densities (rho_g, rho_l) and pressure p0 at T = tr * T_c.

    Equal pressure and equal chemical potential of the two phases, which is
    the Maxwell equal-area rule for the CS EOS.  The coexistence pressure is
    found by bisection on mu(rho_l(P)) - mu(rho_g(P)), with rho_g(P) and
    rho_l(P) the outer roots of p(rho) = P.
    """
    rt = r_gas * tr * critical_temperature(a, b, r_gas)
    r1, r2 = spinodal_densities(rt, a, b)
    p_hi = cs_pressure(r1, rt, a, b)   # local maximum (gas spinodal)
    p_lo = cs_pressure(r2, rt, a, b)   # local minimum (liquid spinodal)
    rho_max = 4.0 / b * (1.0 - 1e-14)

    def outer_roots(P):
        rg = optimize.brentq(lambda r: cs_pressure(r, rt, a, b) - P, 1e-300, r1,
                             xtol=1e-300, rtol=1e-15, maxiter=2000)
        rl = optimize.brentq(lambda r: cs_pressure(r, rt, a, b) - P, r2, rho_max,
                             xtol=1e-300, rtol=1e-15, maxiter=2000)
        return rg, rl

    def dmu(P):
        rg, rl = outer_roots(P)
        return cs_chemical_potential(rl, rt, a, b) - cs_chemical_potential(rg, rt, a, b)

    lo = max(p_lo, 0.0) + 1e-14 * p_hi
    hi = p_hi * (1.0 - 1e-12)
    P = optimize.brentq(dmu, lo, hi, xtol=1e-300, rtol=1e-15, maxiter=2000)
    rg, rl = outer_roots(P)
    return rg, rl, P


def interface_constants(tr, a=1.0, b=4.0, r_gas=1.0):
    """Flat-interface tension C_sigma and 5%-95% thickness C_W at K_EOS = K_INT = 1.

    From the pressure tensor of main Eq. 17 with kappa = G^2 / 4 and
    G^2 = 2 a (main Eq. 21 at K = 1), the planar profile obeys
    (kappa/2) rho'^2 = dOmega(rho) = psi_b - mu0 rho + p0, so
      sigma = int_{rho_g}^{rho_l} sqrt(2 kappa dOmega) d rho,
      W     = int_{rho_5}^{rho_95} sqrt(kappa / (2 dOmega)) d rho,
    with the thickness levels 0.95 rho_g + 0.05 rho_l and 0.05 rho_g + 0.95 rho_l
    used by the paper's measurements.
    """
    rt = r_gas * tr * critical_temperature(a, b, r_gas)
    rg, rl, p0 = maxwell(tr, a, b, r_gas)
    mu0 = cs_chemical_potential(rg, rt, a, b)
    kappa = a / 2.0

    def domega(r):
        return cs_free_energy(r, rt, a, b) - mu0 * r + p0

    c_sigma, _ = integrate.quad(lambda r: math.sqrt(2.0 * kappa * max(domega(r), 0.0)),
                                rg, rl, epsabs=0.0, epsrel=1e-13, limit=400)
    r5 = 0.95 * rg + 0.05 * rl
    r95 = 0.05 * rg + 0.95 * rl
    c_w, _ = integrate.quad(lambda r: math.sqrt(kappa / (2.0 * domega(r))),
                            r5, r95, epsabs=0.0, epsrel=1e-13, limit=400)
    return c_sigma, c_w


def sigma_paper(width, tr, a=1.0, b=4.0, r_gas=1.0):
    """The sigma at which c = 1 under the paper's sound-speed rule (main Eq. 22).

    c^2 = 3 c_s^2 = 3 K_INT^2 K_EOS * RT d(rho phi)/d rho |_{rho_l}; setting
    c = 1 fixes K_EOS, and sigma = C_sigma K_INT K_EOS (main Eq. 23).
    """
    rt = r_gas * tr * critical_temperature(a, b, r_gas)
    _, rl, _ = maxwell(tr, a, b, r_gas)
    c_sigma, c_w = interface_constants(tr, a, b, r_gas)
    k_int = width / c_w
    return c_sigma / (3.0 * k_int * cs_repulsive_slope(rl, rt, b))


# --------------------------------------------------------------------------
# Model coefficients (main Eqs. 7 and 16) and the full parameter map
# --------------------------------------------------------------------------
def model_coefficients(varpi, alpha1=-1.0, beta1=1.0):
    """alpha2, beta2, k, h, b of main Eq. 7 (supplement Eq. 31)."""
    alpha2 = -(2.0 * alpha1 + varpi + 1.0) / (1.0 - varpi)
    beta2 = -2.0 * beta1 / (1.0 - varpi)
    k = 1.0 - varpi
    h = 6.0 * varpi * (1.0 - varpi) / (1.0 - 3.0 * varpi)
    bs = (1.0 - varpi) / (1.0 - 3.0 * varpi)
    return alpha2, beta2, k, h, bs


def relaxation_rates(s_p, varpi):
    """s_q and s_e from tau_p tau_q = (k+1) tau_e tau_q = 1/12 (main Eq. 16),
    with tau = 1/s - 1/2 and k = 1 - varpi."""
    k = 1.0 - varpi
    tau_p = 1.0 / s_p - 0.5
    tau_q = 1.0 / (12.0 * tau_p)
    tau_e = 1.0 / (12.0 * (k + 1.0) * tau_q)
    return 1.0 / (tau_q + 0.5), 1.0 / (tau_e + 0.5)


@dataclass
class Params:
    """The problem statement: lattice, rates, varpi, CS EOS, prescribed sigma and W."""
    nx: int = 64
    ny: int = 64
    s_p: float = 1.0
    s_eps: float | None = None   # None: equal to s_e
    varpi: float = 1.0 / 6.0
    a: float = 1.0
    b: float = 4.0
    r_gas: float = 1.0
    tr: float = 0.8
    sigma: float | None = None   # None: sigma_paper(width, tr)
    width: float = 10.0


@dataclass
class Coeffs:
    """Everything the step needs, in lattice units (c = 1)."""
    rho_g: float
    rho_l: float
    p0: float
    c_sigma: float
    c_w: float
    sigma: float
    width: float
    k_int: float
    k_eos: float
    G2: float        # G'^2 = 2 K_INT^2 K_EOS a  (main Eq. 21 squared)
    Kp: float        # K'   = K_EOS
    RT: float
    a: float
    b: float
    varpi: float
    alpha2: float
    beta2: float
    k: float
    h: float
    bs: float
    s_p: float
    s_q: float
    s_e: float
    s_eps: float


def derive(p: Params) -> Coeffs:
    """Map the problem statement to the lattice coefficients."""
    tr = p.tr
    rg, rl, p0 = maxwell(tr, p.a, p.b, p.r_gas)
    c_sigma, c_w = interface_constants(tr, p.a, p.b, p.r_gas)
    sigma = p.sigma if p.sigma is not None else sigma_paper(p.width, tr, p.a, p.b, p.r_gas)
    k_int = p.width / c_w
    k_eos = sigma / (c_sigma * k_int)
    alpha2, beta2, k, h, bs = model_coefficients(p.varpi)
    s_q, s_e = relaxation_rates(p.s_p, p.varpi)
    s_eps = s_e if p.s_eps is None else p.s_eps
    return Coeffs(rho_g=rg, rho_l=rl, p0=p0, c_sigma=c_sigma, c_w=c_w, sigma=sigma,
                  width=p.width, k_int=k_int, k_eos=k_eos,
                  G2=2.0 * k_int * k_int * k_eos * p.a, Kp=k_eos,
                  RT=p.r_gas * tr * critical_temperature(p.a, p.b, p.r_gas),
                  a=p.a, b=p.b, varpi=p.varpi, alpha2=alpha2, beta2=beta2,
                  k=k, h=h, bs=bs, s_p=p.s_p, s_q=s_q, s_e=s_e, s_eps=s_eps)
