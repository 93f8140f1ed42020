"""Oracle read-outs of macroscopic quantities.  FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).
"""
from __future__ import annotations

import numpy as np

from . import hostmap, lbm


def totals(f):
    """Total mass sum_x rho and total lattice momentum sum_x sum_i e_i f_i."""
    mass = f.sum()
    jx = np.tensordot(lbm.CX.astype(float), f, axes=(0, 0)).sum()
    jy = np.tensordot(lbm.CY.astype(float), f, axes=(0, 0)).sum()
    return mass, jx, jy


def level_crossings(profile, level):
    """Positions where a periodic 1-D profile crosses ``level``, by linear
    interpolation between neighbouring nodes; a node exactly on the level is
    a crossing at that node."""
    p = np.asarray(profile, dtype=np.float64)
    a = p - level
    b = np.roll(a, -1)
    on = np.nonzero(a == 0)[0].astype(np.float64)  # a node exactly on the level
    idx = np.nonzero(a * b < 0)[0]
    return np.sort(np.concatenate([on, idx + a[idx] / (a[idx] - b[idx])]))


def interface_width(profile, rho_g, rho_l):
    """5%-95% thickness of every interface of a periodic 1-D profile.

    Levels 0.95 rho_g + 0.05 rho_l and 0.05 rho_g + 0.95 rho_l, as in the
    paper's thickness measurement; each low-level crossing is paired with the
    nearest high-level crossing.  Returns the mean over interfaces.
    """
    n = len(profile)
    lo = level_crossings(profile, 0.95 * rho_g + 0.05 * rho_l)
    hi = level_crossings(profile, 0.05 * rho_g + 0.95 * rho_l)
    widths = []
    for x in lo:
        d = (hi - x + n / 2) % n - n / 2
        widths.append(np.min(np.abs(d)))
    return float(np.mean(widths))


def bulk_densities(profile):
    """(min, max) of a converged profile: the simulated gas and liquid densities."""
    return float(np.min(profile)), float(np.max(profile))


def droplet_radius(rho, centre, rho_g, rho_l):
    """Radius at the level (rho_g + rho_l)/2, along +-x and +-y through the
    centre (integer node), averaged over the four half-lines."""
    cx, cy = centre
    ny, nx = rho.shape
    level = 0.5 * (rho_g + rho_l)
    radii = []
    for line, c in ((rho[cy, :], cx), (rho[:, cx], cy)):
        n = len(line)
        xs = level_crossings(line, level)
        d = (xs - c + n / 2) % n - n / 2
        radii.append(np.min(d[d > 0]))
        radii.append(-np.max(d[d < 0]))
    return float(np.mean(radii))


def laplace_sigma(rho, centre, co):
    """Surface tension from the 2-D Laplace law sigma = (p_in - p_out) R.

    Pressures are the bulk p_EOS (main Eq. 20, K' = K_EOS) at the centre node
    and at the corner node farthest from it.
    """
    cx, cy = centre
    ny, nx = rho.shape
    p_in = hostmap.cs_pressure(rho[cy, cx], co.RT, co.a, co.b, co.Kp)
    p_out = hostmap.cs_pressure(rho[(cy + ny // 2) % ny, (cx + nx // 2) % nx], co.RT, co.a, co.b, co.Kp)
    R = droplet_radius(rho, centre, co.rho_g, co.rho_l)
    return float((p_in - p_out) * R), R, float(p_in - p_out)


def domain_length(rho):
    """L = 2 pi sum_k S(k) / sum_k |k| S(k), S(k) = |FFT(rho - mean)|^2, k != 0."""
    ny, nx = rho.shape
    s = np.abs(np.fft.fft2(rho - rho.mean())) ** 2
    kx = 2 * np.pi * np.fft.fftfreq(nx)[None, :]
    ky = 2 * np.pi * np.fft.fftfreq(ny)[:, None]
    k = np.sqrt(kx * kx + ky * ky)
    s[0, 0] = 0.0
    return float(2 * np.pi * s.sum() / (k * s).sum())
