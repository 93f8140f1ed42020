"""Seeded synthetic initial fields for the multiphase D2Q9 workloads.

This module is shared by the tests, the benchmark and the oracle-based
checks.  It holds none of the method's arithmetic: coexistence densities,
interface thickness and every other physical constant are arguments, computed
by the caller with whichever parameter map it uses.  All fields are float64
arrays of shape (ny, nx), x the fast axis, rounded through float32 so that a
float32 device buffer and the float64 CPU reference start from identical
values.

Profiles mirror the paper's own test problems: a flat interface (main text,
coexistence curve), a static droplet (Laplace law), spinodal decomposition of
a uniform state with noise, droplet pairs and an elliptic droplet (dynamic
tests), and a head-on collision of two moving droplets.
"""
from __future__ import annotations

import numpy as np

# 5%-95% thickness of a tanh profile: 2 * atanh(0.9) = 2.9444 tanh lengths.
TANH_WIDTH_FACTOR = 2.0 * np.arctanh(0.9)


def _f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def flat_slab(nx, ny, rho_g, rho_l, width, noise=0.0, seed=0):
    """Gas slab in liquid: rho = mean + diff/2 tanh((|y - ny/2| - ny/4) / width).

    ``width`` is used as the tanh length itself; the profile relaxes to the
    model's own thickness.  Uniform noise in [-noise, noise] is added.
    """
    y = np.arange(ny, dtype=np.float64)[:, None] * np.ones((1, nx))
    rho = 0.5 * (rho_l + rho_g) + 0.5 * (rho_l - rho_g) * np.tanh((np.abs(y - ny / 2) - ny / 4) / width)
    if noise:
        rho = rho + np.random.default_rng(seed).uniform(-noise, noise, size=(ny, nx))
    return _f32(rho)


def droplets(nx, ny, rho_g, rho_l, width, centres, radii):
    """Liquid discs in gas with tanh interfaces of 5%-95% thickness ``width``.

    Each disc contributes (rho_l - rho_g)/2 (1 - tanh((r - R) / xi)) with
    xi = width / 2.944, and r the periodic distance to its centre.
    """
    xi = width / TANH_WIDTH_FACTOR
    x = np.arange(nx, dtype=np.float64)[None, :]
    y = np.arange(ny, dtype=np.float64)[:, None]
    rho = np.full((ny, nx), float(rho_g))
    for (cx, cy), r0 in zip(centres, radii):
        dx = (x - cx + nx / 2) % nx - nx / 2
        dy = (y - cy + ny / 2) % ny - ny / 2
        r = np.sqrt(dx * dx + dy * dy)
        rho = rho + 0.5 * (rho_l - rho_g) * (1.0 - np.tanh((r - r0) / xi))
    return _f32(rho)


def ellipse(nx, ny, rho_g, rho_l, width, centre, semi_x, semi_y):
    """Liquid ellipse in gas; the tanh argument is the signed distance
    approximated by (s - 1) * sqrt(semi_x * semi_y) with
    s = sqrt((dx/semi_x)^2 + (dy/semi_y)^2)."""
    xi = width / TANH_WIDTH_FACTOR
    x = np.arange(nx, dtype=np.float64)[None, :] - centre[0]
    y = np.arange(ny, dtype=np.float64)[:, None] - centre[1]
    s = np.sqrt((x / semi_x) ** 2 + (y / semi_y) ** 2)
    d = (s - 1.0) * np.sqrt(semi_x * semi_y)
    rho = rho_g + 0.5 * (rho_l - rho_g) * (1.0 - np.tanh(d / xi))
    return _f32(rho)


def uniform_noise(nx, ny, mean, amplitude, seed=0):
    """mean + U(-amplitude, amplitude): initial state of spinodal decomposition."""
    rng = np.random.default_rng(seed)
    return _f32(mean + rng.uniform(-amplitude, amplitude, size=(ny, nx)))


def random_directions(shape, count, seed=0):
    """``count`` seeded standard-normal fields of ``shape`` (for directional
    derivative checks)."""
    rng = np.random.default_rng(seed)
    return [rng.standard_normal(shape) for _ in range(count)]


# ---------------------------------------------------------------------------
# Named workloads.  Physical constants come from the caller's map ``derived``
# (an object or dict with rho_g, rho_l and width).
# ---------------------------------------------------------------------------
def _get(d, k):
    return d[k] if isinstance(d, dict) else getattr(d, k)


def slab_64(derived, nx=64, ny=64, seed=1):
    """64x64 flat slab at the prescribed width, noise +-1e-4 (seed 1)."""
    return flat_slab(nx, ny, _get(derived, "rho_g"), _get(derived, "rho_l"),
                     _get(derived, "width"), noise=1e-4, seed=seed)


def static_droplet(derived, n=256, radius=40.0):
    """Centred droplet of the given radius on an n x n lattice."""
    return droplets(n, n, _get(derived, "rho_g"), _get(derived, "rho_l"),
                    _get(derived, "width"), [(n / 2, n / 2)], [radius])


def spinodal(derived, n=4096, amplitude=0.01, seed=3):
    """Mean of the coexistence densities plus U(-0.01, 0.01) noise (seed 3)."""
    mean = 0.5 * (_get(derived, "rho_g") + _get(derived, "rho_l"))
    return uniform_noise(n, n, mean, amplitude, seed=seed)


def coalescence(derived, nx=16384, ny=8192, radius=400.0, gap=20.0):
    """Two droplets of radius R, centres 2R + gap apart on the x axis."""
    d = radius + gap / 2
    return droplets(nx, ny, _get(derived, "rho_g"), _get(derived, "rho_l"),
                    _get(derived, "width"),
                    [(nx / 2 - d, ny / 2), (nx / 2 + d, ny / 2)], [radius, radius])


def head_on(derived, speed, n=1024, diameter=128.0, gap=60.0):
    """Two equal droplets on the x axis of an n x n lattice, their surfaces
    ``gap`` apart, approaching each other at relative speed ``speed`` (head-on
    collision).  Each droplet moves at speed/2 towards the other, weighted by
    its own liquid fraction; the gas starts at rest.  Returns (rho, ux, uy)."""
    rg, rl, w = _get(derived, "rho_g"), _get(derived, "rho_l"), _get(derived, "width")
    d = diameter / 2 + gap / 2
    centres = [(n / 2 - d, n / 2), (n / 2 + d, n / 2)]
    rho = droplets(n, n, rg, rl, w, centres, [diameter / 2] * 2)
    left, right = (droplets(n, n, 0.0, 1.0, w, [c], [diameter / 2]) for c in centres)
    ux = _f32(0.5 * speed * (left - right))
    return rho, ux, np.zeros_like(ux)


def sheared_droplet(derived, nx=60, ny=50, radius=14.0, amplitude=0.1):
    """Centred droplet in a smooth periodic velocity field
    u = amplitude * (sin(2 pi y / ny), sin(2 pi x / nx)): the interface moves
    at |u| up to ``amplitude`` in both directions, where the velocity-
    dependent parts of the collision are large.  Returns (rho, ux, uy)."""
    rho = droplets(nx, ny, _get(derived, "rho_g"), _get(derived, "rho_l"), _get(derived, "width"),
                   [(nx / 2, ny / 2)], [radius])
    x = np.arange(nx, dtype=np.float64)[None, :] * np.ones((ny, 1))
    y = np.arange(ny, dtype=np.float64)[:, None] * np.ones((1, nx))
    return rho, _f32(amplitude * np.sin(2 * np.pi * y / ny)), _f32(amplitude * np.sin(2 * np.pi * x / nx))
