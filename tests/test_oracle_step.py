"""Pins of the oracle step (per-node algebra and whole-lattice invariants)
against what the paper and the mathematics fix.  CPU only."""
import dataclasses

import numpy as np
import pytest

from oracle import hostmap as hm
from oracle import lbm

rng = np.random.default_rng(20180907)


def cstep(fn, x, d, h=1e-30):
    """Exact directional derivative of fn at x along d (complex step)."""
    return np.imag(fn(x + 1j * h * d)) / h


@pytest.fixture(scope="module")
def co():
    return hm.derive(hm.Params(tr=0.7, width=10.0))


# ---------------------------------------------------------------------------
# Velocity set and transformation matrix (supplement Eqs. 3-4)
# ---------------------------------------------------------------------------
def test_velocity_set_from_angles():
    i = np.arange(9)
    cx = np.where(i == 0, 0, np.where(i <= 4, np.cos((i - 1) * np.pi / 2), np.sqrt(2) * np.cos((2 * i - 1) * np.pi / 4)))
    cy = np.where(i == 0, 0, np.where(i <= 4, np.sin((i - 1) * np.pi / 2), np.sqrt(2) * np.sin((2 * i - 1) * np.pi / 4)))
    np.testing.assert_allclose(lbm.CX, cx, atol=1e-12)
    np.testing.assert_allclose(lbm.CY, cy, atol=1e-12)


def test_transform_rows_are_velocity_polynomials():
    """Rows of M are 1, -4 + 3c^2, 4 - 21c^2/2 + 9c^4/2, c_x, (3c^2 - 5) c_x,
    c_y, (3c^2 - 5) c_y, c_x^2 - c_y^2, c_x c_y (orthogonal, unweighted)."""
    cx, cy = lbm.CX.astype(float), lbm.CY.astype(float)
    c2 = cx * cx + cy * cy
    rows = np.array([np.ones(9), -4 + 3 * c2, 4 - 10.5 * c2 + 4.5 * c2 * c2, cx, (3 * c2 - 5) * cx,
                     cy, (3 * c2 - 5) * cy, cx * cx - cy * cy, cx * cy])
    np.testing.assert_array_equal(lbm.M, rows)
    np.testing.assert_allclose(lbm.M @ lbm.M.T, np.diag([9, 36, 36, 6, 12, 6, 12, 4, 4]), atol=0)
    np.testing.assert_allclose(lbm.MINV, lbm.M.T @ np.diag(1 / np.array([9, 36, 36, 6, 12, 6, 12, 4, 4.0])),
                               atol=1e-15)


# ---------------------------------------------------------------------------
# Equilibrium, force and consistency moments (main Eqs. 3, 4, 14)
# ---------------------------------------------------------------------------
def product_equilibrium(rho, ux, uy):
    """Tensor-product D2Q9 equilibrium rho Psi_cx(u_x) Psi_cy(u_y) with
    Psi_0 = 2/3 - u^2, Psi_{+-1} = (1 +- 3u + 3u^2)/6: the Hermite-complete
    equilibrium of an ideal gas with c_s^2 = 1/3."""
    def psi(c, u):
        return np.where(c == 0, 2 / 3 - u * u, (1 + 3 * c * u + 3 * u * u) / 6)
    return np.stack([rho * psi(lbm.CX[i], ux) * psi(lbm.CY[i], uy) for i in range(9)])


def test_equilibrium_without_eta_is_product_form(co):
    rho = rng.uniform(0.05, 0.4, 50)
    ux = rng.uniform(-0.2, 0.2, 50)
    uy = rng.uniform(-0.2, 0.2, 50)
    meq = lbm.equilibrium_moments(rho, ux, uy, 0 * rho, co)
    np.testing.assert_allclose(meq, lbm.moments(product_equilibrium(rho, ux, uy)), atol=1e-15)


def test_equilibrium_momentum_flux_gives_p_lbe(co):
    """Momentum flux of m^eq (supplement Eq. 13 combinations) is
    p_LBE I + rho u u with p_LBE = (rho + eta)/3 (main Eq. 9)."""
    rho = rng.uniform(0.05, 0.4, 30)
    ux, uy, eta = rng.uniform(-0.1, 0.1, (3, 30))
    m = lbm.equilibrium_moments(rho, ux, uy, eta, co)
    pxx = 2 / 3 * m[0] + m[1] / 6 + m[7] / 2
    pyy = 2 / 3 * m[0] + m[1] / 6 - m[7] / 2
    p = (rho + eta) / 3
    np.testing.assert_allclose(pxx, p + rho * ux * ux, atol=1e-15)
    np.testing.assert_allclose(pyy, p + rho * uy * uy, atol=1e-15)
    np.testing.assert_allclose(m[8], rho * ux * uy, atol=1e-16)


def test_force_moments_are_equilibrium_derivative(co):
    """F_m = (d m^eq / d j) . F at fixed rho and eta, j = rho u: the force
    term carries the same Hermite orders as the equilibrium."""
    n = 40
    rho = rng.uniform(0.05, 0.4, n)
    ux, uy, eta = rng.uniform(-0.2, 0.2, (3, n))
    Fx, Fy = rng.uniform(-1e-2, 1e-2, (2, n))
    j = np.stack([rho * ux, rho * uy])
    fn = lambda jj: lbm.equilibrium_moments(rho, jj[0] / rho, jj[1] / rho, eta, co)
    deriv = cstep(fn, j, np.stack([Fx, Fy]))
    np.testing.assert_allclose(lbm.force_moments(Fx, Fy, ux, uy), deriv, atol=1e-16, rtol=1e-12)


def test_consistency_term_flux_is_r_add():
    """The momentum flux of Q_m equals (1/24)[2 F~F~ + |F~|^2 I], the tensor of
    R_add (main Eq. 15)."""
    Fx, Fy = rng.uniform(-0.3, 0.3, (2, 25))
    Q = lbm.consistency_moments(Fx, Fy)
    pxx = 2 / 3 * Q[0] + Q[1] / 6 + Q[7] / 2
    pyy = 2 / 3 * Q[0] + Q[1] / 6 - Q[7] / 2
    np.testing.assert_allclose(pxx, (2 * Fx * Fx + Fx * Fx + Fy * Fy) / 24, atol=1e-16)
    np.testing.assert_allclose(pyy, (2 * Fy * Fy + Fx * Fx + Fy * Fy) / 24, atol=1e-16)
    np.testing.assert_allclose(Q[8], 2 * Fx * Fy / 24, atol=1e-16)
    np.testing.assert_array_equal(Q[[0, 3, 4, 5, 6]], 0.0)


def test_consistency_term_is_second_order():
    """The populations M^-1 Q_m of the printed consistency term carry no
    fourth-order Hermite content: their projection on
    H_xxyy(e) = (e_x^2 - 1/3)(e_y^2 - 1/3) is zero, as for the second-order
    tensor of R_add the term produces.  This fixes the epsilon entry (minus
    the e entry), which drops out of the momentum flux."""
    Fx, Fy = rng.uniform(-0.3, 0.3, (2, 25))
    q = lbm.from_moments(lbm.consistency_moments(Fx, Fy))
    hxxyy = (lbm.CX ** 2 - 1 / 3) * (lbm.CY ** 2 - 1 / 3)
    np.testing.assert_allclose(np.tensordot(hxxyy, q, axes=(0, 0)), 0.0, atol=1e-16)
    assert np.max(np.abs(q)) > 1e-3  # and the term itself is not zero


def test_eos_slope_is_derivative_of_pressure(co):
    """d p_LBE / d rho returned by eos is the exact derivative of p_LBE
    (complex step), from the gas to beyond the liquid density."""
    rho = np.linspace(0.5 * co.rho_g, 1.2 * co.rho_l, 41)
    p_lbe, dp_lbe, _ = lbm.eos(rho, co)
    exact = cstep(lambda r: lbm.eos(r, co)[0], rho, np.ones_like(rho))
    np.testing.assert_allclose(dp_lbe, exact, rtol=1e-13, atol=1e-15)


# ---------------------------------------------------------------------------
# Collision matrix and correction matrices (main Eqs. 6, 10-11)
# ---------------------------------------------------------------------------
def test_collision_matrix_inverse_printed(co):
    """S times the printed inverse (supplement Eq. 46) is the identity."""
    c = dataclasses.replace(co, s_eps=1.1)
    for ux, uy in rng.uniform(-0.2, 0.2, (5, 2)):
        S = lbm.collision_matrix(np.array(ux), np.array(uy), c)
        se, sq, sp, seps, k, h, b = c.s_e, c.s_q, c.s_p, c.s_eps, c.k, c.h, c.bs
        Si = np.diag([1, 1 / se, 1 / seps, 1, 1 / sq, 1, 1 / sq, 1 / sp, 1 / sp])
        Si[1, 2] = k * (1 / se - 0.5)
        Si[1, 4] = h * ux * (1 / se - 0.5)
        Si[1, 6] = h * uy * (1 / se - 0.5)
        Si[7, 4] = 2 * b * ux * (1 / sp - 0.5)
        Si[7, 6] = -2 * b * uy * (1 / sp - 0.5)
        Si[8, 4] = b * uy * (1 / sp - 0.5)
        Si[8, 6] = b * ux * (1 / sp - 0.5)
        np.testing.assert_allclose(S @ Si, np.eye(9), atol=1e-14)


def cubic_residuals(c, R, T, X, sample):
    """Correction terms of rows e, p_xx, p_xy plus the cubic velocity terms
    printed in supplement Eqs. 33, 36 and 39, with the leading-order
    relations of supplement Eq. 32 for G-hat_1,7,8 (c = dt = 1); zero when
    R, T, X are right."""
    k, h, b, vp, se, sp = c.k, c.h, c.bs, c.varpi, c.s_e, c.s_p
    ux, uy, rho, drx, dry, dpx, dpy, uxx, uyy, uxy, uyx = sample
    div, dif, sxy = uxx + uyy, uxx - uyy, uxy + uyx
    G1 = -(2 - se) / (2 * se) * 2 * vp * rho * div
    G7 = -(2 - sp) / (2 * sp) * 2 / 3 * rho * dif
    G8 = -(2 - sp) / (2 * sp) * 1 / 3 * rho * sxy

    def corr(r, s):
        return 2 / (2 - s) * (R[r, 1] * G1 + R[r, 7] * G7 + R[r, 8] * G8
                              + T[r, 0] * drx + T[r, 1] * dry + X[r, 0] * dpx + X[r, 1] * dpy)

    cub1 = (-(9 * (2 * k + h) * ux * uy ** 2 * dpx + 9 * (2 * k + h) * ux ** 2 * uy * dpy)
            - (3 * ((1 - k) * ux ** 3 - (2 * k + h) * ux * uy ** 2) * drx
               + 3 * ((1 - k) * uy ** 3 - (2 * k + h) * ux ** 2 * uy) * dry)
            - ((9 * (1 - k) * ux ** 2 - 2 * (3 * k + h) * uy ** 2) * rho * uxx
               + (9 * (1 - k) * uy ** 2 - 2 * (3 * k + h) * ux ** 2) * rho * uyy
               - 4 * (3 * k + h) * ux * uy * rho * sxy))
    cub7 = ((6 * b * ux * uy ** 2 * dpx - 6 * b * ux ** 2 * uy * dpy)
            - ((ux ** 3 + 2 * b * ux * uy ** 2) * drx - (uy ** 3 + 2 * b * ux ** 2 * uy) * dry)
            - ((3 * ux ** 2 + 4 * b * uy ** 2) * rho * uxx - (3 * uy ** 2 + 4 * b * ux ** 2) * rho * uyy))
    cub8 = (-(3 * b * (uy ** 3 + 2 * ux ** 2 * uy) * dpx + 3 * b * (ux ** 3 + 2 * ux * uy ** 2) * dpy)
            + (b * (uy ** 3 + 2 * ux ** 2 * uy) * drx + b * (ux ** 3 + 2 * ux * uy ** 2) * dry)
            + (2 * b * ux * uy * rho * uxx + 2 * b * ux * uy * rho * uyy
               + 2 * b * (ux ** 2 + uy ** 2) * rho * sxy))
    return corr(1, se) + cub1, corr(7, sp) + cub7, corr(8, sp) + cub8


def correction_samples(n=10):
    out = []
    for _ in range(n):
        v = rng.uniform(-1, 1, 11)
        v[2] = abs(v[2]) + 0.1  # rho
        out.append(v)
    return out


# the entries of supplement Eqs. 34, 37, 40 that are not identically zero
CORRECTION_ENTRIES = ([("R", r, q) for r, q in [(1, 1), (1, 7), (1, 8), (7, 1), (7, 7), (8, 1), (8, 8)]]
                      + [(m, r, q) for m in ("T", "X") for r in (1, 7, 8) for q in (0, 1)])


@pytest.mark.parametrize("s_p", [0.8, 1.0, 1.6])
def test_corrections_cancel_printed_cubic_terms(s_p):
    """With the leading-order relations of supplement Eq. 32 for G-hat_1,7,8,
    the R, T, X terms cancel the cubic velocity terms printed in supplement
    Eqs. 33, 36 and 39 exactly (c = dt = 1), and no other entry is nonzero."""
    c = hm.derive(hm.Params(tr=0.7, width=10.0, s_p=s_p))
    for v in correction_samples():
        R, T, X = lbm.correction_matrices(np.array(v[0]), np.array(v[1]), c)
        for res in cubic_residuals(c, R, T, X, v):
            assert res == pytest.approx(0.0, abs=1e-12)
        # every other entry is zero: R acts only on the rows and columns of
        # e, p_xx, p_xy (with R_78 = R_87 = 0), T and X only on those rows
        nonzero = np.zeros((9, 9), dtype=bool)
        nonzero[[1, 1, 1, 7, 7, 8, 8], [1, 7, 8, 1, 7, 1, 8]] = True
        assert np.all(R[~nonzero] == 0)
        others = [0, 2, 3, 4, 5, 6]
        assert np.all(T[others] == 0) and np.all(X[others] == 0)


@pytest.mark.parametrize("mistake", ["sign", "dropped", "factor"])
def test_cancellation_detects_a_wrong_entry(mistake):
    """The pin has power: a sign error, a dropped entry or a wrong factor in
    any single nonzero entry of R, T or X (planted in the oracle's output)
    leaves a residual."""
    c = hm.derive(hm.Params(tr=0.7, width=10.0))
    scale = {"sign": -1.0, "dropped": 0.0, "factor": 2.0}[mistake]
    samples = correction_samples(4)
    for name, r, q in CORRECTION_ENTRIES:
        worst = 0.0
        for v in samples:
            R, T, X = lbm.correction_matrices(np.array(v[0]), np.array(v[1]), c)
            mats = {"R": R.copy(), "T": T.copy(), "X": X.copy()}
            mats[name][r, q] *= scale
            worst = max(worst, max(abs(x) for x in cubic_residuals(c, mats["R"], mats["T"], mats["X"], v)))
        assert worst > 1e-6, (name, r, q, mistake)


# ---------------------------------------------------------------------------
# The two collision forms, invariants and symmetry of the whole step
# ---------------------------------------------------------------------------
def random_state(co, nx=12, ny=10, du=0.05, seed=0, rho_range=None):
    r = np.random.default_rng(seed)
    lo, hi = rho_range or (co.rho_g, co.rho_l)
    rho = r.uniform(lo, hi, (ny, nx))
    ux, uy = r.uniform(-du, du, (2, ny, nx))
    f = lbm.equilibrium(rho, co, ux, uy)
    return f * (1 + r.uniform(-0.02, 0.02, f.shape))


def test_dense_equation_equals_six_step_sequence(co):
    """Supplement Eq. 1 and the six-step recipe of supplement Sec. IV agree."""
    c = dataclasses.replace(co, s_eps=1.37)
    f = random_state(c)
    np.testing.assert_allclose(lbm.collide(f, c), lbm.collide_sequence(f, c), rtol=0, atol=2e-16)


def test_mass_and_momentum_conserved(co):
    """Sum of rho is invariant; total momentum is invariant because the
    pairwise force sums to zero."""
    f = random_state(co, 16, 14, du=0.02, seed=3, rho_range=(0.15, 0.21))
    m0 = f.sum()
    j0 = np.tensordot(lbm.CX, f, axes=(0, 0)).sum(), np.tensordot(lbm.CY, f, axes=(0, 0)).sum()
    for _ in range(50):
        f = lbm.step(f, co)
    assert abs(f.sum() - m0) < 1e-14 * m0 * 50
    j1 = np.tensordot(lbm.CX, f, axes=(0, 0)).sum(), np.tensordot(lbm.CY, f, axes=(0, 0)).sum()
    assert abs(j1[0] - j0[0]) < 1e-13 * m0 and abs(j1[1] - j0[1]) < 1e-13 * m0


def test_force_sums_to_zero(co):
    f = random_state(co, 9, 7, seed=4)
    nf = lbm.node_fields(f, co)
    assert abs(nf["Fx"].sum()) < 1e-16 and abs(nf["Fy"].sum()) < 1e-16


def test_uniform_rest_state_is_fixed_point(co):
    rho = np.full((6, 8), 0.2)
    f = lbm.equilibrium(rho, co)
    np.testing.assert_allclose(lbm.step(f, co), f, rtol=0, atol=1e-16)


def _mirror_x(f):
    perm = [0, 3, 2, 1, 4, 6, 5, 8, 7]
    return np.roll(f[perm][..., ::-1], 1, axis=-1)


def _transpose(f):
    perm = [0, 2, 1, 4, 3, 5, 8, 7, 6]
    return np.swapaxes(f[perm], -1, -2)


def test_step_is_d4_equivariant(co):
    """The step commutes with the mirror x -> -x and with x <-> y."""
    f = random_state(co, 10, 10, du=0.1, seed=5)
    np.testing.assert_allclose(lbm.step(_mirror_x(f), co), _mirror_x(lbm.step(f, co)), atol=1e-15, rtol=0)
    np.testing.assert_allclose(lbm.step(_transpose(f), co), _transpose(lbm.step(f, co)), atol=1e-15, rtol=0)
    g = random_state(co, 10, 10, du=0.1, seed=6)
    a = lbm.step(_mirror_x(_transpose(g)), co)
    b = _mirror_x(_transpose(lbm.step(g, co)))
    np.testing.assert_allclose(a, b, atol=1e-15, rtol=0)


# ---------------------------------------------------------------------------
# Shear waves: viscosity (main Eq. 9) and Galilean invariance (cubic terms)
# ---------------------------------------------------------------------------
def shear_decay_ratio(co, U, rotated=False, n=64, nsteps=300):
    """Measured decay rate of a small shear wave divided by nu k^2,
    nu = (1/s_p - 1/2)/3, on a uniform single-phase state moving at U along
    the wave vector."""
    nu = (1 / co.s_p - 0.5) / 3
    A = 1e-3
    if rotated:
        x = np.arange(n)[None, :]
        y = np.arange(n)[:, None]
        ph = 2 * np.pi * (x + y) / n
        k = 2 * np.pi * np.sqrt(2) / n
        ux = (U + A * np.sin(ph)) / np.sqrt(2) + 0 * y
        uy = (U - A * np.sin(ph)) / np.sqrt(2) + 0 * x
    else:
        x = np.arange(n)[None, :] * 1.0
        k = 2 * np.pi / n
        ux = U + 0 * x
        uy = A * np.sin(k * x)
    rho = np.full(ux.shape, co.rho_l)
    f = lbm.equilibrium(rho, co, ux, uy)
    amps = []
    for _ in range(nsteps):
        _, u, v = lbm.macroscopic(f, co)
        amps.append(np.abs(np.fft.fft2((u - v) / np.sqrt(2))[1, 1]) if rotated else np.abs(np.fft.fft(v[0])[1]))
        f = lbm.step(f, co, lbm.collide_sequence)
    t = np.arange(nsteps)
    slope = np.polyfit(t[50:], np.log(amps[50:]), 1)[0]
    return -slope / (nu * k * k)


@pytest.fixture(scope="module")
def liquid():
    """Single-phase liquid with the non-ideal EOS (eta != 0), no force."""
    return dataclasses.replace(hm.derive(hm.Params(tr=0.8, width=10.0)), G2=0.0)


def test_shear_viscosity(liquid):
    assert shear_decay_ratio(liquid, 0.0) == pytest.approx(1.0, abs=0.005)


def test_galilean_shear_wave_axis(liquid, monkeypatch):
    """A background velocity along the wave vector leaves the shear decay
    rate at nu k^2; with R, T, X removed it does not (the test has power)."""
    assert shear_decay_ratio(liquid, 0.1) == pytest.approx(1.0, abs=0.02)
    orig = lbm.correction_matrices
    monkeypatch.setattr(lbm, "correction_matrices", lambda ux, uy, c: tuple(0 * a for a in orig(ux, uy, c)))
    assert abs(shear_decay_ratio(liquid, 0.1) - 1.0) > 0.05


@pytest.mark.slow
def test_galilean_shear_wave_diagonal(liquid, monkeypatch):
    """Same on the diagonal, where the stress sits in p_xx - p_yy."""
    assert shear_decay_ratio(liquid, 0.15, rotated=True) == pytest.approx(1.0, abs=0.02)
    orig = lbm.correction_matrices
    monkeypatch.setattr(lbm, "correction_matrices", lambda ux, uy, c: tuple(0 * a for a in orig(ux, uy, c)))
    assert abs(shear_decay_ratio(liquid, 0.15, rotated=True) - 1.0) > 0.05


# ---------------------------------------------------------------------------
# Power of a moving-interface parity case over R, T, X (supplement Eqs. 34,
# 37, 40): a wrong sign in any one entry must move the state well beyond
# the FP32 parity gate, or a kernel carrying that mistake would pass parity
# ---------------------------------------------------------------------------
NONZERO_CORRECTIONS = [("R", 1, 1), ("R", 1, 7), ("R", 1, 8), ("T", 1, 0), ("T", 1, 1), ("X", 1, 0), ("X", 1, 1),
                       ("R", 7, 1), ("R", 7, 7), ("T", 7, 0), ("T", 7, 1), ("X", 7, 0), ("X", 7, 1),
                       ("R", 8, 1), ("R", 8, 8), ("T", 8, 0), ("T", 8, 1), ("X", 8, 0), ("X", 8, 1)]
SHEAR_STEPS = 10  # the GPU parity case of tests/test_gpu_step.py runs the same state this long


@pytest.fixture(scope="module")
def sheared():
    import workloads as wl
    c = hm.derive(hm.Params(nx=60, ny=50, tr=0.6, width=6.0))
    rho, ux, uy = wl.sheared_droplet(c)
    return c, lbm.equilibrium(rho, c, ux, uy)


@pytest.mark.parametrize("entry", NONZERO_CORRECTIONS, ids=lambda e: f"{e[0]}{e[1]}{e[2]}")
def test_sheared_droplet_sees_every_correction_entry(sheared, entry, monkeypatch):
    """60 x 50 droplet at T_r = 0.6, W = 6 in a |u| <= 0.1 periodic velocity
    field: flipping the sign of any one of the 19 nonzero R, T, X entries
    moves the populations after 10 steps by at least 5x the FP32 gate
    (1e-5 rho_l), in both collision forms."""
    c, f0 = sheared
    ref = lbm.run(f0, c, SHEAR_STEPS)
    orig = lbm.correction_matrices

    def flipped(ux, uy, co):
        R, T, X = orig(ux, uy, co)
        {"R": R, "T": T, "X": X}[entry[0]][entry[1], entry[2]] *= -1.0
        return R, T, X

    monkeypatch.setattr(lbm, "correction_matrices", flipped)
    for form in (None, lbm.collide_sequence):
        moved = np.abs(lbm.run(f0, c, SHEAR_STEPS, form) - ref).max() / c.rho_l
        assert moved >= 5e-5, (entry, form, moved)


def test_sheared_droplet_corrections_are_not_negligible(sheared, monkeypatch):
    """Removing R, T and X altogether moves the same state by far more than
    the gate: the case sees the velocity-dependent collision as a whole."""
    c, f0 = sheared
    ref = lbm.run(f0, c, SHEAR_STEPS)
    orig = lbm.correction_matrices
    monkeypatch.setattr(lbm, "correction_matrices",
                        lambda ux, uy, co: tuple(np.zeros_like(a) for a in orig(ux, uy, co)))
    moved = np.abs(lbm.run(f0, c, SHEAR_STEPS) - ref).max() / c.rho_l
    assert moved >= 1e-3, moved
