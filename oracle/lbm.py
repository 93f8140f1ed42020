"""Oracle time step of the self-tuning-EOS D2Q9 model.  FP64 (or complex128).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

State convention: ``f`` has shape (9, ny, nx) and holds the post-streaming
distributions f_i(x, t) of main Eq. 1; x is the fast axis.  One call of
``step`` maps f(t) to f(t + dt): density, interaction force (main Eq. 12),
collision in moment space written as the defining equation (supplement
Eq. 1, dense per-node 9x9 matrices), then periodic streaming (supplement
Eq. 2).  Lattice units: dx = dt = c = 1.

Every function accepts real or complex arrays, so that exact derivatives can
be taken with the complex-step method (``oracle/adjoint.py``).
"""
from __future__ import annotations

import numpy as np

# D2Q9 velocity set (supplement Eq. 3): rest, four axes, four diagonals.
CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])

# Transformation matrix (supplement Eq. 4); rows are the moments
# rho, e, eps, j_x, q_x, j_y, q_y, p_xx, p_xy.
M = np.array([
    [1, 1, 1, 1, 1, 1, 1, 1, 1],
    [-4, -1, -1, -1, -1, 2, 2, 2, 2],
    [4, -2, -2, -2, -2, 1, 1, 1, 1],
    [0, 1, 0, -1, 0, 1, -1, -1, 1],
    [0, -2, 0, 2, 0, 1, -1, -1, 1],
    [0, 0, 1, 0, -1, 1, 1, -1, -1],
    [0, 0, -2, 0, 2, 1, 1, -1, -1],
    [0, 1, -1, 1, -1, 0, 0, 0, 0],
    [0, 0, 0, 0, 0, 1, -1, 1, -1],
], dtype=np.float64)
MINV = np.linalg.inv(M)

# Interaction-force weights omega(|e|^2) of main Eq. 12: 1/3 on the axes,
# 1/12 on the diagonals.
W_FORCE = np.array([0.0, 1 / 3, 1 / 3, 1 / 3, 1 / 3, 1 / 12, 1 / 12, 1 / 12, 1 / 12])

# The ordinary choices alpha_1 = -1, beta_1 = 1 (text after main Eq. 9).
ALPHA1 = -1.0
BETA1 = 1.0


def neighbour(a, cx, cy):
    """a(x + c) on the periodic lattice (a has the two lattice axes last)."""
    return np.roll(a, shift=(-cy, -cx), axis=(-2, -1))


def density(f):
    """rho = sum_i f_i (main Eq. 5)."""
    return f.sum(axis=0)


def stencil_gradient(rho):
    """g = sum_i omega_i rho(x + e_i) e_i, the stencil of main Eq. 12.

    g is the local density gradient of supplement Eq. 61; the force is
    F = G^2 rho g.
    """
    gx = np.zeros_like(rho)
    gy = np.zeros_like(rho)
    for i in range(1, 9):
        r = W_FORCE[i] * neighbour(rho, CX[i], CY[i])
        gx = gx + CX[i] * r
        gy = gy + CY[i] * r
    return gx, gy


def eos(rho, co):
    """p_LBE, d p_LBE / d rho and eta at each node.

    p_EOS is the scaled CS EOS of main Eq. 20 (K' = K_EOS in c = 1 units);
    p_LBE = p_EOS + G^2 rho^2 / 2 (main Eq. 18); eta follows from
    p_LBE = c_s^2 [(2 + alpha_1) rho + beta_1 eta] (main Eq. 9), c_s^2 = 1/3.
    """
    v = co.b * rho / 4.0
    one_m = 1.0 - v
    phi = (1.0 + v + v * v - v ** 3) / one_m ** 3
    dphi = (1.0 + 4.0 * v + 4.0 * v * v - 4.0 * v ** 3 + v ** 4) / one_m ** 4  # d(rho phi)/d rho
    p_eos = co.Kp * (rho * co.RT * phi - co.a * rho * rho)
    dp_eos = co.Kp * (co.RT * dphi - 2.0 * co.a * rho)
    p_lbe = p_eos + 0.5 * co.G2 * rho * rho
    dp_lbe = dp_eos + co.G2 * rho
    eta = (3.0 * p_lbe - (2.0 + ALPHA1) * rho) / BETA1
    return p_lbe, dp_lbe, eta


def moments(f):
    """m = M f."""
    return np.einsum("ij,j...->i...", M, f)


def from_moments(m):
    """f = M^{-1} m."""
    return np.einsum("ij,j...->i...", MINV, m)


def equilibrium_moments(rho, ux, uy, eta, co):
    """m^eq of main Eq. 3 (u-hat = u since c = 1)."""
    u2 = ux * ux + uy * uy
    return np.stack([
        rho,
        2.0 * ALPHA1 * rho + 2.0 * BETA1 * eta + 3.0 * rho * u2,
        co.alpha2 * rho + co.beta2 * eta - 3.0 * rho * u2 + 9.0 * rho * ux * ux * uy * uy,
        rho * ux,
        -rho * ux + 3.0 * rho * ux * uy * uy,
        rho * uy,
        -rho * uy + 3.0 * rho * uy * ux * ux,
        rho * (ux * ux - uy * uy),
        rho * ux * uy,
    ])


def force_moments(Fx, Fy, ux, uy):
    """F_m of main Eq. 4.

    The bracket [.] is the sum over distinct index permutations:
    [F u u u]_xxyy = 2 F_x u_x u_y^2 + 2 F_y u_y u_x^2,
    [F u u]_xyy = F_x u_y^2 + 2 F_y u_x u_y, [F u u]_xxy = F_y u_x^2 + 2 F_x u_x u_y.
    """
    Fu = Fx * ux + Fy * uy
    zero = np.zeros_like(Fx)
    return np.stack([
        zero,
        6.0 * Fu,
        -6.0 * Fu + 9.0 * (2.0 * Fx * ux * uy * uy + 2.0 * Fy * uy * ux * ux),
        Fx,
        -Fx + 3.0 * (Fx * uy * uy + 2.0 * Fy * ux * uy),
        Fy,
        -Fy + 3.0 * (Fy * ux * ux + 2.0 * Fx * ux * uy),
        2.0 * (Fx * ux - Fy * uy),
        Fx * uy + Fy * ux,
    ])


def consistency_moments(Ftx, Fty):
    """Q_m of main Eq. 14 from F-tilde = F / (G rho c)."""
    q = Ftx * Ftx + Fty * Fty
    zero = np.zeros_like(Ftx)
    return np.stack([zero, 0.5 * q, -0.5 * q, zero, zero, zero, zero,
                     (Ftx * Ftx - Fty * Fty) / 12.0, Ftx * Fty / 12.0])


def rates(co):
    """Diagonal of S: (s_0, s_e, s_eps, s_j, s_q, s_j, s_q, s_p, s_p).

    s_0 and s_j multiply moments whose non-equilibrium part is zero by the
    definitions of rho and rho u, so their value is immaterial; 1 is used.
    """
    return np.array([1.0, co.s_e, co.s_eps, 1.0, co.s_q, 1.0, co.s_q, co.s_p, co.s_p])


def collision_matrix(ux, uy, co):
    """S of main Eq. 6 at every node, shape (9, 9, ...): node axes last."""
    shape = np.shape(ux)
    S = np.zeros((9, 9) + shape, dtype=np.result_type(ux, float))
    s = rates(co)
    for i in range(9):
        S[i, i] = s[i]
    we = co.s_e / 2.0 - 1.0
    wp = co.s_p / 2.0 - 1.0
    S[1, 2] = co.k * co.s_eps * we
    S[1, 4] = co.h * ux * co.s_q * we
    S[1, 6] = co.h * uy * co.s_q * we
    S[7, 4] = 2.0 * co.bs * ux * co.s_q * wp
    S[7, 6] = -2.0 * co.bs * uy * co.s_q * wp
    S[8, 4] = co.bs * uy * co.s_q * wp
    S[8, 6] = co.bs * ux * co.s_q * wp
    return S


def correction_matrices(ux, uy, co):
    """R (9x9), T (9x2), X (9x2) of main Eqs. 10-11 at every node, node axes last.

    The nonzero entries are those of supplement Eqs. 34, 37 and 40.
    """
    shape = np.shape(ux)
    dt = np.result_type(ux, float)
    R = np.zeros((9, 9) + shape, dtype=dt)
    T = np.zeros((9, 2) + shape, dtype=dt)
    X = np.zeros((9, 2) + shape, dtype=dt)
    se, sp, k, h, b, vp = co.s_e, co.s_p, co.k, co.h, co.bs, co.varpi
    ux2, uy2, uxy = ux * ux, uy * uy, ux * uy
    # row 1 (supplement Eq. 34)
    R[1, 1] = -(se / (4.0 * vp)) * (9.0 * (1.0 - k) - 2.0 * (3.0 * k + h)) * (ux2 + uy2)
    R[1, 7] = (-(3.0 * sp * (2.0 - se)) / (4.0 * (2.0 - sp))
                    * (9.0 * (1.0 - k) + 2.0 * (3.0 * k + h)) * (ux2 - uy2))
    R[1, 8] = (12.0 * sp * (2.0 - se) / (2.0 - sp)) * (3.0 * k + h) * uxy
    T[1, 0] = 1.5 * (2.0 - se) * ((1.0 - k) * ux ** 3 - (2.0 * k + h) * ux * uy2)
    T[1, 1] = 1.5 * (2.0 - se) * ((1.0 - k) * uy ** 3 - (2.0 * k + h) * ux2 * uy)
    X[1, 0] = 4.5 * (2.0 - se) * (2.0 * k + h) * ux * uy2
    X[1, 1] = 4.5 * (2.0 - se) * (2.0 * k + h) * ux2 * uy
    # row 7 (supplement Eq. 37); R_78 = 0
    R[7, 1] = -(se * (2.0 - sp)) / (4.0 * vp * (2.0 - se)) * (3.0 - 4.0 * b) * (ux2 - uy2)
    R[7, 7] = -(3.0 * sp / 4.0) * (3.0 + 4.0 * b) * (ux2 + uy2)
    T[7, 0] = 0.5 * (2.0 - sp) * (ux ** 3 + 2.0 * b * ux * uy2)
    T[7, 1] = 0.5 * (2.0 - sp) * (-uy ** 3 - 2.0 * b * ux2 * uy)
    X[7, 0] = -3.0 * (2.0 - sp) * b * ux * uy2
    X[7, 1] = -3.0 * (2.0 - sp) * b * (-ux2 * uy)
    # row 8 (supplement Eq. 40); R_87 = 0
    R[8, 1] = (se * (2.0 - sp)) / (vp * (2.0 - se)) * b * uxy
    R[8, 8] = 6.0 * sp * b * (ux2 + uy2)
    T[8, 0] = -0.5 * (2.0 - sp) * b * (uy ** 3 + 2.0 * ux2 * uy)
    T[8, 1] = -0.5 * (2.0 - sp) * b * (ux ** 3 + 2.0 * ux * uy2)
    X[8, 0] = 1.5 * (2.0 - sp) * b * (uy ** 3 + 2.0 * ux2 * uy)
    X[8, 1] = 1.5 * (2.0 - sp) * b * (ux ** 3 + 2.0 * ux * uy2)
    return R, T, X


def node_fields(f, co):
    """Per-node quantities the collision needs at time t.

    Returns a dict with rho, g (stencil gradient = grad rho, supplement
    Eq. 61), F (main Eq. 12), F-tilde = G g (F / (G rho c) in c = 1 units),
    u from rho u = sum e_i f_i + F/2 (main Eq. 5), p_LBE, its slope, eta,
    and grad p_LBE = (d p_LBE / d rho) grad rho (supplement Eq. 61).
    """
    rho = density(f)
    gx, gy = stencil_gradient(rho)
    Fx = co.G2 * rho * gx
    Fy = co.G2 * rho * gy
    G = np.sqrt(co.G2)
    jx = np.tensordot(CX.astype(float), f, axes=(0, 0)) + 0.5 * Fx
    jy = np.tensordot(CY.astype(float), f, axes=(0, 0)) + 0.5 * Fy
    ux = jx / rho
    uy = jy / rho
    p_lbe, dp_lbe, eta = eos(rho, co)
    return dict(rho=rho, gx=gx, gy=gy, Fx=Fx, Fy=Fy, Ftx=G * gx, Fty=G * gy,
                ux=ux, uy=uy, p_lbe=p_lbe, dp_lbe=dp_lbe, eta=eta,
                gpx=dp_lbe * gx, gpy=dp_lbe * gy)


def _mv(A, v):
    """Per-node matrix-vector product: A (n, k, ...), v (k, ...) -> (n, ...)."""
    return np.einsum("ij...,j...->i...", A, v)


def collide(f, co):
    """Post-collision f-bar by the defining collision equation (supplement Eq. 1).

    m-bar = m + F_m - S d + S Q_m - R (I - S/2) d - T . grad rho - X . grad p_LBE,
    d = m - m^eq + F_m / 2 (dt = dx = c = 1).
    """
    nf = node_fields(f, co)
    m = moments(f)
    meq = equilibrium_moments(nf["rho"], nf["ux"], nf["uy"], nf["eta"], co)
    Fm = force_moments(nf["Fx"], nf["Fy"], nf["ux"], nf["uy"])
    Qm = consistency_moments(nf["Ftx"], nf["Fty"])
    S = collision_matrix(nf["ux"], nf["uy"], co)
    R, T, X = correction_matrices(nf["ux"], nf["uy"], co)
    d = m - meq + 0.5 * Fm
    I = np.eye(9).reshape((9, 9) + (1,) * (S.ndim - 2))
    grad_rho = np.stack([nf["gx"], nf["gy"]])
    grad_p = np.stack([nf["gpx"], nf["gpy"]])
    mbar = (m + Fm - _mv(S, d) + _mv(S, Qm) - _mv(R, _mv(I - 0.5 * S, d))
            - _mv(T, grad_rho) - _mv(X, grad_p))
    return from_moments(mbar)


def collide_sequence(f, co):
    """Post-collision f-bar by the six-step recipe of supplement Sec. IV.

    An independent second form of ``collide``: the tests require the two to
    agree to rounding.  Indices follow the moment order of ``M``.
    """
    nf = node_fields(f, co)
    ux, uy = nf["ux"], nf["uy"]
    m = moments(f)
    meq = equilibrium_moments(nf["rho"], ux, uy, nf["eta"], co)
    Fm = force_moments(nf["Fx"], nf["Fy"], ux, uy)
    Qm = consistency_moments(nf["Ftx"], nf["Fty"])
    R, T, X = correction_matrices(ux, uy, co)
    s = rates(co)
    # (1)
    mb = m.copy()
    m = m - meq
    mb = mb - 2.0 * m
    m = m + 0.5 * Fm
    # (2) rows 1, 7, 8 use the values of m_2, m_4, m_6 from step (1)
    m = m.copy()
    m[1] = m[1] + 0.5 * co.k * co.s_eps * m[2] + 0.5 * co.h * co.s_q * (ux * m[4] + uy * m[6])
    m[7] = m[7] + co.bs * co.s_q * (ux * m[4] - uy * m[6])
    m[8] = m[8] + 0.5 * co.bs * co.s_q * (uy * m[4] + ux * m[6])
    # (3)
    m = (1.0 - 0.5 * s)[:, None, None] * m
    # (4)
    gr = (nf["gx"], nf["gy"])
    gp = (nf["gpx"], nf["gpy"])
    for r in (1, 7, 8):
        mb[r] = (mb[r] - R[r, 1] * m[1] - R[r, 7] * m[7] - R[r, 8] * m[8]
                 - T[r, 0] * gr[0] - T[r, 1] * gr[1]
                 - X[r, 0] * gp[0] - X[r, 1] * gp[1])
    # (5)
    mb = mb + 2.0 * m
    # (6)
    mb[1] = mb[1] + co.s_e * Qm[1] + co.k * (0.5 * co.s_e - 1.0) * co.s_eps * Qm[2]
    mb[2] = mb[2] + co.s_eps * Qm[2]
    mb[7] = mb[7] + co.s_p * Qm[7]
    mb[8] = mb[8] + co.s_p * Qm[8]
    return from_moments(mb)


def stream(fbar):
    """f_i(x + e_i, t + 1) = f-bar_i(x, t) on the periodic lattice (supplement Eq. 2)."""
    out = np.empty_like(fbar)
    for i in range(9):
        out[i] = np.roll(fbar[i], shift=(CY[i], CX[i]), axis=(-2, -1))
    return out


def step(f, co, collide_fn=None):
    """One full time step f(t) -> f(t + 1).

    ``collide_fn`` selects the collision form: the defining dense equation
    (default) or ``collide_sequence``; the two agree to rounding.
    """
    return stream((collide_fn or collide)(f, co))


def run(f, co, nsteps, collide_fn=None):
    for _ in range(nsteps):
        f = step(f, co, collide_fn)
    return f


def equilibrium(rho, co, ux=None, uy=None):
    """f^eq = M^{-1} m^eq(rho, u, eta(rho)); the initial state used throughout
    (u = 0 unless given)."""
    if ux is None:
        ux = np.zeros_like(rho)
    if uy is None:
        uy = np.zeros_like(rho)
    _, _, eta = eos(rho, co)
    return from_moments(equilibrium_moments(rho, ux, uy, eta, co))


def macroscopic(f, co):
    """rho and the half-force-corrected velocity u of main Eq. 5 at time t."""
    nf = node_fields(f, co)
    return nf["rho"], nf["ux"], nf["uy"]
