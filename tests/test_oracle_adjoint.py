"""Pins of the oracle's exact derivatives (complex step) against central
finite differences, which share nothing with the complex-step code path, and
of the column colouring against the plain dense Jacobian.  CPU only."""
import numpy as np
import pytest

from oracle import adjoint as adj
from oracle import hostmap as hm
from oracle import lbm

rng = np.random.default_rng(7)


@pytest.fixture(scope="module")
def case():
    co = hm.derive(hm.Params(tr=0.7, width=5.0))
    n = 10
    x = np.arange(n)[None, :]
    y = np.arange(n)[:, None]
    rho = 0.18 + 0.12 * np.sin(2 * np.pi * x / n) * np.cos(2 * np.pi * y / n) + 0.01 * rng.standard_normal((n, n))
    f = lbm.equilibrium(rho, co, 0.03 * np.cos(2 * np.pi * y / n) + 0 * x, 0.02 * np.sin(2 * np.pi * x / n) + 0 * y)
    f = f * (1 + 0.01 * rng.standard_normal(f.shape))
    return co, f


def fd(fn, x, d, h):
    return (fn(x + h * d) - fn(x - h * d)) / (2 * h)


def test_step_vjp_dot_product_against_fd(case):
    co, f = case
    lam = rng.standard_normal(f.shape)
    w = rng.standard_normal(f.shape)
    lhs = (adj.step_vjp(f, lam, co) * w).sum()
    rhs = (lam * fd(lambda g: lbm.step(g, co), f, w, 1e-6)).sum()
    assert lhs == pytest.approx(rhs, rel=1e-7)


def test_colouring_equals_dense_jacobian():
    """On a 5 x 5 lattice every colour is one node; the coloured J^T lam must
    equal the transpose of the dense complex-step Jacobian applied to lam."""
    co = hm.derive(hm.Params(tr=0.7, width=5.0))
    rho = 0.18 + 0.02 * rng.standard_normal((5, 5))
    f = lbm.equilibrium(rho, co) * (1 + 0.01 * rng.standard_normal((9, 5, 5)))
    lam = rng.standard_normal(f.shape)
    J = np.zeros((f.size, f.size))
    for c in range(f.size):
        d = np.zeros(f.size, dtype=np.complex128)
        d[c] = 1.0
        J[:, c] = (np.imag(lbm.step(f + 1j * adj.H * d.reshape(f.shape), co)) / adj.H).ravel()
    np.testing.assert_allclose(adj.step_vjp(f, lam, co).ravel(), J.T @ lam.ravel(), rtol=1e-12, atol=1e-12)


def test_param_vjp_against_fd(case):
    co, f = case
    lam = rng.standard_normal(f.shape)
    got = adj.step_param_vjp(f, lam, co)
    th = np.array(adj.theta_of(co))
    for k in range(3):
        e = np.zeros(3)
        e[k] = 1.0
        h = 1e-6 * abs(th[k])
        num = fd(lambda t: (lam * lbm.step(f, adj._with_theta(co, t))).sum(), th, e, h)
        assert got[k] == pytest.approx(num, rel=1e-6)


def test_equilibrium_vjp_against_fd(case):
    co, f = case
    rho0 = f.sum(0)
    lam = rng.standard_normal(f.shape)
    g, dth = adj.equilibrium_vjp(rho0, lam, co)
    d = rng.standard_normal(rho0.shape)
    assert (g * d).sum() == pytest.approx(fd(lambda r: (lam * lbm.equilibrium(r, co)).sum(), rho0, d, 1e-6),
                                          rel=1e-7)
    th = np.array(adj.theta_of(co))
    for k in range(3):
        e = np.zeros(3)
        e[k] = 1.0
        num = fd(lambda t: (lam * lbm.equilibrium(rho0, adj._with_theta(co, t))).sum(), th, e, 1e-6 * abs(th[k]))
        assert dth[k] == pytest.approx(num, rel=1e-6)


def test_reverse_accumulation_equals_directional_derivative(case):
    """Chaining step_vjp backwards from dL/dfT and finishing with
    equilibrium_vjp gives the same dL/drho0 . d as one complex rollout, and
    the accumulated parameter terms match each directional derivative."""
    co, f = case
    rho0 = f.sum(0)
    n = 4
    target = rho0[::-1, :].copy()
    fs = [lbm.equilibrium(rho0, co)]
    for _ in range(n):
        fs.append(lbm.step(fs[-1], co))
    lam = np.broadcast_to(2 * (fs[-1].sum(0) - target), fs[-1].shape).copy()
    dth = np.zeros(3)
    for t in range(n - 1, -1, -1):
        dth += adj.step_param_vjp(fs[t], lam, co)
        lam = adj.step_vjp(fs[t], lam, co)
    g, dth0 = adj.equilibrium_vjp(rho0, lam, co)
    dth += dth0
    d = rng.standard_normal(rho0.shape)
    assert (g * d).sum() == pytest.approx(adj.loss_directional(rho0, co, n, target, drho0=d), rel=1e-10)
    for k in range(3):
        e = np.zeros(3)
        e[k] = 1.0
        assert dth[k] == pytest.approx(adj.loss_directional(rho0, co, n, target, dtheta=e), rel=1e-10)


def test_loss_directional_against_fd(case):
    co, f = case
    rho0 = f.sum(0)
    target = np.full_like(rho0, rho0.mean())
    d = rng.standard_normal(rho0.shape)
    exact = adj.loss_directional(rho0, co, 6, target, drho0=d)
    num = fd(lambda r: adj.loss(r, co, 6, target), rho0, d, 1e-6)
    assert exact == pytest.approx(num, rel=1e-6)
