"""Exact derivatives of the oracle step and of a rollout loss.  FP64/complex128.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Everything here is the complex-step method applied to the oracle's own
functions: for an analytic map F, Im F(x + i h d) / h is the directional
derivative J d to rounding (no subtraction, so h can be 1e-30).  Nothing is
hand-differentiated, so these are independent of any adjoint written by
hand.

* ``step_vjp``: lambda^t = J^T lambda^{t+1} for one step, built column by
  column.  A perturbation of f_i at node z changes f(t+1) only within the
  5 x 5 box around z (streaming moves one node, the force stencil reads one
  more), so nodes whose boxes do not overlap -- congruent modulo 5 in both
  directions -- are perturbed together.
* ``step_param_vjp``: lambda^{t+1} . d step / d theta for theta = (G'^2, K', RT).
* ``loss`` / ``loss_directional``: L = sum (rho_T - target)^2 after n steps
  from f^eq(rho0), and its exact derivative along a direction of
  (rho0, G'^2, K', RT).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import lbm

H = 1e-30
PERIOD = 5  # box of influence of one step is 5 x 5 nodes


def _with_theta(co, theta):
    """Coefficients with (G'^2, K', RT) replaced."""
    g2, kp, rt = theta
    return dataclasses.replace(co, G2=g2, Kp=kp, RT=rt)


def theta_of(co):
    return (co.G2, co.Kp, co.RT)


def step_vjp(f, lam_next, co, collide_fn=None):
    """J^T lam_next with J = d step(f) / d f, shape (9, ny, nx)."""
    _, ny, nx = f.shape
    if nx % PERIOD or ny % PERIOD:
        raise ValueError("lattice sides must be multiples of 5 for the colouring")
    out = np.zeros_like(f)
    xs = np.arange(nx)[None, :]
    ys = np.arange(ny)[:, None]
    for cy in range(PERIOD):
        for cx in range(PERIOD):
            mask = ((xs % PERIOD) == cx) & ((ys % PERIOD) == cy)
            for i in range(9):
                d = np.zeros(f.shape, dtype=np.complex128)
                d[i][mask] = 1.0
                jd = np.imag(lbm.step(f + 1j * H * d, co, collide_fn)) / H
                p = (lam_next * jd).sum(axis=0)          # contribution per output node
                box = np.zeros_like(p)
                for dy in range(-2, 3):
                    for dx in range(-2, 3):
                        box = box + np.roll(p, shift=(-dy, -dx), axis=(0, 1))
                out[i][mask] = box[mask]
    return out


def step_param_vjp(f, lam_next, co, collide_fn=None):
    """lam_next . d step(f) / d theta for theta = (G'^2, K', RT)."""
    th = np.array(theta_of(co), dtype=np.complex128)
    res = []
    for k in range(3):
        t = th.copy()
        t[k] += 1j * H
        jd = np.imag(lbm.step(f.astype(np.complex128), _with_theta(co, t), collide_fn)) / H
        res.append(float((lam_next * jd).sum()))
    return np.array(res)


def equilibrium_vjp(rho0, lam0, co):
    """d/d rho0 and d/d theta of sum lam0 . f^eq(rho0, u = 0, eta(rho0; theta))."""
    drho = np.imag(lbm.equilibrium(rho0 + 1j * H * np.ones_like(rho0), co))  # per-node d f_i / d rho0 * H
    g = (lam0 * drho).sum(axis=0) / H
    th = np.array(theta_of(co), dtype=np.complex128)
    dth = []
    for k in range(3):
        t = th.copy()
        t[k] += 1j * H
        jd = np.imag(lbm.equilibrium(rho0.astype(np.complex128), _with_theta(co, t))) / H
        dth.append(float((lam0 * jd).sum()))
    return g, np.array(dth)


def rollout(rho0, co, nsteps, collide_fn=None):
    f = lbm.equilibrium(rho0, co)
    for _ in range(nsteps):
        f = lbm.step(f, co, collide_fn)
    return f


def loss(rho0, co, nsteps, target, collide_fn=None):
    """L = sum_x (rho_T(x) - target(x))^2."""
    f = rollout(rho0, co, nsteps, collide_fn)
    r = f.sum(axis=0)
    return ((r - target) ** 2).sum()


def loss_directional(rho0, co, nsteps, target, drho0=None, dtheta=(0.0, 0.0, 0.0), collide_fn=None):
    """Exact dL along (drho0, dtheta), by one complex rollout."""
    r0 = rho0 + 0j
    if drho0 is not None:
        r0 = r0 + 1j * H * drho0
    th = np.array(theta_of(co), dtype=np.complex128) + 1j * H * np.asarray(dtheta, dtype=float)
    return float(np.imag(loss(r0, _with_theta(co, th), nsteps, target, collide_fn)) / H)
