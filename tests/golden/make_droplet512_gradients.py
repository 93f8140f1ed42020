"""Write droplet512_gradients.json: exact directional derivatives of the
droplet-to-ellipse loss on the 512 x 512 lattice, from the FP64 oracle only.

Problem: T_r = 0.8, W = 10, sigma = the paper's sound-speed value, a centred
droplet of radius 64 relaxed for 2000 steps; L = sum_x (rho_T - rho_target)^2
with the target an ellipse of the same area (semi-axes 80 and 51.2, same
interface profile).  Directions d = (drho0, dsigma, dW, dT_r): eight seeded
ones (seeds 0..7) with drho0 a standard normal field scaled by
(rho_l - rho_g)/sqrt(N) and each scalar a standard normal times its own
value, then each scalar axis alone.

dL/d(sigma, W, T_r) enters through theta = (G'^2, K', R T); the oracle's
parameter map is differentiated by central differences (h = 1e-6 of each
value), and every derivative along d is one complex-step rollout
(oracle.adjoint.loss_directional with the sequence collision), exact up to
rounding.  Run: python tests/golden/make_droplet512_gradients.py [--jobs 8]
(about half an hour of one core per direction).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import adjoint as adj  # noqa: E402
from oracle import hostmap as hm  # noqa: E402
from oracle import lbm  # noqa: E402
import workloads as wl  # noqa: E402

N_SIDE, TR, WIDTH, NSTEPS, RADIUS, SEMI = 512, 0.8, 10.0, 2000, 64.0, (80.0, 51.2)
OUT = os.path.join(HERE, "droplet512_gradients.json")


def problem(n=N_SIDE, nsteps=NSTEPS):
    sigma = hm.sigma_paper(WIDTH, TR)
    co = hm.derive(hm.Params(tr=TR, width=WIDTH, sigma=sigma))
    scale = n / N_SIDE
    rho0 = wl.droplets(n, n, co.rho_g, co.rho_l, co.width, [(n / 2, n / 2)], [RADIUS * scale])
    target = wl.ellipse(n, n, co.rho_g, co.rho_l, co.width, (n / 2, n / 2), SEMI[0] * scale, SEMI[1] * scale)
    return co, sigma, rho0, target


def theta_jacobian(sigma):
    """d(G'^2, K', RT)/d(sigma, W, T_r) of the oracle's map, central differences."""
    x0 = np.array([sigma, WIDTH, TR])
    J = np.zeros((3, 3))
    for j in range(3):
        h = 1e-6 * x0[j]
        xp, xm = x0.copy(), x0.copy()
        xp[j] += h
        xm[j] -= h
        tp = hm.derive(hm.Params(sigma=xp[0], width=xp[1], tr=xp[2]))
        tm = hm.derive(hm.Params(sigma=xm[0], width=xm[1], tr=xm[2]))
        J[:, j] = (np.array(adj.theta_of(tp)) - np.array(adj.theta_of(tm))) / (2 * h)
    return J


def directions(co, sigma, n=N_SIDE):
    """[(name, drho0 field or None, (dsigma, dW, dT_r))]."""
    out = []
    x0 = np.array([sigma, WIDTH, TR])
    for seed in range(8):
        rng = np.random.default_rng(seed)
        d_rho = rng.standard_normal((n, n)) * (co.rho_l - co.rho_g) / n
        d_par = rng.standard_normal(3) * x0
        out.append((f"seed{seed}", d_rho, d_par))
    for j, name in enumerate(("sigma", "width", "tr")):
        e = np.zeros(3)
        e[j] = 1.0
        out.append((name, None, e))
    return out


def _one(args):
    name, d_rho, d_par, n, nsteps = args
    co, sigma, rho0, target = problem(n, nsteps)
    t = time.time()
    if name == "loss":
        f = adj.rollout(rho0, co, nsteps, collide_fn=lbm.collide_sequence)
        return name, float(((f.sum(0) - target) ** 2).sum()), time.time() - t
    dth = theta_jacobian(sigma) @ np.asarray(d_par)
    v = adj.loss_directional(rho0, co, nsteps, target, drho0=d_rho, dtheta=dth, collide_fn=lbm.collide_sequence)
    return name, v, time.time() - t


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=8)
    ap.add_argument("--n", type=int, default=N_SIDE)
    ap.add_argument("--steps", type=int, default=NSTEPS)
    ap.add_argument("--out", default=OUT)
    a = ap.parse_args()
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    co, sigma, rho0, target = problem(a.n, a.steps)
    dirs = directions(co, sigma, a.n)
    res = {}
    tasks = [(nm, dr, dp, a.n, a.steps) for nm, dr, dp in dirs] + [("loss", None, None, a.n, a.steps)]
    with ProcessPoolExecutor(max_workers=a.jobs) as ex:
        for name, v, dt in ex.map(_one, tasks):
            res[name] = v
            print(f"{name}: {v:.17g} ({dt:.0f} s)", flush=True)
    loss = res.pop("loss")
    doc = {
        "what": "exact dL/d(rho0, sigma, W, T_r) along seeded directions (complex-step FP64 oracle)",
        "n": a.n, "nsteps": a.steps, "tr": TR, "width": WIDTH, "sigma": sigma, "radius": RADIUS * a.n / N_SIDE,
        "semi_axes": [SEMI[0] * a.n / N_SIDE, SEMI[1] * a.n / N_SIDE], "loss": loss,
        "directions": {nm: {"param": list(map(float, dp)), "rho0": dr is not None, "value": res[nm]}
                       for nm, dr, dp in dirs},
    }
    with open(a.out, "w") as fh:
        json.dump(doc, fh, indent=1)
    print("wrote", a.out)


if __name__ == "__main__":
    main()
