"""Dynamic problems of the paper run on the HIP path: oscillation of an
elliptic droplet (main text, dynamic problems: 512^2 lattice, semi-axes 96.0
and 42.7, T_r = 0.6, W = 10).  The velocity-dependent parts of the collision
(R, T, X) act only when the fluid moves, so this is the test that exercises
them at large velocities over a long run.

The period is compared with the linear capillary mode n = 2 of a 2-D
droplet of radius R in a fluid of density rho_g (Lamb, Hydrodynamics):
omega^2 = n (n^2 - 1) sigma / ((rho_l + rho_g) R^3), with R the radius of
the same area, measured late in the run where the oscillation is weak (the
paper measures its own period the same way).  sigma is the paper's
sound-speed value; the paper leaves s_p open and this test uses s_p = 1.4,
the lowest shear viscosity that stays stable at this density ratio
(rho_l/rho_g = 132), where viscous damping shifts the period by well under
1 %."""
import numpy as np
import pytest
from scipy import ndimage

import paper_1809_02390_amd as pkg
import workloads as wl
from oracle import hostmap as hm
from tests._gpu_helpers import lattice

pytestmark = pytest.mark.gpu


def semi_axis(profile, level):
    """Half the distance between the outer level crossings of a 1-D density
    profile through the droplet centre, linearly interpolated."""
    i = np.where(profile > level)[0]
    a, b = i.min(), i.max()
    lo = a - (profile[a] - level) / (profile[a] - profile[a - 1])
    hi = b + (profile[b] - level) / (profile[b] - profile[b + 1])
    return 0.5 * (hi - lo)


def test_elliptic_droplet_period():
    n, tr, width, s_p = 512, 0.6, 10.0, 1.4
    co = hm.derive(hm.Params(tr=tr, width=width, s_p=s_p))
    rho0 = wl.ellipse(n, n, co.rho_g, co.rho_l, co.width, (n / 2, n / 2), 96.0, 42.7)
    lat = lattice(n, n, rho0, tr=tr, width=width, s_p=s_p)
    level = 0.5 * (co.rho_l + co.rho_g)
    every, nsamp = 100, 600
    dev = []
    for _ in range(nsamp):
        lat.step(every)
        r = lat.moments()[0].double().cpu().numpy()
        dev.append(semi_axis(r[n // 2], level) - semi_axis(r[:, n // 2], level))
    dev = np.array(dev)
    t = every * np.arange(1, nsamp + 1)
    cross = [t[i] + every * dev[i] / (dev[i] - dev[i + 1]) for i in range(nsamp - 1)
             if (dev[i] > 0) != (dev[i + 1] > 0)]
    assert len(cross) >= 5, cross
    period = 2 * np.mean(np.diff(cross)[-3:])  # late, weak oscillation
    radius = np.sqrt(96.0 * 42.7)
    analytic = 2 * np.pi * np.sqrt((co.rho_l + co.rho_g) * radius ** 3 / (6 * co.sigma))
    print(f"period {period:.0f} steps, analytic {analytic:.0f} ({period / analytic - 1:+.2%}); "
          f"zero crossings {np.round(cross).astype(int).tolist()}")
    assert period == pytest.approx(analytic, rel=0.03)
    assert abs(dev[-50:]).max() < 0.1 * abs(dev[0])  # the oscillation decays


def liquid_bodies(rho, level):
    """Connected regions with rho > level (4-connected; the droplets stay
    clear of the lattice edges), as (size, x centroid, y centroid), specks
    of up to 20 nodes left out."""
    lab, count = ndimage.label(rho > level)
    idx = range(1, count + 1)
    sizes = ndimage.sum(np.ones_like(rho), lab, idx)
    cm = ndimage.center_of_mass(np.ones_like(rho), lab, idx)
    return [(s, c[1], c[0]) for s, c in zip(sizes, cm) if s > 20]


# We, Re and the dimensionless end time t* = t U / D of each run
HEAD_ON = {"merge": (0.01, 1.0, 2.5), "bounce": (0.1, 1.0, 6.0), "merge_large_deformation": (20.0, 100.0, 12.0),
           "satellite": (60.0, 200.0, 20.0)}


@pytest.mark.parametrize("regime", ["merge", "bounce", "merge_large_deformation", "satellite"])
def test_head_on_collision_regimes(regime):
    """Head-on collision of equal droplets, D = 128 on 1024^2, T_r = 0.7,
    W = 10 (main text, dynamic problems): at We = 0.01, Re = 1 the droplets
    merge; at We = 0.1, Re = 1 they bounce back without merging; at We = 20,
    Re = 100 they merge with large deformation; at We = 60, Re = 200 the
    merged mass splits into two droplets with a satellite at the centre.
    The last two run at s_p = 1.645 and 1.685, near the stability limit at
    this density ratio (from gaps of 80 nodes they diverge).
    We = rho_l U^2 D / sigma and Re = U D / nu fix the relative speed U and
    the shear rate s_p (nu = (1/s_p - 1/2)/3), with sigma the sound-speed
    value.  The paper states neither the initial separation nor the velocity
    field: the droplet surfaces start 60 nodes (6 W) apart, beyond the range
    over which the diffuse interfaces attract each other, each droplet moving
    at U/2 (weighted by its liquid fraction), the gas at rest."""
    n, D, tr, W = 1024, 128.0, 0.7, 10.0
    We, Re, t_end = HEAD_ON[regime]
    d = pkg.lbm_derive(pkg.make_params(n, n, tr=tr, width=W))
    U = np.sqrt(We * d.sigma / (d.rho_l * D))
    s_p = 1.0 / (3.0 * U * D / Re + 0.5)
    rho0, ux0, uy0 = wl.head_on(d, U, n=n, diameter=D, gap=60.0)
    lat = lattice(n, n, rho0, ux0, uy0, tr=tr, width=W, s_p=s_p)
    mass0 = lat.moments()[3][0]
    level = 0.5 * (d.rho_l + d.rho_g)
    nsamp = 12
    every = int(round(t_end * D / U / nsamp))
    history = []
    for _ in range(nsamp):
        lat.step(every)
        rho, _, _, tot = lat.moments()
        history.append(liquid_bodies(rho.double().cpu().numpy(), level))
    counts = [len(h) for h in history]
    sep = [abs(h[1][1] - h[0][1]) if len(h) == 2 else 0.0 for h in history]
    print(f"{regime}: U = {U:.3e}, s_p = {s_p:.4f}, bodies {counts}, centroid distances {np.round(sep, 1).tolist()}")
    # total mass: the collision leaves it unchanged, but each step rounds the
    # nine updated populations in FP32, and steady non-equilibrium regions
    # repeat the same roundings, so the drift grows with the step count:
    # 2.4e-6 over the 0.5M steps of the merge run, 1.9e-4 over the 0.4M steps
    # of the bounce run (s_p = 0.79).  A conservation error of the scheme
    # itself would exceed the bound by orders of magnitude.
    assert abs(tot[0] / mass0 - 1.0) < 1e-3
    if regime == "merge":
        assert counts[0] == 2 and counts[-1] == 1
    elif regime == "bounce":
        assert all(c == 2 for c in counts)
        i = int(np.argmin(sep))
        assert 0 < i < nsamp - 1 and sep[-1] > sep[i] + 5.0  # closest approach, then apart
    elif regime == "merge_large_deformation":
        assert all(c == 1 for c in counts)  # merged by t* = 1 and stays one body
    else:  # the merged mass splits into two droplets with a satellite between them
        print("bodies at the end (size, x, y):", [tuple(round(float(v), 1) for v in b) for b in history[-1]])
        assert counts[0] == 1 and counts[-1] == 3
        # one body at the collision point, two equal ones placed symmetrically about it
        by_dist = sorted(history[-1], key=lambda b: np.hypot(b[1] - n / 2, b[2] - n / 2))
        sat, a, b = by_dist
        assert np.hypot(sat[1] - n / 2, sat[2] - n / 2) < 0.02 * n
        assert np.hypot(0.5 * (a[1] + b[1]) - n / 2, 0.5 * (a[2] + b[2]) - n / 2) < 0.02 * n
        assert abs(a[0] - b[0]) <= 0.05 * max(a[0], b[0])
        assert min(np.hypot(a[1] - n / 2, a[2] - n / 2), np.hypot(b[1] - n / 2, b[2] - n / 2)) > D


def test_elliptic_droplet_window_at_peak_velocity():
    """The elliptic droplet on its full 512^2 lattice: the GPU state at the
    time of largest max|u| over its first 10000 steps (the droplet passing
    through the round shape) is stepped 100 more times on the GPU and by the
    FP64 oracle; every population agrees within 1e-5 rho_l.  The state moves
    at the velocities where the velocity-dependent collision terms act."""
    from oracle import lbm
    n, tr, width, s_p = 512, 0.6, 10.0, 1.4
    co = hm.derive(hm.Params(tr=tr, width=width, s_p=s_p))
    rho0 = wl.ellipse(n, n, co.rho_g, co.rho_l, co.width, (n / 2, n / 2), 96.0, 42.7)
    lat = lattice(n, n, rho0, tr=tr, width=width, s_p=s_p)
    best, t_best, ck = -1.0, 0, lat.checkpoint_buffer()
    for _ in range(50):
        lat.step(200)
        _, ux, uy, _ = lat.moments()
        umax = float(torch_hypot_max(ux, uy))
        if umax > best:
            best, t_best = umax, lat.time
            lat.save_state(ck)
    lat.load_state(ck, t_best)
    f0 = lat.state().double().cpu().numpy()
    lat.step(100)
    got = lat.state().double().cpu().numpy()
    ref = lbm.run(f0, co, 100, lbm.collide_sequence)
    err = np.abs(got - ref).max() / co.rho_l
    print(f"t0 = {t_best}, max|u| = {best:.4f}, max|df|/rho_l after 100 steps = {err:.2e}")
    assert best > 5e-3 and 0 < t_best < 10000
    assert err <= 1e-5, err


def torch_hypot_max(ux, uy):
    return (ux.double() ** 2 + uy.double() ** 2).max().sqrt().item()


def test_head_on_collision_window_at_impact():
    """The We = 60, Re = 200 head-on collision (1024^2, D = 128, T_r = 0.7,
    relative speed U = 0.049, s_p = 1.685): at impact (the 60-node gap closed
    at speed U) two light-cone crops of the GPU state, at the contact point
    and on the rim of the contact zone, run 100 oracle steps; the central
    21 x 21 nodes of each agree with the GPU's next 100 steps within
    1e-5 rho_l on every population.  Crops are 2 x 100 + 13 nodes in
    half-width: one step moves information two nodes (streaming plus
    stencil), so the crop's own periodic seam stays outside the compared
    region."""
    from oracle import lbm
    from tests._gpu_helpers import crop_periodic, params_pair
    n, D, tr, W, We, Re = 1024, 128.0, 0.7, 10.0, 60.0, 200.0
    d = pkg.lbm_derive(pkg.make_params(n, n, tr=tr, width=W))
    U = float(np.sqrt(We * d.sigma / (d.rho_l * D)))
    s_p = 1.0 / (3.0 * U * D / Re + 0.5)
    _, co = params_pair(n, n, tr=tr, width=W, s_p=s_p)
    rho0, ux0, uy0 = wl.head_on(d, U, n=n, diameter=D, gap=60.0)
    lat = lattice(n, n, rho0, ux0, uy0, tr=tr, width=W, s_p=s_p)
    t0, window, inner = int(round(60.0 / U)), 100, 10
    lat.step(t0)
    half = 2 * window + 3 + inner
    centres = [(n // 2, n // 2), (n // 2, n // 2 + 40)]
    st = lat.state()
    crops = [crop_periodic(st, cx, cy, half).double().cpu().numpy() for cx, cy in centres]
    _, ux, uy, _ = lat.moments()
    umax = torch_hypot_max(ux, uy)
    del st
    lat.step(window)
    st = lat.state()
    for (cx, cy), crop in zip(centres, crops):
        with np.errstate(over="ignore", invalid="ignore", divide="ignore"):  # crop seam, outside the light cone
            ref = lbm.run(crop, co, window, lbm.collide_sequence)[:, half - inner:half + inner + 1,
                                                                    half - inner:half + inner + 1]
        assert np.all(np.isfinite(ref))
        got = crop_periodic(st, cx, cy, inner).double().cpu().numpy()
        err = np.abs(got - ref).max() / co.rho_l
        print(f"t0 = {t0}, max|u| = {umax:.4f}, centre ({cx}, {cy}): max|df|/rho_l = {err:.2e}")
        assert err <= 1e-5, (cx, cy, err)
    assert umax > 0.02
