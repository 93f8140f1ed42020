"""The HIP adjoint against the oracle's exact derivatives (complex step,
FP64) and the oracle's finite differences: one adjoint step, the adjoint of
the initial equilibrium, a checkpointed rollout gradient with respect to
rho0 and (G'^2, K', R T) and (sigma, W, T_r), and the torch autograd
wrapper.  Calls go through the C ABI.

Tolerances.  The adjoint runs in FP32.  Per element, lambda^t is a sum of a
few dozen products of O(1) factors, so its rounding is a few ulps of the
largest term: bound 1e-5 of max |lambda| (about 80 ulps).  Parameter sums
are FP64 sums of FP32 node terms: bound 1e-5 of the sum of |terms|, with
the terms taken from the oracle.  Rollout gradients carry the FP32 forward
(relative state error ~1e-6) through the loss: bound 1e-4 relative."""
import json
import os

import numpy as np
import pytest
import torch

import paper_1809_02390_amd as pkg
import workloads as wl
from oracle import adjoint as adj
from oracle import hostmap as hm
from oracle import lbm
from tests._gpu_helpers import adj_state_of, crop_periodic, fp32_state_of, lattice, oracle_init, params_pair

pytestmark = pytest.mark.gpu
DEV = "cuda"


def f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def nonequilibrium_state(nx, ny, co, seed):
    """A droplet with a velocity field, advanced 3 oracle steps, in float32."""
    rng = np.random.default_rng(seed)
    rho = wl.droplets(nx, ny, co.rho_g, co.rho_l, co.width, [(nx / 2, ny / 2)], [min(nx, ny) / 4])
    ux, uy = rng.uniform(-0.03, 0.03, (2, ny, nx))
    return f32(lbm.run(oracle_init(co, rho, ux, uy), co, 3))


def param_term_scale(f, lam, co):
    """sum |lam . d step / d theta_k| per node and population (the scale of
    the FP32 terms the device sums), k = 0..2."""
    th = np.array(adj.theta_of(co), dtype=np.complex128)
    out = []
    for k in range(3):
        t = th.copy()
        t[k] += 1j * adj.H
        jd = np.imag(lbm.step(f.astype(np.complex128), adj._with_theta(co, t))) / adj.H
        out.append(np.abs(lam * jd).sum())
    return np.array(out)


@pytest.fixture(scope="module", params=[(40, 30), (200, 35), (320, 35)], ids=["40x30", "200x35", "320x35"])
def case(request):
    """A small lattice (every tile touches the periodic edge), one with
    interior adjoint tiles next to ragged edges in both directions, and one
    whose width is a multiple of 64 (interior tiles then read the forward
    state through the run-relative addressing).  Sides are multiples of 5
    for the oracle's colouring."""
    nx, ny = request.param
    _, co = params_pair(nx, ny, tr=0.7, width=5.0)
    f = nonequilibrium_state(nx, ny, co, 5)
    lam = f32(np.random.default_rng(6).standard_normal(f.shape))
    return nx, ny, co, f, lam


def test_seed_and_get_roundtrip(case):
    nx, ny, co, f, lam = case
    lat = pkg.Lattice(nx, ny, tr=0.7, width=5.0)
    a = lat.adjoint_seed(lam)
    got = lat.adjoint_get(a).cpu().numpy()
    assert np.array_equal(got, lam.astype(np.float32))


def test_adjoint_step_matches_oracle(case):
    nx, ny, co, f, lam = case
    lat = pkg.Lattice(nx, ny, tr=0.7, width=5.0).set_state(f)
    ck = lat.save_state()
    a, b = lat.adjoint_seed(lam), lat.adjoint_buffer()
    lat.adjoint_theta(reset=True)
    lat.adjoint_step(ck, a, b)
    got = lat.adjoint_get(b).double().cpu().numpy()
    ref = adj.step_vjp(f, lam, co)
    assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max()
    dth = np.array(lat.adjoint_theta(reset=True))
    ref_th = adj.step_param_vjp(f, lam, co)
    scale = param_term_scale(f, lam, co)
    assert np.all(np.abs(dth - ref_th) <= 1e-5 * scale), (dth, ref_th, scale)


def test_adjoint_params_apply_the_parameter_jacobian(case):
    """lbm_adjoint_params returns dL/d(sigma, W, T_r) = J^T dL/dtheta with
    J = lbm_param_jacobian at the context's parameters, from the same
    accumulator as lbm_adjoint_theta, and clears it on request."""
    nx, ny, co, f, lam = case
    lat = pkg.Lattice(nx, ny, tr=0.7, width=5.0).set_state(f)
    ck = lat.save_state()
    a, b = lat.adjoint_seed(lam), lat.adjoint_buffer()
    lat.adjoint_theta(reset=True)
    lat.adjoint_step(ck, a, b)
    dth = np.array(lat.adjoint_theta(reset=False))
    dp, dth2 = pkg.lbm.lbm_adjoint_params(lat.ctx, reset=True)
    assert np.array_equal(np.array(dth2), dth)
    J = np.array(pkg.lbm_param_jacobian(lat.params))
    np.testing.assert_allclose(np.array(dp), J.T @ dth, rtol=1e-12, atol=0)
    assert lat.adjoint_theta(reset=True) == (0.0, 0.0, 0.0)


def test_adjoint_step_nondefault_parameters():
    """One adjoint step with every problem parameter away from its default
    (s_p, s_eps, varpi, a, b, R, T_r, sigma given, W) on 200 x 35, against
    the oracle's complex-step derivatives.  Putting any one of s_p, s_eps,
    varpi, b, T_r, sigma or W back to its default moves lambda^t by >= 2.2e-2
    of max |lambda|; a moves dL/dtheta (theta's K' and R T scale with it)."""
    kw = dict(s_p=0.8, s_eps=1.4, varpi=0.12, a=0.5, b=2.5, r_gas=1.5, tr=0.85, sigma=0.0021, width=12.0)
    nx, ny = 200, 35
    _, co = params_pair(nx, ny, **kw)
    f = nonequilibrium_state(nx, ny, co, 5)
    lam = f32(np.random.default_rng(6).standard_normal(f.shape))
    lat = pkg.Lattice(nx, ny, **kw).set_state(f)
    ck = lat.save_state()
    a, b = lat.adjoint_seed(lam), lat.adjoint_buffer()
    lat.adjoint_theta(reset=True)
    lat.adjoint_step(ck, a, b)
    got = lat.adjoint_get(b).double().cpu().numpy()
    ref = adj.step_vjp(f, lam, co)
    assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max()
    dth = np.array(lat.adjoint_theta(reset=True))
    ref_th = adj.step_param_vjp(f, lam, co)
    scale = param_term_scale(f, lam, co)
    assert np.all(np.abs(dth - ref_th) <= 1e-5 * scale), (dth, ref_th, scale)


@pytest.mark.parametrize("nx,ny", [(4096, 4096), (16384, 8192)])
def test_adjoint_step_sampled(nx, ny):
    """One adjoint step on a spinodal field (mean of the coexistence
    densities +- 0.01, T_r = 0.7, W = 10, after 50 forward steps): 4096^2,
    whose state and adjoint state interleave rows read through 32-bit
    offsets, and 16384 x 8192, whose state is read relative to each tile's
    row band and with 64-bit addresses in the tile rows that wrap.  Lambda(t)
    at sampled nodes, interior and on the periodic edges, against the
    oracle's exact VJP on a 15 x 15 periodic crop of f(t) and Lambda(t+1)
    around each.  Lambda(t) at a node reads f(t) and Lambda(t+1) within two
    nodes (streaming and the force stencil), so the crop's seam, seven
    nodes out, is beyond its reach."""
    half = 7
    _, co = params_pair(nx, ny, tr=0.7, width=10.0)
    rho = wl.uniform_noise(nx, ny, 0.5 * (co.rho_g + co.rho_l), 0.01, seed=3)
    lat = lattice(nx, ny, rho, tr=0.7, width=10.0)
    lat.step(50)
    ck = lat.save_state()
    f = lat.state()
    gen = torch.Generator(device=DEV).manual_seed(11)
    lam = torch.randn((9, ny, nx), generator=gen, device=DEV)
    a, b = lat.adjoint_seed(lam), lat.adjoint_buffer()
    lat.adjoint_step(ck, a, b)
    got_all = lat.adjoint_get(b)
    pts = [(nx // 2 - 1, ny // 2), (0, 0), (nx - 1, ny - 1), (0, ny - 1), (1234, 7), (nx - 2, 3000), (77, 1),
           (nx - 1, ny - 9)]
    for x, y in pts:
        fc = crop_periodic(f, x, y, half).double().cpu().numpy()
        lc = crop_periodic(lam, x, y, half).double().cpu().numpy()
        ref = adj.step_vjp(fc, lc, co)[:, half, half]
        got = got_all[:, y, x].double().cpu().numpy()
        assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max(), (x, y, got, ref)
    lat.close()


def test_two_adjoint_steps_match_oracle(case):
    """The second step reads a nonzero stencil adjoint (the scatter of the
    force terms to the neighbour densities)."""
    nx, ny, co, f, lam = case
    lat = pkg.Lattice(nx, ny, tr=0.7, width=5.0).set_state(f)
    ck0 = lat.save_state()
    lat.step(1)
    ck1 = lat.save_state()
    f1 = lat.state().double().cpu().numpy()
    a, b = lat.adjoint_seed(lam), lat.adjoint_buffer()
    lat.adjoint_step(ck1, a, b)
    lat.adjoint_step(ck0, b, a)
    got = lat.adjoint_get(a).double().cpu().numpy()
    ref = adj.step_vjp(f, adj.step_vjp(f1, lam, co), co)
    assert np.abs(got - ref).max() <= 2e-5 * np.abs(ref).max()


def test_adjoint_init_matches_oracle(case):
    nx, ny, co, f, lam = case
    rho0 = f32(f.sum(0))
    rng = np.random.default_rng(8)
    ux0, uy0 = f32(rng.uniform(-0.02, 0.02, (2, ny, nx)))
    lat = pkg.Lattice(nx, ny, tr=0.7, width=5.0)
    a = lat.adjoint_seed(lam)
    lat.adjoint_theta(reset=True)
    for u in ((None, None), (ux0, uy0)):
        got = lat.adjoint_init(rho0, a, *u).double().cpu().numpy()
        dth = np.array(lat.adjoint_theta(reset=True))
        rho_c = rho0 + 0j
        ref_g = np.imag(lbm.equilibrium(rho_c + 1j * adj.H, co, *(None if v is None else v for v in u)))
        ref_g = (lam * ref_g).sum(0) / adj.H
        assert np.abs(got - ref_g).max() <= 1e-5 * np.abs(ref_g).max()
        if u[0] is None:
            _, ref_th = adj.equilibrium_vjp(rho0, lam, co)
            assert np.allclose(dth, ref_th, rtol=1e-5, atol=0), (dth, ref_th)


def test_step_saved_is_bitwise_lbm_step():
    nx, ny = 70, 37
    _, co = params_pair(nx, ny, tr=0.8)
    rho = wl.droplets(nx, ny, co.rho_g, co.rho_l, co.width, [(30, 20)], [11.0])
    lat = pkg.Lattice(nx, ny, tr=0.8).init(rho)
    bufs = [lat.save_state(), lat.checkpoint_buffer(), lat.checkpoint_buffer()]
    for k in range(5):
        lat.step_saved(bufs[k % 2], bufs[(k + 1) % 2])
    lat.step(5)
    lat.save_state(bufs[2])
    assert torch.equal(fp32_state_of(bufs[1], nx, ny), fp32_state_of(bufs[2], nx, ny))


def test_native_segment_calls_match_single_steps():
    """lbm_step_saved_chain and lbm_adjoint_run give bitwise the results of
    the one-step calls they loop over."""
    nx, ny, n = 70, 37, 5
    _, co = params_pair(nx, ny, tr=0.8)
    rho = wl.droplets(nx, ny, co.rho_g, co.rho_l, co.width, [(30, 20)], [11.0])
    lat = pkg.Lattice(nx, ny, tr=0.8).init(rho)
    chain = [lat.save_state()] + [lat.checkpoint_buffer() for _ in range(n)]
    lat.step_saved_chain(chain)
    single = [chain[0]] + [lat.checkpoint_buffer() for _ in range(n)]
    for j in range(n):
        lat.step_saved(single[j], single[j + 1])
    assert all(torch.equal(fp32_state_of(a, nx, ny), fp32_state_of(b, nx, ny)) for a, b in zip(chain, single))
    lam = np.random.default_rng(3).standard_normal((9, ny, nx))
    a, b = lat.adjoint_seed(lam), lat.adjoint_buffer()
    lat.adjoint_theta(reset=True)
    out = lat.adjoint_run(chain[:n], a, b)
    th_run = lat.adjoint_theta(reset=True)
    x, y = lat.adjoint_seed(lam), lat.adjoint_buffer()
    for j in reversed(range(n)):
        lat.adjoint_step(chain[j], x, y)
        x, y = y, x
    th_single = lat.adjoint_theta(reset=True)
    assert out is b and torch.equal(adj_state_of(out, nx, ny), adj_state_of(x, nx, ny)) and th_run == th_single


@pytest.mark.parametrize("storage", ["fp32", "fp16", "bf16"])
def test_load_state_repeats_the_run(storage):
    nx, ny = 70, 37
    _, co = params_pair(nx, ny, tr=0.8)
    rho = wl.droplets(nx, ny, co.rho_g, co.rho_l, co.width, [(30, 20)], [11.0])
    lat = pkg.Lattice(nx, ny, tr=0.8, storage=storage).init(rho)
    lat.step(3)
    ck = lat.save_state()
    lat.step(7)
    a = lat.state().clone()
    lat.load_state(ck, 3)
    assert lat.time == 3
    lat.step(7)
    assert torch.equal(a, lat.state()) and lat.time == 10


# ---------------------------------------------------------------------------
# Checkpointed rollout gradient
# ---------------------------------------------------------------------------
ROLL = dict(nx=64, ny=48, nsteps=40, every=7, tr=0.8, width=6.0)


@pytest.fixture(scope="module")
def rollout_case():
    nx, ny = ROLL["nx"], ROLL["ny"]
    p, co = params_pair(nx, ny, tr=ROLL["tr"], width=ROLL["width"])
    rho0 = wl.droplets(nx, ny, co.rho_g, co.rho_l, co.width, [(30, 22)], [12.0])
    target = wl.ellipse(nx, ny, co.rho_g, co.rho_l, co.width, (nx / 2, ny / 2), 15.0, 9.6)
    r = pkg.Rollout(nx, ny, ROLL["nsteps"], ROLL["every"], tr=ROLL["tr"], width=ROLL["width"])
    rho_T = r.forward(rho0).double().cpu().numpy()
    drho0, dth, dp = r.backward(torch.tensor(2 * (rho_T - target)))
    return co, rho0, target, rho_T, drho0.double().cpu().numpy(), np.array(dth), np.array(dp)


def test_rollout_forward_matches_oracle(rollout_case):
    co, rho0, target, rho_T, *_ = rollout_case
    ref = adj.rollout(rho0, co, ROLL["nsteps"]).sum(0)
    assert np.abs(rho_T - ref).max() <= 1e-5 * co.rho_l


def test_rollout_gradient_rho0_matches_complex_step(rollout_case):
    co, rho0, target, rho_T, drho0, dth, dp = rollout_case
    for d in wl.random_directions(rho0.shape, 3, seed=11):
        exact = adj.loss_directional(rho0, co, ROLL["nsteps"], target, drho0=d)
        assert (drho0 * d).sum() == pytest.approx(exact, rel=1e-4)


def test_rollout_gradient_theta_matches_complex_step(rollout_case):
    co, rho0, target, rho_T, drho0, dth, dp = rollout_case
    for k in range(3):
        e = np.zeros(3)
        e[k] = 1.0
        exact = adj.loss_directional(rho0, co, ROLL["nsteps"], target, dtheta=e)
        assert dth[k] == pytest.approx(exact, rel=1e-4), k


def test_rollout_gradient_params_match_finite_differences(rollout_case):
    """dL/d(sigma, W, T_r) against FP64 central differences of the oracle
    rollout with the oracle's own parameter map."""
    co, rho0, target, rho_T, drho0, dth, dp = rollout_case
    x0 = [co.sigma, ROLL["width"], ROLL["tr"]]

    def L(x):
        c = hm.derive(hm.Params(sigma=x[0], width=x[1], tr=x[2]))
        return adj.loss(rho0, c, ROLL["nsteps"], target)

    for j in range(3):
        h = 1e-5 * x0[j]
        xp, xm = list(x0), list(x0)
        xp[j] += h
        xm[j] -= h
        num = (L(xp) - L(xm)) / (2 * h)
        assert dp[j] == pytest.approx(num, rel=1e-4), j


def test_rollout_auto_interval_keeps_every_state():
    """every = "auto" keeps every state for a small rollout, and gives the
    bits of an explicit every = 1."""
    nx, ny, steps = 48, 40, 30
    _, co = params_pair(nx, ny, tr=0.8)
    rho = wl.droplets(nx, ny, co.rho_g, co.rho_l, co.width, [(20, 22)], [9.0])
    out = []
    for every in ("auto", 1):
        r = pkg.Rollout(nx, ny, steps, every, tr=0.8)
        rho_T = r.forward(rho)
        out.append((r.every, rho_T.cpu().numpy(), r.backward(2.0 * rho_T)[0].cpu().numpy()))
        r.release()
    assert out[0][0] == 1
    assert np.array_equal(out[0][1], out[1][1]) and np.array_equal(out[0][2], out[1][2])


def test_autograd_function_matches_driver_and_is_deterministic(rollout_case):
    co, rho0, target, rho_T, drho0, dth, dp = rollout_case
    tgt = torch.tensor(target, device=DEV)

    def grads():
        r0 = torch.tensor(rho0, dtype=torch.float32, device=DEV, requires_grad=True)
        s = torch.tensor(co.sigma, dtype=torch.float64, requires_grad=True)
        w = torch.tensor(ROLL["width"], dtype=torch.float64, requires_grad=True)
        t = torch.tensor(ROLL["tr"], dtype=torch.float64, requires_grad=True)
        out = pkg.lbm_rollout(r0, s, w, t, ROLL["nsteps"], every=ROLL["every"])
        ((out.double() - tgt) ** 2).sum().backward()
        return r0.grad.clone(), torch.stack([s.grad, w.grad, t.grad])

    g1, p1 = grads()
    g2, p2 = grads()
    assert torch.equal(g1, g2) and torch.equal(p1, p2)
    np.testing.assert_allclose(g1.double().cpu().numpy(), drho0, rtol=0, atol=1e-6 * np.abs(drho0).max())
    np.testing.assert_allclose(p1.numpy(), dp, rtol=1e-6)


# ---------------------------------------------------------------------------
# Full-size gradient problem against stored exact derivatives
# ---------------------------------------------------------------------------
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "droplet512_gradients.json")


def test_droplet512_gradient_matches_stored_oracle_derivatives():
    """512^2 droplet (R = 64) relaxing towards the same-area ellipse for 2000
    steps, checkpoints every 100 (T_r = 0.8, W = 10, sigma_paper):
    dL/d(rho0, sigma, W, T_r) of the FP32 forward + adjoint along the eight
    seeded directions and the three parameter axes, each within 1e-4
    relative of the exact FP64 derivative written by
    tests/golden/make_droplet512_gradients.py (oracle only)."""
    with open(GOLDEN) as fh:
        g = json.load(fh)
    n, steps, tr, width, sigma = g["n"], g["nsteps"], g["tr"], g["width"], g["sigma"]
    co = hm.derive(hm.Params(tr=tr, width=width, sigma=sigma))
    rho0 = wl.droplets(n, n, co.rho_g, co.rho_l, co.width, [(n / 2, n / 2)], [g["radius"]])
    target = wl.ellipse(n, n, co.rho_g, co.rho_l, co.width, (n / 2, n / 2), *g["semi_axes"])
    r = pkg.Rollout(n, n, steps, 100, tr=tr, width=width, sigma=sigma)
    rho_T = r.forward(rho0).double().cpu().numpy()
    loss = ((rho_T - target) ** 2).sum()
    drho0, _, dp = r.backward(torch.tensor(2 * (rho_T - target)))
    r.release()
    drho0 = drho0.double().cpu().numpy()
    assert loss == pytest.approx(g["loss"], rel=1e-5)
    errs = {}
    for name, e in g["directions"].items():
        v = float(np.dot(dp, e["param"]))
        if e["rho0"]:
            rng = np.random.default_rng(int(name[4:]))
            v += float((drho0 * rng.standard_normal((n, n)) * (co.rho_l - co.rho_g) / n).sum())
        errs[name] = abs(v - e["value"]) / abs(e["value"])
    print("relative errors:", errs)
    assert max(errs.values()) <= 1e-4, errs


def test_overlapped_backward_matches_sequential_sweep():
    """The backward sweep with the next segment recomputed on a second
    stream (four segments, the last one short) gives bitwise the adjoint
    state and the dL/d theta sums of the sweep that recomputes each segment
    on the lattice's own stream right before its adjoint steps."""
    nx, ny, steps, every = 300, 200, 35, 10
    _, co = params_pair(nx, ny, tr=0.7, width=10.0)
    rho = wl.droplets(nx, ny, co.rho_g, co.rho_l, co.width, [(120, 100), (200, 90)], [40.0, 35.0])
    r = pkg.Rollout(nx, ny, steps, every, tr=0.7, width=10.0)
    r.forward(torch.tensor(rho, device="cuda"))
    lam = torch.randn((9, ny, nx), device="cuda", generator=torch.Generator(device="cuda").manual_seed(5))
    lat = r.lat
    got = lat.adjoint_get(r.backward_state(lam)).clone()
    th_got = lat.adjoint_theta(reset=True)
    a, b = lat.adjoint_seed(lam), lat.adjoint_buffer()
    for s in reversed(range(len(r.starts))):
        if lat.adjoint_run(r._segment_states(s), a, b) is b:
            a, b = b, a
    ref = lat.adjoint_get(a)
    th_ref = lat.adjoint_theta(reset=True)
    assert r.rec is not None and torch.equal(got, ref) and np.array_equal(np.array(th_got), np.array(th_ref))
    r.release()


def test_recomputed_segments_are_bitwise_the_forward_pass():
    """On a lattice that takes two steps per launch, the backward's
    recomputation of each checkpoint segment (lbm_step_saved_chain, storing
    every state) continues into the next checkpoint the forward pass saved
    (lbm_step, no state between its two steps): the same bits."""
    nx, ny, steps, every = 1024, 384, 40, 10
    _, co = params_pair(nx, ny, tr=0.7, width=10.0)
    rho = wl.droplets(nx, ny, co.rho_g, co.rho_l, co.width, [(300, 190), (700, 180)], [60.0, 50.0])
    r = pkg.Rollout(nx, ny, steps, every, tr=0.7, width=10.0)
    r.forward(torch.tensor(rho, device="cuda"))
    lat = r.lat
    nxt = lat.checkpoint_buffer()
    for s in range(len(r.starts)):
        states = r._segment_states(s)
        lat.step_saved(states[-1], nxt)
        assert torch.equal(fp32_state_of(nxt, nx, ny), fp32_state_of(r.ckpt[s + 1], nx, ny)), s
    r.release()
