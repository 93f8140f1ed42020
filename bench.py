#!/usr/bin/env python3
"""Benchmark of the self-tuning-EOS D2Q9 path on one MI355X.

Headline workload: spinodal decomposition on a periodic 4096 x 4096 lattice
at T/T_c = 0.7 (mean of the coexistence densities plus seeded uniform noise
+-0.01), W = 10, sigma from the paper's sound-speed rule.  lbm_step(n)
advances FP32 states two steps per launch (density halo, force, collision
and streaming of two time steps in one kernel, the same bits as two single
steps); the 2-byte storages take one step per launch.  Inputs are resident
in HBM before any timed region starts; every timed region is bracketed by
HIP events on the stream the kernels are launched on.

Prints one JSON line:
  value / roofline   MLUPS of the FP32 path (lbm_step) and the roofline of
                     its two-step kernel, which is bound by the vector ALU:
                     230 algorithmic lane-instructions per update (one
                     update's arithmetic in the gfx950 assembly) times the
                     update rate against the non-packed vector peak
                     39.3e12/s; its HBM view beside it (36 algorithmic bytes
                     per update: f read and written once per two updates);
  legs.fp32_single_step  one lbm_step(1) call per step: the one-step kernel,
                     bound by HBM (72 B/LU), with its HBM roofline;
  legs.fp16, .bf16   the step with 2-byte storage of f (40 B/LU, one step per
                     launch), its ratio to both FP32 paths, and the
                     coexistence-density error of a relaxed flat interface
                     against the Maxwell densities; these steps are bound by
                     the vector ALU, and every step leg also carries `alu`,
                     its vector-ALU roofline (lane-instructions per update
                     from the committed rocprofv3 SQ summary times the update
                     rate, against 39.3e12/s);
  legs.fwd_adjoint   checkpointed forward + adjoint over 1000 steps of the
                     2048^2 droplet-pair crop (T/T_c = 0.6, K = 100), the
                     adjoint kernel's own roofline, and the gradient error of
                     the 512^2 droplet-to-ellipse problem (2000 steps, K = 100)
                     against exact oracle derivatives stored in tests/golden;
  legs.fwd_adjoint_keep_all_states  the same crop keeping all 1000 states
                     in HBM (151 GB), so the backward recomputes nothing;
  legs.coalescence_16384x8192  the step on the largest workload over its
                     5000 steps, each storage, with the t = 5000 read-outs of
                     the 2-byte runs against FP32;
  legs.elliptic_droplet  oscillation period of the paper's elliptic droplet
                     against the linear capillary mode;
  legs.head_on_collision  liquid bodies over time in head-on collisions of
                     two droplets at the paper's four (We, Re) pairs;
  legs.graph_replay  256^2 and 1024^2, where launches set the time per step:
                     lbm_step(2000) against a HIP graph of lbm_step(100)
                     captured by the caller and replayed 20 times;
  cpu_baseline       the FP64 oracle timed on a bounded crop.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
METRIC = "MLUPS + % HBM roofline, FP32 vs FP16-storage step; fwd+adjoint MLUPS at stated err"
HBM_PEAK_GBS = 8000.0
# Algorithmic HBM bytes per lattice update (LU):
#   one-step kernel: 9 populations read + 9 written (4 B, or 2 B plus the 2-byte reference density read and written);
#   two-step kernel (FP32): 9 populations read + 9 written per node and launch, two updates;
#   adjoint step: f(t) 9 + L 9 + force adjoint 2 read, L 9 + force adjoint 2 written (4 B each).
BYTES_PER_LU = {"fp32": 72, "fp16": 40, "bf16": 40}
STEP2_BYTES_PER_LU = 36
# Vector instructions of one update's arithmetic (density 8, stencil 13.5,
# forward transform 25.5, node state and EOS 28, six-step collision 123,
# f += M^T w 31.5: the gfx950 assembly of the one-step kernel, per node),
# the algorithmic work against which the two-step kernel's ALU roofline is
# priced (its halo recomputation and addressing are overhead, like re-read
# bytes in an HBM-bound kernel).
ALG_INSTR_PER_LU = 230
ADJ_BYTES_PER_LU = 124
# the same without the two force-adjoint planes: f(t) 9 + lambda 9 read, lambda 9 written
ADJ_MIN_BYTES_PER_LU = 108
# rocprofv3 FETCH_SIZE / WRITE_SIZE summaries of each kernel on the 4096^2 workload
PROFILE_TRAFFIC = {k: os.path.join(ROOT, "profiles", f"traffic_{k}_spinodal4096.json")
                   for k in ("step2_f32", "step_f32", "step_f16", "step_bf16", "adjoint_f32")}
# rocprofv3 SQ summaries: vector instructions per lattice update of each kernel
PROFILE_VALU = {k: os.path.join(ROOT, "profiles", f"valu_{k}_spinodal4096.json")
                for k in ("step2_f32", "step_f32", "step_f16", "step_bf16", "adjoint_f32")}
# Vector-ALU peak without packed FP32: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# = 39.3e12 lane-instructions per second (one FP32 FMA each: 78.6 TFLOP/s,
# half the 157.3 TFLOP/s of packed FP32, which the library is compiled without).
VALU_PEAK_TLANE = 256 * 4 * 16 * 2.4e9 / 1e12
GOLDEN = os.path.join(ROOT, "tests", "golden", "droplet512_gradients.json")


def headline_roofline(fp32):
    """Roofline of the two-step FP32 kernel: bound by the vector ALU, priced
    on ALG_INSTR_PER_LU per update; traffic is its measured HBM bytes per
    launch (two updates per node); its HBM view on 36 B per update beside."""
    achieved = ALG_INSTR_PER_LU * fp32["mlups"] * 1e6 / 1e12
    alu = fp32["alu"] or {}
    return {"bound": "alu", "achieved": round(achieved, 2), "peak": round(VALU_PEAK_TLANE, 2),
            "unit": "T lane-instr/s", "frac": round(achieved / VALU_PEAK_TLANE, 4), "traffic": fp32["traffic"],
            "kernel": fp32["kernel"], "algorithmic_instr_per_lu": ALG_INSTR_PER_LU,
            "executed_instr_per_lu_profiled": alu.get("valu_lane_instr_per_lu"),
            "valu_busy_profiled": alu.get("valu_busy_profiled"),
            "hbm": {"achieved": fp32["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": fp32["frac"],
                    "algorithmic_bytes_per_lu": STEP2_BYTES_PER_LU}}


def kernel_source_hash():
    """The profile summaries' hash of the kernel sources (comments ignored)."""
    sys.path.insert(0, ROOT)
    from paper_1809_02390_amd.profile_summary import kernel_source_hash as h
    return h()


def measured_traffic(kernel, n_nodes):
    """HBM bytes per launch of `kernel` on n_nodes from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source
    and lattice size; else None."""
    t = _profile(PROFILE_TRAFFIC[kernel], n_nodes)
    return None if t is None else round(t["bytes_per_launch"])


def _profile(path, n_nodes):
    """A committed profile summary if it was taken on the current kernel
    source and lattice size, else None."""
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    return t if t.get("kernel_sha") == kernel_source_hash() and t.get("n_nodes") == n_nodes else None


def alu_roofline(kernel, n_nodes, mlups):
    """Vector-ALU roofline of a kernel bound by it: the lane-instructions per
    update counted by rocprofv3 times the measured update rate, against the
    non-packed vector peak; None without a current SQ summary."""
    t = _profile(PROFILE_VALU[kernel], n_nodes)
    if t is None:
        return None
    achieved = mlups * 1e6 * t["valu_lane_instr_per_lu"] / 1e12
    return {"bound": "alu", "achieved": round(achieved, 2), "peak": round(VALU_PEAK_TLANE, 2),
            "unit": "T lane-instr/s", "frac": round(achieved / VALU_PEAK_TLANE, 4),
            "valu_lane_instr_per_lu": round(t["valu_lane_instr_per_lu"], 1),
            "valu_busy_profiled": round(t["valu_busy"], 3)}


class Timer:
    """HIP events on torch's current stream (the stream the library uses).

    Each timed region is preceded by a lead-in: `pacer` steps of a lattice of
    its own, enqueued without a host synchronisation right before the
    region's own (untimed) warm-up work and the timed work.  After any idle
    gap, even 50 ms, the GPU's power management needs about 20 ms of sustained
    work to return to steady clocks (the 4096^2 FP32 step measured 213-236 us
    over its first 100 steps after an idle gap, 201-205 us in steady state),
    and a short timed region would otherwise measure that ramp.  The lead-in
    belongs to no workload and is not timed."""

    def __init__(self, torch, pacer=None, lead_in_steps=500):
        self.torch = torch
        self.stream = torch.cuda.current_stream()
        self.pacer, self.lead_in_steps = pacer, lead_in_steps

    def __call__(self, fn, pre=None):
        torch = self.torch
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        if self.pacer is not None:
            self.pacer.step(self.lead_in_steps)  # asynchronous: no gap before what follows
        if pre is not None:
            pre()
        a.record(self.stream)
        fn()
        b.record(self.stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b)  # ms


def make_pacer(pkg, wl, nx=4096, ny=4080, tr=0.7, width=10.0):
    """The lattice whose steps make the lead-in of every timed region (an
    FP32 spinodal state of its own, seed 4).  16 rows fewer than the 4096^2
    workload: the same work per step within 0.4 %, but another launch grid,
    so a kernel trace keeps its steps apart from the timed ones."""
    d = pkg.lbm_derive(pkg.make_params(nx, ny, tr=tr, width=width))
    rho = wl.uniform_noise(nx, ny, 0.5 * (d.rho_g + d.rho_l), 0.01, seed=4)
    return pkg.Lattice(nx, ny, tr=tr, width=width).init(rho)


def step_leg(pkg, wl, timer, storage, n, steps, warmup, tr=0.7, width=10.0, single=False):
    """`steps` steps of the 4096^2 spinodal workload in one lbm_step call
    (FP32: the two-step kernel), or with single=True one lbm_step(1) call
    per step (the one-step kernel)."""
    d = pkg.lbm_derive(pkg.make_params(n, n, tr=tr, width=width))
    rho0 = wl.spinodal({"rho_g": d.rho_g, "rho_l": d.rho_l, "width": width}, n=n)
    lat = pkg.Lattice(n, n, tr=tr, width=width, storage=storage).init(rho0)

    def run(k):
        if single:
            for _ in range(k):
                lat.step(1)
        else:
            lat.step(k)

    ms = timer(lambda: run(steps), pre=lambda: run(warmup))
    tot = lat.moments(fields=False)
    lat.close()
    if not all(np.isfinite(tot)):
        raise RuntimeError(f"{storage} state diverged")
    per = ms / steps
    two_step = storage == "fp32" and not single
    alg = STEP2_BYTES_PER_LU if two_step else BYTES_PER_LU[storage]
    gbs = alg * n * n / (per * 1e-3) / 1e9
    mlups = round(n * n * steps / (ms * 1e-3) / 1e6, 1)
    kernel = "step2_f32" if two_step else "step_" + storage.replace("fp", "f")
    traffic = measured_traffic(kernel, n * n)
    return d, rho0, {"mlups": mlups, "ms_per_step": round(per, 5),
                     "kernel": ("step2_kernel<F32>, two steps per launch" if two_step
                                else f"step_kernel<{storage.upper()}>, one step per launch"),
                     "achieved_gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                     "algorithmic_bytes_per_lu": alg,
                     "traffic": traffic, "alu": alu_roofline(kernel, n * n, mlups)}


def graph_leg(pkg, wl, timer, torch, n, m=100, reps=20, tr=0.7, width=10.0):
    """Small FP32 lattices, where launches rather than HBM or the ALU set
    the time per step: lbm_step(m * reps) in one call against a HIP graph of
    lbm_step(m), captured on the lattice's stream, replayed reps times on
    torch's current stream, where the eager calls run too."""
    d = pkg.lbm_derive(pkg.make_params(n, n, tr=tr, width=width))
    rho0 = wl.spinodal({"rho_g": d.rho_g, "rho_l": d.rho_l, "width": width}, n=n)
    eager_lat = pkg.Lattice(n, n, tr=tr, width=width).init(rho0)
    ms_eager = timer(lambda: eager_lat.step(m * reps), pre=lambda: eager_lat.step(m))
    eager_lat.close()
    s = torch.cuda.Stream()
    lat = pkg.Lattice(n, n, stream=s, tr=tr, width=width).init(rho0)
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        pkg.lbm.lbm_step(lat.ctx, m)
    torch.cuda.synchronize()

    def replays():
        for _ in range(reps):
            g.replay()

    ms_graph = timer(replays, pre=g.replay)
    tot = lat.moments(fields=False)
    del g
    lat.close()
    if not all(np.isfinite(tot)):
        raise RuntimeError(f"{n}^2 graph leg diverged")
    lu = n * n * m * reps
    eager, graph = lu / (ms_eager * 1e-3) / 1e6, lu / (ms_graph * 1e-3) / 1e6
    return {"lattice": f"{n}x{n} FP32 spinodal", "steps_per_graph": m, "replays": reps,
            "eager_mlups": round(eager, 1), "graph_mlups": round(graph, 1), "ratio": round(graph / eager, 4)}


def _semi_axis(profile, level):
    """Half the distance between the outer level crossings of a 1-D profile."""
    i = np.where(profile > level)[0]
    a, b = i.min(), i.max()
    lo = a - (profile[a] - level) / (profile[a] - profile[a - 1])
    hi = b + (profile[b] - level) / (profile[b] - profile[b + 1])
    return 0.5 * (hi - lo)


def field_bound(rho, ref, d):
    """Pointwise comparison of a density field with ref: the largest ratio
    of |rho - ref| to 1e-3 rho_l + 0.5 |grad ref| (the coexistence bound
    plus an interface displaced by half a lattice spacing), and the largest
    local interface displacement |rho - ref| / |grad ref| over nodes where
    ref lies in the middle 80 % of [rho_g, rho_l]."""
    import torch
    gx = 0.5 * (torch.roll(ref, -1, 1) - torch.roll(ref, 1, 1))
    gy = 0.5 * (torch.roll(ref, -1, 0) - torch.roll(ref, 1, 0))
    g = torch.sqrt(gx * gx + gy * gy)
    diff = (rho - ref).abs()
    span = d.rho_l - d.rho_g
    iface = (ref > d.rho_g + 0.1 * span) & (ref < d.rho_l - 0.1 * span)
    return (diff / (1e-3 * d.rho_l + 0.5 * g)).max().item(), (diff[iface] / g[iface]).max().item()


def coalescence_legs(pkg, wl, timer, nx=16384, ny=8192, steps=5000, warmup=20):
    """The largest workload: two R = 400 droplets 20 nodes apart on
    16384 x 8192 at T/T_c = 0.6 (9.7 GB of FP32 A/B buffers), its 5000 steps
    timed per storage (FP32: the two-step kernel, 36 B/LU), then the
    read-outs at t = 5000 of each 2-byte run against the FP32 run: field
    max |d rho| / rho_l, its largest ratio to the coexistence bound plus a
    half-node interface shift, the largest interface displacement, gap density, liquid bodies, the droplets' vertical semi-axes, liquid and
    gas densities."""
    from scipy import ndimage
    import torch
    d = pkg.lbm_derive(pkg.make_params(nx, ny, tr=0.6, width=10.0))
    rho0 = wl.coalescence({"rho_g": d.rho_g, "rho_l": d.rho_l, "width": 10.0}, nx, ny)
    level = 0.5 * (d.rho_l + d.rho_g)
    cx, cy = nx // 2, ny // 2
    out, ref = {}, None
    for storage in ("fp32", "fp16", "bf16"):
        lat = pkg.Lattice(nx, ny, tr=0.6, width=10.0, storage=storage).init(rho0)
        ms = timer(lambda: lat.step(steps), pre=lambda: lat.step(warmup))
        rho = lat.moments()[0]
        lat.close()
        per = ms / steps
        gbs = (STEP2_BYTES_PER_LU if storage == "fp32" else BYTES_PER_LU[storage]) * nx * ny / (per * 1e-3) / 1e9
        region = rho[cy - 600:cy + 600, cx - 1100:cx + 1100].double().cpu().numpy()
        lab, count = ndimage.label(region > level)
        sizes = ndimage.sum(np.ones_like(region), lab, range(1, count + 1))
        leg = {"mlups": round(nx * ny * steps / (ms * 1e-3) / 1e6, 1), "ms_per_step": round(per, 4),
               "achieved_gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4), "steps_timed": steps,
               "t5000": {"gap_density": float(rho[cy, cx]), "liquid_bodies": int(np.sum(np.asarray(sizes) > 20)),
                         "semi_axes": [round(_semi_axis(rho[:, x].double().cpu().numpy(), level), 4)
                                       for x in (cx - 410, cx + 410)],
                         "liquid_density": [float(rho[cy, x]) for x in (cx - 410, cx + 410)],
                         "gas_density": float(rho[0, 0])}}
        if ref is None:
            ref = rho
        else:
            leg["t5000"]["max_drho_vs_fp32_rel_rho_l"] = float((rho - ref).abs().max().item() / d.rho_l)
            ratio, disp = field_bound(rho, ref, d)
            leg["t5000"]["max_drho_over_coexistence_bound_plus_half_node_shift"] = ratio
            leg["t5000"]["interface_max_displacement_vs_fp32"] = disp
            del rho
        out[storage] = leg
        torch.cuda.empty_cache()
    return out


def ellipse_leg(pkg, wl, n=512, tr=0.6, width=10.0, s_p=1.4, every=100, nsamp=600):
    """Oscillation of an elliptic droplet (semi-axes 96.0 and 42.7): period
    from the late zero crossings of a_x - a_y against the linear capillary
    mode n = 2, omega^2 = 6 sigma / ((rho_l + rho_g) R^3)."""
    d = pkg.lbm_derive(pkg.make_params(n, n, tr=tr, width=width, s_p=s_p))
    rho0 = wl.ellipse(n, n, d.rho_g, d.rho_l, width, (n / 2, n / 2), 96.0, 42.7)
    lat = pkg.Lattice(n, n, tr=tr, width=width, s_p=s_p).init(rho0)
    level = 0.5 * (d.rho_l + d.rho_g)

    def semi(pr):
        i = np.where(pr > level)[0]
        a, b = i.min(), i.max()
        return 0.5 * ((b + (pr[b] - level) / (pr[b] - pr[b + 1])) - (a - (pr[a] - level) / (pr[a] - pr[a - 1])))

    dev = []
    for _ in range(nsamp):
        lat.step(every)
        r = lat.moments()[0].double().cpu().numpy()
        dev.append(semi(r[n // 2]) - semi(r[:, n // 2]))
    lat.close()
    cross = [every * (i + 1) + every * dev[i] / (dev[i] - dev[i + 1]) for i in range(nsamp - 1)
             if (dev[i] > 0) != (dev[i + 1] > 0)]
    period = 2 * float(np.mean(np.diff(cross)[-3:]))
    analytic = 2 * np.pi * np.sqrt((d.rho_l + d.rho_g) * (96.0 * 42.7) ** 1.5 / (6 * d.sigma))
    return {"workload": f"elliptic droplet 96.0 x 42.7 on {n}^2, T/Tc={tr}, W={width}, s_p={s_p}",
            "period_steps": round(period, 1), "analytic_steps": round(float(analytic), 1),
            "rel_err": round(period / analytic - 1, 5)}


# Head-on collision regimes: We, Re, the dimensionless end time t* = t U / D,
# and the outcome the paper describes.
HEAD_ON = {"a": (0.01, 1.0, 2.5, "merge"), "b": (0.1, 1.0, 6.0, "bounce"),
           "c": (20.0, 100.0, 12.0, "merge, large deformation"),
           "d": (60.0, 200.0, 20.0, "two droplets and a central satellite")}


def head_on_leg(pkg, wl, n=1024, diameter=128.0, gap=60.0, tr=0.7, width=10.0, nsamp=12):
    """Head-on collision of equal droplets (1024^2, D = 128, T_r = 0.7,
    W = 10) at the four (We, Re) pairs of the paper: the number of liquid
    bodies (rho above the mean of the coexistence densities, 4-connected)
    at nsamp times up to t*.  U from We = rho_l U^2 D / sigma, s_p from
    Re = U D / nu; the droplet surfaces start `gap` nodes apart."""
    from scipy import ndimage
    d = pkg.lbm_derive(pkg.make_params(n, n, tr=tr, width=width))
    level = 0.5 * (d.rho_l + d.rho_g)
    out = {"workload": f"head-on collision, {n}x{n}, D={diameter:g}, gap={gap:g}, T/Tc={tr}, W={width}"}
    for case, (We, Re, t_end, paper) in HEAD_ON.items():
        U = float(np.sqrt(We * d.sigma / (d.rho_l * diameter)))
        s_p = 1.0 / (3.0 * U * diameter / Re + 0.5)
        rho0, ux0, uy0 = wl.head_on(d, U, n=n, diameter=diameter, gap=gap)
        lat = pkg.Lattice(n, n, tr=tr, width=width, s_p=s_p).init(rho0, ux0, uy0)
        every = int(round(t_end * diameter / U / nsamp))
        bodies = []
        t0 = time.perf_counter()
        try:
            for _ in range(nsamp):
                lat.step(every)
                lab, count = ndimage.label(lat.moments()[0].cpu().numpy() > level)
                sizes = ndimage.sum(np.ones(lab.shape), lab, range(1, count + 1))
                bodies.append(int(np.sum(np.asarray(sizes) > 20)))
            status = "finite"
        except pkg.LbmError as e:
            status = f"diverged ({e})"
        lat.close()
        out[case] = {"We": We, "Re": Re, "U": round(U, 6), "s_p": round(s_p, 4), "t_star": t_end,
                     "steps": every * nsamp, "bodies": bodies, "status": status, "paper": paper,
                     "s": round(time.perf_counter() - t0, 1)}
    return out


def coexistence_leg(pkg, wl, storage, tr=0.7, width=10.0, ny=128, steps=20000):
    """Flat interface relaxed for `steps` steps: bulk densities against the
    Maxwell construction of the library's host map, |d rho| / rho_l."""
    d = pkg.lbm_derive(pkg.make_params(4, ny, tr=tr, width=width))
    rho0 = wl.flat_slab(4, ny, d.rho_g, d.rho_l, width / wl.TANH_WIDTH_FACTOR)
    lat = pkg.Lattice(4, ny, tr=tr, width=width, storage=storage).init(rho0).step(steps)
    rho = lat.moments()[0].double().mean(1).cpu().numpy()
    lat.close()
    liq, gas = rho[0], rho[ny // 2]  # plateau centres, ny/4 from the interfaces
    return {"rho_l_err": float(abs(liq - d.rho_l) / d.rho_l), "rho_g_err": float(abs(gas - d.rho_g) / d.rho_l),
            "rho_g_err_rel_rho_g": float(abs(gas - d.rho_g) / d.rho_g), "steps": steps, "lattice": f"4x{ny}"}


def fwd_adjoint_leg(pkg, wl, timer, torch, n=2048, steps=1000, every=100):
    """Checkpointed forward + adjoint of the droplet-pair crop, whole job
    (every = 1 keeps every state: no recomputation).  Timed on a second run,
    the first having allocated the checkpoint and segment buffers."""
    tr, width = 0.6, 10.0
    need = (steps // every + 2 * every + 6) * 36 * n * n
    torch.cuda.empty_cache()
    free = torch.cuda.mem_get_info()[0]
    if need > 0.9 * free:
        return {"skipped": f"needs {need / 2**30:.1f} GiB of device memory, {free / 2**30:.1f} GiB free"}
    d = pkg.lbm_derive(pkg.make_params(n, n, tr=tr, width=width))
    rho0 = wl.coalescence({"rho_g": d.rho_g, "rho_l": d.rho_l, "width": width}, nx=n, ny=n)
    r = pkg.Rollout(n, n, steps, every, tr=tr, width=width)
    rho0_dev = torch.tensor(rho0, dtype=torch.float32, device="cuda")
    out = {}
    for _ in range(2):  # the first run allocates the checkpoint and segment buffers; the second is timed
        t_f = timer(lambda: r.forward(rho0_dev))
        grad = 2.0 * (r.lat.moments()[0] - rho0_dev)
        t_b = timer(lambda: out.update(zip(("drho0", "dth", "dp"), r.backward(grad))))
    r.release()
    if not np.all(np.isfinite(out["dth"])):
        raise RuntimeError("adjoint diverged")
    return {"workload": f"droplet pair R=400, gap 20, {n}x{n} crop, T/Tc={tr}, W={width}",
            "steps": steps, "checkpoint_every": every,
            "mlups": round(n * n * steps / ((t_f + t_b) * 1e-3) / 1e6, 1),
            "ms_forward": round(t_f, 3), "ms_backward": round(t_b, 3)}


def adjoint_kernel_leg(pkg, wl, timer, torch, n=4096, reps=200, tr=0.7, width=10.0):
    """The adjoint step kernel alone on the 4096^2 spinodal workload (one
    forward checkpoint, alternating adjoint buffers)."""
    d = pkg.lbm_derive(pkg.make_params(n, n, tr=tr, width=width))
    rho0 = wl.spinodal({"rho_g": d.rho_g, "rho_l": d.rho_l, "width": width}, n=n)
    lat = pkg.Lattice(n, n, tr=tr, width=width).init(rho0).step(5)
    ck = lat.save_state()
    gen = torch.Generator(device="cuda").manual_seed(0)
    a = lat.adjoint_seed(torch.randn((9, n, n), device="cuda", generator=gen))
    b = lat.adjoint_buffer()

    def loop():
        x, y = a, b
        for _ in range(reps):
            lat.adjoint_step(ck, x, y)
            x, y = y, x

    loop()  # warm
    ms = timer(loop) / reps
    th = lat.adjoint_theta(reset=True)
    lat.close()
    if not np.all(np.isfinite(th)):
        raise RuntimeError("adjoint diverged")
    gbs = ADJ_BYTES_PER_LU * n * n / (ms * 1e-3) / 1e9
    gbs_min = ADJ_MIN_BYTES_PER_LU * n * n / (ms * 1e-3) / 1e9
    return {"workload": f"spinodal decomposition {n}x{n}, T/Tc={tr}, W={width}", "ms_per_step": round(ms, 5),
            "mlups": round(n * n / (ms * 1e-3) / 1e6, 1), "achieved_gbs": round(gbs, 1),
            "frac": round(gbs / HBM_PEAK_GBS, 4), "algorithmic_bytes_per_lu": ADJ_BYTES_PER_LU,
            "frac_on_lambda_and_state_bytes": round(gbs_min / HBM_PEAK_GBS, 4),
            "lambda_and_state_bytes_per_lu": ADJ_MIN_BYTES_PER_LU,
            "traffic": measured_traffic("adjoint_f32", n * n),
            "alu": alu_roofline("adjoint_f32", n * n, n * n / (ms * 1e-3) / 1e6)}


def gradient_error(pkg, wl, timer, torch):
    """Relative error of the fwd+adjoint directional derivatives of the 512^2
    droplet-to-ellipse loss against the stored exact values, and the rate of
    the second of two identical runs (the first allocates the buffers)."""
    try:
        with open(GOLDEN) as fh:
            g = json.load(fh)
    except (OSError, ValueError):
        return {"error": "golden values missing"}
    n, steps, tr, width, sigma = g["n"], g["nsteps"], g["tr"], g["width"], g["sigma"]
    d = pkg.lbm_derive(pkg.make_params(n, n, tr=tr, width=width, sigma=sigma))
    rho0 = wl.droplets(n, n, d.rho_g, d.rho_l, width, [(n / 2, n / 2)], [g["radius"]])
    target = wl.ellipse(n, n, d.rho_g, d.rho_l, width, (n / 2, n / 2), *g["semi_axes"])
    r = pkg.Rollout(n, n, steps, 100, tr=tr, width=width, sigma=sigma)
    rho0_dev = torch.tensor(rho0, dtype=torch.float32, device="cuda")
    target_dev = torch.tensor(target, device="cuda")
    res = {}

    def run():
        rho_T = r.forward(rho0_dev).double()
        res["loss"] = float(((rho_T - target_dev) ** 2).sum())
        res.update(zip(("drho0", "dth", "dp"), r.backward(2.0 * (rho_T - target_dev))))

    run()  # allocates the checkpoint and segment buffers; the timed run reuses them
    ms = timer(run)
    r.release()
    drho0 = res["drho0"].double().cpu().numpy()
    errs = {}
    for name, e in g["directions"].items():
        seed = int(name[4:]) if name.startswith("seed") else None
        v = float(np.dot(res["dp"], e["param"]))
        if e["rho0"]:
            rng = np.random.default_rng(seed)
            v += float((drho0 * rng.standard_normal((n, n)) * (d.rho_l - d.rho_g) / n).sum())
        errs[name] = abs(v - e["value"]) / abs(e["value"])
    return {"workload": f"droplet R={g['radius']:g} -> ellipse {g['semi_axes']}, {n}x{n}, T/Tc={tr}, "
                        f"{steps} steps, K=100",
            "max_rel_err": max(errs.values()), "per_direction": errs,
            "loss_rel_err": abs(res["loss"] - g["loss"]) / g["loss"], "ms_fwd_adj": round(ms, 2),
            "mlups": round(n * n * steps / (ms * 1e-3) / 1e6, 1)}


def cpu_baseline(rho_full, tr, width, crop=1024, budget_s=20.0):
    """The FP64 oracle (as it stands) on a crop of the same initial field:
    whole steps of the dense per-node form until `budget_s` has passed, with
    its thread pools pinned to one thread (its array operations are single-
    threaded NumPy)."""
    from threadpoolctl import threadpool_limits
    sys.path.insert(0, ROOT)
    from oracle import hostmap as hm
    from oracle import lbm as olbm
    co = hm.derive(hm.Params(tr=tr, width=width))
    rho = np.asarray(rho_full[:crop, :crop], np.float64)
    with threadpool_limits(limits=1):
        f = olbm.equilibrium(rho, co)
        t0 = time.perf_counter()
        n = 0
        while n == 0 or time.perf_counter() - t0 < budget_s:
            f = olbm.step(f, co)
            n += 1
        dt = time.perf_counter() - t0
    return {"value": round(crop * crop * n / dt / 1e6, 4), "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "host_cpu_count": os.cpu_count(),
            "sample": f"{crop}x{crop} crop of the same initial field, {n} dense FP64 steps in {dt:.1f} s "
                      f"on one thread of {os.cpu_count()} host CPUs"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--n", type=int, default=4096, help="lattice side (default: the 4096^2 workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only-fp32", action="store_true", help="skip the 2-byte and adjoint legs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(the lattice would shard as row slabs with a halo exchange per step)", file=sys.stderr)
        sys.exit(2)

    import torch
    sys.path.insert(0, ROOT)
    import paper_1809_02390_amd as pkg
    import workloads as wl

    tr, width, n = 0.7, 10.0, args.n
    pacer = make_pacer(pkg, wl)
    timer = Timer(torch, pacer)
    t_wall = time.perf_counter()
    derived, rho0, fp32 = step_leg(pkg, wl, timer, "fp32", n, args.steps, args.warmup, tr, width)
    t_wall = time.perf_counter() - t_wall
    t_start = time.perf_counter()

    def done(what):
        print(f"bench.py: {what} done ({time.perf_counter() - t_start:.0f} s)", file=sys.stderr, flush=True)

    done("fp32 step leg")
    legs = {}
    _, _, single = step_leg(pkg, wl, timer, "fp32", n, args.steps, args.warmup, tr, width, single=True)
    legs["fp32_single_step"] = single
    done("fp32 single-step leg")
    if not args.only_fp32:
        for st in ("fp16", "bf16"):
            _, _, leg = step_leg(pkg, wl, timer, st, n, args.steps, args.warmup, tr, width)
            leg["ratio_vs_fp32"] = round(leg["mlups"] / fp32["mlups"], 4)
            leg["ratio_vs_fp32_single_step"] = round(leg["mlups"] / single["mlups"], 4)
            leg["coexistence"] = coexistence_leg(pkg, wl, st)
            legs[st] = leg
            done(f"{st} step leg")
        legs["graph_replay"] = [graph_leg(pkg, wl, timer, torch, k) for k in (256, 1024)]
        done("graph replay legs")
        legs["fp32_coexistence"] = coexistence_leg(pkg, wl, "fp32")
        legs["coalescence_16384x8192"] = coalescence_legs(pkg, wl, timer)
        done("16384x8192 legs")
        legs["elliptic_droplet"] = ellipse_leg(pkg, wl)
        done("elliptic droplet")
        legs["head_on_collision"] = head_on_leg(pkg, wl)
        done("head-on collisions")
        legs["fwd_adjoint"] = fwd_adjoint_leg(pkg, wl, timer, torch)
        legs["fwd_adjoint_keep_all_states"] = fwd_adjoint_leg(pkg, wl, timer, torch, every=1)
        done("forward + adjoint legs")
        legs["fwd_adjoint"]["adjoint_kernel"] = adjoint_kernel_leg(pkg, wl, timer, torch)
        legs["fwd_adjoint"]["gradient"] = gradient_error(pkg, wl, timer, torch)
        done("adjoint kernel and gradient legs")
    pacer.close()

    out = {
        "metric": METRIC,
        "value": fp32["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": fp32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"spinodal decomposition {n}x{n}, T/Tc={tr}, W={width}, "
                               f"sigma={derived.sigma:.6g}", "nx": n, "ny": n, "storage": "fp32"},
        "roofline": headline_roofline(fp32),
        "legs": legs,
        "wall_s_fp32_leg": round(t_wall, 3),
        "lead_in": {"steps": timer.lead_in_steps, "lattice": "4096x4080 FP32, its own spinodal state",
                    "note": "untimed steps of another lattice enqueued right before each timed region"},
        "paper_figures": {"relative_cost_vs_pseudopotential_mrt": 1.178,
                          "source": "supplement Sec. IV: cost of the model relative to the pseudopotential MRT "
                                    "model of Li et al.; hardware, precision and workload not stated",
                          "absolute_rates": None},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(rho0, tr, width)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
