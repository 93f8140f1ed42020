"""Shared helpers of the GPU tests: run the HIP path and the oracle on the
same seeded input and compare."""
from __future__ import annotations

import numpy as np
import torch

import paper_1809_02390_amd as pkg
from oracle import hostmap as hm
from oracle import lbm


def params_pair(nx, ny, **kw):
    """Library params and the oracle's coefficients for the same problem."""
    p = pkg.make_params(nx, ny, **kw)
    sigma = kw.get("sigma", 0.0)
    s_eps = kw.get("s_eps", 0.0)
    co = hm.derive(hm.Params(nx=nx, ny=ny, s_p=kw.get("s_p", 1.0), s_eps=s_eps if s_eps > 0 else None,
                             varpi=kw.get("varpi", 1 / 6), a=kw.get("a", 1.0), b=kw.get("b", 4.0),
                             r_gas=kw.get("r_gas", 1.0), tr=kw.get("tr", 0.8),
                             sigma=sigma if sigma > 0 else None, width=kw.get("width", 10.0)))
    return p, co


def lattice(nx, ny, rho0, ux0=None, uy0=None, **kw):
    lat = pkg.Lattice(nx, ny, **kw)
    lat.init(rho0, ux0, uy0)
    return lat


def oracle_init(co, rho0, ux0=None, uy0=None):
    """The oracle's initial state from the same float32-rounded inputs."""
    f32 = lambda a: None if a is None else np.asarray(a, np.float32).astype(np.float64)
    return lbm.equilibrium(f32(rho0), co, f32(ux0), f32(uy0))


def crop_periodic(a, cx, cy, half):
    """(2 half + 1)^2 crop of the last two axes of a, centred on (cx, cy),
    taken with periodic wrap."""
    ny, nx = a.shape[-2:]
    ys = np.arange(cy - half, cy + half + 1) % ny
    xs = np.arange(cx - half, cx + half + 1) % nx
    if isinstance(a, torch.Tensor):
        ys, xs = (torch.as_tensor(v, device=a.device) for v in (ys, xs))
    return a[..., ys[:, None], xs[None, :]]


def sampled_oracle(co, rho0, points, nsteps):
    """Oracle f at each sample point after nsteps, from light-cone crops of the
    initial field (dependence radius 2 nodes per step, plus a margin)."""
    half = 2 * nsteps + 3
    out = []
    for (x, y) in points:
        crop = crop_periodic(np.asarray(rho0, np.float64), x, y, half)
        f = lbm.run(lbm.equilibrium(crop, co), co, nsteps, lbm.collide_sequence)
        out.append(f[:, half, half])
    return np.array(out)


def sampled_oracle_moments(co, rho0, points, nsteps):
    """Oracle rho, u_x, u_y (main Eq. 5) at each sample point after nsteps,
    from the same light-cone crops as sampled_oracle (the force stencil
    reads one node beyond the point, inside the crop's valid region)."""
    half = 2 * nsteps + 3
    out = []
    for (x, y) in points:
        crop = crop_periodic(np.asarray(rho0, np.float64), x, y, half)
        f = lbm.run(lbm.equilibrium(crop, co), co, nsteps, lbm.collide_sequence)
        r, u, v = lbm.macroscopic(f, co)
        out.append((r[half, half], u[half, half], v[half, half]))
    return np.array(out)


def device_samples(f_dev, points):
    """f at the sample points from a device state tensor (9, ny, nx)."""
    xs = torch.tensor([p[0] for p in points], device=f_dev.device)
    ys = torch.tensor([p[1] for p in points], device=f_dev.device)
    return f_dev[:, ys, xs].T.double().cpu().numpy()


def fp32_state_of(buf, nx, ny):
    """The nine populations (9, ny*nx) held by an FP32 state or checkpoint
    buffer.  Its internal layout interleaves rows: population i of node
    (x, y) at element (9 y + i) nx + x; the rest of the buffer holds no
    data."""
    n = nx * ny
    return buf[: 9 * n * 4].view(torch.float32).view(ny, 9, nx).permute(1, 0, 2).reshape(9, n)


def adj_state_of(buf, nx, ny):
    """The eleven fields (11, ny*nx) of an adjoint state buffer (L_0..L_8,
    A_x, A_y): rows interleaved (field i of node (x, y) at element
    (11 y + i) nx + x) when 44 nx ny < 2^32, else eleven padded planes."""
    n = nx * ny
    if 44 * n <= 0xFFFFFFFF:
        return buf[: 11 * n * 4].view(torch.float32).view(ny, 11, nx).permute(1, 0, 2).reshape(11, n)
    return planes_of(buf, nx, ny, 11)


def planes_of(buf, nx, ny, nplanes, es=4):
    """The nplanes data regions (nplanes, ny*nx) of an internal byte buffer
    in plane layout (adjoint states of lattices too large for interleaved
    rows): planes P elements apart,
    with P = nx*ny rounded up to 64 plus 16640 bytes' worth of elements
    (include/lbm.h); the padding between planes holds no data."""
    p = -(-nx * ny // 64) * 64 + 16640 // es
    dtype = torch.float32 if es == 4 else torch.int16
    return buf[: nplanes * p * es].view(dtype).reshape(nplanes, p)[:, : nx * ny]
