"""The allocation-free moments entry point (lbm_moments_noalloc) against
lbm_moments, through the C ABI: identical fields and totals on two calls in
a row, the second on a smaller lattice; oversized lattices are refused
before any launch."""
import numpy as np
import pytest
import torch

import paper_1809_02390_amd as pkg
import workloads as wl
from paper_1809_02390_amd import lbm as L
from tests._gpu_helpers import lattice, params_pair

pytestmark = pytest.mark.gpu


def _noalloc(lat):
    dev = lat.f_a.device
    rho, ux, uy = (torch.full((lat.ny, lat.nx), float("nan"), dtype=torch.float32, device=dev) for _ in range(3))
    tot = torch.full((3,), float("nan"), dtype=torch.float64, device=dev)
    L.lbm_moments_noalloc(lat.ctx, rho, ux, uy, tot, n=lat.n)
    torch.cuda.synchronize()
    return rho, ux, uy, tuple(tot.cpu().tolist())


@pytest.mark.parametrize("storage", ["fp32", "fp16"])
def test_noalloc_moments_match_moments_two_calls(storage):
    """Two calls in a row: 700 x 300 (231 workgroups, several tiles and a
    ragged tail), then 70 x 37; each against lbm_moments on the same state,
    bit for bit (the same kernels in the same order)."""
    for nx, ny, steps in ((700, 300, 30), (70, 37, 20)):
        _, co = params_pair(nx, ny, tr=0.7)
        rho0 = wl.droplets(nx, ny, co.rho_g, co.rho_l, co.width, [(nx * 0.4, ny * 0.5)], [min(nx, ny) * 0.3])
        lat = lattice(nx, ny, rho0, tr=0.7, storage=storage).step(steps)
        r_ref, u_ref, v_ref, tot_ref = lat.moments()
        r, u, v, tot = _noalloc(lat)
        assert torch.equal(r, r_ref) and torch.equal(u, u_ref) and torch.equal(v, v_ref)
        assert tot == tuple(tot_ref), (tot, tot_ref)
        assert np.isclose(tot[0], float(np.asarray(rho0, np.float32).astype(np.float64).sum()), rtol=1e-6)
        lat.close()


def test_noalloc_moments_refuse_oversized_lattice():
    """16384 x 5600 needs 89600 workgroups of partials, beyond the static
    2 MiB: LBM_EINVAL from the host check, nothing launched (the state is not
    even initialised)."""
    lat = pkg.Lattice(16384, 5600, tr=0.7, storage="fp16")
    out = torch.empty((5600, 16384), dtype=torch.float32, device="cuda")
    with pytest.raises(pkg.LbmError) as e:
        L.lbm_moments_noalloc(lat.ctx, out, None, None, None, n=lat.n)
    assert e.value.status == L.LBM_EINVAL and "static maximum" in str(e.value)
    lat.close()
