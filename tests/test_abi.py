"""The C-ABI library loads, exports every symbol its header declares, and its
host-only parameter map agrees with the oracle.  CPU only: nothing here
launches a kernel."""
import ctypes
import os
import re

import pytest

import paper_1809_02390_amd as pkg
from oracle import hostmap as hm
from paper_1809_02390_amd import lbm as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", src))
    return names


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert {"lbm_create", "lbm_step", "lbm_moments", "lbm_init", "lbm_destroy"} <= names
    lib = ctypes.CDLL(L._LIB_PATH)
    for n in sorted(names):
        assert hasattr(lib, n), f"{n} declared in include/ but not exported"
    assert names <= set(L.EXPORTED), "binding does not wrap every declared entry point"


def test_struct_layouts_match_header():
    assert ctypes.sizeof(L.lbm_params) == 4 * 4 + 9 * 8
    assert ctypes.sizeof(L.lbm_derived) == 22 * 8


@pytest.mark.parametrize("tr,width,sigma", [(0.8, 10.0, None), (0.7, 10.0, None), (0.6, 10.0, None),
                                            (0.9, 8.0, 2e-3), (0.5, 30.0, 5e-3), (0.75, 15.0, 1e-2)])
def test_host_map_matches_oracle(tr, width, sigma):
    lib = pkg.lbm_derive(pkg.make_params(32, 32, tr=tr, width=width, sigma=sigma or 0.0, s_p=0.8))
    ora = hm.derive(hm.Params(tr=tr, width=width, sigma=sigma, s_p=0.8))
    for name, ref in [("rho_g", ora.rho_g), ("rho_l", ora.rho_l), ("p0", ora.p0), ("c_sigma", ora.c_sigma),
                      ("c_w", ora.c_w), ("sigma", ora.sigma), ("k_int", ora.k_int), ("k_eos", ora.k_eos),
                      ("g2", ora.G2), ("kp", ora.Kp), ("rt", ora.RT), ("beta2", ora.beta2), ("k", ora.k),
                      ("h", ora.h), ("bs", ora.bs), ("s_q", ora.s_q), ("s_e", ora.s_e), ("s_eps", ora.s_eps)]:
        assert getattr(lib, name) == pytest.approx(ref, rel=1e-10), name


def test_sigma_paper_matches_oracle():
    for tr in (0.9, 0.8, 0.7, 0.6, 0.5):
        assert pkg.lbm_sigma_paper(10.0, tr) == pytest.approx(hm.sigma_paper(10.0, tr), rel=1e-10)


@pytest.mark.parametrize("bad", [dict(nx=0), dict(ny=-3), dict(s_p=2.0), dict(s_p=0.0), dict(tr=1.0),
                                 dict(tr=0.0), dict(varpi=1.0), dict(varpi=1 / 3), dict(width=0.0),
                                 dict(a=-1.0), dict(storage=7), dict(nx=20000, ny=20000)])
def test_invalid_parameters_rejected(bad):
    kw = dict(nx=16, ny=16)
    kw.update(bad)
    nx, ny = kw.pop("nx"), kw.pop("ny")
    with pytest.raises(pkg.LbmError) as e:
        pkg.lbm_derive(pkg.make_params(nx, ny, **kw))
    assert e.value.status == L.LBM_EINVAL
    assert "invalid parameter" in pkg.lbm_last_error()
    assert pkg.lbm_state_bytes(pkg.make_params(nx, ny, **kw)) == 0


def plane(nx, ny, es):
    """P of the internal buffer sizes (9 P or 11 P elements): nx*ny rounded
    up to 64 plus a 16640-byte pad (include/lbm.h)."""
    return -(-nx * ny // 64) * 64 + 16640 // es


def test_buffer_sizes():
    p = pkg.make_params(100, 30)
    assert pkg.lbm_state_bytes(p) == 9 * plane(100, 30, 4) * 4
    assert pkg.lbm_ref_bytes(p) == 0
    p16 = pkg.make_params(100, 30, storage="fp16")
    assert pkg.lbm_state_bytes(p16) == 9 * plane(100, 30, 2) * 2
    assert pkg.lbm_ref_bytes(p16) == 2 * 100 * 30 * 2


def test_largest_lattice_accepted():
    """9 nx ny < 2^31 is the size limit: 16384 x 14563 (9 nx ny = 2147401728)
    is accepted, one row more is not."""
    assert pkg.lbm_state_bytes(pkg.make_params(16384, 14563)) == 9 * plane(16384, 14563, 4) * 4
    assert pkg.lbm_state_bytes(pkg.make_params(16384, 14564)) == 0


def test_null_context_rejected():
    assert L._lib.lbm_step(None, 1) == L.LBM_EINVAL
    assert L._lib.lbm_time(None) == -1


def test_checkpoint_and_adjoint_sizes():
    p = pkg.make_params(100, 30)
    assert pkg.lbm_checkpoint_bytes(p) == 9 * plane(100, 30, 4) * 4
    assert pkg.lbm_adjoint_bytes(p) == 11 * plane(100, 30, 4) * 4
    p16 = pkg.make_params(100, 30, storage="bf16")
    assert pkg.lbm_checkpoint_bytes(p16) == 9 * plane(100, 30, 2) * 2 + 100 * 30 * 2
    assert pkg.lbm_adjoint_bytes(p16) == 0  # the adjoint is FP32-only
    assert pkg.lbm_checkpoint_bytes(pkg.make_params(0, 3)) == 0


def test_adjoint_calls_without_context_rejected():
    assert L._lib.lbm_adjoint_step(None, None, None, None) == L.LBM_EINVAL
    assert L._lib.lbm_adjoint_theta(None, None, 1) == L.LBM_EINVAL
    assert L._lib.lbm_save_state(None, None) == L.LBM_EINVAL


@pytest.mark.parametrize("tr,width,sigma", [(0.8, 10.0, None), (0.7, 10.0, 1.8e-3), (0.6, 14.0, 3e-3)])
def test_param_jacobian_against_oracle_map(tr, width, sigma):
    """d(G'^2, K', RT)/d(sigma, W, T_r) of the library against central
    differences of the oracle's own parameter map (FP64)."""
    p = pkg.make_params(16, 16, tr=tr, width=width, sigma=sigma or 0.0)
    jac = pkg.lbm_param_jacobian(p)
    s0 = pkg.lbm_derive(p).sigma  # the sigma the context uses, held independent

    def theta(s, w, t):
        co = hm.derive(hm.Params(tr=t, width=w, sigma=s))
        return [co.G2, co.Kp, co.RT]

    x0 = [s0, width, tr]
    for j in range(3):
        h = 1e-4 * x0[j]
        xp, xm = list(x0), list(x0)
        xp[j] += h
        xm[j] -= h
        num = [(a - b) / (2 * h) for a, b in zip(theta(*xp), theta(*xm))]
        for k in range(3):
            assert jac[k][j] == pytest.approx(num[k], rel=1e-6, abs=1e-12), (k, j)
