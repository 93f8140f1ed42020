"""Ablation of the reference of the 2-byte storages, on the CPU.

The FP64 oracle runs the 4 x 128 flat interface (T_r = 0.7, W = 10, 20000
steps, the coexistence workload), and after every step each population is
replaced by what a 2-byte storage returns for it:

    f_i <- f_ref,i + round16(S (f_i - f_ref,i)) / S

with binary16 (S = 2^12) or bfloat16 (S = 1), round to nearest even.  Two
references:

  global  one rest equilibrium f^eq(rho_bar, eta(rho_bar), u = 0) for the
          whole lattice, rho_bar = (rho_g + rho_l)/2 (36 bytes per update);
  local   the rest equilibrium at rho~ = binary16(rho(x)) of the node's
          previous density, with the exact eta(rho~) (40 bytes per update;
          the library fits eta by a cubic, which changes only how far the
          reference is from f).

Prints the bulk densities' offsets from the unrounded run and from the
Maxwell construction, in units of rho_l.  Run by hand:

    python tests/ablation/storage_reference.py

(about 2.5 minutes on one core).  Test infrastructure: it uses the oracle
only.
"""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
import workloads as wl  # noqa: E402
from oracle import hostmap as hm  # noqa: E402
from oracle import lbm  # noqa: E402


def round_bf16(x):
    """Round FP64 values to bfloat16 (nearest even) via binary32."""
    a = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((a + 0x7FFF + ((a >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def round16(x, fmt):
    return x.astype(np.float16).astype(np.float64) if fmt == "fp16" else round_bf16(x)


def rest_equilibrium(rho, co):
    """f^eq(rho, eta(rho), u = 0) for a density field (ny, nx)."""
    return lbm.equilibrium(rho, co)


def run(co, fmt=None, reference=None, ny=128, steps=20000):
    rho0 = wl.flat_slab(4, ny, co.rho_g, co.rho_l, co.width / wl.TANH_WIDTH_FACTOR)
    f = lbm.equilibrium(rho0, co)
    S = 4096.0 if fmt == "fp16" else 1.0
    if reference == "global":
        ref = rest_equilibrium(np.full((1, 1), 0.5 * (co.rho_g + co.rho_l)), co)
    for _ in range(steps):
        rho_prev = f.sum(0)
        f = lbm.step(f, co)
        if fmt is None:
            continue
        if reference == "local":
            ref = rest_equilibrium(rho_prev.astype(np.float16).astype(np.float64), co)
        f = ref + round16(S * (f - ref), fmt) / S
    rho = f.sum(0).mean(1)
    return rho[0], rho[ny // 2]  # plateau centres, ny/4 from the interfaces


def main():
    co = hm.derive(hm.Params(tr=0.7, width=10.0))
    base_l, base_g = run(co)
    print(f"FP64: rho_l {base_l:.8f}, rho_g {base_g:.8f}  (Maxwell {co.rho_l:.8f}, {co.rho_g:.8f})")
    for reference in ("global", "local"):
        for fmt in ("fp16", "bf16"):
            l, g = run(co, fmt, reference)
            print(f"{reference:6s} {fmt}: |d rho_l| / rho_l = {abs(l - base_l) / co.rho_l:.2e}, "
                  f"|d rho_g| / rho_l = {abs(g - base_g) / co.rho_l:.2e} (vs the unrounded run)", flush=True)


if __name__ == "__main__":
    main()
