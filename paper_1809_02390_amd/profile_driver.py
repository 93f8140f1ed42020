"""Fixed workload for hardware-counter profiling (run under rocprofv3).

Runs, on the current GPU:
  1. a plain device-to-device copy of ``--copy-mib`` MiB, ``--copies`` times
     (the runtime's copy kernel: reads and writes exactly that many bytes),
     used to calibrate the FETCH_SIZE / WRITE_SIZE counters;
  2. ``--steps`` steps of one library kernel on the 4096 x 4096 spinodal
     workload (T/T_c = 0.7, W = 10):
       --what step     lbm_step(steps) with the chosen --storage (FP32: the
                       two-step kernel, steps / 2 launches);
       --what step1    FP32 single steps, one lbm_step(1) call each (the
                       one-step kernel);
       --what adjoint  the FP32 adjoint step (forward state of the workload,
                       seeded adjoint, alternating adjoint buffers).

Example:
    rocprofv3 --pmc FETCH_SIZE -d out -o pmc -- python -m paper_1809_02390_amd.profile_driver
"""
from __future__ import annotations

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--storage", default="fp32")
    ap.add_argument("--what", choices=("step", "step1", "adjoint"), default="step")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--copies", type=int, default=3)
    args = ap.parse_args()

    import torch
    sys.path.insert(0, ROOT)
    import paper_1809_02390_amd as pkg
    import workloads as wl

    a = torch.empty(args.copy_mib << 20, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    for _ in range(args.copies):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b

    n, tr, width = args.n, 0.7, 10.0
    d = pkg.lbm_derive(pkg.make_params(n, n, tr=tr, width=width))
    rho0 = wl.spinodal({"rho_g": d.rho_g, "rho_l": d.rho_l, "width": width}, n=n)
    storage = args.storage if args.what == "step" else "fp32"
    lat = pkg.Lattice(n, n, tr=tr, width=width, storage=storage).init(rho0)
    if args.what == "step":
        lat.step(args.steps)
    elif args.what == "step1":
        for _ in range(args.steps):
            lat.step(1)
    else:
        lat.step(5)
        ck = lat.save_state()
        gen = torch.Generator(device="cuda").manual_seed(0)
        lam = torch.randn((9, n, n), device="cuda", generator=gen)
        bufs = [lat.adjoint_seed(lam), lat.adjoint_buffer()]
        del lam
        for _ in range(args.steps):
            lat.adjoint_step(ck, bufs[0], bufs[1])
            bufs.reverse()
        lat.adjoint_theta(reset=True)
    torch.cuda.synchronize()
    print(f"profile_driver: copy {args.copies} x {args.copy_mib} MiB, {args.steps} x {args.what} of {n}x{n} "
          f"({storage})", flush=True)


if __name__ == "__main__":
    main()
