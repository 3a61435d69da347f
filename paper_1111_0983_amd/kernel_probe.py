"""Launch one kernel of the multigrid cycle in isolation, for hardware-counter profiles.

Builds the tank workload (step 0 of the 384^3 sequence, FP32 cycles in FP64 defect
correction: the benchmark's headline) or the 2D flower, then launches the requested kernel
`--reps` times at one level through mg_time_kernel, and finally copies a buffer of
known size `--copy-mb` MiB with torch (three launches), whose FETCH_SIZE / WRITE_SIZE
readings calibrate the counters (bytes read = bytes written = the buffer size).  The
default 2 GiB is far larger than the 256 MiB last-level cache, so the copy's reads all
reach HBM.

  python -m paper_1111_0983_amd.kernel_probe --workload tank --kernel relax --level 0
"""
from __future__ import annotations

import argparse
import json
import sys


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--kernel", default="relax",
                    choices=["relax", "defect", "restrict", "prolong", "residual",
                             "relax_prolong", "relax_restrict", "coarse"])
    ap.add_argument("--level", type=int, default=0)
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--workload", choices=["tank", "flower"], default="tank")
    ap.add_argument("--n", type=int, default=0, help="grid (default 384 tank, 2048 flower)")
    ap.add_argument("--nc", type=int, default=0, help="coarsest grid (default 24 / 128)")
    ap.add_argument("--fp32", action="store_true", help="flower: FP32 cycles (the tank always)")
    ap.add_argument("--copy-mb", type=int, default=2048)
    args = ap.parse_args(argv)

    import torch

    from paper_1111_0983_amd import ghostmg as gm
    from workloads import problems as pr

    if args.workload == "tank":
        from workloads import tank

        n, nc = args.n or 384, args.nc or 24
        seq = tank.TankSequence(n)
        grid = gm.mg_grid_default(3, n, nc, precision=gm.MG_FP32_DC, inner_cycles=3)
        s = gm.Solver(seq.phi(0, "cuda"), [seq.rule], grid)
    else:
        n, nc = args.n or 2048, args.nc or 128
        w = pr.flower(n, nc)
        phi = w.domain.nodal_phi(n)
        grid = gm.mg_grid_default(2, n, nc,
                                  precision=gm.MG_FP32_DC if args.fp32 else gm.MG_FP64)
        s = gm.Solver(torch.from_numpy(phi).cuda(), [w.rule], grid)
    ms, nbytes = s.time_kernel(args.kernel, args.level, args.reps)
    info = s.level(args.level)
    n = args.copy_mb * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"kernel": args.kernel, "level": args.level, "avg_ms": ms,
                      "algorithmic_bytes": nbytes, "GBs": nbytes / (ms * 1e-3) / 1e9,
                      "level_info": info, "copy_bytes": n * 4}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
