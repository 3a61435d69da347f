"""Launch one kernel of the multigrid cycle in isolation, for hardware-counter profiles.

Builds the flower workload (the headline benchmark problem), then launches the requested
kernel `--reps` times at one level through mg_time_kernel, and finally copies a buffer of
known size `--copy-mb` MiB with torch (three launches), whose FETCH_SIZE / WRITE_SIZE
readings calibrate the counters (bytes read = bytes written = the buffer size).  The
default 2 GiB is far larger than the 256 MiB last-level cache, so the copy's reads all
reach HBM.

  python -m paper_1111_0983_amd.kernel_probe --kernel relax --level 0
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
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--nc", type=int, default=128)
    ap.add_argument("--fp32", action="store_true")
    ap.add_argument("--copy-mb", type=int, default=2048)
    args = ap.parse_args(argv)

    import numpy as np
    import torch

    from paper_1111_0983_amd import ghostmg as gm
    from workloads import problems as pr

    w = pr.flower(args.n, args.nc)
    phi = w.domain.nodal_phi(args.n)
    grid = gm.mg_grid_default(2, args.n, args.nc,
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
