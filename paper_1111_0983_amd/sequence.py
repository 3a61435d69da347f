"""3D projection-style sequence: one pressure solve per step of a moving ellipsoidal tank.

Every step builds the hierarchy of the tank's current position (mg_setup), takes the
previous step's solution as the initial iterate (mg_warm_start extrapolates it linearly to
the nodes the boundary has moved over), and solves with FP32 cycles inside FP64 defect
correction to the tolerance.  Inputs come from workloads/tank.py; every arithmetic step of the solve runs in
the HIP library.

  python -m paper_1111_0983_amd.sequence --steps 4 --n 384
"""
from __future__ import annotations

import time

import torch

from . import ghostmg as gm


def run(steps: int = 4, n: int = 384, n_coarse: int = 24, warm: bool = True,
        tol: float = 1e-10, precision: int = gm.MG_FP32_DC, device: str = "cuda:0",
        keep_last: bool = False, start: int = 0, log=print) -> dict:
    """Returns per-step setup seconds, solve milliseconds, cycles, residuals (and, with
    keep_last, the last step's phi, f and solution)."""
    from workloads import tank

    seq = tank.TankSequence(n)
    rows = dict(setup_s=[], solve_ms=[], cycles=[], outer=[], rel=[], unknowns=[])
    prev_u = prev_s = None
    out = {}
    for t in range(start, start + steps):
        t0 = time.perf_counter()
        phi = seq.phi(t, device)
        s = gm.Solver(phi, [seq.rule],
                      gm.mg_grid_default(3, n, n_coarse, precision=precision, inner_cycles=3,
                                         max_cycles=300))
        c = torch.from_numpy(s.classes()).to(device)
        f = torch.where(c == 1, seq.f(t, device), torch.zeros((), dtype=torch.float64,
                                                               device=device)).contiguous()
        g = torch.zeros_like(f)
        setup = time.perf_counter() - t0
        u = torch.zeros_like(f)
        if warm and prev_u is not None:
            u.copy_(prev_u)
            s.warm_start(prev_s, u)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        info = s.solve(f, g, u, tol=tol)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t1)
        rows["setup_s"].append(setup)
        rows["solve_ms"].append(ms)
        rows["cycles"].append(info["cycles"])
        rows["outer"].append(info["outer"])
        rows["rel"].append(info["rel"])
        rows["unknowns"].append(int((c > 0).sum().item()))
        if log:
            log(f"[sequence] step {t}: setup {setup:.1f}s, solve {ms:.1f} ms, "
                f"{info['cycles']} cycles, rel {info['rel']:.2e}")
        if prev_s is not None:
            prev_s.close()
        prev_u, prev_s = u, s
        if keep_last and t == start + steps - 1:
            out["phi"], out["f"], out["u"] = phi, f, u
    if prev_s is not None:
        prev_s.close()
    out.update(rows)
    return out


def main(argv=None):
    import argparse
    import json

    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--n", type=int, default=384)
    ap.add_argument("--cold", action="store_true", help="zero initial iterate at every step")
    args = ap.parse_args(argv)
    res = run(args.steps, args.n, warm=not args.cold)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
