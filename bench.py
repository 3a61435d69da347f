"""Benchmark: unknowns/s to 1e-10 relative residual on one MI355X.

Workload (the single-GPU headline configuration): 2D flower r < 0.5 + 0.15 sin(5 theta)
on [-1, 1]^2 with 2048 x 2048 intervals, Dirichlet where x > 0 and Neumann elsewhere,
manufactured u = sin(3x) cos(2y) + x y, V(2,1) cycles with lambda = 5 boundary sweeps down
to a 128 x 128 coarsest grid (5 levels; --nc), zero initial guess, until
||r||_inf / ||(f_h, g_h)||_inf <= 1e-10.
One step = one complete solve (mg_solve) with inputs resident in HBM.

Prints one JSON line on stdout.  Extra fields: the FP32-in-FP64 defect-correction solve of
the same problem, the roofline of the dominant kernel (the fine-level red-black
relaxation) and the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "unknowns/s to 1e-10 rel. residual: plain FP64 vs FP32+learned guess; HBM GB/s"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def bench_torus(args, gm, pr, geo, np, torch, dev, step):
    """3D torus (R, r) = (0.5, 0.25) on [-1, 1]^3, Neumann where z < 0, Dirichlet where
    z >= 0, u = exp(x + y) cos(z), coarsest grid 16: FP64 cycles against FP32 cycles inside
    FP64 defect correction, both to 1e-10."""
    n = args.n3d
    w = pr.torus(n, 16)
    phi = w.domain.nodal_phi(n)
    out = {}
    ref = None
    for name, prec in (("fp64", gm.MG_FP64), ("fp32dc", gm.MG_FP32_DC)):
        grid = gm.mg_grid_default(3, n, 16, precision=prec, inner_cycles=2)
        t0 = time.time()
        s = gm.Solver(torch.from_numpy(phi).to(dev), [w.rule], grid)
        setup = time.time() - t0
        if ref is None:
            c = s.classes()
            G = s.ghosts()
            P = geo.grid_points(3, n)
            f = torch.from_numpy(np.where(c == 1, w.solution.f(P), 0.0)).to(dev)
            g = torch.from_numpy(pr.rhs_from_ghosts(3, n, c, G["node"], G["B"], G["type"],
                                                    w.solution, w.domain)).to(dev)
            unknowns = int((c > 0).sum())
        u = torch.zeros_like(f)
        for _ in range(args.warmup):
            info = step_fg(s, u, f, g)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            info = step_fg(s, u, f, g)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        if ref is None:
            ref = u.clone()
            err = float(np.abs(u.cpu().numpy() - w.solution.u(P))[c == 1].max())
            out["torus_max_error_vs_exact"] = err
        else:
            out["torus_fp32dc_vs_fp64_rel_diff"] = float((u - ref).abs().max() / ref.abs().max())
        out[f"torus_{name}_unknowns_per_s"] = unknowns / dt
        out[f"torus_{name}_ms"] = 1e3 * dt
        out[f"torus_{name}_cycles"] = info["cycles"]
        out[f"torus_{name}_rel_residual"] = info["rel"]
        out[f"torus_{name}_setup_s"] = setup
        log(f"[bench] torus {n}^3 {name}: {1e3 * dt:.1f} ms, {info['cycles']} cycles, "
            f"rel {info['rel']:.2e}, setup {setup:.1f}s")
        if name == "fp64":
            # every launch sequence of one FP64 cycle, per level (microseconds; a relaxation
            # is a tile launch plus one chunk launch per phase range)
            per_level = {}
            for lev in range(s.nlev - 1):
                names = ["relax_restrict" if lev > 0 else "relax", "relax", "defect", "relax_prolong"]
                per_level[str(lev)] = {k: round(s.time_kernel(k, lev, 5)[0] * 1e3, 1)
                                       for k in dict.fromkeys(names)}
            per_level[str(s.nlev - 1)] = {
                "coarse_with_restriction": round(s.time_kernel("coarse", s.nlev - 1, 5)[0] * 1e3, 1)}
            out["torus_fp64_launch_us_by_level"] = per_level
        s.close()
    out["torus_unknowns"] = unknowns
    out["torus_workload"] = f"torus-{n}^3 3D V(2,1) lambda=5 Nc=16 tol=1e-10"
    return out


def bench_learned(args, torch):
    """The learned-guess workload: ellipse-union problems at 512^2 (evaluation seeds), each
    solved on its own to 1e-10: FP64 and FP32-DC from the zero guess, FP32-DC and FP64 from
    the guess of the committed network (inference included)."""
    import numpy as np

    from paper_1111_0983_amd import cnn, learned
    from workloads import ellipses as el

    w = os.path.join(ROOT, "paper_1111_0983_amd", "weights", "guessnet.npz")
    net = cnn.GuessNet(seed=0)
    net.load(dict(np.load(w)))
    seeds, s = [], 1_000_000
    while len(seeds) < args.learned_problems:
        p = el.draw(s)
        if el.accept(el.nodal_phi(p, learned.N_FINE, device="cuda:0"), learned.N_FINE,
                     3.0 * 2.0 / learned.N_COARSE):
            seeds.append(s)
        s += 1
    s64, f, g, probs = learned.build_batch(seeds)
    s64.close()
    pp = learned.evaluate_each(net, probs, f, g, reps=2)
    out = {f"learned_{k}": round(v, 3) for k, v in pp.items() if k.endswith(("_mean", "_median"))}
    out["learned_problems"] = len(probs)
    out["learned_workload"] = "ellipse unions 512^2, Nc=32, per-problem solves to 1e-10"
    log(f"[bench] learned guess: zero FP64 {pp['zero64_cycles_mean']:.1f} cycles "
        f"{pp['zero64_ms_mean']:.2f} ms, zero FP32-DC {pp['zero_dc_cycles_mean']:.1f} cycles "
        f"{pp['zero_dc_ms_mean']:.2f} ms, learned FP32-DC {pp['learned_dc_cycles_mean']:.1f} "
        f"cycles {pp['learned_dc_ms_mean']:.2f} ms (means over {len(probs)} problems)")
    return out


def step_fg(solver, uu, f, g):
    uu.zero_()
    return solver.solve(f, g, uu, tol=1e-10)


def measured_traffic(summary: str):
    """HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE counter summary (each
    scaled by what the counter reads for a copy of known size), or None when the summary is
    missing or the kernel sources changed since the counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", summary)
    if not os.path.exists(path):
        return None
    rec = json.loads(open(path).read().strip().splitlines()[-1])
    h = hashlib.sha256()
    for f in ("kernels.hip", "setup.cpp"):
        h.update(open(os.path.join(ROOT, "paper_1111_0983_amd", "csrc", f), "rb").read())
    if h.hexdigest()[:16] != rec.get("source_sha"):
        return None
    return rec["traffic_bytes"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--nc", type=int, default=128, help="coarsest grid (intervals per axis)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dc", action="store_true")
    ap.add_argument("--no-3d", action="store_true")
    ap.add_argument("--n3d", type=int, default=256)
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--learned-problems", type=int, default=16)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the solver runs on a single MI355X)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1111_0983_amd import ghostmg as gm
    from workloads import geometry as geo, problems as pr

    dev = torch.device("cuda:0")
    n = args.n
    w = pr.flower(n, 32)
    t0 = time.time()
    phi = w.domain.nodal_phi(n)
    log(f"[bench] phi {n}^2 in {time.time() - t0:.1f}s")
    grid = gm.mg_grid_default(2, n, args.nc)
    t0 = time.time()
    s = gm.Solver(torch.from_numpy(phi).to(dev), [w.rule], grid)
    setup_s = time.time() - t0
    c = s.classes()
    G = s.ghosts()
    P = geo.grid_points(2, n)
    f = torch.from_numpy(np.where(c == 1, w.solution.f(P), 0.0)).to(dev)
    g = torch.from_numpy(pr.rhs_from_ghosts(2, n, c, G["node"], G["B"], G["type"],
                                            w.solution, w.domain)).to(dev)
    unknowns = int((c > 0).sum())
    u = torch.zeros_like(f)
    log(f"[bench] setup {setup_s:.2f}s, {unknowns} unknowns, {s.nlev} levels")

    def step(solver, uu):
        uu.zero_()
        info = solver.solve(f, g, uu, tol=1e-10)
        return info

    for _ in range(args.warmup):
        info = step(s, u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        info = step(s, u)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = 1e3 * dt / args.steps
    value = unknowns * args.steps / dt
    err = float(np.abs(u.cpu().numpy() - w.solution.u(P))[c == 1].max())
    log(f"[bench] FP64: {ms:.2f} ms/solve, {info['cycles']} cycles, rel {info['rel']:.2e}, "
        f"error vs exact {err:.2e}")

    # the same number of cycles queued as graph launches with a single read-back at the end:
    # the cycle itself, without the residual checks of the stopping test
    uc = torch.zeros_like(u)
    s.cycles(f, g, uc, info["cycles"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.cycles(f, g, uc, info["cycles"])
    torch.cuda.synchronize()
    cycle_us = 1e6 * (time.perf_counter() - t0) / info["cycles"]
    log(f"[bench] {info['cycles']} cycles queued at once: {cycle_us:.1f} us per cycle")

    # roofline of the dominant kernel: the fine-level relaxation (one launch: interior
    # tiles and the boundary chunks); the other launches of the cycle are timed alongside
    k_ms, k_bytes = s.time_kernel("relax", 0, 50)
    achieved = k_bytes / (k_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "kernel": "k_relax<2,double> (finest level)", "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic("k_relax_flower2048_level0_counters.txt"),
            "avg_us": round(k_ms * 1e3, 2), "bytes_per_launch": k_bytes}
    # the launches of one V(2,1) cycle on every level (microseconds): the first
    # pre-relaxation restricts (coarse levels), the first post-relaxation interpolates
    per_level = {}
    for lev in range(s.nlev - 1):
        row = {}
        names = ["relax_restrict" if lev > 0 else "relax", "relax", "defect", "relax_prolong"]
        for name in dict.fromkeys(names):
            ms_k, _ = s.time_kernel(name, lev, 20)
            row[name] = round(ms_k * 1e3, 2)
        per_level[str(lev)] = row
    # the coarsest level: the solve with the inverse, which restricts its right-hand side
    per_level[str(s.nlev - 1)] = {
        "coarse_with_restriction": round(s.time_kernel("coarse", s.nlev - 1, 20)[0] * 1e3, 2)}
    roof["launch_us_by_level"] = per_level
    log(f"[bench] k_relax level 0: {k_ms * 1e3:.2f} us, {achieved:.0f} GB/s; per level {per_level}")

    extra = {}
    if not args.no_dc:
        gdc = gm.mg_grid_default(2, n, args.nc, precision=gm.MG_FP32_DC, inner_cycles=2)
        sdc = gm.Solver(torch.from_numpy(phi).to(dev), [w.rule], gdc)
        udc = torch.zeros_like(f)
        for _ in range(args.warmup):
            idc = step(sdc, udc)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            idc = step(sdc, udc)
        torch.cuda.synchronize()
        dtdc = time.perf_counter() - t0
        diff = float((udc - u).abs().max().item() / u.abs().max().item())
        extra = {"fp32dc_unknowns_per_s": unknowns * args.steps / dtdc,
                 "fp32dc_ms_per_step": 1e3 * dtdc / args.steps,
                 "fp32dc_cycles": idc["cycles"], "fp32dc_outer": idc["outer"],
                 "fp32dc_rel_residual": idc["rel"], "fp32dc_vs_fp64_rel_diff": diff}
        log(f"[bench] FP32-DC: {1e3 * dtdc / args.steps:.2f} ms/solve, {idc['cycles']} FP32 "
            f"cycles in {idc['outer']} steps, diff vs FP64 {diff:.2e}")
        sdc.close()

    if not args.no_3d:
        extra.update(bench_torus(args, gm, pr, geo, np, torch, dev, step))
    if not args.no_learned:
        extra.update(bench_learned(args, torch))

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import Oracle, default_grid

        t0 = time.perf_counter()
        o = Oracle(phi, default_grid(2, n, args.nc), w.rule)
        oc, _ = o.cls(0)
        OG = o.ghosts(0)
        rhs = pr.rhs_from_ghosts(2, n, oc, OG["node"], OG["B"], OG["type"], w.solution, w.domain)
        t1 = time.perf_counter()
        st, uo, hist = o.solve(rhs, tol=1e-10, max_cycles=60)
        t2 = time.perf_counter()
        cpu = {"value": unknowns / (t2 - t1), "unit": "unknowns/s", "cores": 1, "kind": "oracle",
               "sample": f"one complete FP64 red-black V(2,1) solve of the same {n}^2 flower "
                         f"problem to 1e-10 ({len(hist) - 1} cycles, {t2 - t1:.1f} s, status "
                         f"{st}; setup {t1 - t0:.1f} s not counted)"}
        d = float(np.abs(uo - u.cpu().numpy()).max() / np.abs(uo).max())
        cpu["gpu_vs_oracle_rel_diff"] = d
        log(f"[bench] oracle: {t2 - t1:.1f}s, GPU vs oracle {d:.2e}")

    out = {"metric": METRIC, "value": value, "unit": "unknowns/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": f"flower-{n} 2D FP64 V(2,1) lambda=5 Nc={args.nc} tol=1e-10 zero guess",
                      "n": n, "unknowns": unknowns, "cycles": info["cycles"],
                      "rel_residual": info["rel"], "max_error_vs_exact": err,
                      "setup_s": round(setup_s, 3), "parallelism": "single GPU"},
           "roofline": roof, "cpu_baseline": cpu, "cycle_us_without_checks": round(cycle_us, 1)}
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
