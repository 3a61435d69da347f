"""Benchmark: unknowns/s to 1e-10 relative residual on one MI355X.

Headline workload (the largest single-GPU configuration): the 3D projection-style sequence,
one pressure solve per step of an ellipsoidal tank (semi-axes 0.8, 0.6, 0.5) moving 0.002
per step through [-1, 1]^3 on a 384^3 grid (7.27M unknowns), Dirichlet p = 0 on the free
surface z > 0.2, homogeneous Neumann on the walls, f = 20 Gaussians moving with the tank;
V(2,1) cycles with lambda = 5 boundary sweeps down to a 24^3 coarsest grid, FP32 cycles
inside FP64 defect correction, each step started from the previous step's solution (warm
start: mg_warm_start extends it to the nodes the boundary moved over), until
||r||_inf / ||(f_h, g_h)||_inf <= 1e-10.  One step = the warm start and one complete solve
(mg_solve) with its inputs resident in HBM; every step's hierarchy is built (mg_setup, timed
separately) before the timed region.

Prints one JSON line on stdout.  Extra fields: the same sequence step in FP64 and from a
cold start, the roofline of the dominant kernel, the FP64 CPU oracle on all host cores,
and the other workloads (2D flower 2048^2, 3D torus 256^3, the learned-guess batch).
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
TOL = 1e-10


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def measured_traffic(summary: str):
    """HBM bytes per launch from a committed FETCH_SIZE / WRITE_SIZE counter summary (each
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


def per_level_launches(s, reps=5):
    """Every launch sequence of one cycle, per level (microseconds, HIP events): the first
    pre-relaxation restricts (coarse levels), the first post-relaxation interpolates."""
    out = {}
    for lev in range(s.nlev - 1):
        names = ["relax_restrict" if lev > 0 else "relax", "relax", "defect", "relax_prolong"]
        out[str(lev)] = {k: round(s.time_kernel(k, lev, reps)[0] * 1e3, 1)
                         for k in dict.fromkeys(names)}
    out[str(s.nlev - 1)] = {
        "coarse_with_restriction": round(s.time_kernel("coarse", s.nlev - 1, reps)[0] * 1e3, 1)}
    return out


# ---------------------------------------------------------------------------------------
# headline: the 384^3 tank sequence
# ---------------------------------------------------------------------------------------
def bench_tank(args, gm, torch, dev):
    from workloads import tank

    n, nc = args.n3, 24
    seq = tank.TankSequence(n)
    nsteps = args.warmup + args.steps
    zero = torch.zeros((), dtype=torch.float64, device=dev)
    handles, fs, setup_s, unknowns = [], [], [], []
    g = None
    for t in range(nsteps):
        phi = seq.phi(t, dev)
        t0 = time.perf_counter()
        s = gm.Solver(phi, [seq.rule], gm.mg_grid_default(3, n, nc, precision=gm.MG_FP32_DC,
                                                          inner_cycles=args.inner,
                                                          max_cycles=300))
        setup_s.append(time.perf_counter() - t0)
        c = torch.from_numpy(s.classes()).to(dev)
        f = torch.where(c == 1, seq.f(t, dev), zero).contiguous()
        if g is None:
            g = torch.zeros_like(f)  # g = 0 on every ghost (p = 0, homogeneous Neumann)
        unknowns.append(int((c > 0).sum().item()))
        # capture the handle's cycle graphs now, outside the timed region
        tmp = torch.zeros_like(f)
        s.cycles(f, g, tmp, 1)
        handles.append(s)
        fs.append(f)
        del phi, c, tmp
        log(f"[bench] tank step {t}: setup {setup_s[-1]:.1f}s, {unknowns[-1]} unknowns")
    u = torch.zeros_like(fs[0])
    infos = []
    # the last warm-up step is also solved in FP64 below (from the same warm start)
    cmp_step = args.warmup - 1
    # a step: the previous solution mapped onto the new unknowns (mg_warm_start), then the solve
    for t in range(args.warmup):
        if t > 0:
            handles[t].warm_start(handles[t - 1], u)
        if t == cmp_step:
            u_cmp_start = u.clone()
        infos.append(handles[t].solve(fs[t], g, u, tol=TOL))
        if t == cmp_step:
            u_cmp = u.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(args.warmup, nsteps):
        handles[t].warm_start(handles[t - 1], u)
        infos.append(handles[t].solve(fs[t], g, u, tol=TOL))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    timed = infos[args.warmup:]
    tot_unknowns = sum(unknowns[args.warmup:])
    res = {"value": tot_unknowns / dt, "ms_per_step": 1e3 * dt / args.steps,
           "unknowns": unknowns[args.warmup], "cycles": [i["cycles"] for i in timed],
           "outer": [i["outer"] for i in timed], "rel": max(i["rel"] for i in timed),
           "setup_s": [round(x, 2) for x in setup_s], "nlev": handles[0].nlev}
    log(f"[bench] tank {n}^3 FP32-DC warm: {res['ms_per_step']:.2f} ms/step, FP32 cycles "
        f"{res['cycles']}, rel {res['rel']:.2e}")
    last = nsteps - 1
    s = handles[last]
    # the last step from a cold start (zero guess), same handle
    uc = torch.zeros_like(u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ic = s.solve(fs[last], g, uc, tol=TOL)
    torch.cuda.synchronize()
    res["cold_ms"] = 1e3 * (time.perf_counter() - t0)
    res["cold_cycles"] = ic["cycles"]
    res["warm_vs_cold_rel_diff"] = float((uc - u).abs().max() / u.abs().max())
    log(f"[bench] tank last step cold: {res['cold_ms']:.2f} ms, {ic['cycles']} FP32 cycles")
    # the dominant launches: one relaxation of the finest level (tile launch and chunk
    # launches) and the finest defect with its extension, FP32 as in the cycle
    k_ms, k_bytes = s.time_kernel("relax", 0, 20)
    d_ms, d_bytes = s.time_kernel("defect", 0, 20)
    res["relax_l0"] = (k_ms, k_bytes)
    res["defect_l0"] = (d_ms, d_bytes)
    res["launch_us_by_level"] = per_level_launches(s, 5)
    for h in handles[:-1]:
        h.close()
    handles = handles[-1:]
    # the last warm-up step in FP64 cycles, warm (from the same start) and cold
    phi = seq.phi(cmp_step, dev)
    t0 = time.perf_counter()
    s64 = gm.Solver(phi, [seq.rule], gm.mg_grid_default(3, n, nc, max_cycles=200))
    res["fp64_setup_s"] = time.perf_counter() - t0
    del phi
    tmp = torch.zeros_like(u)
    s64.cycles(fs[cmp_step], g, tmp, 1)
    res["fp64_step"] = cmp_step
    res["fp32dc_warm_cycles"] = infos[cmp_step]["cycles"]
    for name, start in (("fp64_warm", u_cmp_start), ("fp64_cold", None)):
        w = start.clone() if start is not None else torch.zeros_like(u)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        i64 = s64.solve(fs[cmp_step], g, w, tol=TOL)
        torch.cuda.synchronize()
        res[f"{name}_ms"] = 1e3 * (time.perf_counter() - t0)
        res[f"{name}_cycles"] = i64["cycles"]
        res[f"{name}_vs_fp32dc_rel_diff"] = float((w - u_cmp).abs().max() / u_cmp.abs().max())
    log(f"[bench] tank step {cmp_step} FP64: warm {res['fp64_warm_ms']:.2f} ms "
        f"{res['fp64_warm_cycles']} cycles, cold {res['fp64_cold_ms']:.2f} ms "
        f"{res['fp64_cold_cycles']} cycles (FP32-DC warm: {res['fp32dc_warm_cycles']} FP32 "
        f"cycles)")
    s64.close()
    s.close()
    res["last_step"] = last
    res["f_last"] = fs[last]
    res["u_last"] = u
    return res


def tank_cpu_baseline(args, res):
    """The FP64 oracle (red-black V(2,1), all host cores, gcc -O3 -march=native) solving the
    last timed step of the sequence from the zero guess: unknowns / its solve time."""
    import numpy as np

    import oracle
    from oracle import Oracle, default_grid
    from workloads import tank

    oracle.use_native()
    cores = os.cpu_count() or 1
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        pass
    cores = min(cores, 16)
    oracle.threads(cores)
    n = args.n3
    seq = tank.TankSequence(n)
    t0 = time.perf_counter()
    phi = seq.phi(res["last_step"], "cuda:0").cpu().numpy()
    o = Oracle(phi, default_grid(3, n, 24), tank.RULE)
    oc, _ = o.cls(0)
    rhs = np.where(oc == 1, res["f_last"].cpu().numpy(), 0.0)
    t1 = time.perf_counter()
    st, uo, hist = o.solve(rhs, tol=TOL, max_cycles=args.cpu_cycles)
    t2 = time.perf_counter()
    ncyc = len(hist) - 1
    unknowns = int((oc > 0).sum())
    # a solve cut short by the cycle budget is scaled to the cycles the rate predicts
    done = st == 0
    need = ncyc
    if not done and ncyc >= 2 and hist[-1] < hist[0]:
        rate = (hist[-1] / hist[0]) ** (1.0 / ncyc)
        need = int(np.ceil(np.log(TOL / hist[0]) / np.log(rate)))
    t_solve = (t2 - t1) * need / max(ncyc, 1)
    d = float(np.abs(uo - res["u_last"].cpu().numpy()).max() / np.abs(uo).max()) if done else None
    cpu = {"value": unknowns / t_solve, "unit": "unknowns/s", "cores": oracle.threads(),
           "kind": "oracle", "cpu_model": cpu_model(),
           "sample": f"the FP64 oracle (red-black V(2,1), gcc -O3 -march=native, OpenMP on "
                     f"{oracle.threads()} threads) solving step {res['last_step']} of the "
                     f"{n}^3 tank sequence from the zero guess: {ncyc} cycles in "
                     f"{t2 - t1:.1f} s, status {st}"
                     + ("" if done else f", scaled to the {need} cycles its rate predicts")
                     + f"; setup {t1 - t0:.1f} s not counted",
           "gpu_vs_oracle_rel_diff": d}
    log(f"[bench] oracle {n}^3: {ncyc} cycles {t2 - t1:.1f}s on {oracle.threads()} threads "
        f"({cpu_model()}), status {st}, GPU vs oracle {d}")
    return cpu


# ---------------------------------------------------------------------------------------
# other workloads (extra fields)
# ---------------------------------------------------------------------------------------
def timed_solves(torch, s, f, g, u, warmup, steps):
    info = None
    for _ in range(warmup):
        u.zero_()
        info = s.solve(f, g, u, tol=TOL)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        u.zero_()
        info = s.solve(f, g, u, tol=TOL)
    torch.cuda.synchronize()
    return info, (time.perf_counter() - t0) / steps


def bench_flower(args, gm, pr, geo, np, torch, dev):
    """2D flower r < 0.5 + 0.15 sin(5 theta), 2048^2, Dirichlet where x > 0, manufactured
    u = sin(3x) cos(2y) + x y, coarsest grid 128: FP64 and FP32-DC from the zero guess."""
    n, nc = 2048, args.nc2d
    w = pr.flower(n, nc)
    phi = w.domain.nodal_phi(n)
    out = {"flower_workload": f"flower-{n}^2 2D V(2,1) lambda=5 Nc={nc} tol=1e-10 zero guess"}
    ref = None
    for name, prec in (("fp64", gm.MG_FP64), ("fp32dc", gm.MG_FP32_DC)):
        t0 = time.time()
        s = gm.Solver(torch.from_numpy(phi).to(dev), [w.rule],
                      gm.mg_grid_default(2, n, nc, precision=prec, inner_cycles=args.inner))
        setup = time.time() - t0
        if ref is None:
            c = s.classes()
            G = s.ghosts()
            P = geo.grid_points(2, n)
            f = torch.from_numpy(np.where(c == 1, w.solution.f(P), 0.0)).to(dev)
            g = torch.from_numpy(pr.rhs_from_ghosts(2, n, c, G["node"], G["B"], G["type"],
                                                    w.solution, w.domain)).to(dev)
            unknowns = int((c > 0).sum())
        u = torch.zeros_like(f)
        info, dt = timed_solves(torch, s, f, g, u, 2, args.steps)
        if ref is None:
            ref = u.clone()
            out["flower_max_error_vs_exact"] = float(
                np.abs(u.cpu().numpy() - w.solution.u(P))[c == 1].max())
            # one cycle without the stopping test's read-backs
            uc = torch.zeros_like(u)
            s.cycles(f, g, uc, info["cycles"])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.cycles(f, g, uc, info["cycles"])
            torch.cuda.synchronize()
            out["flower_cycle_us_without_checks"] = round(
                1e6 * (time.perf_counter() - t0) / info["cycles"], 1)
            k_ms, k_bytes = s.time_kernel("relax", 0, 50)
            out["flower_relax_l0"] = {"avg_us": round(k_ms * 1e3, 2), "bytes": k_bytes,
                                      "GBs": round(k_bytes / (k_ms * 1e-3) / 1e9, 1)}
            out["flower_fp64_launch_us_by_level"] = per_level_launches(s, 20)
        else:
            out["flower_fp32dc_vs_fp64_rel_diff"] = float((u - ref).abs().max() / ref.abs().max())
        out[f"flower_{name}_unknowns_per_s"] = unknowns / dt
        out[f"flower_{name}_ms"] = 1e3 * dt
        out[f"flower_{name}_cycles"] = info["cycles"]
        out[f"flower_{name}_rel_residual"] = info["rel"]
        out[f"flower_{name}_setup_s"] = round(setup, 2)
        log(f"[bench] flower {n}^2 {name}: {1e3 * dt:.2f} ms, {info['cycles']} cycles, "
            f"rel {info['rel']:.2e}")
        s.close()
    out["flower_unknowns"] = unknowns
    return out


def bench_torus(args, gm, pr, geo, np, torch, dev):
    """3D torus (R, r) = (0.5, 0.25), 256^3, Neumann where z < 0, Dirichlet where z >= 0,
    u = exp(x + y) cos(z), coarsest grid 16: FP64 and FP32-DC from the zero guess."""
    n = 256
    w = pr.torus(n, 16)
    phi = w.domain.nodal_phi(n)
    out = {"torus_workload": f"torus-{n}^3 3D V(2,1) lambda=5 Nc=16 tol=1e-10 zero guess"}
    ref = None
    for name, prec in (("fp64", gm.MG_FP64), ("fp32dc", gm.MG_FP32_DC)):
        t0 = time.time()
        s = gm.Solver(torch.from_numpy(phi).to(dev), [w.rule],
                      gm.mg_grid_default(3, n, 16, precision=prec, inner_cycles=args.inner))
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
        info, dt = timed_solves(torch, s, f, g, u, 1, args.steps)
        if ref is None:
            ref = u.clone()
            out["torus_max_error_vs_exact"] = float(
                np.abs(u.cpu().numpy() - w.solution.u(P))[c == 1].max())
            out["torus_fp64_launch_us_by_level"] = per_level_launches(s, 5)
        else:
            out["torus_fp32dc_vs_fp64_rel_diff"] = float((u - ref).abs().max() / ref.abs().max())
        out[f"torus_{name}_unknowns_per_s"] = unknowns / dt
        out[f"torus_{name}_ms"] = 1e3 * dt
        out[f"torus_{name}_cycles"] = info["cycles"]
        out[f"torus_{name}_rel_residual"] = info["rel"]
        out[f"torus_{name}_setup_s"] = round(setup, 2)
        log(f"[bench] torus {n}^3 {name}: {1e3 * dt:.1f} ms, {info['cycles']} cycles, "
            f"rel {info['rel']:.2e}, setup {setup:.1f}s")
        s.close()
    out["torus_unknowns"] = unknowns
    return out


def bench_learned(args, torch):
    """The learned-guess workload: ellipse-union problems at 512^2 (evaluation seeds, the
    workload's rejections only), each solved on its own to 1e-10: FP64 and FP32-DC from the
    zero guess, FP32-DC and FP64 from the guess of the committed network (inference
    included)."""
    import numpy as np

    from paper_1111_0983_amd import cnn, learned
    from workloads import ellipses as el

    wpath = os.path.join(ROOT, "paper_1111_0983_amd", "weights", "guessnet.npz")
    net = cnn.GuessNet(seed=0)
    net.load(dict(np.load(wpath)))
    seeds, s, drawn = [], 1_000_000, 0
    while len(seeds) < args.learned_problems:
        p = el.draw(s)
        drawn += 1
        if el.accept(el.nodal_phi(p, learned.N_FINE, device="cuda:0"), learned.N_FINE,
                     3.0 * 2.0 / learned.N_COARSE):
            seeds.append(s)
        s += 1
    s64, f, g, probs = learned.build_batch(seeds)
    s64.close()
    pp = learned.evaluate_each(net, probs, f, g, reps=2)
    out = {f"learned_{k}": round(v, 3) for k, v in pp.items() if k.endswith(("_mean", "_median"))}
    out["learned_problems"] = len(probs)
    out["learned_failed"] = pp.get("failed", [])
    out["learned_zero64_cycles_max"] = max(pp["zero64_cycles"]) if pp.get("zero64_cycles") else None
    out["learned_rejected"] = {"box_margin": drawn - len(seeds),
                               "singular_or_merging": len(seeds) - len(probs)}
    out["learned_workload"] = "ellipse unions 512^2, Nc=32, per-problem solves to 1e-10"
    log(f"[bench] learned guess: zero FP64 {pp['zero64_cycles_mean']:.1f} cycles "
        f"{pp['zero64_ms_mean']:.2f} ms, zero FP32-DC {pp['zero_dc_cycles_mean']:.1f} cycles "
        f"{pp['zero_dc_ms_mean']:.2f} ms, learned FP32-DC {pp['learned_dc_cycles_mean']:.1f} "
        f"cycles {pp['learned_dc_ms_mean']:.2f} ms (means over {len(probs)} problems)")
    return out


def bench_paper_rho(gm, torch, dev):
    """The convergence factors of the paper's tables measured on the GPU cycle (red-black
    ordering, W-cycle, lambda = 5, delta = 3h, D/N-split transfers, coarsest grid 8 and the
    diagonal Nc = N/2), beside the printed GS-LEX values (tests/golden/rho_tables.txt)."""
    import numpy as np

    from workloads import geometry as geo, problems as pr

    printed = {}
    for line in open(os.path.join(ROOT, "tests", "golden", "rho_tables.txt")):
        if line.startswith("#") or not line.strip():
            continue
        t, dom, a, b, cyc, lam, nc, n, v = line.split()
        printed[(dom, int(a), int(b), cyc, int(lam), nc, int(n))] = v
    doms = {"circle": geo.paper_circle(), "ellipse": geo.rotated_ellipse_paper(),
            "saddle": geo.saddle_domain(), "flower": geo.Flower(0.5, 0.2, 5)}
    rows = []
    t0 = time.perf_counter()
    for key, v in sorted(printed.items()):
        dom, a, b, cyc, lam, nc, n = key
        ncv = n // 2 if cyc == "TGCS" else int(nc)
        grid = gm.mg_grid_default(2, n, ncv, nu1=a, nu2=b, gamma=2 if cyc == "W" else 1, lam=lam)
        phi = doms[dom].nodal_phi(n)
        try:
            s = gm.Solver(torch.from_numpy(phi).to(dev), [pr.paper_rule()], grid)
        except gm.GhostMGError as e:
            rows.append([dom, a + b, cyc, lam, ncv, n, v, f"setup {e.code}"])
            continue
        c = s.classes()
        u0 = torch.from_numpy(np.where(c > 0, np.random.default_rng(1).uniform(-1, 1, c.size),
                                       0.0)).to(dev)
        r, hist = s.rho(u0, max_cycles=100, rtol=1e-3)
        s.close()
        rows.append([dom, a + b, cyc, lam, ncv, n, v, round(r, 3)])
    log(f"[bench] paper rho tables on the GPU: {len(rows)} entries in "
        f"{time.perf_counter() - t0:.1f}s")
    return {"paper_rho_gpu": {"columns": ["domain", "nu", "cycle", "lambda", "Nc", "N",
                                          "printed (GS-LEX)", "GPU red-black"],
                              "rows": rows}}


def bench_reinit(gm, torch, dev, n=384, iters=100):
    """Eq. (sdf) on the GPU at the headline size: the tank's quadratic level set
    (x/a)^2 + (y/b)^2 + (z/c)^2 - 1 reinitialised by `iters` steps."""
    from workloads import tank

    x = torch.linspace(-1.0, 1.0, n + 1, dtype=torch.float64, device=dev)
    Z, Y, X = torch.meshgrid(x, x, x, indexing="ij")
    a, b, c = tank.AXES
    phi0 = ((X / a) ** 2 + ((Y + 0.2) / b) ** 2 + (Z / c) ** 2 - 1.0).reshape(-1).contiguous()
    del X, Y, Z
    gm.reinit(phi0, 3, n, 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    phi = gm.reinit(phi0, 3, n, iters)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ex = tank.ellipsoid_sdf(n, (0.0, -0.2, 0.0), device=dev)
    h = 2.0 / n
    near = ex.abs() < 3 * h
    err = float((phi - ex).abs()[near].max())
    nodes = (n + 1) ** 3
    out = {"reinit_workload": f"ellipsoid level set {n}^3, {iters} steps of Eq. (sdf)",
           "reinit_ms": 1e3 * dt, "reinit_us_per_step": 1e6 * dt / iters,
           "reinit_GBs_per_step": 24.0 * nodes / (dt / iters) / 1e9,
           "reinit_max_err_within_3h_over_h": err / h}
    log(f"[bench] reinit {n}^3: {1e3 * dt:.1f} ms for {iters} steps "
        f"({out['reinit_GBs_per_step']:.0f} GB/s), error within 3h = {err / h:.3f} h")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n3", type=int, default=384, help="tank sequence grid (intervals per axis)")
    ap.add_argument("--nc2d", type=int, default=128, help="flower coarsest grid")
    ap.add_argument("--inner", type=int, default=3,
                    help="FP32 cycles per defect-correction step (every FP32-DC leg)")
    ap.add_argument("--cpu-cycles", type=int, default=40,
                    help="cycle budget of the CPU oracle's solve (scaled beyond it)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-flower", action="store_true")
    ap.add_argument("--no-torus", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--learned-problems", type=int, default=64)
    ap.add_argument("--no-paper-rho", action="store_true")
    ap.add_argument("--no-reinit", action="store_true")
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
    res = bench_tank(args, gm, torch, dev)
    k_ms, k_bytes = res.pop("relax_l0")
    d_ms, d_bytes = res.pop("defect_l0")
    achieved = k_bytes / (k_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "kernel": "finest-level relaxation, FP32 (tile launch + chunk launches)",
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic("k_relax_tank384_level0_counters.txt"),
            "avg_us": round(k_ms * 1e3, 2), "bytes_per_launch": k_bytes,
            "defect_l0": {"avg_us": round(d_ms * 1e3, 2), "bytes": d_bytes,
                          "GBs": round(d_bytes / (d_ms * 1e-3) / 1e9, 1)},
            "launch_us_by_level": res.pop("launch_us_by_level")}
    log(f"[bench] tank relax level 0: {k_ms * 1e3:.1f} us, {achieved:.0f} GB/s; defect "
        f"{d_ms * 1e3:.1f} us")
    cpu = None if args.no_cpu_baseline else tank_cpu_baseline(args, res)
    res.pop("f_last")
    res.pop("u_last")
    extra = {}
    if not args.no_flower:
        extra.update(bench_flower(args, gm, pr, geo, np, torch, dev))
    if not args.no_torus:
        extra.update(bench_torus(args, gm, pr, geo, np, torch, dev))
    if not args.no_learned:
        extra.update(bench_learned(args, torch))
    if not args.no_paper_rho:
        extra.update(bench_paper_rho(gm, torch, dev))
    if not args.no_reinit:
        extra.update(bench_reinit(gm, torch, dev))
    out = {"metric": METRIC, "value": res["value"], "unit": "unknowns/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
           "data": "synthetic",
           "config": {"workload": f"tank-sequence-{args.n3}^3 3D V(2,1) lambda=5 Nc=24 "
                                  "FP32 cycles in FP64 defect correction, warm start, tol=1e-10",
                      "n": args.n3, "unknowns_per_step": res["unknowns"],
                      "fp32_cycles_per_step": res["cycles"], "dc_steps": res["outer"],
                      "max_rel_residual": res["rel"], "setup_s_per_step": res["setup_s"],
                      "levels": res["nlev"], "parallelism": "single GPU"},
           "roofline": roof, "cpu_baseline": cpu,
           # times rounded; the solution differences (rounding-level) keep their value
           "tank_last_step": {k: (round(v, 4) if isinstance(v, float) and "rel_diff" not in k
                                  else v)
                              for k, v in res.items()
                              if k.startswith(("cold", "fp64", "fp32dc", "warm_vs", "last"))}}
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
