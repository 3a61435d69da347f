"""Training and evaluation of the learned initial guess (random ellipse-union problems).

* generate(): seeded batches of problems are solved by the GPU solver itself (FP64, zero
  guess); the network inputs and targets are taken on one coarse level of each problem's
  hierarchy and kept on the GPU.
* train(): minibatch Adam with the project's BF16 MFMA kernels.
* evaluate(): cycles and time to the tolerance with the zero guess (FP64 cycles) against
  the learned guess (FP32 cycles inside FP64 defect correction).

Samples whose domain comes within 3 coarsest mesh widths of the box, which have a connected
component without a Dirichlet ghost (a singular problem), or whose interior components merge
on a coarser level of the hierarchy (a topology the coarsest grid does not resolve) are
rejected; all three are decided from phi and the boundary partition alone.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import cnn, ghostmg as gm

N_FINE, N_COARSE, LEVEL = 512, 32, 3   # the network works on the 65 x 65 level
# cycle budget of a training-target solve (to 1e-8; the median problem needs about 15)
GEN_CYCLES = 150
# first validation seed (training draws from seed0 upwards, evaluation from 1,000,000)
VAL_SEED0 = 500_000


def _components_ok(cls: np.ndarray, ghosts: dict, n: int) -> bool:
    from scipy import ndimage

    inside = (cls == 1).reshape(n + 1, n + 1)
    lab, nlab = ndimage.label(inside)
    if nlab == 0:
        return False
    dirich = ghosts["node"][ghosts["type"] == 1]
    if len(dirich) == 0:
        return False
    # a Dirichlet ghost is attached to the components of its interior neighbours
    has = np.zeros(nlab + 1, bool)
    gy, gx = np.divmod(dirich, n + 1)
    for dy, dx in ((0, 1), (0, -1), (1, 0), (-1, 0)):
        yy, xx = gy + dy, gx + dx
        ok = (yy >= 0) & (yy <= n) & (xx >= 0) & (xx <= n)
        has[lab[yy[ok], xx[ok]]] = True
    has[0] = False
    return bool(has[1:].all())


def components_merge(cls_levels) -> bool:
    """True when interior components of the finest grid merge on a coarser level of the
    hierarchy: the number of connected components of Omega_h (4-connected interior nodes)
    drops from one level to the next.  The coarse grid then cannot represent the domain:
    its correction couples pieces that are separate on the fine grid, and the cycle
    converges slowly or diverges (as for the paper's flower on too coarse a grid, Table
    rhoSF3).  cls_levels: the node classes of every level, finest first, as square 2D
    arrays.  A property of phi alone."""
    from scipy import ndimage

    prev = None
    for c in cls_levels:
        k = ndimage.label(np.asarray(c) == 1)[1]
        if prev is not None and k < prev:
            return True
        prev = k
    return False


def _merges(solver, problem: int) -> bool:
    levels = []
    for lev in range(solver.nlev):
        nl = solver.level(lev)["n"]
        levels.append(solver.classes(problem, lev).reshape(nl + 1, nl + 1))
    return components_merge(levels)


def build_batch(seeds, n=N_FINE, nc=N_COARSE, device="cuda:0", precision=gm.MG_FP64,
                inner_cycles=2, screen=True, max_cycles=1000):
    """Solver handle plus f, g for the accepted problems among `seeds`."""
    from workloads import ellipses as el

    probs, phis, fs = [], [], []
    for s in seeds:
        p = el.draw(int(s))
        phi = el.nodal_phi(p, n, device=device)
        if not el.accept(phi, n, 3.0 * 2.0 / nc):
            continue
        probs.append(p)
        phis.append(phi)
        fs.append(el.nodal_f(p, n, device=device))
    while probs:
        # a few accepted problems converge slowly (rho 0.9-0.95: concave corners where two
        # ellipses meet, around 500 cycles to 1e-10); the default budget lets every one finish
        grid = gm.mg_grid_default(2, n, nc, batch=len(probs), precision=precision,
                                  inner_cycles=inner_cycles, max_cycles=max_cycles)
        try:
            solver = gm.Solver(torch.cat(phis), [p.rule for p in probs], grid)
        except gm.GhostMGError as e:
            if e.code != gm.MG_EGEOM:
                raise
            # find the offending problems one by one
            keep = []
            for i, (p, phi) in enumerate(zip(probs, phis)):
                try:
                    gm.Solver(phi, [p.rule], gm.mg_grid_default(2, n, nc)).close()
                    keep.append(i)
                except gm.GhostMGError:
                    pass
            if len(keep) == len(probs):
                raise
            probs = [probs[i] for i in keep]
            phis = [phis[i] for i in keep]
            fs = [fs[i] for i in keep]
            continue
        bad = [i for i in range(len(probs))
               if not _components_ok(solver.classes(i), solver.ghosts(i), n)]
        if not bad and screen:
            bad = [i for i in range(len(probs)) if _merges(solver, i)]
        if bad:
            solver.close()
            probs = [p for i, p in enumerate(probs) if i not in bad]
            phis = [p for i, p in enumerate(phis) if i not in bad]
            fs = [p for i, p in enumerate(fs) if i not in bad]
            continue
        f = torch.cat(fs)
        # f on the interior nodes only; g = 0 on every ghost
        cls = torch.from_numpy(np.concatenate([solver.classes(i) for i in range(len(probs))]))
        f = torch.where(cls.to(f.device) == 1, f, torch.zeros_like(f)).contiguous()
        g = torch.zeros_like(f)
        return solver, f, g, probs
    return None, None, None, []


def _targets(solver, f, g, probs, device, max_cycles=1000):
    """Solve one built batch to 1e-8 for its training targets.  Problems on which the cycle
    diverges (a few percent of the ellipse unions: concave corners, coarse components without
    a Dirichlet condition) have no target: the batch is solved again without them.  Returns
    (features, targets, masks, kept count, dropped count, cycles) or None."""
    dropped = 0
    u = torch.zeros_like(f)
    # 1e-8 is far below what the network can reproduce; a batch whose slowest problem misses
    # it within the cycle budget keeps the problems that reached it
    info = solver.solve(f, g, u, tol=1e-8, check=False)
    while info["status"] == gm.MG_EDIVERGED:
        B0 = len(probs)
        fmax = f.reshape(B0, -1).abs().max(dim=1).values.cpu().numpy()
        rel = solver.residual(f, g, u).max(axis=1) / np.maximum(fmax, 1e-300)
        keep = [p.seed for p, r in zip(probs, rel) if r < 1.0]
        solver.close()
        dropped += B0 - len(keep)
        if not keep or len(keep) == B0:
            return None, dropped
        solver, f, g, probs = build_batch(keep, device=device, max_cycles=max_cycles)
        if solver is None:
            return None, dropped
        u = torch.zeros_like(f)
        info = solver.solve(f, g, u, tol=1e-8, check=False)
    if info["status"] not in (gm.MG_OK, gm.MG_ENOCONV):
        raise gm.GhostMGError(info["status"], "mg_solve")
    B0 = len(probs)
    norms = solver.residual(f, g, u).max(axis=1)
    fmax = f.reshape(B0, -1).abs().max(dim=1).values.cpu().numpy()
    good = torch.from_numpy(norms <= 1e-8 * np.maximum(fmax, 1e-300)).to(f.device)
    x, scale, (B, H, W) = cnn.features(solver, LEVEL, f, g)
    tgt, mask = cnn.target(solver, LEVEL, u, scale / cnn.GuessNet.GAIN)
    solver.close()
    return (x.reshape(B, H * W * 8)[good], tgt.reshape(B, H * W)[good],
            mask.reshape(B, H * W)[good], (H, W), info["cycles"]), \
        dropped + int(B0 - good.sum().item())


def generate(n_samples: int, seed0: int = 0, batch: int = 64, device="cuda:0", log=print,
             threads: int = 12, max_cycles: int = GEN_CYCLES, max_seconds: float = 0.0):
    """Solver-generated training samples.  The hierarchies of `threads` batches are built at
    once (the host setup of a batch is the slow part, and mg_setup runs outside the Python
    lock), then solved one after the other.  A batch is solved together, so its slowest
    problem sets its cycle count: a problem that has not reached the target tolerance within
    max_cycles gives no sample (counted as rejected), instead of holding its batch for
    hundreds of cycles.  max_seconds > 0: stop after the round that passes that time, with
    the samples generated so far."""
    from concurrent.futures import ThreadPoolExecutor

    from workloads import ellipses as el

    xs, ts, ms = [], [], []
    seed = seed0
    t0 = time.time()
    total = 0
    rejected = 0
    H = W = None
    last = 0
    with ThreadPoolExecutor(max_workers=threads) as pool:
        while total < n_samples:
            if max_seconds > 0 and time.time() - t0 > max_seconds:
                break
            want = min(batch * threads, n_samples - total)
            seeds = []
            while len(seeds) < want:  # screen the box margin cheaply before building solvers
                p = el.draw(seed)
                if el.accept(el.nodal_phi(p, N_FINE, device=device), N_FINE,
                             3.0 * 2.0 / N_COARSE):
                    seeds.append(seed)
                else:
                    rejected += 1
                seed += 1
            groups = [seeds[i:i + batch] for i in range(0, len(seeds), batch)]
            built = list(pool.map(
                lambda sd: build_batch(sd, device=device, max_cycles=max_cycles), groups))
            for sd, (solver, f, g, probs) in zip(groups, built):
                rejected += len(sd) - len(probs)
                if solver is None:
                    continue
                out, drop = _targets(solver, f, g, probs, device, max_cycles)
                rejected += drop
                if out is None:
                    continue
                x, t, m, (H, W), last = out
                xs.append(x)
                ts.append(t)
                ms.append(m)
                total += x.shape[0]
            if log:
                log(f"[learned] generated {total}/{n_samples} ({rejected} rejected, "
                    f"last solve {last} cycles) {time.time() - t0:.1f}s")
    return dict(x=torch.cat(xs)[:n_samples], t=torch.cat(ts)[:n_samples],
                m=torch.cat(ms)[:n_samples], H=H, W=W, rejected=rejected,
                seconds=time.time() - t0)


def train(net: cnn.GuessNet, data: dict, steps: int, batch: int = 64, lr: float = 2e-3,
          seed: int = 0, log=print, val: dict | None = None):
    H, W = data["H"], data["W"]
    n = data["x"].shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed)
    hist = []
    t0 = time.time()
    for step in range(steps):
        idx = torch.randint(0, n, (batch,), generator=g).to(data["x"].device)
        x = data["x"][idx].reshape(-1)
        t = data["t"][idx].reshape(-1)
        m = data["m"][idx].reshape(-1)
        warm = min(1.0, (step + 1) / 100.0)
        lr_t = lr * warm * 0.5 * (1 + np.cos(np.pi * step / steps))
        pred = net.forward(x, batch, H, W)
        out, dy = cnn.loss(pred, t, m)
        net.adam(net.backward(dy, batch, H, W), lr=lr_t)
        if step % 100 == 0 or step == steps - 1:
            rec = dict(step=step, loss=out[0].item())
            if val is not None:
                rec["val"] = validate(net, val)
            hist.append(rec)
            if log:
                log(f"[learned] step {step} loss {rec['loss']:.4e}"
                    + (f" val {rec['val']:.4e}" if "val" in rec else "")
                    + f" {time.time() - t0:.1f}s")
    return hist


def validate(net: cnn.GuessNet, data: dict, batch: int = 64) -> float:
    H, W = data["H"], data["W"]
    tot, cnt = 0.0, 0
    for s in range(0, data["x"].shape[0], batch):
        x = data["x"][s:s + batch]
        B = x.shape[0]
        pred = net.forward(x.reshape(-1), B, H, W)
        out, _ = cnn.loss(pred, data["t"][s:s + batch].reshape(-1),
                          data["m"][s:s + batch].reshape(-1), with_grad=False)
        tot += out[0].item() * B
        cnt += B
    return tot / max(cnt, 1)


def evaluate(net: cnn.GuessNet | None, seeds, tol: float = 1e-10, device="cuda:0", reps: int = 3):
    """Solve the batch with (a) FP64 cycles from the zero guess and (b) FP32 defect
    correction from the learned guess (and from the zero guess); returns cycles and times."""
    out = {}
    s64, f, g, probs = build_batch(seeds, device=device)
    sdc, _, _, _ = build_batch([p.seed for p in probs], device=device, precision=gm.MG_FP32_DC,
                               screen=False)
    B = len(probs)
    u = torch.zeros_like(f)

    def timed(fn):
        best = None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = fn()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        return info, best

    def zero64():
        u.zero_()
        return s64.solve(f, g, u, tol=tol)

    info, dt = timed(zero64)
    ref = u.clone()
    out["fp64_zero"] = dict(cycles=info["cycles"], ms=1e3 * dt, rel=info["rel"])

    def zerodc():
        u.zero_()
        return sdc.solve(f, g, u, tol=tol)

    info, dt = timed(zerodc)
    out["fp32dc_zero"] = dict(cycles=info["cycles"], outer=info["outer"], ms=1e3 * dt,
                              rel=info["rel"])
    if net is not None:
        def learned():
            cnn.guess(net, sdc, LEVEL, f, g, u)
            return sdc.solve(f, g, u, tol=tol)

        info, dt = timed(learned)
        out["fp32dc_learned"] = dict(cycles=info["cycles"], outer=info["outer"], ms=1e3 * dt,
                                     rel=info["rel"],
                                     diff_vs_fp64=(u - ref).abs().max().item() / ref.abs().max().item())
        # error of the initial guess itself (relative, on the unknowns)
        u0 = torch.zeros_like(u)
        cnn.guess(net, sdc, LEVEL, f, g, u0)
        out["guess_rel_error"] = ((u0 - ref).abs().max() / ref.abs().max()).item()

        def learned64():
            cnn.guess(net, s64, LEVEL, f, g, u)
            return s64.solve(f, g, u, tol=tol)

        info, dt = timed(learned64)
        out["fp64_learned"] = dict(cycles=info["cycles"], ms=1e3 * dt, rel=info["rel"])
    unknowns = int(sum((s64.classes(i) > 0).sum() for i in range(B)))
    out["problems"] = B
    out["unknowns"] = unknowns
    s64.close()
    sdc.close()
    out["per_problem"] = evaluate_each(net, probs, f, g, tol=tol, device=device, reps=reps)
    return out


def evaluate_each(net, probs, f, g, tol=1e-10, device="cuda:0", reps=3):
    """Cycles and time to the tolerance of every problem solved on its own (a batch solve
    runs until its slowest problem converges): FP64 and FP32 defect correction from the zero
    guess, FP32 defect correction and FP64 from the learned guess (network inference
    included in the time).  Returns per-problem lists and their means / medians; problems on
    which the zero-guess FP64 cycle does not reach the tolerance are listed under "failed"
    (seed, status) and left out of the lists."""
    from workloads import ellipses as el

    nn = (N_FINE + 1) ** 2
    rows = {k: [] for k in ("zero64_cycles", "zero64_ms", "zero_dc_cycles", "zero_dc_ms",
                            "learned_dc_cycles", "learned_dc_ms", "learned64_cycles",
                            "learned64_ms", "guess_rel_error")}
    failed = []
    for i, p in enumerate(probs):
        phi = el.nodal_phi(p, N_FINE, device=device)
        fi = f[i * nn:(i + 1) * nn].contiguous()
        gi = g[i * nn:(i + 1) * nn].contiguous()
        s64 = gm.Solver(phi, [p.rule], gm.mg_grid_default(2, N_FINE, N_COARSE, max_cycles=1000))
        u = torch.zeros_like(fi)
        first = s64.solve(fi, gi, u, tol=tol, check=False)
        if first["status"] != gm.MG_OK:
            failed.append((p.seed, first["status"]))
            s64.close()
            continue
        sdc = gm.Solver(phi, [p.rule], gm.mg_grid_default(2, N_FINE, N_COARSE, max_cycles=1000,
                                                          precision=gm.MG_FP32_DC))

        def timed(fn):
            best, info = None, None
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                info = fn()
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                best = dt if best is None else min(best, dt)
            return info, best

        def zero64():
            u.zero_()
            return s64.solve(fi, gi, u, tol=tol)

        info, dt = timed(zero64)
        ref = u.clone()
        rows["zero64_cycles"].append(info["cycles"])
        rows["zero64_ms"].append(1e3 * dt)

        def zero_dc():
            u.zero_()
            return sdc.solve(fi, gi, u, tol=tol)

        info, dt = timed(zero_dc)
        rows["zero_dc_cycles"].append(info["cycles"])
        rows["zero_dc_ms"].append(1e3 * dt)
        if net is not None:
            def learned_dc():
                cnn.guess(net, sdc, LEVEL, fi, gi, u)
                return sdc.solve(fi, gi, u, tol=tol)

            info, dt = timed(learned_dc)
            rows["learned_dc_cycles"].append(info["cycles"])
            rows["learned_dc_ms"].append(1e3 * dt)

            def learned64():
                cnn.guess(net, s64, LEVEL, fi, gi, u)
                return s64.solve(fi, gi, u, tol=tol)

            info, dt = timed(learned64)
            rows["learned64_cycles"].append(info["cycles"])
            rows["learned64_ms"].append(1e3 * dt)
            u0 = torch.zeros_like(u)
            cnn.guess(net, s64, LEVEL, fi, gi, u0)
            rows["guess_rel_error"].append(((u0 - ref).abs().max() / ref.abs().max()).item())
        s64.close()
        sdc.close()
    res = {k: v for k, v in rows.items() if v}
    for k, v in list(res.items()):
        res[k + "_mean"] = float(np.mean(v))
        res[k + "_median"] = float(np.median(v))
    res["failed"] = failed
    return res


def mfma_rate(net: cnn.GuessNet, B: int = 64, reps: int = 20, device="cuda:0") -> dict:
    """Measured throughput of the network's BF16 MFMA kernels at the training shape (B
    problems of the 65 x 65 level): forward, and forward + backward (data and weight
    gradients), in TFLOP/s counted as 2 x (multiply-adds of the 3 x 3 convolutions), against
    the dense BF16 peak of 2.5 PFLOP/s."""
    H = W = 65
    x = torch.randn(B * H * W * 8, device=device).to(torch.bfloat16)
    fwd = sum(2.0 * B * H * W * 9 * cin * cout for cin, cout, _ in net.layers)
    tgt = torch.zeros(B * H * W, device=device)
    mask = torch.ones_like(tgt)

    def run(back):
        pred = net.forward(x, B, H, W)
        if back:
            _, dy = cnn.loss(pred, tgt, mask)
            net.backward(dy, B, H, W)

    out = {}
    for name, back, flops in (("forward", False, fwd), ("train_step", True, 3.0 * fwd)):
        run(back)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            run(back)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[f"{name}_ms"] = ms
        out[f"{name}_tflops"] = flops / (ms * 1e-3) / 1e12
        out[f"{name}_mfma_util"] = out[f"{name}_tflops"] / 2500.0
    return out


def main(argv=None):
    import argparse
    import json
    import os

    ap = argparse.ArgumentParser(description="train and evaluate the learned initial guess")
    ap.add_argument("--samples", type=int, default=20000)
    ap.add_argument("--gen-seconds", type=float, default=0.0,
                    help="stop generating training samples after this many seconds (0: no limit)")
    ap.add_argument("--seed0", type=int, default=0, help="first training seed")
    ap.add_argument("--val", type=int, default=512)
    ap.add_argument("--steps", type=int, default=6000)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--eval", type=int, default=64, help="evaluation problems (0: none)")
    ap.add_argument("--out", default="learned_out")
    ap.add_argument("--init", default=None, help="start training from these weights")
    ap.add_argument("--weights", default=None, help="skip training, load these weights")
    ap.add_argument("--arch", choices=["base", "large"], default="base",
                    help="base: 5 layers, receptive field 33; large: 8 layers, field 131")
    ap.add_argument("--rate-only", action="store_true",
                    help="print the MFMA kernels' measured throughput at the training shape "
                         "(randomly initialised network) and exit")
    args = ap.parse_args(argv)
    net = cnn.GuessNet(seed=0, layers=cnn.LAYERS_LARGE if args.arch == "large" else cnn.LAYERS)
    if args.rate_only:
        print(json.dumps({"arch": args.arch, "mfma": mfma_rate(net)}), flush=True)
        return
    os.makedirs(args.out, exist_ok=True)
    res = {}
    if args.weights:
        net.load(dict(np.load(args.weights)))
    else:
        if args.init:
            net.load(dict(np.load(args.init)))
        t0 = time.time()
        data = generate(args.samples, seed0=args.seed0, max_seconds=args.gen_seconds)
        # validation seeds far from the training seeds (about 3.5 seeds are drawn per sample)
        val = generate(args.val, seed0=VAL_SEED0) if args.val else None
        res["generate_s"] = time.time() - t0
        res["samples"] = int(data["x"].shape[0])
        res["rejected"] = data["rejected"]
        t0 = time.time()
        res["train_hist"] = train(net, data, args.steps, batch=args.batch, lr=args.lr, val=val)
        res["train_s"] = time.time() - t0
        np.savez(os.path.join(args.out, "guessnet.npz"), **net.state())
        del data
    res["mfma"] = mfma_rate(net)
    print(json.dumps({"mfma": res["mfma"]}), flush=True)
    if args.eval:
        seeds = []
        s = 1_000_000
        from workloads import ellipses as el
        while len(seeds) < args.eval:
            p = el.draw(s)
            if el.accept(el.nodal_phi(p, N_FINE, device="cuda:0"), N_FINE, 3.0 * 2.0 / N_COARSE):
                seeds.append(s)
            s += 1
        res["eval"] = evaluate(net, seeds)
        print(json.dumps(res["eval"]))
    with open(os.path.join(args.out, "learned.json"), "w") as f:
        json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
