"""The learned-closure experiment: train on exact stresses, judge against them.

    python -m paper_1902_02508_amd.experiment [--train 32] [--heldout 4] [--steps 20000] [--production 8]

Training snapshots (seeded synthetic channel fields) go through the exact
path (filtered velocity and tau_ij), their gradient features are built on
the device, and the perceptron is trained on (features -> tau_ij). On
held-out snapshots the exact tau_ij judges the closure: pointwise relative
error per component and the relative error of the plane-averaged
<tau_12>(y) profile in the form of eq. (14) of the paper (full channel and
the wall-to-centreline half). Two baselines are reported beside it: tau = 0
and the gradient model tau_ij = sum_k (Delta_k^2 / 12) d_k ubar_i d_k ubar_j
(the leading term of the small-width expansion of a filtered product). The
exact path and the closure inference are timed on the same snapshot.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np
import torch

from . import eles, synth



def trapezoid(y):
    w = np.empty(len(y))
    w[1:-1] = 0.5 * (y[2:] - y[:-2])
    w[0] = 0.5 * (y[1] - y[0])
    w[-1] = 0.5 * (y[-1] - y[-2])
    return w


def profile_error(a, b, y, half=False):
    """sqrt(int (a - b)^2 dy / int b^2 dy), trapezoid rule; half: lower wall to centreline."""
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    if half:
        k = y <= 0.0
        y, a, b = y[k], a[k], b[k]
    w = trapezoid(y)
    return math.sqrt(np.sum(w * (a - b) ** 2) / np.sum(w * b * b))


def init_params(seed: int) -> np.ndarray:
    """U(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases from PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for a, b in zip((10, 64, 64, 64), (64, 64, 64, 6)):
        lim = 1.0 / math.sqrt(a)
        parts.append(rng.uniform(-lim, lim, size=(b, a)).ravel())
        parts.append(rng.uniform(-lim, lim, size=(b,)))
    return np.concatenate(parts)


def exact_snapshot(f, cfg, seed, dev):
    y, terms = synth.snapshot_factors(cfg, seed)
    du = synth.assemble_on_device(cfg, terms, dev)
    ub, tau, st = f.sgs_stress(du)
    return du, ub, tau, st


def build_dataset(f, cfg, seeds, dev, log=print):
    feats = torch.empty((len(seeds), 10) + f.shape, dtype=torch.float32, device=dev)
    taus = torch.empty((len(seeds), 6) + f.shape, dtype=torch.float32, device=dev)
    for k, s in enumerate(seeds):
        du, ub, tau, _ = exact_snapshot(f, cfg, s, dev)
        eles.features(f, ub, out=feats[k])
        taus[k].copy_(tau)
        del du, ub, tau
    torch.cuda.synchronize()
    log(f"dataset: {len(seeds)} snapshots of {cfg.nx}x{cfg.ny}x{cfg.nz}")
    return feats, taus


def widths_coef(cfg):
    """c_k = Delta_k^2 / 12 of the configuration's filter widths."""
    return np.array([cfg.delta_x ** 2 / 12.0, cfg.delta_y ** 2 / 12.0, cfg.delta_z ** 2 / 12.0])


def gradient_model_closure(cfg, norms, dev):
    """The gradient model alone, run by the library's inference: a closure
    whose network outputs zero (last layer and bias zero) and whose target
    mean is zero, so its prediction is G = sum_k c_k d_k ubar_i d_k ubar_j."""
    theta = init_params(0)
    theta[-(6 * 64 + 6):] = 0.0
    n = np.array(norms, dtype=np.float64)
    n[20:26] = 0.0
    return eles.Closure(theta, n, device=dev, gm_coef=widths_coef(cfg))


def evaluate(cl, f, cfg, seeds, dev, baseline=None):
    """Closure and baselines against the exact stress on held-out snapshots
    (host-side metrics of the device outputs): pointwise relative L2 per
    component and the eq. (14)-form error of <tau_12>(y) from the FP64
    plane statistics; tau = 0 has profile error 1 by definition."""
    y = synth.ygrid(cfg.ny, cfg.ykind, cfg.stretch)
    w = trapezoid(y)
    rows = []
    for s in seeds:
        du, ub, tau, st = exact_snapshot(f, cfg, s, dev)
        pred, pst = cl.infer(f, ub)
        pred, pst = pred.cpu().numpy().astype(np.float64), pst.cpu().numpy()
        gm, gst = baseline.infer(f, ub) if baseline is not None else (None, None)
        ref = tau.cpu().numpy().astype(np.float64)
        ref12 = st[4].cpu().numpy()                  # <tau_12>(y), FP64 plane sums of the exact path
        row = {"seed": s,
               "tau12_profile_error": profile_error(pst[1], ref12, y),
               "tau12_profile_error_half": profile_error(pst[1], ref12, y, half=True)}
        den = [np.sum(w * np.mean(ref[q] ** 2, axis=(0, 2))) for q in range(6)]
        row["pointwise_rel_l2"] = [math.sqrt(np.sum(w * np.mean((pred[q] - ref[q]) ** 2, axis=(0, 2))) / den[q])
                                   for q in range(6)]
        if baseline is not None:
            gm = gm.cpu().numpy().astype(np.float64)
            row["tau12_profile_error_gradient_model"] = profile_error(gst[1].cpu().numpy(), ref12, y)
            row["pointwise_rel_l2_gradient_model"] = [
                math.sqrt(np.sum(w * np.mean((gm[q] - ref[q]) ** 2, axis=(0, 2))) / den[q]) for q in range(6)]
        # size of the mean profile relative to the pointwise field
        row["tau12_profile_to_field_ratio"] = math.sqrt(np.sum(w * ref12 ** 2) / den[1])
        rows.append(row)
        del du, ub, tau
    return rows


def time_paths(cl, f, cfg, dev, reps=20):
    y, u = synth.make_snapshot(cfg, synth.SEEDS["heldout"][0])
    du = torch.from_numpy(u).to(dev)
    ub = torch.empty((3,) + f.shape, dtype=torch.float32, device=dev)
    tau = torch.empty((6,) + f.shape, dtype=torch.float32, device=dev)
    st = torch.empty((9, cfg.ny), dtype=torch.float64, device=dev)
    pred = torch.empty_like(tau)
    pst = torch.empty((6, cfg.ny), dtype=torch.float64, device=dev)
    for _ in range(3):
        f.sgs_stress(du, ub, tau, st)
        cl.infer(f, ub, pred, pst)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        f.sgs_stress(du, ub, tau, st)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(reps):
        cl.infer(f, ub, pred, pst)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    exact = cfg.points * reps / (t1 - t0)
    learned = cfg.points * reps / (t2 - t1)
    return {"exact_points_per_s": exact, "closure_points_per_s": learned, "speedup": learned / exact}


def production(cl, n_snap=8, tail=1e-8, workload="dns1024", log=print):
    """Exact path vs closure inference at the production shape.

    n_snap snapshots are staged in HBM first (host-to-device copies from
    pinned buffers timed on their own); the exact path is timed over all of
    them with the FP32 and the BF16x3 y pass, the closure's inference
    (features from ubar + perceptron + plane means) over the same filtered
    velocities, and each snapshot's closure <tau_12>(y) is compared with the
    exact FP64 plane statistics.
    """
    dev = torch.device("cuda", torch.cuda.current_device())
    cfg = synth.config(workload)
    y = synth.ygrid(cfg.ny, cfg.ykind, cfg.stretch)
    seeds = synth.SEEDS[workload][:n_snap]
    us, h2d_s, nbytes = [], 0.0, 0
    for s in seeds:
        _, u = synth.make_snapshot(cfg, s)
        host = torch.from_numpy(u).pin_memory()
        d = torch.empty(host.shape, dtype=host.dtype, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        d.copy_(host, non_blocking=True)
        torch.cuda.synchronize()
        h2d_s += time.perf_counter() - t0
        nbytes += host.numel() * 4
        us.append(d)
        del host, u
        log(f"  staged snapshot {s} ({len(us)}/{len(seeds)})")
    pts = cfg.points * len(us)
    res = {"workload": f"channel {cfg.nx}x{cfg.ny}x{cfg.nz}", "snapshots": len(us),
           "h2d_GBps": nbytes / h2d_s / 1e9}
    shape = (cfg.nx, cfg.ny, cfg.nz)
    tau = torch.empty((6,) + shape, dtype=torch.float32, device=dev)
    for mode in ("fp32", "bf16x3"):
        f = eles.Filter.from_config(cfg, tail_tol=tail, ygemm=mode, device=dev)
        ub = torch.empty((3,) + shape, dtype=torch.float32, device=dev)
        st = torch.empty((9, cfg.ny), dtype=torch.float64, device=dev)
        f.sgs_stress(us[0], ub, tau, st)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for u in us:
            f.sgs_stress(u, ub, tau, st)
        torch.cuda.synchronize()
        res[f"exact_{mode}_points_per_s"] = pts / (time.perf_counter() - t0)
        log(f"  exact {mode}: {res[f'exact_{mode}_points_per_s']:.3e} points/s")
        del f, ub, st
        torch.cuda.empty_cache()
    f = eles.Filter.from_config(cfg, tail_tol=tail, device=dev)
    ubs, stats = [], []
    for u in us:
        ub = torch.empty((3,) + shape, dtype=torch.float32, device=dev)
        st = torch.empty((9, cfg.ny), dtype=torch.float64, device=dev)
        f.sgs_stress(u, ub, tau, st)
        ubs.append(ub)
        stats.append(st)
    del tau
    torch.cuda.empty_cache()
    pred = torch.empty((6,) + shape, dtype=torch.float32, device=dev)
    pst = [torch.empty((6, cfg.ny), dtype=torch.float64, device=dev) for _ in ubs]
    cl.infer(f, ubs[0], pred, pst[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for ub, ps in zip(ubs, pst):
        cl.infer(f, ub, pred, ps)
    torch.cuda.synchronize()
    res["closure_points_per_s"] = pts / (time.perf_counter() - t0)
    errs = [profile_error(ps[1].cpu().numpy(), st[4].cpu().numpy(), y) for ps, st in zip(pst, stats)]
    res["tau12_profile_error"] = float(np.mean(errs))
    res["tau12_profile_error_max"] = float(np.max(errs))
    res["speedup_vs_fp32"] = res["closure_points_per_s"] / res["exact_fp32_points_per_s"]
    res["speedup_vs_bf16x3"] = res["closure_points_per_s"] / res["exact_bf16x3_points_per_s"]
    log(f"  closure: {res['closure_points_per_s']:.3e} points/s, <tau12> profile error {res['tau12_profile_error']:.3f}")
    return res


def run(n_train=32, n_heldout=4, steps=20000, batch=65536, lr=1e-3, seed=1, workload="dns192",
        tail=1e-8, physics=True, log=print):
    dev = torch.device("cuda", torch.cuda.current_device())
    cfg = synth.config(workload)
    f = eles.Filter.from_config(cfg, tail_tol=tail, device=dev)
    t0 = time.perf_counter()
    feats, taus = build_dataset(f, cfg, synth.SEEDS["train"][:n_train], dev, log)
    fm = eles.moments(feats).cpu().numpy()
    tm = eles.moments(taus).cpu().numpy()
    norms = np.concatenate([fm[0], fm[1], tm[0], tm[1]])
    cl = eles.Closure(init_params(seed), norms, device=dev, gm_coef=widths_coef(cfg) if physics else None)
    t1 = time.perf_counter()
    chunks = []
    done = 0
    while done < steps:
        n = min(2000, steps - done)
        chunks.append(cl.train(feats, taus, steps=n, batch=batch, seed=seed, lr=lr))
        torch.cuda.synchronize()
        done += n
        log(f"  {done} steps, {time.perf_counter() - t1:.1f} s, loss {chunks[-1][-50:].mean().item():.4f}")
    t2 = time.perf_counter()
    lh = torch.cat(chunks).cpu().numpy()
    log(f"trained {steps} steps of {batch} in {t2 - t1:.2f} s; loss {lh[:10].mean():.4f} -> {lh[-100:].mean():.4f}")
    del feats, taus
    torch.cuda.empty_cache()
    rows = evaluate(cl, f, cfg, synth.SEEDS["heldout"][:n_heldout], dev,
                    baseline=gradient_model_closure(cfg, norms, dev))
    speed = time_paths(cl, f, cfg, dev)
    res = {
        "workload": f"channel {cfg.nx}x{cfg.ny}x{cfg.nz}", "physics_term": bool(physics),
        "train_snapshots": n_train, "heldout_snapshots": n_heldout, "steps": steps, "batch": batch,
        "train_seconds": t2 - t1, "dataset_seconds": t1 - t0,
        "loss_first": float(lh[:10].mean()), "loss_last": float(lh[-100:].mean()),
        "tau12_profile_error": float(np.mean([r["tau12_profile_error"] for r in rows])),
        "tau12_profile_error_half": float(np.mean([r["tau12_profile_error_half"] for r in rows])),
        "tau12_profile_error_gradient_model": float(np.mean([r["tau12_profile_error_gradient_model"] for r in rows])),
        "pointwise_rel_l2": [float(np.mean([r["pointwise_rel_l2"][q] for r in rows])) for q in range(6)],
        "pointwise_rel_l2_gradient_model": [float(np.mean([r["pointwise_rel_l2_gradient_model"][q] for r in rows]))
                                            for q in range(6)],
        "tau12_profile_to_field_ratio": float(np.mean([r["tau12_profile_to_field_ratio"] for r in rows])),
        **speed,
    }
    return res, cl, f


def time_inference(workload: str, reps: int = 20, seed: int = 1):
    """Exact stress path against the closure's inference on one snapshot of
    a workload, with random weights (the cost does not depend on their
    values) and unit feature / output normalisation."""
    dev = torch.device("cuda", torch.cuda.current_device())
    cfg = synth.config(workload)
    f = eles.Filter.from_config(cfg, tail_tol=1e-8, device=dev)
    norms = np.concatenate([np.zeros(10), np.ones(10), np.zeros(6), np.ones(6)])
    cl = eles.Closure(init_params(seed), norms, device=dev)
    out = time_paths(cl, f, cfg, dev, reps=reps)
    out["workload"] = f"{cfg.nx}x{cfg.ny}x{cfg.nz}"
    return out


def main(argv=None):
    p = argparse.ArgumentParser()
    p.add_argument("--time-inference", metavar="WORKLOAD", default=None,
                   help="only time the exact path against the closure's inference (random weights) and exit")
    p.add_argument("--train", type=int, default=32)
    p.add_argument("--heldout", type=int, default=4)
    p.add_argument("--steps", type=int, default=20000)
    p.add_argument("--batch", type=int, default=65536)
    p.add_argument("--lr", type=float, default=1e-3)
    p.add_argument("--seed", type=int, default=1)
    p.add_argument("--no-physics", action="store_true",
                   help="train the plain network, without the gradient-model term")
    p.add_argument("--production", type=int, default=0, metavar="N",
                   help="also time exact path vs closure on N staged 1024x385x768 snapshots")
    a = p.parse_args(argv)
    if a.time_inference:
        print(json.dumps(time_inference(a.time_inference)), flush=True)
        return
    log = lambda m: print(m, file=sys.stderr, flush=True)
    res, cl, f = run(a.train, a.heldout, a.steps, a.batch, a.lr, a.seed, physics=not a.no_physics, log=log)
    if a.production > 0:
        del f
        torch.cuda.empty_cache()
        res["production"] = production(cl, a.production, log=log)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
