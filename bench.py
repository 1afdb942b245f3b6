"""Throughput of the exact filtered velocity + subgrid stress path on one GPU.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--filter gaussian|differential]

A step is one exact-stress evaluation (filtered velocity, the six stress
components and their plane averages) of one 192 x 129 x 192 channel
snapshot; four seeded snapshots stay resident in HBM and are cycled. The
timed region is K steps bracketed by device synchronisations; HIP events on
the library's stream time the dominant pass inside it. Prints one JSON line.

Beside the headline (unless --skip-extras): the stress on the LES2 / LES4
grids; the production shape 1024 x 385 x 768 (one snapshot in HBM, BF16x3
and FP32 y passes, rooflines tied to the committed counter summaries); and
the learned closure, trained on exact stresses of 192 x 129 x 192
snapshots, judged on held-out snapshots and on the production snapshot by
the <tau_12>(y) profile error, and timed against the exact path there.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "points/s for filt(u_i)+tau_ij filtering; MLP-closure speedup at stated tau error"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_VALU_PEAK_TF = 157.3      # MI355X vector FP32 (counts packed FP32: two FMAs per lane per cycle)
FP32_VALU_NONPACKED_TF = 78.6  # 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz: non-packed FMA issue
                               # limit (a wave64 v_fma_f32 takes four cycles; measured 72.6 TFLOP/s)
FP32_MFMA_PEAK_TF = 157.3      # dense FP32 matrix rate
BF16_MFMA_PEAK_TF = 2500.0     # dense BF16 matrix rate


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=50)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--workload", default="dns192")
    p.add_argument("--ygemm", default="fp32", choices=["fp32", "bf16", "bf16x3"])
    p.add_argument("--tail", type=float, default=1e-8)
    p.add_argument("--filter", default="gaussian", choices=["gaussian", "differential"],
                   help="the Gaussian filter of the benchmark configuration, or the paper's own "
                        "differential filter (1 - a^2 lap) ubar = u, a = 0.1")
    p.add_argument("--xz", default="matrix", choices=["matrix", "vector"],
                   help="x/z pass on the matrix cores (where it covers the grid) or the vector units")
    p.add_argument("--snapshots", type=int, default=4)
    p.add_argument("--skip-extras", action="store_true",
                   help="time only the stress (no LES-grid, production-shape, closure, inverse-filter or "
                        "error measurements): for profiler runs whose per-kernel figures must cover the "
                        "stress alone")
    p.add_argument("--production-steps", type=int, default=5,
                   help="timed steps of the 1024x385x768 production block")
    p.add_argument("--closure-train", type=int, default=32,
                   help="192x129x192 training snapshots of the closure block")
    p.add_argument("--closure-steps", type=int, default=20000, help="Adam steps of the closure block")
    p.add_argument("--cpu-seconds", type=float, default=12.0,
                   help="budget of the oracle CPU baseline (0 disables it)")
    p.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                   help="only run plain device-to-device copies of this many MiB "
                        "(reference dispatches for scaling the HBM byte counters)")
    return p.parse_args()


def copy_calibration(mib):
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": n * 4, "bytes_written": n * 4, "dispatches": 3}))


def pass_model(cfg, f, ops_nnz):
    """Algorithmic flops and bytes per grid point of each pass."""
    mx, mz = f.layout.mx, f.layout.mz
    return {
        # read u (3 x 4 B), write nine x/z-filtered fields (9 x 4 B);
        # 9 fields x (x taps + z taps) FMAs + 7 flops forming u1' and the products
        "xz": dict(bytes=48.0, flops=2.0 * 9 * ((2 * mx + 1) + (2 * mz + 1)) + 7.0),
        # read nine fields, write 3 ubar + 6 tau; 12 banded operator products
        "y": dict(bytes=72.0, flops=2.0 * 12 * ops_nnz + 12.0),
    }


def host_cpu():
    """nproc (the cores this process may use) and the CPU model name."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return len(os.sched_getaffinity(0)), model


def _time_oracle(fn, budget_s, max_reps=64):
    reps, t0 = 0, time.perf_counter()
    out = None
    while True:
        out = fn()
        reps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or reps >= max_reps:
            return reps, el, out


def cpu_baseline(cfg, u_host, budget_s):
    """The FP64 oracle timed on the host cores over whole snapshots: with the
    BLAS threads it uses by default, then on one thread."""
    from threadpoolctl import threadpool_info, threadpool_limits
    import numpy as np
    from oracle import filter_ref as R
    ops = R.Operators.from_config(cfg)
    u64 = u_host.astype(np.float64)
    reps, el, out = _time_oracle(lambda: R.sgs_stress(u64, ops), budget_s)
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    with threadpool_limits(limits=1):
        reps1, el1, _ = _time_oracle(lambda: R.sgs_stress(u64, ops), budget_s / 4, max_reps=8)
    nproc, model = host_cpu()
    return {"value": cfg.points * reps / el, "unit": "points/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"{reps} full {cfg.nx}x{cfg.ny}x{cfg.nz} snapshot(s), FP64 dense sums, {el:.1f} s",
            "nproc": nproc, "cpu_model": model,
            "one_thread": {"value": cfg.points * reps1 / el1, "unit": "points/s",
                           "sample": f"{reps1} snapshot(s), {el1:.1f} s"}}, out


def fast_transforms(cfg):
    """The library transforms x and z by FFTs when both lengths factor into
    2, 3 and 5 (and fit a block), else by the folded table products."""
    def smooth(n):
        for r in (2, 3, 5):
            while n % r == 0:
                n //= r
        return n == 1
    return all(smooth(n) and 2 <= n <= 8192 for n in (cfg.nx, cfg.nz))


def dfilter_pass_model(cfg, nf=9, products=True):
    """Algorithmic bytes and matrix-core flops per grid point of each pass of
    the differential filter: the stress (nine filtered fields, the first pass
    forming them from u) or plain filtering / inverse filtering of nf
    fields. Fast transforms are counted by their bytes alone (their vector
    work, O(log n) per point, is not the bound)."""
    fast = fast_transforms(cfg)
    def fwd(n):   # folded forward transform: cosines 0..h and sines 1..hs over nodes 1..h
        h, hs = n // 2, (n - 1) // 2
        return 0.0 if fast else 2.0 * h * (h + 1 + hs) / n
    def inv(n):   # folded inverse: P and Q sums for nodes 0..h over coefficients 1..h / 1..hs
        h, hs = n // 2, (n - 1) // 2
        return 0.0 if fast else 2.0 * (h + 1) * (h + hs) / n
    fb = 8.0 * nf   # one read and one write of the fields
    m = {
        # stress: reads u (3 fields), writes 9
        "x_fwd": dict(bytes=48.0 if products else fb, flops=nf * fwd(cfg.nx), kernel="dfilter_xf" if products else None),
        "z_fwd": dict(bytes=fb, flops=nf * fwd(cfg.nz), kernel="dfilter_zf" if products else None),
        "y_solve": dict(bytes=fb, flops=0.0, kernel="dfilter_y" if products else None),
        "z_inv": dict(bytes=fb, flops=nf * inv(cfg.nz), kernel="dfilter_zi" if products else None),
        "x_inv": dict(bytes=fb, flops=nf * inv(cfg.nx), kernel="dfilter_xi" if products else None),
    }
    if products:
        m["epilogue"] = dict(bytes=72.0, flops=0.0, kernel="dfilter_epi")   # 9 fields in, ubar + tau out
    return m


def dfilter_rooflines(cfg, model, prof, traffic_rec, counters):
    """Per pass: the larger of the matrix-core and HBM fractions, from the
    library's event timings."""
    roofs = {}
    for k, m in model.items():
        ms, nl = prof[k]
        t_k = ms / 1e3 / max(nl, 1)
        gbs = m["bytes"] * cfg.points / t_k / 1e9
        r = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS}
        if m["flops"] > 0:
            tfs = m["flops"] * cfg.points / t_k / 1e12
            if tfs / FP32_MFMA_PEAK_TF >= r["frac"]:
                r = {"bound": "mfma", "achieved": tfs, "peak": FP32_MFMA_PEAK_TF, "unit": "TFLOP/s",
                     "frac": tfs / FP32_MFMA_PEAK_TF,
                     "note": "folded real-transform multiply-adds on FP32 matrix cores; padding of the "
                             "16x16 tiles and the K steps past n/2 are not counted"}
        r["kernel"] = m["kernel"]
        r["us_avg"] = 1e6 * t_k
        tr = counters.current(traffic_rec, m["kernel"]) if m["kernel"] else None
        r["traffic"] = tr["bytes"] if tr else None
        roofs[k] = r
    return roofs


def dfilter_cpu_baseline(cfg, u_host, budget_s):
    """The FP64 differential-filter oracle timed on the host cores."""
    from threadpoolctl import threadpool_info
    import numpy as np
    from oracle import dfilter_ref as D
    ops = D.DOperators.from_config(cfg)
    u64 = u_host.astype(np.float64)
    reps, el, out = _time_oracle(lambda: D.sgs_stress(u64, ops), budget_s)
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    nproc, model = host_cpu()
    return {"value": cfg.points * reps / el, "unit": "points/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{reps} full {cfg.nx}x{cfg.ny}x{cfg.nz} snapshot(s), FP64 FFT + Thomas, {el:.1f} s",
            "nproc": nproc, "cpu_model": model}, out


def les_grid_measure(cfg, eles, torch, ubar, tau, steps):
    """The stress on the LES2 and LES4 grids (coarser by 2 and 4, linear
    interpolation as the discretization operator) from this run's DNS-grid
    outputs, timed with events on the library's stream, and the commutation
    error of the interpolation with the y derivative for ubar_1 and tau_12.
    Bytes: nine fields read at the DNS nodes the interpolation touches (the
    eight corners of every LES node, at most every DNS node) and nine LES
    fields written."""
    out = {}
    ns = len(ubar)
    for r in (2, 4):
        g = eles.LesGrid.coarsened(cfg, r)
        ul, T = g.stress(ubar[0], tau[0])
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for i in range(steps):
            g.stress(ubar[i % ns], tau[i % ns], ul, T)
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) / steps * 1e-3
        nles = g.les_shape[0] * g.les_shape[1] * g.les_shape[2]
        byt = 36.0 * (min(cfg.points, 8 * nles) + nles)
        c_u = float(g.commutation(ubar[0][0])[0])
        c_t = float(g.commutation(tau[0][1])[0])
        out[f"les{r}"] = {"shape": list(g.les_shape), "us": 1e6 * t, "bytes": byt,
                          "hbm_frac": byt / t / 1e9 / HBM_PEAK_GBS,
                          "commutation_error_ubar1": c_u, "commutation_error_tau12": c_t}
    return out


def run_differential(a):
    import numpy as np
    import torch
    from paper_1902_02508_amd import counters, eles, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cfg = synth.config(a.workload)
    seeds = synth.SEEDS.get(a.workload, [0, 1, 2, 3])[: a.snapshots]
    while len(seeds) < a.snapshots:
        seeds.append(seeds[-1] + 1)
    hosts, us = [], []
    for sd in seeds:
        y, u = synth.make_snapshot(cfg, sd)
        hosts.append(u)
        us.append(torch.from_numpy(u).to(dev))
    f = eles.DFilter.from_config(cfg, a=0.1, device=dev)
    ns = len(us)
    ubar = [torch.empty((3,) + f.shape, dtype=torch.float32, device=dev) for _ in range(ns)]
    tau = [torch.empty((6,) + f.shape, dtype=torch.float32, device=dev) for _ in range(ns)]
    stats = [torch.empty((9, cfg.ny), dtype=torch.float64, device=dev) for _ in range(ns)]

    def step(i):
        k = i % ns
        f.sgs_stress(us[k], ubar[k], tau[k], stats[k])

    for i in range(a.warmup):
        step(i)
    torch.cuda.synchronize()
    print(f"warmup done ({a.warmup} steps)", file=sys.stderr, flush=True)
    # per-pass durations in a loop of their own; the timed region brackets
    # only the dominant pass (each event pair adds a few microseconds)
    model = dfilter_pass_model(cfg)
    eles.dfilter_profile_begin(f.h, a.steps)
    for i in range(a.steps):
        step(i)
    prof_all = eles.dfilter_profile_end(f.h)
    dom = max(model, key=lambda k: prof_all[k][0] / max(prof_all[k][1], 1))

    eles.dfilter_profile_begin(f.h, a.steps, passes=[eles.DPASS_NAMES.index(dom)])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        step(i)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof_dom = eles.dfilter_profile_end(f.h)
    el = t1 - t0
    ms_per_step = 1e3 * el / a.steps
    value = cfg.points * a.steps / el
    print(f"timed {a.steps} steps: {ms_per_step:.4f} ms/step", file=sys.stderr, flush=True)
    prof = dict(prof_all)
    prof[dom] = prof_dom[dom]

    traffic_rec = counters.read_summary(os.path.join(ROOT, "profiles", f"hbm_traffic_{a.workload}_differential.md"))
    roofs = dfilter_rooflines(cfg, model, prof, traffic_rec, counters)
    for k in roofs:
        roofs[k]["timed"] = "timed region" if k == dom else "per-pass loop"
    passes = {k: {"us_avg": 1e3 * ms / max(n, 1), "launches": n} for k, (ms, n) in prof_all.items()}

    inverse, errors, two = None, None, None
    if not a.skip_extras:
        inverse, errors = dfilter_extras(cfg, eles, torch, f, us, ubar, a.steps, counters)
        f2 = eles.DFilter.from_config(cfg, a=0.1, device=dev)
        two = two_streams_block(cfg, a, f, f2, us, ubar, tau, stats, torch,
                                lambda msg: print(msg, file=sys.stderr, flush=True))
        del f2

    cpu = None
    parity = None
    if a.cpu_seconds > 0:
        from oracle import filter_ref as R
        cpu, (rub, rtau) = dfilter_cpu_baseline(cfg, hosts[0], a.cpu_seconds)
        f.sgs_stress(us[0], ubar[0], tau[0], stats[0])
        torch.cuda.synchronize()
        yv = synth.ygrid(cfg.ny, cfg.ykind, cfg.stretch)
        gu = ubar[0].cpu().numpy().astype(np.float64)
        gt = tau[0].cpu().numpy().astype(np.float64)
        parity = max([R.rel_l2(gu[k], rub[k], yv) for k in range(3)] +
                     [R.rel_l2(gt[k], rtau[k], yv) for k in range(6)])
    return cfg, value, ms_per_step, ns, roofs, dom, passes, cpu, parity, inverse, errors, two


def dfilter_extras(cfg, eles, torch, f, us, ubar, steps, counters):
    """The inverse filter of the three filtered velocities and the error
    measures of eqs. (13)-(15) against the unfiltered field, timed."""
    ns = len(us)
    back = torch.empty_like(ubar[0])
    eles.dfilter_profile_begin(f.h, steps)
    for i in range(steps):
        f.inverse(ubar[i % ns], [1, -1, 1], out=back)
    prof_i = eles.dfilter_profile_end(f.h)
    model_i = dfilter_pass_model(cfg, nf=3, products=False)
    roofs_i = dfilter_rooflines(cfg, model_i, prof_i, None, counters)
    dom_i = max(model_i, key=lambda k: prof_i[k][0])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    f.errors(back, us[0], 1.0, 1.0)
    e0.record()
    for i in range(steps):
        err = f.errors(back, us[(steps - 1) % ns], 1.0, 1.0)
    e1.record()
    torch.cuda.synchronize()
    t_err = e0.elapsed_time(e1) / steps * 1e-3
    err_bytes = 24.0 * cfg.points   # two velocity fields read once
    inverse = {"us_per_call": sum(1e3 * ms / max(n, 1) for ms, n in prof_i.values()),
               "passes": {k: round(1e3 * ms / max(n, 1), 2) for k, (ms, n) in prof_i.items() if n},
               "roofline": roofs_i[dom_i], "fields": 3,
               "round_trip_errors_eq13_15": [float(v) for v in err.cpu().numpy()]}
    errors = {"us_per_call": 1e6 * t_err, "bytes": err_bytes,
              "roofline": {"bound": "hbm", "achieved": err_bytes / t_err / 1e9, "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": err_bytes / t_err / 1e9 / HBM_PEAK_GBS}}
    return inverse, errors


def main_differential(a):
    cfg, value, ms_per_step, ns, roofs, dom, passes, cpu, parity, inverse, errors, two = run_differential(a)
    line = {
        "metric": METRIC, "value": value, "unit": "points/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "fp32", "data": "synthetic",
        "config": {"workload": f"channel {cfg.nx}x{cfg.ny}x{cfg.nz} exact filtered velocity + tau_ij, "
                               "differential filter",
                   "filter": "differential", "a": 0.1,
                   "box": f"{cfg.lx:.4f}x2x{cfg.lz:.4f}", "snapshots": ns, "parallelism": "none"},
        "roofline": roofs[dom],
        "rooflines": roofs,
        "cpu_baseline": cpu,
        "passes": passes,
        "max_rel_l2_vs_oracle": parity,
        "inverse_filter": inverse,
        "errors_eq13_15": errors,
        "two_streams": two,
    }
    print(json.dumps(line), flush=True)


def measure_exact(cfg, ygemm, tail, xz, snapshots, steps, warmup, seeds, torch, eles, synth, counters,
                  np, traffic_name, log):
    """Time the exact stress path (sgs_stress: shift, x/z, y, statistics) on
    snapshots resident in HBM. Per-pass durations come from a loop of their
    own (an event pair between two kernels adds a few microseconds); the
    timed region brackets only the dominant pass with events, so its
    roofline is measured live."""
    dev = torch.device("cuda:0")
    us = []
    for s in seeds[:snapshots]:
        y, terms = synth.snapshot_factors(cfg, s)
        us.append(synth.assemble_on_device(cfg, terms, dev))
    f = eles.Filter.from_config(cfg, tail_tol=tail, ygemm=ygemm, device=dev)
    matrix_xz = xz == "matrix" and f.layout.xz_waves > 0
    if f.layout.xz_waves > 0:
        f.set_xz(matrix_xz)
    ns = len(us)
    ubar = [torch.empty((3,) + f.shape, dtype=torch.float32, device=dev) for _ in range(ns)]
    tau = [torch.empty((6,) + f.shape, dtype=torch.float32, device=dev) for _ in range(ns)]
    stats = [torch.empty((9, cfg.ny), dtype=torch.float64, device=dev) for _ in range(ns)]

    def step(i):
        k = i % ns
        f.sgs_stress(us[k], ubar[k], tau[k], stats[k])

    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    log(f"warmup done ({warmup} steps)")
    eles.filter_profile_begin(f.h, steps)
    for i in range(steps):
        step(i)
    prof_all = eles.filter_profile_end(f.h)
    dom = max(("xz", "y"), key=lambda k: prof_all[k][0] / max(prof_all[k][1], 1))

    eles.filter_profile_begin(f.h, steps, passes=[eles.PASS_NAMES.index(dom)])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step(i)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof_dom = eles.filter_profile_end(f.h)
    el = t1 - t0
    ms_per_step = 1e3 * el / steps
    value = cfg.points * steps / el
    log(f"timed {steps} steps: {ms_per_step:.4f} ms/step")
    prof = dict(prof_all)
    prof[dom] = prof_dom[dom]

    ops = f.operators()
    nnz = float(np.count_nonzero(ops["wp"])) / cfg.ny
    model = pass_model(cfg, f, nnz)
    passes = {k: {"us_avg": 1e3 * ms / max(n, 1), "launches": n} for k, (ms, n) in prof_all.items()}
    traffic_rec = counters.read_summary(os.path.join(ROOT, "profiles", f"hbm_traffic_{traffic_name}.md"))
    staged = f.layout.y_groups > 0 and ygemm == "fp32"
    xz_name = ("k_xzw" if f.layout.xz_wide else "k_xzm") if matrix_xz else "k_xz"
    names = {"xz": xz_name, "y": "k_ys" if staged else "k_y_" + ygemm}
    roofs = {}
    for k in ("xz", "y"):
        t_k = prof[k][0] / 1e3 / max(prof[k][1], 1)
        gbs = model[k]["bytes"] * cfg.points / t_k / 1e9
        r = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS}
        if k == "xz":
            tfs = model[k]["flops"] * cfg.points / t_k / 1e12
            if matrix_xz:
                if tfs / FP32_MFMA_PEAK_TF >= r["frac"]:
                    r = {"bound": "mfma", "achieved": tfs, "peak": FP32_MFMA_PEAK_TF, "unit": "TFLOP/s",
                         "frac": tfs / FP32_MFMA_PEAK_TF,
                         "note": "algorithmic stencil flops on FP32 matrix cores; the 16x16 band "
                                 "products also multiply the zero taps at the band edges"}
            elif tfs / FP32_VALU_PEAK_TF >= r["frac"]:
                r = {"bound": "alu", "achieved": tfs, "peak": FP32_VALU_PEAK_TF, "unit": "TFLOP/s",
                     "frac": tfs / FP32_VALU_PEAK_TF,
                     "note": "peak counts packed FP32; with packed FP32 disabled the issue limit is "
                             f"{FP32_VALU_NONPACKED_TF} TFLOP/s"}
        r["kernel"] = names[k]
        r["us_avg"] = 1e6 * t_k
        r["timed"] = "timed region" if k == dom else "per-pass loop"
        tr = counters.current(traffic_rec, names[k])
        r["traffic"] = tr["bytes"] if tr else None
        if tr:
            r["traffic_source_sha256"] = tr["source_sha256"]
        roofs[k] = r
    return dict(f=f, us=us, ubar=ubar, tau=tau, stats=stats, value=value, ms_per_step=ms_per_step,
                roofs=roofs, dom=dom, passes=passes, matrix_xz=matrix_xz, ns=ns)


def two_streams_block(cfg, a, f, f2, us, ubar, tau, stats, torch, log):
    """The same exact path with snapshots alternating between two streams,
    each with a filter handle of its own (f2 a second handle of f's
    configuration: a handle's per-call state is not shared between calls in
    flight), so that one snapshot's later passes can run beside the next
    snapshot's first ones: steady-state throughput of one and of two streams
    over the same resident snapshots (at least 200 snapshots each, the
    overlap needs a few to fill), and the outputs compared bitwise with the
    one-stream run's."""
    fs = [f, f2]
    ns = len(us)
    ub2 = [torch.empty_like(t) for t in ubar]
    ta2 = [torch.empty_like(t) for t in tau]
    st2 = [torch.empty_like(t) for t in stats]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]

    def step(i):
        # snapshot k, its outputs and its handle stay on stream k mod 2
        k = i % ns
        with torch.cuda.stream(streams[k % 2]):
            fs[k % 2].sgs_stress(us[k], ub2[k], ta2[k], st2[k])

    def one(i):
        k = i % ns
        f.sgs_stress(us[k], ubar[k], tau[k], stats[k])

    n = max(a.steps, 200)
    el = {}
    for name, fn in (("one", one), ("two", step)):
        torch.cuda.synchronize()
        for i in range(max(a.warmup, 4)):
            fn(i)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(n):
            fn(i)
        torch.cuda.synchronize()
        el[name] = time.perf_counter() - t0
    # both loops covered every snapshot (n >= ns), one after the other, so
    # ubar/tau/stats hold the one-stream outputs and ub2/ta2/st2 the
    # two-stream ones; f is never used on two streams at once
    same = all(torch.equal(x, y) for x, y in zip(ubar + tau + stats, ub2 + ta2 + st2))
    v1, v2 = cfg.points * n / el["one"], cfg.points * n / el["two"]
    log(f"two streams: {1e3 * el['two'] / n:.4f} ms per snapshot (one stream {1e3 * el['one'] / n:.4f})")
    return {"points_per_s": v2, "ms_per_snapshot": 1e3 * el["two"] / n, "one_stream_points_per_s": v1,
            "speedup_vs_one_stream": v2 / v1, "snapshots_timed": n, "streams": 2, "handles": 2,
            "bitwise_equal_to_one_stream": same}


def production_block(a, torch, eles, synth, counters, np, log):
    """The production shape, 1024 x 385 x 768 (one snapshot resident in
    HBM): the exact path with the BF16x3 y pass (the configured production
    arithmetic) and with FP32, per-pass rooflines tied to the committed
    counter summaries."""
    cfg = synth.config("dns1024")
    seeds = synth.SEEDS["dns1024"]
    out = {"workload": f"channel {cfg.nx}x{cfg.ny}x{cfg.nz} exact filtered velocity + tau_ij",
           "snapshots": 1, "steps": a.production_steps}
    keep = None
    for mode in ("bf16x3", "fp32"):
        r = measure_exact(cfg, mode, a.tail, "matrix", 1, a.production_steps, 1, seeds, torch, eles, synth,
                          counters, np, "dns1024" if mode == "fp32" else "dns1024_bf16x3", log)
        out[mode] = {"points_per_s": r["value"], "ms_per_step": r["ms_per_step"], "roofline": r["roofs"][r["dom"]],
                     "rooflines": r["roofs"], "passes": r["passes"]}
        if mode == "fp32":
            keep = r
        else:
            del r
        torch.cuda.empty_cache()
    return out, cfg, keep


def closure_block(a, torch, eles, synth, np, prod_cfg, prod, log):
    """The learned closure (row a8/a9): trained on exact stresses of
    192 x 129 x 192 snapshots, judged on held-out ones and on the production
    snapshot by the eq. (14)-form error of <tau_12>(y) against the exact
    path's FP64 statistics, and timed against the exact path."""
    from paper_1902_02508_amd import experiment as X
    dev = torch.device("cuda:0")
    cfg = synth.config("dns192")
    f = eles.Filter.from_config(cfg, tail_tol=a.tail, device=dev)
    t0 = time.perf_counter()
    feats, taus = X.build_dataset(f, cfg, synth.SEEDS["train"][:a.closure_train], dev, log=log)
    fm, tm = eles.moments(feats).cpu().numpy(), eles.moments(taus).cpu().numpy()
    norms = np.concatenate([fm[0], fm[1], tm[0], tm[1]])
    cl = eles.Closure(X.init_params(1), norms, device=dev, gm_coef=X.widths_coef(cfg))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lh = cl.train(feats, taus, steps=a.closure_steps, batch=65536, seed=1, lr=1e-3)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    loss = lh.cpu().numpy()
    del feats, taus
    torch.cuda.empty_cache()
    rows = X.evaluate(cl, f, cfg, synth.SEEDS["heldout"], dev, baseline=X.gradient_model_closure(cfg, norms, dev))
    res = {"train": {"snapshots": a.closure_train, "steps": a.closure_steps, "batch": 65536,
                     "seconds": t2 - t1, "dataset_seconds": t1 - t0,
                     "loss_first": float(loss[:10].mean()), "loss_last": float(loss[-100:].mean())},
           "heldout": {"snapshots": len(rows),
                       "tau12_profile_error": float(np.mean([r["tau12_profile_error"] for r in rows])),
                       "tau12_profile_error_gradient_model":
                           float(np.mean([r["tau12_profile_error_gradient_model"] for r in rows])),
                       "tau12_profile_error_zero": 1.0,
                       "pointwise_rel_l2": [float(np.mean([r["pointwise_rel_l2"][q] for r in rows]))
                                            for q in range(6)],
                       "pointwise_rel_l2_gradient_model": [
                           float(np.mean([r["pointwise_rel_l2_gradient_model"][q] for r in rows])) for q in range(6)]}}
    if prod is not None:
        # closure inference on the production snapshot's filtered velocity,
        # the exact path (FP32 y pass) as the judge
        pf, ub, st = prod["f"], prod["ubar"][0], prod["stats"][0]
        pred = torch.empty((6,) + pf.shape, dtype=torch.float32, device=dev)
        pst = torch.empty((6, prod_cfg.ny), dtype=torch.float64, device=dev)
        for mode in (eles.INFER_UNCHECKED, eles.INFER_CHECK):
            cl.infer(pf, ub, pred, pst, fallback=mode)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(a.production_steps):
                cl.infer(pf, ub, pred, pst, fallback=mode)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            key = "closure_points_per_s" if mode == eles.INFER_CHECK else "closure_points_per_s_unchecked"
            res.setdefault("production", {})[key] = prod_cfg.points * a.production_steps / el
        y = synth.ygrid(prod_cfg.ny, prod_cfg.ykind, prod_cfg.stretch)
        p = res["production"]
        p["tau12_profile_error"] = X.profile_error(pst[1].cpu().numpy(), st[4].cpu().numpy(), y)
        p["exact_fp32_points_per_s"] = prod["value"]
        p["speedup_vs_exact_fp32"] = p["closure_points_per_s"] / prod["value"]
        p["workload"] = f"channel {prod_cfg.nx}x{prod_cfg.ny}x{prod_cfg.nz}, seed {synth.SEEDS['dns1024'][0]}"
    return res


def main():
    a = parse()
    if a.copy_calibration:
        copy_calibration(a.copy_calibration)
        return
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {a.gpus} is not supported "
              "(snapshots are independent: run one process per GPU)", file=sys.stderr)
        sys.exit(2)
    if a.filter == "differential":
        main_differential(a)
        return
    import numpy as np
    import torch
    from paper_1902_02508_amd import counters, eles, synth

    def log(m):
        print(m, file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cfg = synth.config(a.workload)
    seeds = list(synth.SEEDS.get(a.workload, [0, 1, 2, 3]))
    while len(seeds) < a.snapshots:
        seeds.append(seeds[-1] + 1)
    traffic = a.workload if a.ygemm == "fp32" else f"{a.workload}_{a.ygemm}"
    m = measure_exact(cfg, a.ygemm, a.tail, a.xz, a.snapshots, a.steps, a.warmup, seeds, torch, eles, synth,
                      counters, np, traffic, log)
    f, us, ubar, tau, stats = m["f"], m["us"], m["ubar"], m["tau"], m["stats"]

    les = None if a.skip_extras else les_grid_measure(cfg, eles, torch, ubar, tau, a.steps)

    cpu = None
    parity = None
    if a.cpu_seconds > 0:
        cpu, (rub, rtau) = cpu_baseline(cfg, us[0].cpu().numpy(), a.cpu_seconds)
        from oracle import filter_ref as R
        f.sgs_stress(us[0], ubar[0], tau[0], stats[0])
        torch.cuda.synchronize()
        yv = synth.ygrid(cfg.ny, cfg.ykind, cfg.stretch)
        gu = ubar[0].cpu().numpy().astype(np.float64)
        gt = tau[0].cpu().numpy().astype(np.float64)
        parity = max([R.rel_l2(gu[k], rub[k], yv) for k in range(3)] +
                     [R.rel_l2(gt[k], rtau[k], yv) for k in range(6)])

    two = None
    if not a.skip_extras:
        f2 = eles.Filter.from_config(cfg, tail_tol=a.tail, ygemm=a.ygemm, device=dev)
        if f2.layout.xz_waves > 0:
            f2.set_xz(m["matrix_xz"])
        two = two_streams_block(cfg, a, f, f2, us, ubar, tau, stats, torch, log)
        del f2

    head = {"value": m["value"], "ms_per_step": m["ms_per_step"], "roofline": m["roofs"][m["dom"]],
            "rooflines": m["roofs"], "passes": m["passes"], "matrix_xz": m["matrix_xz"], "ns": m["ns"],
            "layout": f.layout}
    production = closure = None
    if not a.skip_extras and a.workload == "dns192":
        del m, f, us, ubar, tau, stats
        torch.cuda.empty_cache()
        production, pcfg, prod = production_block(a, torch, eles, synth, counters, np, log)
        closure = closure_block(a, torch, eles, synth, np, pcfg, prod, log)
        del prod
        torch.cuda.empty_cache()

    lay = head["layout"]
    line = {
        "metric": METRIC, "value": head["value"], "unit": "points/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "fp32" if a.ygemm == "fp32" else a.ygemm, "data": "synthetic",
        "config": {"workload": f"channel {cfg.nx}x{cfg.ny}x{cfg.nz} exact filtered velocity + tau_ij",
                   "box": f"{cfg.lx:.4f}x2x{cfg.lz:.4f}", "widths": [cfg.delta_x, cfg.delta_y, cfg.delta_z],
                   "tail_tol": a.tail, "ygemm": a.ygemm, "xz": "matrix" if head["matrix_xz"] else "vector",
                   "snapshots": head["ns"], "stencil_half_widths": [lay.mx, lay.mz], "parallelism": "none"},
        "roofline": head["roofline"],
        "rooflines": head["rooflines"],
        "cpu_baseline": cpu,
        "passes": head["passes"],
        "max_rel_l2_vs_oracle": parity,
        "les_grid": les,
        "two_streams": two,
        "production": production,
        "closure": closure,
    }
    print(json.dumps(line), flush=True)

if __name__ == "__main__":
    main()
