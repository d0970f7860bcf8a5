"""Benchmark: site updates/s of the metric semi-Lagrangian Vlasov-Poisson
engine on one MI355X, mixed precision next to plain FP64, with the roofline
of the dominant kernel and the CPU oracle timed on the host.

A step is one drift-kick-drift step of the whole hot path over the grid
(element predictor and records, nearest-element query + inverse map +
six-point interpolation + column sums, cumulative-mass force, kick and
corrector), with the resampling (remap evaluation + cubic B-spline fit)
every n_s steps included in the timed region.  A site update is one grid
site reconstructed in one step.

Workload: 2048^2 grid on [-1, 1]^2, elements every 8th site (256^2), a seeded
sum of 4 Gaussian halos (synthetic; it stands in for the paper's random set
of clouds), dt = 5e-4, remap every 50 steps; the default 2000 timed steps are
the whole run.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("site updates/s mixed vs FP64 at 2048^2 (% HBM peak); "
          "p50/p99 solve latency")
HBM_PEAK_GBS = 8000.0


def kernel_source_hash() -> str:
    """Hash of the engine's code with comments and trailing blanks removed,
    so that a traffic record stays valid across comment-only edits."""
    import re
    h = hashlib.sha256()
    for f in ("paper_1705_03750_amd/csrc/vp_kernels.hpp",
              "paper_1705_03750_amd/csrc/vp_engine.hip"):
        with open(os.path.join(ROOT, f), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        lines = [ln.rstrip() for ln in text.splitlines()]
        h.update("\n".join(ln for ln in lines if ln).encode())
    return h.hexdigest()[:16]


WARM_S = 0.5                    # least seconds of warm-up per timed run
FP64_PEAK_TFLOPS = 78.6          # MI355X FP64 vector, FMA counted as 2
FLOPS_PER_EVAL = 34             # one full candidate evaluation, FP64
EVALS_PER_SITE = 4              # windows holding a site (2 per axis)


def recon_algorithmic_bytes(n: int, s: int, fbytes: int) -> dict:
    """Bytes one launch of the transport reconstruction must move: F_ini
    read once, each element's query data (position, A, H: 12 doubles) read
    once, and the column partial sums (one double per column per 64-row
    group) written once."""
    E = (n // s) ** 2
    ngy = n // 64 + 1
    b_f = n * n * fbytes
    b_e = E * 12 * 8
    b_p = ngy * n * 8
    return {"F_ini": b_f, "elements": b_e, "partials": b_p,
            "total": b_f + b_e + b_p}


def recon_algorithmic_flops(n: int) -> float:
    """FP64 flops one launch must do: every site lies in the validity
    windows of 4 elements (half-width = element spacing, 2 per axis), and
    each of them needs the full inverse map and distance (2 sub, 2 mul +
    2 fma for l, 3 mul for the monomials, 2 x (mul + 2 fma) for u, 4 fma
    for dQ, 2 mul + mul + fma for d^2: 34 flops).  The six-point
    interpolation and the column sums are not counted."""
    return float(n) * n * EVALS_PER_SITE * FLOPS_PER_EVAL


def run_gpu(precision: str, cfg, f0, steps: int, warmup: int, **extra):
    """Warm up, then time the whole run twice from t = 0: once plain (the
    reported throughput), once with the engine's per-launch HIP events on
    its stream (the per-kernel durations; the events add a few microseconds
    of gap per launch, so this pass is not the throughput)."""
    import torch
    import paper_1705_03750_amd as vp
    p = cfg.params(precision)
    p.update(extra)
    run = vp.VlasovRun(device="cuda:0", **{k: v for k, v in p.items()
                                           if k != "precision"},
                       precision=precision)
    f0t = torch.as_tensor(f0, device="cuda:0")
    run.init_conditions(f0t)
    if warmup:
        # the warm-up steps, repeated until the device has been busy for
        # WARM_S seconds: its clocks rise under sustained load, and the
        # first leg measured would otherwise run partly before they have
        t_w = time.perf_counter()
        run.step(warmup)
        torch.cuda.synchronize()
        while time.perf_counter() - t_w < WARM_S:
            run.step(warmup)
            torch.cuda.synchronize()
    out = {}
    for prof in (False, True):
        run.init_conditions(f0t)        # timed region = the run from t = 0
        run.sync()
        torch.cuda.synchronize()
        if prof:
            run.prof_begin(steps + 8)
        t0 = time.perf_counter()
        run.step(steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if prof:
            out["kernels"] = run.prof_end()
            out["ms_per_step_profiled"] = 1e3 * (t1 - t0) / steps
        else:
            dt = t1 - t0
            out.update({"seconds": dt, "ms_per_step": 1e3 * dt / steps,
                        "value": cfg.n * cfg.n * steps / dt})
    run.sync()
    out["diag"] = run.diagnostics()
    run.close()
    return out


def whole_cycles(steps: int, n_s: int) -> int:
    """The timed window rounded up to whole resampling cycles, so that the
    resampling (remap evaluation and spline fit, every n_s steps) is part of
    every measured rate in its own proportion."""
    if n_s <= 0:
        return steps
    return max(1, -(-steps // n_s)) * n_s


def mixed_error_leg(plan=(("c2_halos_2048", None), ("c3_halos_sheet_8192",
                                                    None))):
    """Error of the mixed-precision path against the FP64 path on the GPU
    (which the tests hold to the FP64 oracle at 1e-12), over whole runs of
    the workloads: the 2048^2 halo run (2000 steps) and the 8192^2 halo +
    sheet run (4000 steps), each from the same f0.  Reported: relative L2
    of f at the end, |drift_mixed - drift_fp64| of the total energy
    (drift = (E_end - E_0) / |E_0|, section 3.2), the same for the mass,
    and the fraction of sites whose nearest element differs at the end."""
    import torch
    import paper_1705_03750_amd as vp
    import workloads as W
    out = {}
    for name, steps in plan:
        cfg, f0 = W.config(name)
        steps = steps or cfg.steps
        f0t = torch.as_tensor(f0, device="cuda:0")
        del f0
        res = {}
        for prec in ("mixed", "fp64"):
            p = {k: v for k, v in cfg.params(prec).items() if k != "precision"}
            g = vp.VlasovRun(device="cuda:0", precision=prec, **p)
            g.init_conditions(f0t)
            d0 = g.diagnostics()
            t0 = time.perf_counter()
            g.step(steps)
            g.sync()
            secs = time.perf_counter() - t0
            d1 = g.diagnostics()
            res[prec] = {"f": g.reconstruct_f().to(torch.float64),
                         "assign": g.assignment(),
                         "e0": d0["energy"], "e1": d1["energy"],
                         "m0": d0["mass"], "m1": d1["mass"],
                         "seconds": secs, "t": d1["t"]}
            g.sync()
            g.close()
            del g
        m, f = res["mixed"], res["fp64"]
        rel_l2 = float(torch.linalg.vector_norm(m["f"] - f["f"]) /
                       torch.linalg.vector_norm(f["f"]))
        drift = {k: (r["e1"] - r["e0"]) / abs(r["e0"]) for k, r in res.items()}
        mdrift = {k: (r["m1"] - r["m0"]) / abs(r["m0"]) for k, r in res.items()}
        out[name] = {
            "grid": cfg.n, "element_stride": cfg.s, "steps": steps,
            "resamplings": steps // cfg.n_s if cfg.n_s else 0,
            "t_end": f["t"],
            "rel_l2_f": rel_l2, "rel_l2_f_target": 1e-5,
            "energy_drift_mixed": drift["mixed"],
            "energy_drift_fp64": drift["fp64"],
            "energy_drift_diff": abs(drift["mixed"] - drift["fp64"]),
            "energy_drift_diff_target": 1e-6,
            "mass_drift_diff": abs(mdrift["mixed"] - mdrift["fp64"]),
            "assignment_differs_frac": float(
                (m["assign"] != f["assign"]).double().mean()),
            "seconds": {k: r["seconds"] for k, r in res.items()},
            "within_targets": bool(rel_l2 <= 1e-5 and
                                   abs(drift["mixed"] - drift["fp64"]) <= 1e-6),
        }
        del res, m, f, f0t
        torch.cuda.empty_cache()
    return out


def host_io_leg(cfg, f0, steps: int, warmup: int):
    """The same run with its input and output in host memory: f0 handed
    over as a host pointer (the library stages it through device memory
    itself), the steps, then f reconstructed and copied back to host memory.
    The rate counts the transfers; the device-resident figure (the initial
    condition already on the device, f left there) is timed beside it with
    the same clock, so the two differ only by the host hand-over."""
    import ctypes as C
    import torch
    import paper_1705_03750_amd as vp
    p = cfg.params("mixed")
    run = vp.VlasovRun(device="cuda:0", **{k: v for k, v in p.items()
                                           if k != "precision"},
                       precision="mixed")
    f0h = np.ascontiguousarray(f0, dtype=np.float64)
    f0t = torch.as_tensor(f0h, device="cuda:0")
    run.init_conditions(f0t)
    run.step(warmup)
    run.sync()
    out = {}
    for where in ("device", "host"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if where == "host":
            rc = vp.lib().vp_init_conditions(
                run.h, f0h.ctypes.data_as(C.c_void_p), 0)
            if rc != 0:
                raise RuntimeError(f"vp_init_conditions (host): {rc}")
        else:
            run.init_conditions(f0t)
        run.sync()
        t1 = time.perf_counter()
        run.step(steps)
        run.sync()
        t2 = time.perf_counter()
        f = run.reconstruct_f()
        if where == "host":
            f = f.cpu()
        run.sync()
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        out[where] = {"init_ms": 1e3 * (t1 - t0), "steps_ms": 1e3 * (t2 - t1),
                      "f_out_ms": 1e3 * (t3 - t2),
                      "value": cfg.n * cfg.n * steps / (t3 - t0)}
    run.close()
    h, d = out["host"], out["device"]
    return {"what": f"one {steps}-step run from f0 to f: host f0 (FP64, "
                    f"{f0h.nbytes >> 20} MiB, pageable) in, f (FP32) out, "
                    "against the same run device-resident; init includes "
                    "the spline fit and the element reset",
            "unit": "site updates/s", "steps": steps,
            "value": h["value"], "device_resident_value": d["value"],
            "host": h, "device": d,
            "transfer_ms": (h["init_ms"] - d["init_ms"]) +
                           (h["f_out_ms"] - d["f_out_ms"])}


def large_grid_leg(plan=(("c3_halos_sheet_8192", 200),
                         ("c5_halos_cold_16384", 100))):
    """The two large workloads, mixed and FP64, each timed over a bounded
    prefix of its run from t = 0 (resamplings included): the 8192^2 halo +
    sheet workload (s = 8, remap every 50 steps) and the 16384^2 halo + cold
    workload (s = 16, remap every 20 steps).  Reconstruction rates are the
    same algorithmic flop and byte counts as the headline's, per launch."""
    import torch
    import workloads as W
    out = {}
    for name, steps in plan:
        cfg, f0 = W.config(name)
        row = {"grid": cfg.n, "element_stride": cfg.s, "n_s": cfg.n_s,
               "steps": steps}
        for prec in ("mixed", "fp64"):
            r = run_gpu(prec, cfg, f0, steps, 10)
            ms, cnt = r["kernels"]["recon"]
            avg_s = ms / cnt / 1e3
            flops = recon_algorithmic_flops(cfg.n)
            alg = recon_algorithmic_bytes(cfg.n, cfg.s,
                                          4 if prec == "mixed" else 8)
            row[prec] = {
                "value": r["value"], "ms_per_step": r["ms_per_step"],
                "recon_avg_launch_us": avg_s * 1e6,
                "recon_alu_frac": flops / avg_s / 1e12 / FP64_PEAK_TFLOPS,
                "recon_hbm_GBps": alg["total"] / avg_s / 1e9,
                "kernels_ms_per_step": {k: v[0] / steps for k, v in
                                        r["kernels"].items() if v[1]}}
            del r
            torch.cuda.empty_cache()
        row["mixed_over_fp64"] = row["mixed"]["value"] / row["fp64"]["value"]
        out[name] = row
        del f0
    return out


def variable_step_leg(cfg, f0, steps: int, warmup: int, fixed: dict):
    """The same workload with the variable step of section 2.4: C_dyn set so
    that the first step is half the nominal dt (which becomes the cap); the
    steps then follow the density.  Same step count as the fixed run."""
    g = np.array(f0, dtype=np.float64)
    g[0, :] = g[-1, :] = 0.0
    g[:, 0] = g[:, -1] = 0.0
    dv = 2.0 / cfg.n
    c_dyn = 0.5 * cfg.dt * math.sqrt((dv * g.sum(axis=0)).max())
    r = run_gpu("mixed", cfg, f0, steps, warmup, c_dyn=c_dyn)
    return {"c_dyn": c_dyn, "value": r["value"],
            "ms_per_step": r["ms_per_step"],
            "over_fixed_step_time": r["ms_per_step"] / fixed["ms_per_step"],
            "t_end": r["diag"]["t"], "dt_end": r["diag"]["dt"],
            "dt_first": min(cfg.dt, c_dyn / math.sqrt(
                (dv * g.sum(axis=0)).max())),
            "simulated_time_per_s": r["diag"]["t"] / r["seconds"]}


def emap_leg(cfg, f0, steps: int, warmup: int, fixed: dict,
             every: int = 10):
    """Adaptive resampling (end of section 2.3.3) on the same workload: no
    fixed schedule; every `every` steps E_map of the current elements is
    computed and the run resamples when it exceeds the value the fixed
    schedule reaches one step before its first resampling.  Same step
    count as the fixed run; the resamplings are counted from the engine's
    per-launch events (second pass)."""
    import torch
    import paper_1705_03750_amd as vp
    p = {k: v for k, v in cfg.params("mixed").items() if k != "precision"}
    f0t = torch.as_tensor(f0, device="cuda:0")
    g = vp.VlasovRun(device="cuda:0", precision="mixed", **p)
    g.init_conditions(f0t)
    g.step(cfg.n_s - 1)
    thr = g.diagnostics()["emap"]
    g.close()
    pa = dict(p, n_s=0, emap_max=thr, emap_every=every)
    g = vp.VlasovRun(device="cuda:0", precision="mixed", **pa)
    g.init_conditions(f0t)
    if warmup:
        g.step(warmup)
    out = {"emap_max": thr, "emap_every": every}
    for prof in (False, True):
        g.init_conditions(f0t)
        g.sync()
        torch.cuda.synchronize()
        if prof:
            g.prof_begin(3 * steps + 16)
        t0 = time.perf_counter()
        g.step(steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if prof:
            kern = g.prof_end()
            n_rm = kern["remap_eval"][1]
            out.update({"resamplings": n_rm,
                        "steps_per_resampling": steps / max(1, n_rm),
                        "fixed_schedule_resamplings": steps // cfg.n_s})
        else:
            out.update({"value": cfg.n * cfg.n * steps / (t1 - t0),
                        "ms_per_step": 1e3 * (t1 - t0) / steps,
                        "over_fixed_step_time": 1e3 * (t1 - t0) / steps /
                        fixed["ms_per_step"]})
    d = g.diagnostics()
    out.update({"mass": d["mass"], "energy": d["energy"], "emap_end": d["emap"]})
    g.close()
    return out


def periodic_leg(steps: int, warmup: int):
    """The periodic-x variant at the same size: an electron plasma on a ring
    (two-stream instability, 2048^2, elements every 8th site, dt 0.05,
    remap every 50 steps), mixed precision; its reconstruction kernel is the
    nearest-image instantiation."""
    import workloads as W
    cfg, f0 = W.config("p2_two_stream_2048")
    r = run_gpu("mixed", cfg, f0, steps, warmup)
    ms, n = r["kernels"]["recon"]
    avg_s = ms / n / 1e3
    achieved = recon_algorithmic_flops(cfg.n) / avg_s / 1e12
    return {"workload": "p2_two_stream_2048: 2048^2 on [0, 10 pi) x [-8, 8], "
                        "x periodic, G = -1/2 (electron plasma), beams at "
                        "+-2.4, dt 0.05, remap every 50 steps",
            "value": r["value"], "unit": "site updates/s",
            "ms_per_step": r["ms_per_step"],
            "recon_avg_launch_us": avg_s * 1e6,
            "recon_alu_frac": achieved / FP64_PEAK_TFLOPS,
            "t_end": r["diag"]["t"],
            "energy": r["diag"]["energy"],
            "kernels_ms_per_step": {k: v[0] / steps
                                    for k, v in r["kernels"].items() if v[1]}}


# 4D reconstruction: one full candidate evaluation (l = A dP 28, u = l^T H l
# 140, dQ 48, d^2 10 FP64 flops) for each of the 2^4 windows holding a site
FLOPS_PER_EVAL_4D = 226
EVALS_PER_SITE_4D = 16


def four_d_leg(steps: int = 20):
    """The 4D phase-space engine (2D periodic space x 2D velocity): a
    Maxwellian plasma with seeded low-mode perturbations on 64^4 sites,
    elements every 4th site per axis, dt 0.1, resampling every 10 steps,
    mixed precision.  Times the run from t = 0 (plain pass), then the
    per-kernel durations with HIP events (second pass)."""
    import torch
    import paper_1705_03750_amd.vp4 as v4
    import workloads as W
    ns = nv = 64
    L, vmax = 4.0 * math.pi, 6.0
    f0 = torch.as_tensor(W.landau4(ns, nv, L, vmax, 0.05, seed=1),
                         device="cuda:0")
    g = v4.VlasovRun4(device="cuda:0", ns=ns, nv=nv, L=L, vmax=vmax, ss=4,
                      sv=4, G=-0.5, dt=0.1, n_s=10, precision="mixed")
    g.init_conditions(f0)
    g.step(2)
    out = {}
    for prof in (False, True):
        g.init_conditions(f0)
        g.sync()
        torch.cuda.synchronize()
        if prof:
            g.prof_begin(2 * steps + 8)
        t0 = time.perf_counter()
        g.step(steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if prof:
            kern = g.prof_end()
        else:
            secs = t1 - t0
    n4 = ns * ns * nv * nv
    ms, n = kern["recon"]
    avg_s = ms / n / 1e3
    flops = FLOPS_PER_EVAL_4D * EVALS_PER_SITE_4D * n4
    achieved = flops / avg_s / 1e12
    d = g.diagnostics()
    g.close()
    return {"workload": "q4_landau_64: 64^4 sites, x, y periodic on [0, 4 pi), "
                        "u, w on [-6, 6), G = -1/2, elements every 4th site, "
                        "dt 0.1, resampling every 10 steps, mixed precision",
            "value": n4 * steps / secs, "unit": "site updates/s",
            "ms_per_step": 1e3 * secs / steps, "steps": steps,
            "recon_avg_launch_us": avg_s * 1e6,
            "recon_roofline": {"bound": "alu", "achieved": achieved,
                               "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                               "frac": achieved / FP64_PEAK_TFLOPS,
                               "algorithmic_flops_per_launch": flops},
            "kernels_ms_per_step": {k: v[0] / steps for k, v in kern.items()
                                    if v[1]},
            "mass": d["mass"], "energy": d["energy"]}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, f0, steps: int, threads: int, single_steps: int):
    """The oracle on the host: `steps` steps with `threads` OpenMP threads
    (the reported value), then `single_steps` steps on one thread."""
    import oracle
    p = cfg.params()
    p.pop("precision")
    rates = {}
    for nthr, nst in ((threads, steps), (1, single_steps)):
        if nst <= 0:
            continue
        used = oracle.set_threads(nthr)
        o = oracle.Oracle(**p)
        o.init_conditions(f0)
        t0 = time.perf_counter()
        o.step(nst)
        rates[nthr] = (used, nst, time.perf_counter() - t0)
    used, nst, dt = rates[threads]
    out = {"value": cfg.n * cfg.n * nst / dt, "unit": "site updates/s",
           "cores": used, "kind": "oracle",
           "sample": f"{nst} steps of the same 2048^2 run from t = 0 "
                     f"(remap at step {cfg.n_s} included when reached), "
                     f"{dt:.2f} s wall",
           "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}
    if 1 in rates and threads != 1:
        _, n1, dt1 = rates[1]
        out["single_thread"] = {"value": cfg.n * cfg.n * n1 / dt1,
                                "steps": n1, "seconds": dt1}
    oracle.set_threads(threads)
    return out


def cpu_baseline_large(threads: int, plan=(("c3_halos_sheet_8192", 2),
                                            ("c5_halos_cold_16384", 1))):
    """The oracle on the host (`threads` OpenMP threads) over a short prefix
    of each large workload from t = 0 (bounded so that the default run stays
    within minutes): site updates/s, to set beside the GPU rates of the
    large-grid leg.  The initial condition (spline fit of F_ini) is not
    timed."""
    import oracle
    import workloads as W
    out = {}
    used = oracle.set_threads(threads)
    for name, nst in plan:
        cfg, f0 = W.config(name)
        p = cfg.params()
        p.pop("precision")
        o = oracle.Oracle(**p)
        o.init_conditions(f0)
        del f0
        t0 = time.perf_counter()
        o.step(nst)
        dt = time.perf_counter() - t0
        out[name] = {"value": cfg.n * cfg.n * nst / dt,
                     "unit": "site updates/s", "cores": used, "steps": nst,
                     "seconds": dt, "kind": "oracle"}
        del o
    return out


def serve_leg(count: int, step_scale: float, seed: int, occupancy: float,
              max_active: int, pool_gb: float, tol: float = 0.05,
              max_passes: int = 3):
    """Continuous-batching leg: `count` independent mixed-precision runs drawn
    from the serving mix (N in {256, 512, 1024, 2048}, element stride 4 or 8,
    steps ~ U{200..2000} times step_scale, remap every 25-50 steps, 1-6
    seeded halos).  A first pass with every request arriving at t = 0 gives
    the device time per site update at full load; then the requests arrive
    as a Poisson process (one seeded draw of unit-rate gaps, scaled by the
    rate) at the rate that targets the requested device occupancy
    (device-busy time / wall time).  Busier batching at full load makes the
    first estimate low, so the rate is rescaled by target / measured and the
    arrival pass repeated until the measured occupancy lies within
    target +- tol (at most max_passes arrival passes; the last is reported).
    Reports p50/p99 latency (arrival to final f on the device) and the
    aggregate site updates/s at that rate."""
    from concurrent.futures import ThreadPoolExecutor
    import numpy as np
    import torch
    import paper_1705_03750_amd as vp
    import workloads as W
    mix = W.serving_requests(count, sizes=(256, 512, 1024, 2048),
                             strides=(4, 8), steps=(200, 2000), remap=(25, 50))
    with ThreadPoolExecutor(max_workers=8) as ex:
        f0s = list(ex.map(lambda ck: W.request_f0(*ck), mix))
    reqs = []
    for (cfg, k), f0 in zip(mix, f0s):
        nsteps = max(1, int(round(cfg.steps * step_scale)))
        reqs.append(dict(
            params=dict(nx=cfg.n, sx=cfg.s, dt=cfg.dt, n_s=cfg.n_s,
                        precision="mixed"),
            f0=torch.as_tensor(f0, device="cuda:0"),
            out=torch.empty((cfg.n, cfg.n), dtype=torch.float32,
                            device="cuda:0"),
            nsteps=nsteps, tag=int(cfg.seed), arrival_s=0.0))
    del f0s
    work = np.array([r["params"]["nx"] ** 2 * r["nsteps"] for r in reqs],
                    dtype=np.float64)
    srv = vp.Server(precision="mixed", max_active=max_active,
                    pool_bytes=int(pool_gb * (1 << 30)))
    torch.cuda.synchronize()
    _, cal = srv.run(reqs)                       # full load, all at t = 0
    cost = cal["gpu_busy_s"] / cal["site_updates"]
    lam = occupancy / (cost * work.mean())
    gaps = np.random.default_rng(seed).exponential(1.0, size=len(reqs))
    gaps[0] = 0.0
    unit_t = np.cumsum(gaps)
    passes = []
    for _ in range(max_passes):
        for r, a in zip(reqs, unit_t / lam):
            r["arrival_s"] = float(a)
        res, st = srv.run(reqs)
        torch.cuda.synchronize()
        occ = st["gpu_busy_s"] / st["wall_s"] if st["wall_s"] else 0.0
        passes.append({"arrival_rate_per_s": lam, "occupancy": occ})
        print(f"[bench] serving pass: rate {lam:.2f}/s, occupancy {occ:.3f}",
              file=sys.stderr, flush=True)
        if abs(occ - occupancy) <= tol or occ <= 0.0:
            break
        lam *= occupancy / occ
    lat = np.array([x["done_s"] - x["arrival_s"] for x in res])
    wait = np.array([x["admit_s"] - x["arrival_s"] for x in res])
    srv.close()
    del reqs
    torch.cuda.empty_cache()
    return {
        "requests": len(res),
        "mix": "N in {256,512,1024,2048}, stride 4 or 8, steps "
               f"U{{200..2000}} x {step_scale}, remap every 25-50, 1-6 halos, "
               "mixed precision",
        "arrival_rate_per_s": passes[-1]["arrival_rate_per_s"],
        "target_occupancy": occupancy,
        "occupancy": passes[-1]["occupancy"],
        "occupancy_within_tolerance": abs(passes[-1]["occupancy"] -
                                          occupancy) <= tol,
        "rate_passes": passes,
        "p50_latency_s": float(np.percentile(lat, 50)),
        "p99_latency_s": float(np.percentile(lat, 99)),
        "p50_queue_wait_s": float(np.percentile(wait, 50)),
        "site_updates_per_s": st["site_updates"] / st["wall_s"],
        "full_load_site_updates_per_s": cal["site_updates"] / cal["wall_s"],
        "site_updates": st["site_updates"],
        "max_active": st["max_active"],
        "ticks": st["ticks"],
        "graph_replay": bool(st["graph_replay"]),
        "wall_s": st["wall_s"],
    }


def load_traffic(kind: str, precision: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary,
    when it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "recon_traffic_c2.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get(precision, {}).get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--cpu-steps", type=int, default=150)
    ap.add_argument("--cpu-single-steps", type=int, default=8)
    ap.add_argument("--cpu-threads", type=int,
                    default=min(16, os.cpu_count() or 1))
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--only", choices=["mixed", "fp64"], default=None)
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--serve-step-scale", type=float, default=1.0)
    ap.add_argument("--serve-occupancy", type=float, default=0.8)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--copy-cal", action="store_true",
                    help="run only a plain 1 GiB device-to-device copy (5x), "
                         "the reference for scaling rocprofv3 FETCH_SIZE / "
                         "WRITE_SIZE counters to bytes")
    ap.add_argument("--leg", choices=["periodic", "four_d", "serve", "emap",
                                      "host_io", "large", "mixed_error"],
                    default=None,
                    help="run only this extra leg (for profiling) and print "
                         "its JSON")
    args = ap.parse_args()
    if args.leg and args.gpus == 1:
        if args.leg == "periodic":
            res = periodic_leg(args.steps, args.warmup)
        elif args.leg == "four_d":
            res = four_d_leg(args.steps)
        elif args.leg == "large":
            res = large_grid_leg()
        elif args.leg == "mixed_error":
            res = mixed_error_leg()
        elif args.leg == "host_io":
            import workloads as W
            cfg, f0 = W.config("c2_halos_2048")
            res = host_io_leg(cfg, f0, args.steps, args.warmup)
        elif args.leg == "emap":
            import workloads as W
            cfg, f0 = W.config("c2_halos_2048")
            fixed = run_gpu("mixed", cfg, f0, args.steps, args.warmup)
            res = emap_leg(cfg, f0, args.steps, args.warmup, fixed)
        else:
            res = serve_leg(args.serve_requests, args.serve_step_scale, seed=4,
                            occupancy=args.serve_occupancy, max_active=64,
                            pool_gb=8.0)
        print(json.dumps(res))
        return
    if args.copy_cal:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 5
        print(json.dumps({"copy_bytes_read": src.numel() * 4,
                          "copy_bytes_written": src.numel() * 4,
                          "seconds_per_copy": dt,
                          "GBps_read_plus_write": 2 * src.numel() * 4 / dt / 1e9}))
        return
    if args.gpus != 1:
        print("bench.py: this engine runs one run on one GPU; multi-GPU "
              "figures are not part of this build (use --gpus 1).",
              file=sys.stderr)
        sys.exit(2)

    import workloads as W
    cfg, f0 = W.config("c2_halos_2048")
    steps = whole_cycles(args.steps, cfg.n_s)
    # the warm-up also covers a whole cycle, so that the first launches of
    # the resampling kernels (code-object loading) happen before the timing
    warm = whole_cycles(args.warmup, cfg.n_s) if args.warmup > 0 else 0
    res = {}
    for prec in (["mixed", "fp64"] if args.only is None else [args.only]):
        res[prec] = run_gpu(prec, cfg, f0, steps, warm)
        print(f"[bench] {prec}: {res[prec]['ms_per_step']:.4f} ms/step, "
              f"{res[prec]['value']:.4e} site updates/s", file=sys.stderr,
              flush=True)
    main_prec = "mixed" if "mixed" in res else "fp64"
    m = res[main_prec]
    fb = 4 if main_prec == "mixed" else 8
    ms_recon, n_recon = m["kernels"]["recon"]
    avg_s = ms_recon / n_recon / 1e3
    alg = recon_algorithmic_bytes(cfg.n, cfg.s, fb)
    flops = recon_algorithmic_flops(cfg.n)
    achieved = flops / avg_s / 1e12
    gbps = alg["total"] / avg_s / 1e9
    traffic = load_traffic("recon", main_prec)
    out = {
        "metric": METRIC,
        "value": m["value"],
        "unit": "site updates/s",
        "n_gpus": 1,
        "steps": steps,
        "steps_requested": args.steps,
        "resamplings_in_window": steps // cfg.n_s,
        "warmup": warm,
        "warmup_requested": args.warmup,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 f/interp + f64 elements/query/force" if main_prec ==
        "mixed" else "f64",
        "data": "synthetic (seeded 4-halo sum)",
        "config": {"workload": "c2_halos_2048: 2048^2 grid on [-1,1]^2, "
                               "elements every 8th site, 4 Gaussian halos, "
                               "dt 5e-4, remap every 50 steps",
                   "grid": cfg.n, "element_stride": cfg.s, "dt": cfg.dt,
                   "n_s": cfg.n_s, "precision": main_prec},
        "roofline": {"bound": "alu", "achieved": achieved,
                     "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS, "traffic": traffic,
                     "kernel": "k_recon (nearest element, inverse map, "
                               "six-point interpolation, column partials)",
                     "avg_launch_us": avg_s * 1e6,
                     "timing": "HIP events around each k_recon launch on the "
                               "run's stream, over a second pass of the "
                               "same timed run",
                     "ms_per_step_with_events": m["ms_per_step_profiled"],
                     "algorithmic_flops_per_launch": flops,
                     "algorithmic_bytes_per_launch": alg["total"],
                     "hbm_achieved_GBps": gbps,
                     "hbm_frac": gbps / HBM_PEAK_GBS},
    }
    if "fp64" in res and main_prec != "fp64":
        f = res["fp64"]
        fms, fn = f["kernels"]["recon"]
        out["fp64"] = {"value": f["value"], "ms_per_step": f["ms_per_step"],
                       "recon_avg_launch_us": fms / fn * 1e3,
                       "mixed_over_fp64": m["value"] / f["value"]}
    out["kernels_ms_per_step"] = {
        k: v[0] / steps for k, v in m["kernels"].items() if v[1]}
    if args.only is None:
        out["mixed_error"] = mixed_error_leg()
        for k, v in out["mixed_error"].items():
            print(f"[bench] mixed vs FP64, {k} ({v['steps']} steps): rel L2 "
                  f"{v['rel_l2_f']:.2e}, energy drift difference "
                  f"{v['energy_drift_diff']:.2e}", file=sys.stderr, flush=True)
    if args.only is None:
        out["host_io"] = host_io_leg(cfg, f0, steps, warm)
        print(f"[bench] host in/out: {out['host_io']['value']:.4e} site "
              f"updates/s with transfers, "
              f"{out['host_io']['transfer_ms']:.2f} ms of them",
              file=sys.stderr, flush=True)
    if args.only is None:
        out["variable_step"] = variable_step_leg(cfg, f0, steps,
                                                 warm, m)
        print(f"[bench] variable step: "
              f"{out['variable_step']['ms_per_step']:.4f} ms/step",
              file=sys.stderr, flush=True)
    if args.only is None:
        out["adaptive_resampling"] = emap_leg(cfg, f0, steps,
                                              warm, m)
        print(f"[bench] adaptive resampling: "
              f"{out['adaptive_resampling']['ms_per_step']:.4f} ms/step, "
              f"{out['adaptive_resampling']['resamplings']} resamplings",
              file=sys.stderr, flush=True)
    if args.only is None:
        out["periodic"] = periodic_leg(steps, warm)
        print(f"[bench] periodic plasma: "
              f"{out['periodic']['ms_per_step']:.4f} ms/step",
              file=sys.stderr, flush=True)
    if args.only is None:
        out["large_grids"] = large_grid_leg()
        for k, v in out["large_grids"].items():
            print(f"[bench] {k}: mixed {v['mixed']['ms_per_step']:.3f} / "
                  f"FP64 {v['fp64']['ms_per_step']:.3f} ms/step",
                  file=sys.stderr, flush=True)
    if args.only is None:
        out["four_d"] = four_d_leg()
        print(f"[bench] 4D: {out['four_d']['ms_per_step']:.3f} ms/step",
              file=sys.stderr, flush=True)
    if not args.no_serve and args.only is None:
        out["serving"] = serve_leg(args.serve_requests, args.serve_step_scale,
                                   seed=4, occupancy=args.serve_occupancy,
                                   max_active=64, pool_gb=8.0)
        print(f"[bench] serving: p50 {out['serving']['p50_latency_s']:.3f} s,"
              f" p99 {out['serving']['p99_latency_s']:.3f} s",
              file=sys.stderr, flush=True)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cfg, f0, args.cpu_steps,
                                           args.cpu_threads,
                                           args.cpu_single_steps)
        if args.only is None:
            out["cpu_baseline"]["large_grids"] = cpu_baseline_large(
                args.cpu_threads)
            for k, v in out["cpu_baseline"]["large_grids"].items():
                print(f"[bench] oracle on the host, {k}: {v['value']:.3e} "
                      f"site updates/s ({v['steps']} steps, "
                      f"{v['seconds']:.1f} s)", file=sys.stderr, flush=True)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
