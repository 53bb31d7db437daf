#!/usr/bin/env python
"""Benchmark of the Spectral Ewald k-space path on one MI355X.

One step = one evaluation of the whole path (bin, spread, transforms with
scaling, gather of potentials and forces, FP64 energy) on one batch of
synthetic input already resident in HBM.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline] [--no-tune]
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

METRIC = "particles/s, SE potential+force at 1e-6 rms err; FP32/batched vs plain FP64"
HBM_PEAK = 8.0e12           # B/s, MI355X HBM3E
ALU_PEAK = {"f32": 157.3e12, "f64": 78.6e12}   # published vector peaks, FLOP/s


def rel_rms(a, b):
    import numpy as np
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def roofline(stages, prec, workload_P=None):
    """Roofline object for the stage with the largest total time."""
    dom = max(stages, key=lambda s: s["ms_total"])
    t = dom["ms_avg"] * 1e-3
    bw = dom["bytes"] / t
    fl = dom["flops"] / t
    f_hbm = bw / HBM_PEAK
    f_alu = fl / ALU_PEAK[prec]
    traffic = None
    tpath = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tpath):
        try:
            tr = json.load(open(tpath))
            ent = tr.get(dom["name"])
            if ent and ent.get("source_sha") == _source_sha() and ent.get("P") == workload_P:
                traffic = ent["bytes_per_launch"]
        except Exception:
            traffic = None
    if f_hbm >= f_alu:
        r = {"bound": "hbm", "achieved": bw / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": f_hbm}
    else:
        r = {"bound": "alu", "achieved": fl / 1e12, "peak": ALU_PEAK[prec] / 1e12, "unit": "TFLOP/s",
             "frac": f_alu}
    r["traffic"] = traffic
    r["traffic_unit"] = "bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
    r["kernel"] = dom["name"]
    r["ms_avg"] = dom["ms_avg"]
    r["alg_bytes"] = dom["bytes"]
    r["alg_flops"] = dom["flops"]
    return r


def stage_table(stages, prec, workload_P=None):
    """Per-stage rooflines: algorithmic bytes and flops of one launch over its
    average HIP-event time, as fractions of the HBM and vector peaks; the
    binding fraction is the larger.  Stored HBM byte counts (rocprofv3
    FETCH_SIZE + WRITE_SIZE, copy-calibrated) for the same sources and
    workload add the counter-to-algorithmic ratio."""
    traffic = {}
    tpath = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tpath):
        try:
            sha = _source_sha()
            traffic = {k: v for k, v in json.load(open(tpath)).items()
                       if v.get("source_sha") == sha and v.get("P") == workload_P}
        except Exception:
            traffic = {}
    rows = []
    for r in stages:
        t = max(r["ms_avg"], 1e-9) * 1e-3
        bw, fl = r["bytes"] / t, r["flops"] / t
        fh, fa = bw / HBM_PEAK, fl / ALU_PEAK[prec]
        row = {"stage": r["name"], "ms_avg": r["ms_avg"], "alg_bytes": r["bytes"], "alg_flops": r["flops"],
               "GB_s": bw / 1e9, "frac_hbm": fh, "TFLOP_s": fl / 1e12, "frac_alu": fa,
               "bound": "hbm" if fh >= fa else "alu", "frac": max(fh, fa)}
        ent = traffic.get(r["name"])
        if ent and r["bytes"] > 0:
            row["traffic"] = ent["bytes_per_launch"]
            row["traffic_ratio"] = ent["bytes_per_launch"] / r["bytes"]
        rows.append(row)
    return rows


def host_cpu():
    """Model name of the host CPU (from /proc/cpuinfo)."""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _source_sha(files=("se_kernels.hip", "se_fft.hip", "se_plan.cpp", "se_internal.h", "se_device.h")):
    """Hash of the kernel and planner sources without comments and blank lines
    (a stored HBM byte count stays valid across comment edits only)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in files:
        text = open(os.path.join(ROOT, "paper_1712_04732_amd", "csrc", f)).read()
        code = [ln.rstrip() for ln in (re.sub(r"//.*", "", x) for x in text.split("\n"))]
        h.update("\n".join(ln for ln in code if ln.strip()).encode())
    return h.hexdigest()[:16]


def run_path(plan, x, q, steps, warmup, profile=True):
    import torch
    N = x.shape[0]
    out = (torch.empty(N, dtype=plan.dtype, device=x.device),
           torch.empty((N, 3), dtype=plan.dtype, device=x.device),
           torch.empty((), dtype=torch.float64, device=x.device))
    plan(x, q, out=out, check=True)            # validates the inputs once
    for _ in range(warmup):
        plan(x, q, out=out, check=False)
    torch.cuda.synchronize()
    plan.profile(reset=True)
    t0 = time.perf_counter()
    for _ in range(steps):
        plan(x, q, out=out, check=False, profile=profile)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stages = plan.profile(reset=True) if profile else None
    return (t1 - t0) * 1e3 / steps, out, stages


def cpu_baseline(cfg, x, q, budget_s=15.0):
    """The direct FP64 oracle on the host cores, on a bounded target sample."""
    import numpy as np
    from oracle import direct
    N = x.shape[0]
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    # calibrate on a small sample, then size the sample to the budget
    t_small = max(16, min(N, 64))
    tg = np.arange(t_small)
    t0 = time.perf_counter()
    direct.kspace(cfg["D"], cfg["L"], cfg["xi"], x, q, targets=tg)
    dt = time.perf_counter() - t0
    T = int(min(N, max(t_small, t_small * budget_s / max(dt, 1e-6))))
    tg = np.sort(np.random.default_rng(7).choice(N, size=T, replace=False)) if T < N else np.arange(N)
    t0 = time.perf_counter()
    phi, grad = direct.kspace(cfg["D"], cfg["L"], cfg["xi"], x, q, targets=tg)
    dt = time.perf_counter() - t0
    return {"value": T / dt, "unit": "particles/s", "cores": cores, "kind": "oracle",
            "sample": f"direct FP64 k-space sum (closed forms) for {T} of {N} targets against all "
                      f"{N} sources, potential and gradient, {dt:.1f} s"}, tg, phi, grad


def batch_cpu_baseline(systems, budget_s=10.0, per_sys_targets=256):
    """The direct FP64 oracle on the host cores for sampled targets of batch
    systems, until the time budget is used.  Its cost per system spans five
    orders of magnitude (the lattice sums grow as N (xi L)^D), so systems are
    taken from each periodicity in turn, cheapest first by that measure; the
    budget is then overrun by at most one small system."""
    import numpy as np
    from oracle import direct
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    by_d = [sorted((k for k, s in enumerate(systems) if s["D"] == D),
                   key=lambda k: systems[k]["N"] * (systems[k]["xi"] * systems[k]["L"]) ** systems[k]["D"])
            for D in (0, 1, 2, 3)]
    order = [lst[r] for r in range(max(len(l) for l in by_d)) for lst in by_d if r < len(lst)]
    t_tot, n_tot, used, res = 0.0, 0, 0, []
    for k in order:
        s = systems[k]
        T = min(per_sys_targets, s["N"])
        tg = np.sort(np.random.default_rng(100 + k).choice(s["N"], size=T, replace=False))
        t0 = time.perf_counter()
        phi, grad = direct.kspace(s["D"], s["L"], s["xi"], s["x"], s["q"], targets=tg)
        dt = time.perf_counter() - t0
        t_tot += dt
        n_tot += T
        used += 1
        res.append((k, tg, phi, grad, dt))
        if t_tot > budget_s:
            break
    return {"value": n_tot / t_tot, "unit": "particles/s", "cores": cores, "kind": "oracle",
            "systems": [r[0] for r in res],
            "sample": f"direct FP64 k-space sums (closed forms, potential and gradient) for {n_tot} "
                      f"targets: up to {per_sys_targets} per system of {used} systems (each periodicity "
                      f"in turn, cheapest first by N (xi L)^D), each against all of its sources, "
                      f"{t_tot:.1f} s"}, res


def batch_o2_baseline(systems, params, budget_s=8.0):
    """The discrete SE oracle (numpy FP64, one thread: the method's own
    algorithm on the CPU) on whole batch systems, each periodicity in turn,
    smallest grid first, until the time budget is used."""
    from oracle import se_discrete as se
    by_d = [sorted((k for k, s in enumerate(systems) if s["D"] == D),
                   key=lambda k: params[k].M ** 3) for D in (0, 1, 2, 3)]
    order = [lst[r] for r in range(max(len(l) for l in by_d)) for lst in by_d if r < len(lst)]
    t_tot, n_tot, used = 0.0, 0, 0
    for k in order:
        s, pp = systems[k], params[k]
        extra = {"s": pp.s, "n_l": pp.n_l} if s["D"] in (1, 2) else {}
        p = se.Params(D=s["D"], L=s["L"], xi=s["xi"], M=pp.M, P=pp.P, window="pkb", **extra)
        t0 = time.perf_counter()
        se.spectral_ewald(s["x"], s["q"], p)
        t_tot += time.perf_counter() - t0
        n_tot += s["N"]
        used += 1
        if t_tot > budget_s:
            break
    return {"value": n_tot / t_tot, "unit": "particles/s", "cores": 1, "kind": "oracle (discrete SE, numpy)",
            "sample": f"discrete SE oracle (Algorithms 1-4, FP64, numpy FFTs) on {used} whole systems "
                      f"({n_tot} particles, potential and gradient, each periodicity in turn, smallest grid "
                      f"first), {t_tot:.1f} s"}


def oracle_one_core(res, budget_s=6.0):
    """The direct oracle's batch sample timed with one thread, in a child
    process (OpenMP takes its thread count when the library loads): the same
    systems in the same order and the same targets as the all-core sample,
    until the budget is used; the all-core rate over the same systems is
    reported beside it."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        out = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-oracle-sample", str(budget_s)],
                             env=env, capture_output=True, text=True, timeout=300)
        one = json.loads(out.stdout.strip().splitlines()[-1])
    except Exception as e:   # reported, not fatal: the main baseline stands
        return {"error": str(e)[:200]}
    same = [r for r in res if r[0] in set(one.get("systems", []))]
    if same:
        one["all_cores_same_sample"] = sum(len(r[1]) for r in same) / sum(r[4] for r in same)
    return one


def _cpu_oracle_sample(budget_s):
    """Child process of oracle_one_core: no GPU, prints one JSON line."""
    import workloads as wl
    systems = wl.batch_systems()
    cb, _ = batch_cpu_baseline(systems, budget_s=budget_s)
    print(json.dumps(cb), flush=True)


_KNOBS = ("tile3", "fft_cap", "xcd_tiles", "xcd_fft", "spread_mode")


def _save_schedule(path, params):
    """The autotuner's knobs, one entry per system (with D and M to check
    that a stored schedule belongs to the same batch)."""
    rows = [dict(D=p.D, M=p.M, tile3=list(p.tile3), fft_cap=p.fft_cap, xcd_tiles=p.xcd_tiles, xcd_fft=p.xcd_fft,
                 spread_mode=p.spread_mode) for p in params]
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "w") as f:
        f.write('{"device": "MI355X (gfx950)", "systems": [\n')
        f.write(",\n".join(json.dumps(r) for r in rows))
        f.write("\n]}\n")


def _load_schedule(path, params):
    rows = json.load(open(path))["systems"]
    if len(rows) != len(params) or any(r["D"] != p.D or r["M"] != p.M for r, p in zip(rows, params)):
        return False
    for r, p in zip(rows, params):
        for d in range(3):
            p.tile3[d] = r["tile3"][d]
        p.fft_cap, p.xcd_tiles, p.xcd_fft = r["fft_cap"], r["xcd_tiles"], r["xcd_fft"]
        p.spread_mode = r.get("spread_mode", 0)
    return True


def main_batch(args):
    import numpy as np
    import torch

    import workloads as wl
    from paper_1712_04732_amd import SpectralEwald, SpectralEwaldBatch, params_for_tolerance
    from paper_1712_04732_amd import _lib

    cfg = wl.BATCH
    systems = wl.batch_systems()
    dev = torch.device("cuda:0")
    N = [s["N"] for s in systems]
    tot = sum(N)
    p32 = [params_for_tolerance(s["D"], s["L"], s["xi"], float((s["q"] ** 2).sum()), cfg["tol_rel"],
                                cfg["P"], cfg["window"], "f32") for s in systems]
    p64 = [params_for_tolerance(s["D"], s["L"], s["xi"], float((s["q"] ** 2).sum()), cfg["tol_rel"],
                                cfg["P"], cfg["window"], "f64") for s in systems]
    x = torch.tensor(np.concatenate([s["x"] for s in systems]), device=dev)
    q = torch.tensor(np.concatenate([s["q"] for s in systems]), device=dev)
    t0 = time.perf_counter()
    b32 = SpectralEwaldBatch(p32, N)
    t_plan = time.perf_counter() - t0
    tune_rep = None
    sched_path = args.schedule or os.path.join(ROOT, "paper_1712_04732_amd", "schedules", "c5_batch.json")
    if args.no_tune:
        schedule = "default"
    elif os.path.exists(sched_path) and not args.retune and _load_schedule(sched_path, p32):
        schedule = f"autotuned, stored ({os.path.relpath(sched_path, ROOT)})"
        b32 = SpectralEwaldBatch(p32, N)
    else:
        t0 = time.perf_counter()
        b32, tune_rep = SpectralEwaldBatch.tuned(p32, N, x, q)
        tune_rep["seconds"] = time.perf_counter() - t0
        schedule = "autotuned"
        print(f"bench: autotuner {tune_rep['candidates']} candidates in {tune_rep['seconds']:.1f} s: "
              f"{tune_rep['ms_default']:.2f} -> {tune_rep['ms_tuned']:.2f} ms", file=sys.stderr, flush=True)
        if args.save_schedule:
            _save_schedule(args.save_schedule, b32.params)
    tiles = sorted({tuple(b32.info(k).tile) for k in range(len(N))})
    caps = sorted({b32.info(k).fft_cap for k in range(len(N))})
    modes = sorted({b32.info(k).spread_mode for k in range(len(N))})
    print(f"bench: schedule {schedule}: tiles {tiles} fft_cap {caps} spread modes {modes}", file=sys.stderr,
          flush=True)
    print(f"bench: batch of {len(N)} systems, sum N = {tot}, D counts "
          f"{np.bincount([s['D'] for s in systems], minlength=4).tolist()}, M {min(p.M for p in p32)}.."
          f"{max(p.M for p in p32)}, plan {t_plan:.1f} s",
          file=sys.stderr, flush=True)

    out32 = (torch.empty(tot, dtype=torch.float32, device=dev), torch.empty((tot, 3), dtype=torch.float32, device=dev),
             torch.empty(len(N), dtype=torch.float64, device=dev))
    b32(x, q, out=out32, check=True)
    for _ in range(args.warmup):
        b32(x, q, out=out32, check=False)
    torch.cuda.synchronize()
    b32.profile(reset=True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b32(x, q, out=out32, check=False, profile=True)
    torch.cuda.synchronize()
    ms32 = (time.perf_counter() - t0) * 1e3 / args.steps
    rec = b32.profile(reset=True)
    print(f"bench: FP32 batched {ms32:.3f} ms/step", file=sys.stderr, flush=True)

    # the plain FP64 path: one plan per system, evaluated one after another
    plans = []
    for k, s in enumerate(systems):
        p = p64[k]
        plans.append(SpectralEwald(s["D"], s["L"], s["xi"], p.M, cfg["P"], window=cfg["window"], prec="f64",
                                   n_max=s["N"], s=p.s, n_l=p.n_l))
    offs = np.concatenate([[0], np.cumsum(N)])
    out64 = [(torch.empty(n, dtype=torch.float64, device=dev), torch.empty((n, 3), dtype=torch.float64, device=dev),
              torch.empty((), dtype=torch.float64, device=dev)) for n in N]
    xs = [x[offs[k]:offs[k + 1]] for k in range(len(N))]
    qs = [q[offs[k]:offs[k + 1]] for k in range(len(N))]
    for k, pl in enumerate(plans):
        pl(xs[k], qs[k], out=out64[k], check=True)
    torch.cuda.synchronize()
    steps64 = max(1, args.steps // 2)
    t0 = time.perf_counter()
    for _ in range(steps64):
        for k, pl in enumerate(plans):
            pl(xs[k], qs[k], out=out64[k], check=False)
    torch.cuda.synchronize()
    ms64 = (time.perf_counter() - t0) * 1e3 / steps64
    print(f"bench: FP64 plain loop {ms64:.3f} ms/step", file=sys.stderr, flush=True)

    # the same batch in FP64 (batching without the precision change)
    b64 = SpectralEwaldBatch(p64, N)
    o64b = b64(x, q)
    for _ in range(args.warmup):
        b64(x, q, out=o64b, check=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps64):
        b64(x, q, out=o64b, check=False)
    torch.cuda.synchronize()
    ms64b = (time.perf_counter() - t0) * 1e3 / steps64
    del b64, o64b
    print(f"bench: FP64 batched {ms64b:.3f} ms/step", file=sys.stderr, flush=True)

    phi32 = out32[0].double().cpu().numpy()
    f32 = out32[1].double().cpu().numpy()
    e32 = out32[2].cpu().numpy()
    phi64 = np.concatenate([o[0].cpu().numpy() for o in out64])
    f64 = np.concatenate([o[1].cpu().numpy() for o in out64])
    e64 = np.array([float(o[2]) for o in out64])
    err = {"phi_f32_vs_f64": rel_rms(phi32, phi64), "force_f32_vs_f64": rel_rms(f32, f64),
           "energy_f32_vs_f64_max": float(np.max(np.abs(e32 - e64) / np.abs(e64)))}

    stages = [r for r in rec if r["name"] != "batch_all_stages"]
    whole = [r for r in rec if r["name"] == "batch_all_stages"][0]
    for r in stages:
        t = max(r["ms_avg"], 1e-9) * 1e-3
        print(f"bench:   {r['name']:8s} {r['ms_avg'] * 1e3:9.1f} us  {r['bytes'] / t / 1e9:8.1f} GB/s  "
              f"{r['flops'] / t / 1e12:7.2f} TFLOP/s", file=sys.stderr, flush=True)
    roof = roofline(stages, "f32", cfg["P"])
    stage_ids = {n: k for k, n in enumerate(["zero", "bin", "scan1", "scan2", "scatter", "order", "spread", "fold",
                                             "fft0", "fft1", "fft2", "fft3", "fft4", "gather", "energy"])}
    st_name = roof["kernel"]
    if st_name == "fft2":
        roof["kernel"] = "batch_fft_kernel<float, 4, unsigned int> (fft2: fused forward transform, scaling, inverse transform)"
    elif st_name.startswith("fft"):
        roof["kernel"] = f"batch_fft_kernel<float, *> ({st_name}: one launch per transform kind)"
    else:
        roof["kernel"] = f"batch_stage_kernel<float, {cfg['P']}, {stage_ids[st_name]}> ({st_name})"
    roof["whole_eval_ms"] = whole["ms_avg"]

    result = {
        "metric": METRIC,
        "value": tot / (ms32 * 1e-3),
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms32,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "C5_batch", "n_sys": len(N), "sum_N": tot, "P": cfg["P"], "window": cfg["window"],
                   "tol_rel": cfg["tol_rel"], "xi": "1.2 N^(1/3)/L", "charges": cfg["charges"],
                   "outputs": "potential+force+energy", "launch": "one launch per stage over all systems",
                   "schedule": schedule},
        "fp64_plain_value": tot / (ms64 * 1e-3),
        "fp64_plain_ms_per_step": ms64,
        "speedup_vs_fp64_plain": ms64 / ms32,
        "fp64_batched_value": tot / (ms64b * 1e-3),
        "fp64_batched_ms_per_step": ms64b,
        "speedup_batching_fp64": ms64 / ms64b,
        "speedup_precision_batched": ms64b / ms32,
        "roofline": roof,
        "stages": stage_table(stages, "f32", cfg["P"]),
        "errors": err,
        "autotune": tune_rep,
    }
    if not args.no_single:
        result["single_systems"] = single_systems(args)
    if not args.no_cpu_baseline:
        cb, res = batch_cpu_baseline(systems)
        cb["host_cpu"] = host_cpu()
        cb["one_core"] = oracle_one_core(res)
        cb["discrete_se"] = batch_o2_baseline(systems, p64)
        result["cpu_baseline"] = cb
        e_phi32, e_phi64, e_f32, ref_n = 0.0, 0.0, 0.0, 0.0
        for k, tg, phi_o, grad_o, _ in res:
            sl = offs[k] + tg
            e_phi32 += float(np.sum((phi32[sl] - phi_o) ** 2))
            e_phi64 += float(np.sum((phi64[sl] - phi_o) ** 2))
            e_f32 += float(np.sum((f32[sl] + systems[k]["q"][tg, None] * grad_o) ** 2))
            ref_n += float(np.sum(phi_o ** 2))
        g_n = sum(float(np.sum((systems[k]["q"][tg, None] * grad_o) ** 2)) for k, tg, phi_o, grad_o, _ in res)
        e_f64 = sum(float(np.sum((f64[offs[k] + tg] + systems[k]["q"][tg, None] * grad_o) ** 2))
                    for k, tg, phi_o, grad_o, _ in res)
        err["phi_f32_vs_oracle"] = (e_phi32 / ref_n) ** 0.5
        err["phi_f64_vs_oracle"] = (e_phi64 / ref_n) ** 0.5
        err["force_f32_vs_oracle"] = (e_f32 / g_n) ** 0.5
        err["force_f64_vs_oracle"] = (e_f64 / g_n) ** 0.5
    print(json.dumps(result), flush=True)


SINGLE_SCHEDULE = os.path.join(ROOT, "paper_1712_04732_amd", "schedules", "single_systems.json")
SINGLE_NAMES = ("C1_3P", "C2_0P", "C3_2P", "C4_1P")
KNOBS = ("tile", "fft_cap", "xcd_tiles", "xcd_fft", "spread_mode")


def _single_plan(name, prec, stored=None):
    """The plan of a single-system configuration: default knobs, or the
    autotuner's knobs stored for (name, prec) when given."""
    import workloads as wl
    from paper_1712_04732_amd import SpectralEwald, _lib
    cfg = wl.CONFIGS[name]
    D, N, L, M, P, xi, win = cfg["D"], cfg["N"], cfg["L"], cfg["M"], cfg["P"], cfg["xi"], cfg["window"]
    kw = dict(window=win, n_max=N)
    if D in (1, 2):
        x, q = wl.config_system(name)
        Q = float((q * q).sum())
        kw.update(Q=Q, tol=1e-6 * _lib.se_error_scale(Q, xi, L))
    plan = SpectralEwald(D, L, xi, M, P, prec=prec, **kw)
    row = (stored or {}).get(name, {}).get(prec)
    if row is None or row.get("M") != plan.params.M:
        return plan, False
    p = plan.params
    for d in range(3):
        p.tile3[d] = row["tile3"][d]
    for k in KNOBS:
        setattr(p, k, row[k])
    return SpectralEwald.from_params(p, N), True


def main_retune_singles(args):
    """Run the single-plan autotuner on C1-C4 in both precisions and store the
    chosen knobs (the single-system lines then time these plans)."""
    import torch

    import workloads as wl
    dev = torch.device("cuda:0")
    out = {}
    for name in SINGLE_NAMES:
        x, q = wl.config_system(name)
        x64, q64 = torch.tensor(x, device=dev), torch.tensor(q, device=dev)
        for prec in ("f32", "f64"):
            plan, _ = _single_plan(name, prec)
            tuned, rep = plan.autotune(x64, q64)
            p = tuned.params
            row = dict(M=p.M, tile3=list(p.tile3), **{k: getattr(p, k) for k in KNOBS})
            out.setdefault(name, {})[prec] = row
            print(f"bench: {name} {prec} autotuner {rep['candidates']} candidates: {rep['ms_default']:.3f} -> "
                  f"{rep['ms_tuned']:.3f} ms {row}", file=sys.stderr, flush=True)
    path = args.retune_singles
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "w") as f:
        json.dump(dict(device="MI355X (gfx950)", systems=out), f, indent=1)


def single_systems(args, names=SINGLE_NAMES):
    """The four single-system configurations in FP32 and FP64 (one plan each,
    inputs resident): particles/s with the stored autotuned knobs where
    present (and with the default knobs beside them), per-stage rooflines of
    the FP32 run and the FP32 error against FP64."""
    import numpy as np
    import torch

    import workloads as wl
    from paper_1712_04732_amd import _lib
    out = {}
    dev = torch.device("cuda:0")
    steps = max(5, args.steps // 2)
    stored = json.load(open(SINGLE_SCHEDULE))["systems"] if os.path.exists(SINGLE_SCHEDULE) else {}
    for name in names:
        cfg = wl.CONFIGS[name]
        D, N, L, M, P, xi, win = cfg["D"], cfg["N"], cfg["L"], cfg["M"], cfg["P"], cfg["xi"], cfg["window"]
        x, q = wl.config_system(name)
        x64 = torch.tensor(x, device=dev)
        q64 = torch.tensor(q, device=dev)
        row = {"workload": name, "D": D, "N": N, "M": M, "P": P, "window": win, "xi": xi,
               "config": {"workload": name, "D": D, "N": N, "L": L, "M": M, "P": P, "window": win, "xi": xi,
                          "charges": cfg["charges"], "outputs": "potential+force+energy"}}
        res = {}
        for prec in ("f32", "f64"):
            plan, tuned = _single_plan(name, prec, stored)
            # timed without per-stage events (for a small system their
            # records cost more than its kernels); the stage table comes
            # from a profiled run of its own
            ms, o, _ = run_path(plan, x64, q64, steps, args.warmup, profile=False)
            row[f"value_{prec}"] = N / (ms * 1e-3)
            row[f"ms_per_step_{prec}"] = ms
            row[f"schedule_{prec}"] = "autotuned, stored" if tuned else "default"
            if tuned:
                dplan, _ = _single_plan(name, prec)
                row[f"ms_per_step_{prec}_default"], _, _ = run_path(dplan, x64, q64, steps, args.warmup,
                                                                    profile=False)
                del dplan
            if prec == "f32":
                row["Mt"] = plan.info.Mt
                _, _, st = run_path(plan, x64, q64, steps, 0)
                row["stages_f32"] = stage_table(st, "f32", P)
            res[prec] = [t.double().cpu().numpy() for t in o]
            del plan
        row["phi_f32_vs_f64"] = rel_rms(res["f32"][0], res["f64"][0])
        row["force_f32_vs_f64"] = rel_rms(res["f32"][1], res["f64"][1])
        out[name] = row
        print(f"bench: {name} f32 {row['ms_per_step_f32']:.3f} ms ({row['value_f32']:.3g} particles/s), "
              f"f64 {row['ms_per_step_f64']:.3f} ms", file=sys.stderr, flush=True)
    return out


def pairs_within(D, L, rc, x, n_sample=20000, seed=11):
    """Mean number of other charges within rc of a charge (periodic images in
    the first D directions), counted exactly for a sample of charges."""
    import numpy as np
    from scipy.spatial import cKDTree
    pts = [x]
    for d in range(D):                  # images across the periodic faces within rc
        new = []
        for p in pts:
            lo = p[p[:, d] < rc].copy()
            lo[:, d] += L
            hi = p[p[:, d] >= L - rc].copy()
            hi[:, d] -= L
            new += [lo, hi]
        pts += new
    tree = cKDTree(np.concatenate(pts))
    idx = np.random.default_rng(seed).choice(x.shape[0], size=min(n_sample, x.shape[0]), replace=False)
    cnt = tree.query_ball_point(x[idx], rc, return_length=True)
    return float(np.mean(cnt)) - 1.0


# Arithmetic of one pair term of Eq. (real_space_ewald) and its gradient as
# written: difference (3), r^2 (5), r and 1/r (2), erfc and exp (1 each),
# the potential term (2), the gradient factor (5) and its three products and
# sums (6).
PAIR_FLOPS = 25


RS_SOURCES = ("se_real.hip", "se_device.h", "se_internal.h")


def _rs_traffic(workload):
    """Stored HBM bytes per launch of the FP32 pair kernel (FETCH_SIZE +
    WRITE_SIZE, copy-calibrated) when they were taken on these sources and
    this workload, else None."""
    tpath = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        ent = json.load(open(tpath)).get("rs_pairs")
        if ent and ent.get("source_sha") == _source_sha(RS_SOURCES) and ent.get("workload") == workload:
            return ent["bytes_per_launch"]
    except Exception:
        pass
    return None


# Kernels whose HBM counters become traffic.json entries: the FP32 C5 batch
# stages (one launch per evaluation each; the transform kinds map one to one
# onto the five transform stages of the batch) and the FP32 real-space pairs.
TRAFFIC_KERNELS = {
    "batch_stage_kernel<float, 10, 6>": ("spread", "C5_batch", "spreading (column mode)"),
    "batch_fft_kernel<float, 2, unsigned int>": ("fft0", "C5_batch", "R2C transforms"),
    "batch_fft_kernel<float, 0, unsigned int>": ("fft1", "C5_batch", "forward C2C transforms"),
    "batch_fft_kernel<float, 4, unsigned int>": ("fft2", "C5_batch",
                                                 "fused forward transform, scaling, inverse transform"),
    "batch_fft_kernel<float, 1, unsigned int>": ("fft3", "C5_batch", "inverse C2C transforms"),
    "batch_fft_kernel<float, 3, unsigned int>": ("fft4", "C5_batch", "C2R transforms"),
    "batch_stage_kernel<float, 10, 13>": ("gather", "C5_batch", "gathering"),
    "rs_sum_kernel<float, true>": ("rs_pairs", "C4_1P", "real-space pair sums"),
}


def _pmc_means(path, counter):
    """Mean value per dispatch of one rocprofv3 --pmc counter (KiB) by kernel
    name, from its counter_collection CSV."""
    import csv
    sums, cnt = {}, {}
    with open(path) as f:
        for row in csv.DictReader(f):
            if row["Counter_Name"] != counter:
                continue
            k = row["Kernel_Name"]
            for short in TRAFFIC_KERNELS:
                if short in k:
                    k = short
                    break
            else:
                if "copyBuffer" not in k:
                    continue
            sums[k] = sums.get(k, 0.0) + float(row["Counter_Value"])
            cnt[k] = cnt.get(k, 0) + 1
    return {k: sums[k] / cnt[k] for k in sums}


def main_traffic_from(paths):
    """profiles/traffic.json from four rocprofv3 --pmc runs (counter CSVs):
    FETCH_SIZE and WRITE_SIZE of a workload run, and of --copy-calibration
    (256 MiB read and written per copy), which scales each counter to bytes.
    Entries carry the hash of the kernel sources they were taken on; the
    bench reports them only while that hash matches."""
    fetch, write, cfetch, cwrite = (_pmc_means(pth, c) for pth, c in
                                    zip(paths, ("FETCH_SIZE", "WRITE_SIZE", "FETCH_SIZE", "WRITE_SIZE")))
    copy_kib = (64 << 20) * 4 / 1024   # KiB read (and written) per copy of --copy-calibration
    ck = [k for k in cfetch if "copyBuffer" in k]
    if not ck or not [k for k in cwrite if "copyBuffer" in k]:
        raise SystemExit("no copy kernel in the calibration counters")
    fs = copy_kib / cfetch[ck[0]]
    ws = copy_kib / cwrite[[k for k in cwrite if "copyBuffer" in k][0]]
    tpath = os.path.join(ROOT, "profiles", "traffic.json")
    out = json.load(open(tpath)) if os.path.exists(tpath) else {}
    for k, (stage, workload, what) in TRAFFIC_KERNELS.items():
        if k not in fetch or k not in write:
            continue
        sha = _source_sha(RS_SOURCES) if stage == "rs_pairs" else _source_sha()
        ent = {"kernel": f"{k} ({what})", "workload": workload, "fetch_bytes": fetch[k] * 1024 * fs,
               "write_bytes": write[k] * 1024 * ws, "fetch_scale": fs, "write_scale": ws, "source_sha": sha}
        if workload == "C5_batch":
            ent["P"] = 10
        ent["bytes_per_launch"] = ent["fetch_bytes"] + ent["write_bytes"]
        out[stage] = ent
        print(f"{stage:8s} fetch {ent['fetch_bytes'] / 1e9:.3f} GB write {ent['write_bytes'] / 1e9:.3f} GB "
              f"per launch ({k})", flush=True)
    with open(tpath, "w") as f:
        json.dump(out, f, indent=1)
    print(f"copy calibration: FETCH_SIZE scale {fs:.3f}, WRITE_SIZE scale {ws:.3f}; wrote {tpath}", flush=True)


def main_real_space(args):
    """The real-space part (Eq. real_space_ewald) on the GPU for one of the
    single-system workloads, at the cutoff of Eq. (KP_real_space) for the same
    1e-6 relative tolerance as the k-space part."""
    import numpy as np
    import torch

    import workloads as wl
    from paper_1712_04732_amd import RealSpace, _lib

    name = args.workload if args.workload in wl.CONFIGS else "C4_1P"
    cfg = wl.CONFIGS[name]
    D, N, L, xi = cfg["D"], cfg["N"], cfg["L"], cfg["xi"]
    x, q = wl.config_system(name)
    Q = float((q * q).sum())
    rc = _lib.se_rs_cutoff_for_tolerance(L, xi, Q, 1e-6)
    dev = torch.device("cuda:0")
    xt = torch.tensor(x, dtype=torch.float64, device=dev)
    qt = torch.tensor(q, dtype=torch.float64, device=dev)
    res = {}
    for prec in ("f32", "f64"):
        rs = RealSpace(D, L, xi, rc, prec=prec, n_max=N)
        dt = rs.dtype
        out = (torch.empty(N, dtype=dt, device=dev), torch.empty((N, 3), dtype=dt, device=dev),
               torch.empty((), dtype=torch.float64, device=dev))
        rs(xt, qt, out=out, check=True)
        for _ in range(args.warmup):
            rs(xt, qt, out=out, check=False)
        torch.cuda.synchronize()
        rs.profile(reset=True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            rs(xt, qt, out=out, check=False, profile=True)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        st = {r["name"]: r["ms_avg"] for r in rs.profile(reset=True)}
        res[prec] = (ms, st, [t.double().cpu().numpy() for t in out], rs.cells, rs.span)
        print(f"bench real space {prec}: {ms:.4f} ms/step, stages {st}", file=sys.stderr, flush=True)
    ms32, st32, (phi32, f32, e32), cells, span = res["f32"]
    ms64, st64, (phi64, f64, e64), _, _ = res["f64"]
    npair = pairs_within(D, L, rc, x)
    flops = N * npair * PAIR_FLOPS
    t_pairs = st32["rs_pairs"] * 1e-3
    err = {"phi_f32_vs_f64": rel_rms(phi32, phi64), "force_f32_vs_f64": rel_rms(f32, f64),
           "energy_f32_vs_f64": float(abs(e32 - e64) / abs(e64))}
    result = {
        "metric": "particles/s, real-space part (potential+force+energy) at the 1e-6 cutoff",
        "value": N / (ms32 * 1e-3), "unit": "particles/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms32, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": name + "_real_space", "D": D, "N": N, "L": L, "xi": xi, "rc": rc,
                   "cells": cells, "span": span, "pairs_per_particle": npair},
        "fp64_value": N / (ms64 * 1e-3), "fp64_ms_per_step": ms64,
        "stages_ms": st32, "stages_ms_fp64": st64,
        "roofline": {"bound": "alu", "achieved": flops / t_pairs / 1e12, "peak": ALU_PEAK["f32"] / 1e12,
                     "unit": "TFLOP/s", "frac": flops / t_pairs / ALU_PEAK["f32"], "traffic": _rs_traffic(name),
                     "kernel": "rs_sum_kernel<float, true> (rs_pairs)", "ms_avg": st32["rs_pairs"],
                     "alg_flops": flops},
        "errors": err,
    }
    if not args.no_cpu_baseline:
        from oracle import direct
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        tg = np.sort(np.random.default_rng(7).choice(N, size=min(N, 2048), replace=False))
        t0 = time.perf_counter()
        phi_o, grad_o = direct.real_space(D, L, xi, rc, x, q, targets=tg)
        dt = time.perf_counter() - t0
        result["cpu_baseline"] = {"value": len(tg) / dt, "unit": "particles/s", "cores": cores, "kind": "oracle",
                                  "sample": f"direct FP64 real-space sum for {len(tg)} of {N} targets against "
                                            f"all {N} sources and their images within rc, {dt:.1f} s"}
        err["phi_f32_vs_oracle"] = rel_rms(phi32[tg], phi_o)
        err["phi_f64_vs_oracle"] = rel_rms(phi64[tg], phi_o)
        err["force_f32_vs_oracle"] = rel_rms(f32[tg], -q[tg, None] * grad_o)
        err["force_f64_vs_oracle"] = rel_rms(f64[tg], -q[tg, None] * grad_o)
    print(json.dumps(result), flush=True)


def main_xi_balance(args):
    """Total time of the full potential (k space + real space + self term) of
    one workload against the Ewald parameter: for each xi the grid M comes
    from the k-space estimate (Eq. KP_fourier_space, se_params_for_tolerance)
    and rc from the real-space estimate (Eq. KP_rc, se_rs_cutoff_for_tolerance), both at 1e-6 B,
    so that the balance point the paper tunes xi for is measured.  One JSON
    line per xi."""
    import torch

    import workloads as wl
    from paper_1712_04732_amd import RealSpace, SpectralEwald, _lib, params_for_tolerance

    name = args.workload if args.workload in wl.CONFIGS else "C4_1P"
    cfg = wl.CONFIGS[name]
    D, N, L, xi0, P = cfg["D"], cfg["N"], cfg["L"], cfg["xi"], cfg["P"]
    x, q = wl.config_system(name)
    Q = float((q * q).sum())
    dev = torch.device("cuda:0")
    xt = torch.tensor(x, dtype=torch.float32, device=dev)
    qt = torch.tensor(q, dtype=torch.float32, device=dev)
    for f in (0.5, 0.7, 0.85, 1.0, 1.2, 1.45, 1.75):
        xi = xi0 * f
        p = params_for_tolerance(D, L, xi, Q, 1e-6, P=P, window=cfg["window"], prec="f32")
        if p.M > 400:
            continue
        rc = _lib.se_rs_cutoff_for_tolerance(L, xi, Q, 1e-6)
        ks = SpectralEwald.from_params(p, N)
        rs = RealSpace(D, L, xi, rc, prec="f32", n_max=N)
        out = ks(xt, qt, add_self=True)
        ms = {}
        for label, fn in (("kspace", lambda: ks(xt, qt, add_self=True, check=False, out=out)),
                          ("real", lambda: rs(xt, qt, accumulate=True, check=False, out=out))):
            for _ in range(args.warmup):
                fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                fn()
            torch.cuda.synchronize()
            ms[label] = (time.perf_counter() - t0) * 1e3 / args.steps
        print(json.dumps({"workload": name, "xi": xi, "M": p.M, "rc": rc, "cells": rs.cells,
                          "ms_kspace": ms["kspace"], "ms_real": ms["real"],
                          "ms_total": ms["kspace"] + ms["real"],
                          "particles_per_s": N / ((ms["kspace"] + ms["real"]) * 1e-3)}), flush=True)
        del ks, rs


def main_force_methods(args):
    """Section 7.2, Fig. force: the two ways of computing the k-space force on
    the paper's workload (3P, N = 1e4 uniform in the unit box, charges uniform
    in [-1, 1] re-centred, xi = 8, M = 64, PKB window).  For each P, the
    force error of method 1 (gradient of the gathering window) and method 2
    (i k in the scaling step, three inverse transforms and three gatherings)
    against a high-accuracy GPU FP64 reference (method 1, P = 16, nu = 9; its
    own parity with the oracles is tested), and the time of an evaluation of
    the forces alone.  One JSON line per P and precision."""
    import torch

    import workloads as wl
    from paper_1712_04732_amd import SpectralEwald

    N, L, xi, M = 10000, 1.0, 8.0, 64
    x, q = wl.system(N, L, 171204732 + 7, "uniform")
    dev = torch.device("cuda:0")
    x64, q64 = torch.tensor(x, device=dev), torch.tensor(q, device=dev)
    ref_plan = SpectralEwald(3, L, xi, M, 16, nu=9, prec="f64", n_max=N)
    _, fref, _ = ref_plan(x64, q64)
    fref = fref.cpu().numpy()

    def timed(plan, xt, qt):
        f = torch.empty((N, 3), dtype=plan.dtype, device=dev)
        out = (None, f, None)
        plan(xt, qt, out=out)
        for _ in range(args.warmup):
            plan(xt, qt, out=out, check=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            plan(xt, qt, out=out, check=False)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / args.steps, f.double().cpu().numpy()

    for prec in ("f64", "f32"):
        xt, qt = x64, q64     # FP64 inputs (binning forms cell offsets in FP64 for both precisions)
        for P in (4, 6, 8, 10, 12, 14):
            row = {"workload": "W3_force_3P", "N": N, "xi": xi, "M": M, "P": P, "prec": prec}
            for m in (1, 2):
                plan = SpectralEwald(3, L, xi, M, P, prec=prec, n_max=N, force_method=m)
                ms, f = timed(plan, xt, qt)
                row[f"method{m}_ms"] = ms
                row[f"method{m}_force_err"] = rel_rms(f, fref)
                del plan
            print(json.dumps(row), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="C5_batch")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="batch: keep the default schedule knobs")
    ap.add_argument("--retune", action="store_true", help="batch: run the autotuner even if a schedule is stored")
    ap.add_argument("--schedule", default=None, help="batch: stored schedule (JSON) to use")
    ap.add_argument("--save-schedule", default=None, help="batch: write the autotuner's schedule here")
    ap.add_argument("--real-space", action="store_true",
                    help="time the real-space part instead (single-system workloads; default C4_1P)")
    ap.add_argument("--xi-balance", action="store_true",
                    help="time k space + real space against xi (single-system workloads; default C4_1P)")
    ap.add_argument("--no-single", action="store_true", help="batch: skip the C1-C4 single-system lines")
    ap.add_argument("--retune-singles", default=None,
                    help="run the single-plan autotuner on C1-C4 and write the chosen knobs to this path")
    ap.add_argument("--cpu-oracle-sample", type=float, default=None, help=argparse.SUPPRESS)
    ap.add_argument("--force-methods", action="store_true",
                    help="force method 1 vs method 2 against P on the paper's 3P workload (Section 7.2)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 256 MiB device to device 5 times (reference for HBM byte counters)")
    ap.add_argument("--traffic-from", nargs=4, default=None,
                    metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    help="write profiles/traffic.json from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE "
                         "counter CSVs of a bench run and of --copy-calibration (no GPU needed)")
    args = ap.parse_args()
    if args.cpu_oracle_sample is not None:
        return _cpu_oracle_sample(args.cpu_oracle_sample)
    if args.traffic_from:
        return main_traffic_from(args.traffic_from)
    if args.copy_calibration:
        import torch
        a = torch.empty(64 << 20, dtype=torch.float32, device="cuda:0").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": 2 * a.numel() * 4}), flush=True)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the Spectral Ewald path here runs on a single "
              "MI355X; multi-GPU sharding is a design note, not a measured configuration.",
              file=sys.stderr)
        sys.exit(2)
    if args.real_space:
        return main_real_space(args)
    if args.retune_singles:
        return main_retune_singles(args)
    if args.xi_balance:
        return main_xi_balance(args)
    if args.force_methods:
        return main_force_methods(args)
    if args.workload == "C5_batch":
        return main_batch(args)

    import numpy as np
    import torch

    import workloads as wl
    from paper_1712_04732_amd import SpectralEwald

    cfg = wl.CONFIGS[args.workload]
    D, N, L, M, P, xi, win = cfg["D"], cfg["N"], cfg["L"], cfg["M"], cfg["P"], cfg["xi"], cfg["window"]
    x, q = wl.config_system(args.workload)
    Q = float((q * q).sum())
    from paper_1712_04732_amd import _lib
    tol = 1e-6 * _lib.se_error_scale(Q, xi, L)
    dev = torch.device("cuda:0")
    prec = "f32"
    kw = dict(window=win, n_max=N)
    if D in (1, 2):
        kw.update(Q=Q, tol=tol)

    plan32 = SpectralEwald(D, L, xi, M, P, prec="f32", **kw)
    plan64 = SpectralEwald(D, L, xi, M, P, prec="f64", **kw)
    x64 = torch.tensor(x, dtype=torch.float64, device=dev)
    q64 = torch.tensor(q, dtype=torch.float64, device=dev)
    print(f"bench: {args.workload} D={D} N={N} M={M} Mt={plan32.info.Mt} P={P} xi={xi} "
          f"tile={list(plan32.info.tile)}", file=sys.stderr, flush=True)

    ms32, out32, stages32 = run_path(plan32, x64, q64, args.steps, args.warmup)
    ms64, out64, stages64 = run_path(plan64, x64, q64, args.steps, args.warmup)
    print(f"bench: f32 {ms32:.4f} ms/step, f64 {ms64:.4f} ms/step", file=sys.stderr, flush=True)

    phi32, f32, e32 = (t.double().cpu().numpy() for t in out32)
    phi64, f64, e64 = (t.double().cpu().numpy() for t in out64)
    err = {"phi_f32_vs_f64": rel_rms(phi32, phi64), "force_f32_vs_f64": rel_rms(f32, f64),
           "energy_f32_vs_f64": float(abs(e32 - e64) / abs(e64))}

    result = {
        "metric": METRIC,
        "value": N / (ms32 * 1e-3),
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms32,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic",
        "config": {"workload": args.workload, "D": D, "N": N, "L": L, "M": M, "Mt": plan32.info.Mt,
                   "P": P, "window": win, "xi": xi, "charges": cfg["charges"],
                   "outputs": "potential+force+energy"},
        "fp64_value": N / (ms64 * 1e-3),
        "fp64_ms_per_step": ms64,
        "roofline": roofline(stages32, prec),
        "roofline_fp64": roofline(stages64, "f64"),
        "stages": [{k: (round(v, 6) if isinstance(v, float) else v) for k, v in s.items()}
                   for s in stages32],
        "errors": err,
    }
    if not args.no_cpu_baseline:
        cb, tg, phi_o, grad_o = cpu_baseline(cfg, x, q)
        result["cpu_baseline"] = cb
        err["phi_f32_vs_oracle"] = rel_rms(phi32[tg], phi_o)
        err["phi_f64_vs_oracle"] = rel_rms(phi64[tg], phi_o)
        err["force_f32_vs_oracle"] = rel_rms(f32[tg], -q[tg, None] * grad_o)
        err["force_f64_vs_oracle"] = rel_rms(f64[tg], -q[tg, None] * grad_o)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
