"""Benchmark: pressure-projection solves/s on the 512 x 512 x 768 stretched grid.

One step = one full projection (divergence + x/y transforms + per-mode z
tridiagonals + inverse transforms + gradient correction) of one provisional
velocity field that is already resident in HBM.  Each timed step projects its
own copy of the input (the projection works in place), so no copy runs inside
the timed region.  Both precision modes are measured in the same run:

  * fp32_refine : FP32 transforms/tridiagonals (near-singular mode lines in
                  FP64), FP64 residual, correction solves to ||r||/||f|| <= 1e-10
                  (the mode this workload is specified with; reported as value)
  * fp64        : every step in FP64

Beside the projection the line carries: the Poisson solve on the 768 x 768 x
1024 grid (power-law right-hand side, FP32+refine and FP64; not in value),
the error of both modes against the FP64 oracle on a 96-plane slab of the
512 x 512 x 768 grid, the bandwidth of a plain copy kernel as a second
denominator, and the legs of the fractional step around the projection
(viscous step, momentum right-hand side, IB-MLS transfer).

Prints ONE JSON line.  `--gpus N` with N > 1 exits: the path runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0     # MI355X HBM3E, GB/s
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_c3_512x512x768.json")

# Kernel that each timing slot launches at the 512 x 512 x 768 workload (the
# hardware-counter summary is keyed by kernel name)
SLOT_KERNEL = {
    "fp64": {"xfwd": "k_xfwd<double, double, 1, 2048, 256, 512>", "yfwd": "k_yfwd<double, 4096, 512, 512, 4>",
             "zsolve": "k_zsolvev_pf<double, double, 2, 16, 24, 512, 12>", "yinv": "k_yinv<double, 4096, 512, 512, 4>",
             "xinv": "k_xinv<double, double, 0, 2048, 256, 512>", "grad": "k_grad_row2<double, double, 256, 16>",
             "xinv_grad": "k_xinv_grad<512>"},
    "fp32_refine": {"xfwd": "k_xfwd<double, float, 1, 2048, 256, 512>", "yfwd": "k_yfwd<float, 8192, 1024, 512, 6>",
                    "zsolve": "k_zsolvev_pf<float, float, 4, 16, 24, 512, 12>", "yinv": "k_yinv<float, 8192, 1024, 512, 4>",
                    "xinv": "k_xinv<float, float, 0, 2048, 256, 512>", "xinv_acc": "k_xinv<float, double, 2, 2048, 256, 512>",
                    "resid": "k_resid_pairs<256, 8, true, float, 2>",
                    "resid_norm": "k_resid_pairs<256, 8, false, double, 2>",
                    "xfwd_r": "k_xfwd<float, float, 4, 2048, 256, 512>", "grad": "k_grad_row2<double, double, 256, 16>",
                    "grad_resid": "k_grad_resid<256, 16, false>", "xinv_grad_resid": "k_xinv_grad_resid<512>"},
    "viscous_fp64": {"visc_x": "k_visc_x<16>", "visc_y": "k_visc_strided<2, 16>",
                     "visc_z": "k_visc_strided_pf<24, 12>"},
    "momentum_fp64": {"momentum_rhs": "k_momentum_rhs_pairs<64, 16, true>"},
}

# Algorithmic HBM bytes per cell of each kernel launch (minimum pass model:
# every operand read once, every result written once).
BYTES_PER_CELL = {
    "fp64": {"xfwd": 32, "yfwd": 16, "zsolve": 16, "yinv": 16, "xinv": 16, "grad": 56, "xinv_grad": 64},
    # refinement at this workload (pair tiling): the first solve's pressure is
    # FP32 (x inverse writes 4 B; the first residual reads it: f 8 + p 4, r 4
    # written; the first correction reads p32 + delta and writes p 8)
    "fp32_refine": {"xfwd": 36, "yfwd": 8, "zsolve": 8, "yinv": 8, "xinv": 8, "resid_xfwd": 20,
                    "resid": 16, "xfwd_r": 8, "resid_norm": 16, "xinv_acc": 16, "grad": 56, "grad_resid": 64,
                    # first correction + gradient + check in one pass: correction 4, p32 4, f 8 and
                    # u, v, w 24 read; u, v, w 24 and p 8 written
                    "xinv_grad_resid": 72},
    # implicit viscous step: every line solve of one component reads and
    # writes the field once (3 components x 3 directions = 144 B/cell)
    # Poisson solves (f read, p written): FP64 and FP32+refine (FP64 input,
    # an FP64 copy of f kept for the residual)
    "solve_fp64": {"xfwd": 16, "yfwd": 16, "zsolve": 16, "yinv": 16, "xinv": 16},
    "solve_fp32_refine": {"xfwd": 20, "yfwd": 8, "zsolve": 8, "yinv": 8, "xinv": 8, "resid": 16, "xfwd_r": 8,
                          "resid_norm": 16, "xinv_acc": 16},
    "viscous_fp64": {"visc_x": 16, "visc_y": 16, "visc_z": 16},
    # explicit momentum right-hand side: u, v, w and N^{n-1} read, rhs and N^n written
    "momentum_fp64": {"momentum_rhs": 96},
}


# Minimum-pass model of a whole step (bytes per cell; every field crossing HBM
# once per pass the method needs): the FP64 projection 144 (divergence + x
# transform 32, y 16, z 16, y inverse 16, x inverse + gradient 64); the
# FP32+refine projection with FP64 input and output 72 for the first solve
# (including storing f in FP64), 64 per correction beyond the last, and 64 for
# the last correction fused with the gradient and the convergence check
# (136 + 64 k for k corrections); the Poisson solves 80 (FP64) and 48 + 64 k +
# 16 (FP32+refine).
def model_bytes_per_cell(mode, iterations):
    k = max(int(iterations or 0), 1)
    return {"fp64": 144, "fp32_refine": 136 + 64 * k, "solve_fp64": 80,
            "solve_fp32_refine": 64 + 64 * k}.get(mode)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed_steps(step, steps, warmup, plan, torch):
    """Run `warmup` untimed then `steps` timed calls of step(i); the library
    records HIP events around every launch on the plan's stream during the
    timed region (per-kernel times), and an event pair on the same stream
    brackets every step (median step time).  Returns (wall ms per step,
    median event ms per step, kernel times)."""
    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    plan.reset_timing()
    plan.set_timing(True)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        ev[i][0].record()
        step(warmup + i)
        ev[i][1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plan.set_timing(False)
    med = float(np.median([a.elapsed_time(b) for a, b in ev]))
    return (t1 - t0) * 1e3 / steps, med, plan.kernel_times()


def gpu_mode(mode, spec, u0, v0, w0, steps, warmup, torch, fsei):
    """Time `steps` projections of resident copies of (u0, v0, w0)."""
    prec = fsei.PREC_FP64 if mode == "fp64" else fsei.PREC_FP32_REFINE
    plan = fsei.Plan.from_spec(spec, precision=prec, rtol=1e-10, max_iter=4)
    ncopy = steps + warmup
    bufs = [(u0.clone(), v0.clone(), w0.clone()) for _ in range(ncopy)]
    p = torch.empty_like(u0)
    torch.cuda.synchronize()
    infos = []

    def step(i):
        # refine mode reads one residual norm per iteration back to the host;
        # FP64 mode runs without any host synchronisation
        if mode == "fp64":
            plan.project(*bufs[i], p=p)
        else:
            infos.append(plan.project(*bufs[i], p=p, info=True)[1])
    ms, med, ktimes = timed_steps(step, steps, warmup, plan, torch)
    res = {"ms_per_step": ms, "median_step_ms": med, "kernels": ktimes, "kernel_steps": steps}
    res["last_info"] = infos[-1] if infos else None
    # check the last output: divergence of the projected field
    u, v, w = bufs[-1]
    res["div_check"] = float(divergence_max(u, v, w, spec, torch))
    del bufs
    torch.cuda.empty_cache()
    return res, plan


def gpu_solve(mode, spec, f0, steps, warmup, torch, fsei):
    """Time `steps` Poisson solves p = L^+ f of a resident right-hand side
    (the solve reads f and writes p; f is not modified)."""
    prec = fsei.PREC_FP64 if mode == "solve_fp64" else fsei.PREC_FP32_REFINE
    plan = fsei.Plan.from_spec(spec, precision=prec, rtol=1e-10, max_iter=6, accept_floor=True)
    p = torch.empty_like(f0)
    infos = []

    def step(i):
        if mode == "solve_fp64":
            plan.poisson_solve(f0, p)
        else:
            infos.append(plan.poisson_solve(f0, p, info=True)[1])
    import warnings
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", RuntimeWarning)   # refinement stopping at the FP64 floor
        ms, med, ktimes = timed_steps(step, steps, warmup, plan, torch)
    res = {"ms_per_step": ms, "median_step_ms": med, "kernels": ktimes, "kernel_steps": steps,
           "last_info": infos[-1] if infos else None, "div_check": None}
    del p
    torch.cuda.empty_cache()
    return res


def copy_bandwidth(field, torch, reps=10):
    """GB/s of a plain device copy of one FP64 field (8 B read + 8 B written
    per cell), median of `reps` copies timed with events: the streaming
    ceiling the kernels are also compared with."""
    dst = torch.empty_like(field)
    dst.copy_(field)
    torch.cuda.synchronize()
    t = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(field)
        b.record()
        torch.cuda.synchronize()
        t.append(a.elapsed_time(b))
    del dst
    return 2.0 * field.numel() * field.element_size() / (float(np.median(t)) / 1e3) / 1e9


def gpu_viscous(spec, u0, v0, w0, steps, warmup, torch, fsei):
    """Time `steps` implicit viscous steps (fsei_viscous_solve of u, v, w) on
    resident copies of the input (the solve does the same work whatever the
    values, so each step re-solves the previous step's output)."""
    plan = fsei.Plan.from_spec(spec)
    beta = 0.5 * spec.dx ** 2
    u, v, w = u0.clone(), v0.clone(), w0.clone()
    ms, med, kt = timed_steps(lambda i: plan.viscous_step(u, v, w, beta), steps, warmup, plan, torch)
    res = {"ms_per_step": ms, "median_step_ms": med, "kernels": kt, "kernel_steps": steps,
           "last_info": None, "div_check": None, "beta": beta}
    del u, v, w
    torch.cuda.empty_cache()
    return res


def gpu_momentum(spec, u0, v0, w0, steps, warmup, torch, fsei):
    """Time `steps` explicit momentum right-hand sides (fsei_momentum_rhs) on
    resident fields (N^{n-1} taken from the previous call)."""
    plan = fsei.Plan.from_spec(spec)
    n = [torch.zeros_like(u0) for _ in range(3)]
    r = [torch.empty_like(u0) for _ in range(3)]
    dt, re = 1e-3, 1000.0
    ms, med, kt = timed_steps(lambda i: plan.momentum_rhs(u0, v0, w0, n, r, dt, re), steps, warmup, plan, torch)
    res = {"ms_per_step": ms, "median_step_ms": med, "kernels": kt, "kernel_steps": steps,
           "last_info": None, "div_check": None}
    del n, r
    torch.cuda.empty_cache()
    return res


def gpu_ib(spec, u0, steps, warmup, torch, fsei):
    """Time `steps` IB-MLS transfers (interpolation of the three velocity
    components at the markers, then spreading of one value per marker and
    component back to the grid).  Markers: the ~10^6 triangle centroids of a
    prolate spheroid surface centred in the domain, about one triangle per
    grid cell face, in mesh order."""
    from paper_2103_15187_amd import workloads as W
    plan = fsei.Plan.from_spec(spec)
    xb, dv = W.spheroid_markers(spec)
    nb = len(xb)
    xd = torch.from_numpy(xb).to(u0.device)
    fb = torch.ones(nb, dtype=torch.float64, device=u0.device)
    dvb = torch.from_numpy(dv).to(u0.device)
    ub = torch.empty(nb, dtype=torch.float64, device=u0.device)
    f = torch.zeros_like(u0)

    def step(i):
        for c in range(3):
            plan.ib_interpolate(u0, c, xd, ub)
            plan.ib_spread(f, c, xd, fb, dvb)
    ms, med, kt = timed_steps(step, steps, warmup, plan, torch)
    del f, xd, fb, dvb, ub
    torch.cuda.empty_cache()
    return {"ms_per_step": round(ms, 4), "median_step_ms": round(med, 4), "markers": nb,
            "markers_per_s": round(nb / (ms / 1e3), 1),
            "kernel_ms_per_step": {k: round(v[0] / steps, 4) for k, v in kt.items()},
            "note": "one step = interpolation of u, v, w at every marker + spreading of one value per marker "
                    "and component (27-node MLS supports, FP64 atomics); markers: triangle centroids of a prolate "
                    "spheroid (semi-axes 1.2, 1.2, 2.4) centred in the 512x512x768 domain, mesh order"}


def divergence_max(u, v, w, spec, torch):
    """max |D u| of the projected field, relative to max |D u*| scale 1 (GPU,
    torch ops; a property check, not part of the timed path)."""
    zc = torch.tensor(spec.zc(), dtype=torch.float64, device=u.device)
    dz = (zc[1:] - zc[:-1]).view(-1, 1, 1)
    uh = torch.roll(u, -1, 2)
    if spec.bcx == 1:
        uh[:, :, -1] = 0
        u = u.clone()
        u[:, :, 0] = 0
    vh = torch.roll(v, -1, 1)
    if spec.bcy == 1:
        vh[:, -1, :] = 0
        v = v.clone()
        v[:, 0, :] = 0
    wh = torch.roll(w, -1, 0)
    wh[-1] = 0
    w = w.clone()
    w[0] = 0
    d = (uh - u) / spec.dx + (vh - v) / spec.dy + (wh - w) / dz
    return d.abs().max().item()


def kernel_source_hash():
    """sha256 of the HIP/C++ sources of the library (the counters in the
    traffic summary belong to the sources they were measured on)."""
    csrc = os.path.join(ROOT, "paper_2103_15187_amd", "csrc")
    h = hashlib.sha256()
    for fn in sorted(os.listdir(csrc)):
        if fn.endswith((".hip", ".h", ".cpp")):
            h.update(fn.encode())
            with open(os.path.join(csrc, fn), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def measured_traffic(mode, slot, ncells):
    """Calibrated HBM bytes per launch of the slot's kernel from the committed
    counter summary, or None when there is none for it, the sources have
    changed since the counters were taken, or the run is not the profiled
    512x512x768 workload."""
    from paper_2103_15187_amd import workloads as W
    if ncells != W.CONFIGS["C3"].ncells:
        return None
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != kernel_source_hash():
        return None
    k = t.get("kernels", {}).get(SLOT_KERNEL.get(mode, {}).get(slot, ""))
    return None if k is None else round(k["fetch_bytes"] + k["write_bytes"])


def roofline_for(mode, res, ncells, copy_gbs=None):
    """Dominant kernel (largest total time in the timed region) and its
    achieved algorithmic bandwidth: algorithmic bytes per launch over its
    average launch duration (HIP events on the plan's stream)."""
    kt = res["kernels"]
    bpc = BYTES_PER_CELL[mode]
    name = max((k for k in kt if k in bpc), key=lambda k: kt[k][0])
    total_ms, n = kt[name]
    avg_s = total_ms / n / 1e3
    bytes_per_launch = bpc[name] * ncells
    achieved = bytes_per_launch / avg_s / 1e9
    out = {"kernel": name, "bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
           "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": measured_traffic(mode, name, ncells),
           "bytes_per_launch": bytes_per_launch, "avg_launch_ms": round(avg_s * 1e3, 4)}
    if copy_gbs:
        out["copy_ceiling"] = round(copy_gbs, 1)
        out["frac_of_copy"] = round(achieved / copy_gbs, 4)
    return out


def _short_kernel(name):
    return name.split("(")[0].replace("void ", "").replace("fsei::dev::", "").strip()


def summarize_profiles(d, cmd_trace, cmd_pmc):
    """Turn the rocprofv3 outputs under `d` (prof/, pmc_FETCH_SIZE/,
    pmc_WRITE_SIZE/) into the committed summaries under profiles/."""
    import csv
    out = os.path.join(ROOT, "profiles")
    rows = list(csv.DictReader(open(os.path.join(d, "prof", "c3_kernel_stats.csv"))))
    md = ["# Kernel trace: projection (FP32+refine and FP64 modes), viscous step, momentum right-hand side "
          "and IB-MLS transfer, 512x512x768 walls tanh 2.5", "",
          "Command (run from the repository root on one MI355X):", "", "```", cmd_trace, "```", "",
          "| kernel | calls | avg (us) | total (ms) | % |", "|---|---:|---:|---:|---:|"]
    for r in rows:
        name = _short_kernel(r["Name"])
        if len(name) > 70:
            name = name[:70] + "..."
        md.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                  f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.1f} |")
    with open(os.path.join(out, "projection_c3_512x512x768_kernel_stats.md"), "w") as fh:
        fh.write("\n".join(md) + "\n")
    # hardware byte counters (KiB per dispatch), calibrated on torch.neg over
    # one FP64 field of the workload (reads and writes 8 B per cell)
    spec_cells = 512 * 512 * 768
    vals = {}
    for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
        for r in csv.DictReader(open(os.path.join(d, f"pmc_{ctr}", "c3_counter_collection.csv"))):
            full = r["Kernel_Name"]
            key = "CALIB" if "neg_kernel" in full else _short_kernel(full)
            vals.setdefault((key, ctr), []).append(float(r["Counter_Value"]) * 1024.0)
    cal = {c: 8.0 * spec_cells / (sum(vals[("CALIB", c)]) / len(vals[("CALIB", c)]))
           for c in ("FETCH_SIZE", "WRITE_SIZE")}
    kern = {}
    for (key, ctr), v in vals.items():
        if key == "CALIB" or not key.startswith("k_"):
            continue
        e = kern.setdefault(key, {"dispatches": len(v)})
        e["fetch_bytes" if ctr == "FETCH_SIZE" else "write_bytes"] = sum(v) / len(v) * cal[ctr]
    res = {"workload": "512x512x768 cells, walls, tanh 2.5", "source_sha256": kernel_source_hash(),
           "command": cmd_pmc, "calibration": {"kernel": "torch.neg over one FP64 field (8 B read + 8 B written per cell)",
                                               "fetch_factor": round(cal["FETCH_SIZE"], 4),
                                               "write_factor": round(cal["WRITE_SIZE"], 4)},
           "kernels": kern}
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(res, fh, indent=1, sort_keys=True)
    md = ["# HBM traffic per kernel launch: projection and implicit viscous step, 512x512x768 walls tanh 2.5", "",
          "Commands (run from the repository root on one MI355X; one counter per run):", "", "```", cmd_pmc, "```", "",
          f"Counters scaled by the reading of a plain streaming kernel of known size (torch.neg over one FP64 "
          f"field, 8 B read + 8 B written per cell): FETCH_SIZE x{cal['FETCH_SIZE']:.3f}, "
          f"WRITE_SIZE x{cal['WRITE_SIZE']:.3f}. Bytes per cell = bytes per launch / {spec_cells}.", "",
          f"Kernel sources sha256: `{res['source_sha256']}`", "",
          "| kernel | launches | read B/cell | write B/cell | total GB/launch |", "|---|---:|---:|---:|---:|"]
    for key in sorted(kern):
        e = kern[key]
        md.append(f"| `{key[:70]}` | {e['dispatches']} | {e.get('fetch_bytes', 0) / spec_cells:.2f} | "
                  f"{e.get('write_bytes', 0) / spec_cells:.2f} | "
                  f"{(e.get('fetch_bytes', 0) + e.get('write_bytes', 0)) / 1e9:.3f} |")
    with open(os.path.join(out, "hbm_traffic_c3_512x512x768.md"), "w") as fh:
        fh.write("\n".join(md) + "\n")
    ab_csv = os.path.join(d, "prof_ab", "ab_kernel_stats.csv")
    if os.path.exists(ab_csv):
        summarize_transform_ab(d, ab_csv, out)


def summarize_transform_ab(d, ab_csv, out):
    """profiles/transform_ab_768x768x1024.md from the kernel trace of
    `bench.py --transform-ab` and the JSON line it printed."""
    import csv
    rows = list(csv.DictReader(open(ab_csv)))
    res = None
    log_path = os.path.join(d, "prof_ab.log")
    if os.path.exists(log_path):
        for ln in open(log_path):
            if ln.startswith("{") and "transform_ab" in ln:
                res = json.loads(ln)["transform_ab"]
    md = ["# Transform A/B: the 768-point y transform as LDS FFT kernels and as transform-as-GEMM on the "
          "matrix cores, 768x768x1024", "",
          "Command (run from the repository root on one MI355X):", "", "```",
          "rocprofv3 --kernel-trace --stats -d gpurun_out/prof_ab -o ab --output-format csv -- "
          "python3 bench.py --transform-ab", "python3 bench.py --summarize gpurun_out", "```", ""]
    if res:
        md += ["Event-timed medians printed by the run (ms per forward y transform of the whole grid):", "",
               "| variant | FP32 | FP64 |", "|---|---:|---:|"]
        for key, name in (("lds_fft_ms", "LDS FFT (`k_yfwd`, this library)"),
                          ("gemm_dense_ms", "dense GEMM, M (768x768) X_k per plane"),
                          ("gemm_four_step_ms", "four-step 24x32 GEMMs + twiddles (transposes not counted)")):
            md.append(f"| {name} | {res[key].get('fp32', float('nan')):.3f} | {res[key].get('fp64', float('nan')):.3f} |")
        md.append("")
    md += ["Kernel trace (all kernels of the run; the projections that time the LDS kernels also run their other "
           "kernels):", "", "| kernel | calls | avg (us) | total (ms) |", "|---|---:|---:|---:|"]
    for r in rows:
        name = _short_kernel(r["Name"])
        if len(name) > 80:
            name = name[:80] + "..."
        md.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                  f"{float(r['TotalDurationNs']) / 1e6:.2f} |")
    with open(os.path.join(out, "transform_ab_768x768x1024.md"), "w") as fh:
        fh.write("\n".join(md) + "\n")


def mode_summary(mode, res, ncells, copy_gbs=None):
    """Rates of one leg.  hbm_frac_of_peak prices the step at the minimum-pass
    model of the method (model_bytes_per_cell) where there is one; the bytes
    of the launches this build actually makes are reported beside it."""
    kt = res["kernels"]
    bpc = BYTES_PER_CELL.get(mode, {})
    sec = res["ms_per_step"] / 1e3
    ks = res["kernel_steps"]   # steps the kernel times cover
    build_step = sum(bpc.get(k, 0) * ncells * n for k, (ms, n) in kt.items()) / ks
    iters = res["last_info"]["iterations"] if res.get("last_info") else 0
    mb = model_bytes_per_cell(mode, iters)
    model_step = mb * ncells if mb else build_step
    out = {
        "solves_per_s": round(1.0 / sec, 3),
        "gpts_per_s": round(ncells / sec / 1e9, 3),
        "ms_per_step": round(res["ms_per_step"], 4),
        "median_step_ms": round(res["median_step_ms"], 4),
        "model_bytes_per_cell": mb if mb else round(build_step / ncells, 2),
        "model_bytes_per_step_GB": round(model_step / 1e9, 3),
        "hbm_frac_of_peak": round(model_step / sec / 1e9 / PEAK_HBM_GBS, 4),
        "build_bytes_per_cell": round(build_step / ncells, 2),
        "kernel_ms_per_step": {k: round(ms / ks, 4) for k, (ms, n) in kt.items()},
    }
    if copy_gbs:
        out["frac_of_copy"] = round(model_step / sec / 1e9 / copy_gbs, 4)
    if res.get("div_check") is not None:
        out["max_abs_div_after"] = res["div_check"]
    if res["last_info"]:
        out["iterations"] = res["last_info"]["iterations"]
        out["rel_residual"] = res["last_info"]["rel_residual"]
        if res["last_info"].get("floor_reached"):
            out["floor_reached"] = True
    return out


def cpu_baseline(spec):
    """The FP64 CPU oracle, timed on a bounded sample of the same workload:
    the full projection of the bottom 96 of the 768 z-planes of the same grid
    (same x,y lengths and stretched faces, 1/8 of the cells), scaled to
    solves/s of the whole grid.  Also returns the sample and the oracle's
    result (for the GPU's error against it)."""
    import oracle
    from paper_2103_15187_amd import workloads as W
    nzs = 96
    sub = W.GridSpec(spec.nx, spec.ny, nzs, spec.bcx, spec.bcy, spec.lx, spec.ly, spec.lz, spec.stretch)
    zc = spec.zc()[: nzs + 1]
    g = oracle.Grid(sub.nx, sub.ny, nzs, sub.bcx, sub.bcy, sub.dx, sub.dy, zc)
    u, v, w = W.random_velocity(sub, W.SEEDS["C3"])
    threads = None
    try:
        from threadpoolctl import threadpool_info
        threads = max((i.get("num_threads", 0) for i in threadpool_info()), default=None)
    except Exception:
        pass
    t0 = time.perf_counter()
    ref = oracle.project(u, v, w, g)
    dt = time.perf_counter() - t0
    frac = nzs / spec.nz
    cb = {"value": round(frac / dt, 6), "unit": "solves/s", "cores": threads or len(os.sched_getaffinity(0)),
          "kind": "oracle", "sample": f"full FP64 oracle projection of the bottom {nzs} of {spec.nz} z-planes "
          f"({spec.nx}x{spec.ny}x{nzs}, same grid), {dt:.2f} s, scaled by {spec.nz // nzs}",
          "seconds_for_sample": round(dt, 3), "host_cores": len(os.sched_getaffinity(0))}
    return cb, (sub, zc, (u, v, w), ref)


def cpu_baseline_viscous(spec, beta):
    """The FP64 CPU oracle of the implicit viscous step, timed on a bounded
    sample: for each component and direction, the oracle's line solve
    (numpy.linalg.solve with the dense factor) of 4096 lines at the true line
    length, scaled by that direction's line count, summed over the three
    components and directions (steps/s of the whole grid)."""
    import numpy as np
    import oracle
    from oracle import viscous as V
    from paper_2103_15187_amd import workloads as W
    g = oracle.Grid(spec.nx, spec.ny, spec.nz, spec.bcx, spec.bcy, spec.dx, spec.dy, spec.zc())
    rng = W.rng(7)
    sample = 4096
    lens = {"x": spec.nx, "y": spec.ny, "z": spec.nz}
    nlines = {"x": spec.ny * spec.nz, "y": spec.nx * spec.nz, "z": spec.nx * spec.ny}
    total = 0.0
    t_all = 0.0
    for comp in range(3):
        for d in ("x", "y", "z"):
            b = rng.standard_normal((lens[d], sample))
            t0 = time.perf_counter()
            np.linalg.solve(V.helmholtz_factor(g, comp, d, beta), b)
            dt = time.perf_counter() - t0
            t_all += dt
            total += dt * nlines[d] / sample
    return {"value": round(1.0 / total, 6), "unit": "steps/s", "cores": len(os.sched_getaffinity(0)),
            "kind": "oracle", "sample": f"oracle line solves of {sample} lines per component and direction at the "
            f"true line lengths, scaled by the line counts ({t_all:.2f} s measured)",
            "seconds_for_sample": round(t_all, 3)}


def cpu_baseline_momentum(spec, planes=16):
    """The FP64 CPU oracle of the momentum right-hand side, timed on a slab of
    `planes` z-planes of the same grid (every plane costs the same), scaled by
    nz / planes (steps/s of the whole grid)."""
    import numpy as np
    import oracle
    from oracle import momentum as MO
    from paper_2103_15187_amd import workloads as W
    zc = spec.zc()
    lo = spec.nz // 2 - planes // 2
    g = oracle.Grid(spec.nx, spec.ny, planes, spec.bcx, spec.bcy, spec.dx, spec.dy, zc[lo:lo + planes + 1])
    r = W.rng(11)
    shape = (planes, spec.ny, spec.nx)
    u, v, w = (r.standard_normal(shape) for _ in range(3))
    prev = tuple(r.standard_normal(shape) for _ in range(3))
    t0 = time.perf_counter()
    MO.momentum_rhs(u, v, w, prev, g, dt=1e-3, re=300.0)
    dt = time.perf_counter() - t0
    total = dt * spec.nz / planes
    return {"value": round(1.0 / total, 6), "unit": "steps/s", "cores": len(os.sched_getaffinity(0)),
            "kind": "oracle", "sample": f"oracle right-hand side of {planes} of {spec.nz} z-planes "
            f"({spec.nx}x{spec.ny}x{planes}, same spacing), {dt:.2f} s, scaled by {spec.nz / planes:g}",
            "seconds_for_sample": round(dt, 3)}


def cpu_baseline_ib(spec, planes=24, max_markers=1500):
    """The FP64 CPU oracle of the IB-MLS step (interpolation of u, v, w and
    spreading of one value per marker and component), timed on the surface
    markers of a slab of z-planes (markers two planes or more from the slab's
    ends, so their supports are those of the whole grid), scaled by the
    marker count (steps/s for all markers)."""
    import numpy as np
    import oracle
    from oracle import ibm as IB
    from paper_2103_15187_amd import workloads as W
    xb, dv = W.spheroid_markers(spec)
    zc = spec.zc()
    lo = spec.nz // 2 - planes // 2
    sel = np.nonzero((xb[:, 2] > zc[lo + 3]) & (xb[:, 2] < zc[lo + planes - 3]))[0][:max_markers]
    g = oracle.Grid(spec.nx, spec.ny, planes, spec.bcx, spec.bcy, spec.dx, spec.dy, zc[lo:lo + planes + 1])
    r = W.rng(12)
    field = r.standard_normal((planes, spec.ny, spec.nx))
    fb = r.standard_normal(len(sel))
    t0 = time.perf_counter()
    for comp in range(3):
        IB.interpolate(field, g, comp, xb[sel])
        IB.spread(g, comp, xb[sel], fb, dv[sel])
    dt = time.perf_counter() - t0
    total = dt * len(xb) / len(sel)
    return {"value": round(1.0 / total, 6), "unit": "steps/s", "cores": len(os.sched_getaffinity(0)),
            "kind": "oracle", "sample": f"oracle transfer of {len(sel)} of the {len(xb)} surface markers (those "
            f"in a {planes}-plane slab, on that slab's grid), {dt:.2f} s, scaled by the marker count",
            "seconds_for_sample": round(dt, 3)}


def err_vs_oracle(spec, oracle_out, torch, fsei):
    """Relative L2 errors of the GPU projection (FP64 and FP32+refine, the
    benchmark's launch configuration) against the oracle's result on the
    cpu_baseline sample (the bottom 96 z-planes of the grid)."""
    sub, zc, (u, v, w), ref = oracle_out
    out = {"sample": f"bottom {sub.nz} of {spec.nz} z-planes ({sub.nx}x{sub.ny}x{sub.nz}, same grid), "
                     f"u* N(0,1), against the FP64 oracle's projection"}
    for mode, prec in (("fp64", fsei.PREC_FP64), ("fp32_refine", fsei.PREC_FP32_REFINE)):
        plan = fsei.Plan(sub.nx, sub.ny, sub.nz, (sub.bcx, sub.bcy), sub.dx, sub.dy, zc, precision=prec,
                         rtol=1e-10, max_iter=4)
        d = [torch.from_numpy(a).cuda() for a in (u, v, w)]
        p, info = plan.project(*d, p=torch.empty_like(d[0]), info=True)
        torch.cuda.synchronize()
        e = {k: float(np.linalg.norm(t.cpu().numpy() - r) / np.linalg.norm(r))
             for k, t, r in zip("uvwp", (*d, p), ref)}
        out[mode] = {k: float(f"{x:.3e}") for k, x in e.items()}
        if mode == "fp32_refine":
            out[mode]["rel_residual"] = float(f"{info['rel_residual']:.3e}")
        del plan, d, p
    torch.cuda.empty_cache()
    return out


def transform_ab(torch, fsei):
    """The y transform of the 768 x 768 x 1024 grid two ways: this library's
    LDS FFT kernels (forward + inverse, from the per-kernel times of FP64 and
    FP32 projections) and transform-as-GEMM on the matrix cores through the
    platform GEMM library (torch.matmul): (a) dense, Y_k = M (768 x 768) X_k
    per z-plane; (b) four-step, 768 = 24 x 32 on complex sequences (two real
    lines each): 32-point DFTs as a GEMM, the twiddle multiply, 24-point DFTs
    as a GEMM, transposes not counted.  Median of 5 event-timed runs."""
    from paper_2103_15187_amd import workloads as W
    spec = W.CONFIGS["C5"]
    nx, ny, nz = spec.nx, spec.ny, spec.nz

    def timeit(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        return float(np.median(ts))
    out = {"workload": f"y transform of {nx}x{ny}x{nz} (lines of {ny} points), forward",
           "lds_fft_ms": {}, "gemm_dense_ms": {}, "gemm_four_step_ms": {}}
    for name, prec, dt in (("fp64", fsei.PREC_FP64, torch.float64), ("fp32", fsei.PREC_FP32, torch.float32)):
        plan = fsei.Plan.from_spec(spec, precision=prec)
        u, v, w = (torch.randn(spec.shape, dtype=dt, device="cuda") for _ in range(3))
        for a, m in zip((u, v, w), W.dead_face_masks(spec)):
            a[torch.from_numpy(m).cuda()] = 0
        plan.project(u, v, w, want_p=False)
        torch.cuda.synchronize()
        plan.reset_timing()
        plan.set_timing(True)
        for _ in range(3):
            plan.project(u, v, w, want_p=False)
        torch.cuda.synchronize()
        plan.set_timing(False)
        kt = plan.kernel_times()
        out["lds_fft_ms"][name] = round(kt["yfwd"][0] / kt["yfwd"][1], 4)
        del plan, u, v, w
        torch.cuda.empty_cache()
        X = torch.randn(nz, ny, nx, dtype=dt, device="cuda")
        M = torch.randn(ny, ny, dtype=dt, device="cuda")
        Y = torch.empty_like(X)
        out["gemm_dense_ms"][name] = round(timeit(lambda: torch.matmul(M, X, out=Y)), 4)
        del X, Y
        torch.cuda.empty_cache()
        ct = torch.complex128 if dt == torch.float64 else torch.complex64
        Z = torch.randn(nz * nx // 2, 24, 32, dtype=ct, device="cuda")
        F32, F24, T = (torch.randn(s, dtype=ct, device="cuda") for s in ((32, 32), (24, 24), (24, 32)))

        def four_step():
            A = torch.matmul(Z, F32)
            A.mul_(T)
            return torch.matmul(F24, A)
        out["gemm_four_step_ms"][name] = round(timeit(four_step), 4)
        del Z
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="C3")
    ap.add_argument("--modes", default="fp32_refine,fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-viscous", action="store_true",
                    help="skip the implicit viscous step, the momentum right-hand side and the IB-MLS transfer "
                         "(reported beside the projection, not in value)")
    ap.add_argument("--no-c5", action="store_true",
                    help="skip the 768x768x1024 Poisson solves (reported beside the projection, not in value)")
    ap.add_argument("--c5-steps", type=int, default=4)
    ap.add_argument("--calib", action="store_true",
                    help="also run torch.neg over one field (a plain streaming kernel of known size: "
                         "reads and writes 8 B per cell) to calibrate hardware byte counters")
    ap.add_argument("--transform-ab", action="store_true",
                    help="time the 768-point y transform as this library's LDS FFT and as transform-as-GEMM on "
                         "the matrix cores (dense and four-step), print that as the one JSON line and exit")
    ap.add_argument("--summarize", metavar="DIR",
                    help="write profiles/ summaries from the rocprofv3 outputs under DIR and exit")
    args = ap.parse_args()
    if args.summarize:
        summarize_profiles(
            args.summarize,
            "rocprofv3 --kernel-trace --stats -d gpurun_out/prof -o c3 --output-format csv -- "
            "python3 bench.py --steps 3 --warmup 1 --no-cpu-baseline --no-c5",
            "rocprofv3 --pmc FETCH_SIZE -d gpurun_out/pmc_FETCH_SIZE -o c3 --output-format csv -- "
            "python3 bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-c5 --calib\n"
            "rocprofv3 --pmc WRITE_SIZE -d gpurun_out/pmc_WRITE_SIZE -o c3 --output-format csv -- "
            "python3 bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-c5 --calib\n"
            "python3 bench.py --summarize gpurun_out")
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the projection runs on one GPU only; multi-GPU runs are not supported "
              "(the slab decomposition is a design note, not built)", file=sys.stderr)
        sys.exit(2)
    if args.steps + args.warmup > 30:
        print("bench.py: steps + warmup <= 30 (each step keeps its own resident input copy)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2103_15187_amd import fsei, workloads as W
    if args.transform_ab:
        print(json.dumps({"transform_ab": transform_ab(torch, fsei)}), flush=True)
        return
    spec = W.CONFIGS[args.config]
    log(f"[bench] generating {args.config} input {spec.shape}")
    if args.config == "C3":
        u, v, w = W.c3_velocity(spec, W.SEEDS["C3"])
        recipe = "u* N(0,1) + Gaussian jet (amplitude 10, width 0.05 Lx)"
    else:
        u, v, w = W.random_velocity(spec, W.SEEDS.get(args.config, 1))
        recipe = "u* N(0,1)"
    dev = torch.device("cuda:0")
    u0, v0, w0 = (torch.from_numpy(a).to(dev) for a in (u, v, w))
    del u, v, w
    ncells = spec.ncells
    if args.calib:
        tmp = torch.empty_like(u0)
        torch.neg(u0, out=tmp)
        torch.cuda.synchronize()
        del tmp
    copy_gbs = copy_bandwidth(u0, torch)
    log(f"[bench] plain copy of one field: {copy_gbs:.0f} GB/s")
    modes = [m for m in args.modes.split(",") if m]
    results = {}
    for m in modes:
        log(f"[bench] mode {m}: warmup {args.warmup}, steps {args.steps}")
        res, _ = gpu_mode(m, spec, u0, v0, w0, args.steps, args.warmup, torch, fsei)
        results[m] = res
        log(f"[bench] mode {m}: {res['ms_per_step']:.3f} ms/step (median {res['median_step_ms']:.3f})")
    head = modes[0]
    hres = results[head]
    grid = f"{spec.nx}x{spec.ny}x{spec.nz}"
    line = {
        "metric": f"Poisson-projection solves/s & Gpts/s at {grid}; FP32+refine vs FP64, %HBM peak",
        "value": round(1e3 / hres["ms_per_step"], 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(hres["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if head == "fp32_refine" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {grid} cells, bc x/y "
                   f"{'wall' if spec.bcx else 'periodic'}/{'wall' if spec.bcy else 'periodic'}, z walls "
                   f"tanh {spec.stretch}, {recipe}, dt=1; value = {head}",
                   "grid": [spec.nx, spec.ny, spec.nz], "mode": head},
        "roofline": roofline_for(head, hres, ncells, copy_gbs),
        "modes": {m: mode_summary(m, results[m], ncells, copy_gbs) for m in modes},
        "gpts_per_s": round(ncells * 1e3 / hres["ms_per_step"] / 1e9, 3),
        "copy_GBs": round(copy_gbs, 1),
    }
    for m in modes:
        line["modes"][m]["roofline"] = roofline_for(m, results[m], ncells, copy_gbs)
    if not args.no_viscous:
        log(f"[bench] viscous step: warmup {args.warmup}, steps {args.steps}")
        vres = gpu_viscous(spec, u0, v0, w0, args.steps, args.warmup, torch, fsei)
        log(f"[bench] viscous step: {vres['ms_per_step']:.3f} ms/step")
        vs = mode_summary("viscous_fp64", vres, ncells, copy_gbs)
        vs["steps_per_s"] = vs.pop("solves_per_s")
        vs["beta"] = vres["beta"]
        vs["roofline"] = roofline_for("viscous_fp64", vres, ncells, copy_gbs)
        if not args.no_cpu_baseline:
            vs["cpu_baseline"] = cpu_baseline_viscous(spec, vres["beta"])
        line["modes"]["viscous_fp64"] = vs
        log(f"[bench] momentum right-hand side: warmup {args.warmup}, steps {args.steps}")
        mres = gpu_momentum(spec, u0, v0, w0, args.steps, args.warmup, torch, fsei)
        log(f"[bench] momentum right-hand side: {mres['ms_per_step']:.3f} ms/step")
        ms = mode_summary("momentum_fp64", mres, ncells, copy_gbs)
        ms["steps_per_s"] = ms.pop("solves_per_s")
        ms["roofline"] = roofline_for("momentum_fp64", mres, ncells, copy_gbs)
        if not args.no_cpu_baseline:
            ms["cpu_baseline"] = cpu_baseline_momentum(spec)
        line["modes"]["momentum_fp64"] = ms
        log("[bench] IB-MLS transfer of ~10^6 surface markers")
        ib = gpu_ib(spec, u0, args.steps, args.warmup, torch, fsei)
        ib["steps_per_s"] = round(1e3 / ib["ms_per_step"], 2)
        if not args.no_cpu_baseline:
            ib["cpu_baseline"] = cpu_baseline_ib(spec)
        line["modes"]["ib_mls_fp64"] = ib
        log(f"[bench] IB-MLS: {ib['ms_per_step']:.3f} ms/step")
    del u0, v0, w0
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle on a bounded sample) and the GPU's error against it")
        cb, oracle_out = cpu_baseline(spec)
        line["cpu_baseline"] = cb
        line["err_vs_oracle"] = err_vs_oracle(spec, oracle_out, torch, fsei)
        del oracle_out
    if not args.no_c5:
        line["c5_solve"] = c5_leg(args, torch, fsei)
    print(json.dumps(line), flush=True)


def c5_leg(args, torch, fsei):
    """Poisson solves on the 768 x 768 x 1024 grid (walls, tanh 3.0, power-law
    right-hand side): FP32+refine (to rtol 1e-10 or the FP64 rounding floor
    of this right-hand side) and FP64, each timed over its own steps."""
    from paper_2103_15187_amd import workloads as W
    spec = W.CONFIGS["C5"]
    log(f"[bench] C5 {spec.shape}: power-law right-hand side")
    f0 = torch.from_numpy(W.rhs_powerlaw(spec, W.SEEDS["C5"])).cuda()
    copy_gbs = copy_bandwidth(f0, torch)
    out = {"workload": f"C5: {spec.nx}x{spec.ny}x{spec.nz} cells, walls, z tanh {spec.stretch}, right-hand "
                       f"side k^-5/3 over 64 modes per axis; one step = one fsei_poisson_solve",
           "copy_GBs": round(copy_gbs, 1)}
    for m in ("solve_fp32_refine", "solve_fp64"):
        log(f"[bench] C5 {m}: warmup 1, steps {args.c5_steps}")
        res = gpu_solve(m, spec, f0, args.c5_steps, 1, torch, fsei)
        s = mode_summary(m, res, spec.ncells, copy_gbs)
        s["roofline"] = roofline_for(m, res, spec.ncells, copy_gbs)
        out[m] = s
        log(f"[bench] C5 {m}: {res['ms_per_step']:.3f} ms/step")
    del f0
    torch.cuda.empty_cache()
    return out


if __name__ == "__main__":
    main()
