"""Benchmark: pressure-projection solves/s on the 512 x 512 x 768 stretched grid.

One step = one full projection (divergence + x/y transforms + per-mode z
tridiagonals + inverse transforms + gradient correction) of one provisional
velocity field that is already resident in HBM.  Each timed step projects its
own copy of the input (the projection works in place), so no copy runs inside
the timed region.  Both precision modes are measured in the same run:

  * fp32_refine : FP32 transforms/tridiagonals (lowest-mode lines in FP64),
                  FP64 residual, correction solves to ||r||/||f|| <= 1e-10
                  (the mode this workload is specified with; reported as value)
  * fp64        : every step in FP64

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
             "zsolve": "k_zsolvev<double, double, 2, 16, 24, 512>", "yinv": "k_yinv<double, 4096, 512, 512, 4>",
             "xinv": "k_xinv<double, double, 0, 2048, 256, 512>", "grad": "k_grad_row2<double, double, 256, 16>"},
    "fp32_refine": {"xfwd": "k_xfwd<double, float, 1, 2048, 256, 512>", "yfwd": "k_yfwd<float, 8192, 1024, 512, 6>",
                    "zsolve": "k_zsolvev<float, float, 4, 16, 24, 512>", "yinv": "k_yinv<float, 8192, 1024, 512, 4>",
                    "xinv": "k_xinv<float, float, 0, 2048, 256, 512>", "xinv_acc": "k_xinv<float, double, 2, 2048, 256, 512>",
                    "resid": "k_resid_pairs<256, 8, true, float, 2>",
                    "resid_norm": "k_resid_pairs<256, 8, false, double, 2>",
                    "xfwd_r": "k_xfwd<float, float, 4, 2048, 256, 512>", "grad": "k_grad_row2<double, double, 256, 16>",
                    "grad_resid": "k_grad_resid<256, 16, false>"},
    "viscous_fp64": {"visc_x": "k_visc_x<16>", "visc_y": "k_visc_strided<2, 16>",
                     "visc_z": "k_visc_strided<2, 24>"},
    "momentum_fp64": {"momentum_rhs": "k_momentum_rhs_pairs<64, 16, true>"},
}

# Algorithmic HBM bytes per cell of each kernel launch (minimum pass model:
# every operand read once, every result written once).
BYTES_PER_CELL = {
    "fp64": {"xfwd": 32, "yfwd": 16, "zsolve": 16, "yinv": 16, "xinv": 16, "grad": 56},
    # refinement at this workload (pair tiling): the first solve's pressure is
    # FP32 (x inverse writes 4 B; the first residual reads it: f 8 + p 4, r 4
    # written; the first correction reads p32 + delta and writes p 8)
    "fp32_refine": {"xfwd": 36, "yfwd": 8, "zsolve": 8, "yinv": 8, "xinv": 8, "resid_xfwd": 20,
                    "resid": 16, "xfwd_r": 8, "resid_norm": 16, "xinv_acc": 16, "grad": 56, "grad_resid": 64},
    # implicit viscous step: every line solve of one component reads and
    # writes the field once (3 components x 3 directions = 144 B/cell)
    "viscous_fp64": {"visc_x": 16, "visc_y": 16, "visc_z": 16},
    # explicit momentum right-hand side: u, v, w and N^{n-1} read, rhs and N^n written
    "momentum_fp64": {"momentum_rhs": 96},
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def gpu_mode(mode, spec, u0, v0, w0, steps, warmup, torch, fsei):
    """Time `steps` projections of resident copies of (u0, v0, w0)."""
    prec = fsei.PREC_FP64 if mode == "fp64" else fsei.PREC_FP32_REFINE
    plan = fsei.Plan.from_spec(spec, precision=prec, rtol=1e-10, max_iter=4)
    ncopy = steps + warmup
    bufs = [(u0.clone(), v0.clone(), w0.clone()) for _ in range(ncopy)]
    p = torch.empty_like(u0)
    torch.cuda.synchronize()
    infos = []
    for i in range(warmup):
        _, info = plan.project(*bufs[i], p=p, info=True)
        infos.append(info)
    torch.cuda.synchronize()
    # refine mode reads one residual norm per iteration back to the host;
    # FP64 mode runs without any host synchronisation inside the loop
    t0 = time.perf_counter()
    for i in range(warmup, ncopy):
        if mode == "fp64":
            plan.project(*bufs[i], p=p)
        else:
            _, info = plan.project(*bufs[i], p=p, info=True)
            infos.append(info)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # per-kernel times from HIP events the library records around every
    # launch, in a separate instrumented pass over fresh copies of the input
    # (the events are kept out of the timed loop above)
    nk = min(steps, 3)
    for i in range(nk):
        for dst, src in zip(bufs[i], (u0, v0, w0)):
            dst.copy_(src)
    torch.cuda.synchronize()
    plan.reset_timing()
    plan.set_timing(True)
    for i in range(nk):
        plan.project(*bufs[i], p=p)
    torch.cuda.synchronize()
    plan.set_timing(False)
    ktimes = plan.kernel_times()
    # check the last output: divergence of the projected field, V-mean of p
    res = {"ms_per_step": (t1 - t0) * 1e3 / steps, "kernels": ktimes, "kernel_steps": nk}
    res["last_info"] = infos[-1] if infos else None
    u, v, w = bufs[-1]
    res["div_check"] = float(divergence_max(u, v, w, spec, torch))
    del bufs
    torch.cuda.empty_cache()
    return res, plan


def gpu_viscous(spec, u0, v0, w0, steps, warmup, torch, fsei):
    """Time `steps` implicit viscous steps (fsei_viscous_solve of u, v, w) on
    resident copies of the input (the solve does the same work whatever the
    values, so each step re-solves the previous step's output)."""
    plan = fsei.Plan.from_spec(spec)
    beta = 0.5 * spec.dx ** 2
    u, v, w = u0.clone(), v0.clone(), w0.clone()
    for _ in range(warmup):
        plan.viscous_step(u, v, w, beta)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.viscous_step(u, v, w, beta)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    nk = min(steps, 3)
    plan.reset_timing()
    plan.set_timing(True)
    for _ in range(nk):
        plan.viscous_step(u, v, w, beta)
    torch.cuda.synchronize()
    plan.set_timing(False)
    res = {"ms_per_step": (t1 - t0) * 1e3 / steps, "kernels": plan.kernel_times(), "kernel_steps": nk,
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
    for _ in range(warmup):
        plan.momentum_rhs(u0, v0, w0, n, r, dt, re)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.momentum_rhs(u0, v0, w0, n, r, dt, re)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    nk = min(steps, 3)
    plan.reset_timing()
    plan.set_timing(True)
    for _ in range(nk):
        plan.momentum_rhs(u0, v0, w0, n, r, dt, re)
    torch.cuda.synchronize()
    plan.set_timing(False)
    res = {"ms_per_step": (t1 - t0) * 1e3 / steps, "kernels": plan.kernel_times(), "kernel_steps": nk,
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

    def step():
        for c in range(3):
            plan.ib_interpolate(u0, c, xd, ub)
            plan.ib_spread(f, c, xd, fb, dvb)
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plan.reset_timing()
    plan.set_timing(True)
    step()
    torch.cuda.synchronize()
    plan.set_timing(False)
    kt = plan.kernel_times()
    ms = (t1 - t0) * 1e3 / steps
    del f, xd, fb, dvb, ub
    torch.cuda.empty_cache()
    return {"ms_per_step": round(ms, 4), "markers": nb, "markers_per_s": round(nb / (ms / 1e3), 1),
            "kernel_ms_per_step": {k: round(v[0], 4) for k, v in kt.items()},
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


def roofline_for(mode, res, ncells):
    """Dominant kernel (largest total time) and its achieved algorithmic
    bandwidth over the timed region."""
    kt = res["kernels"]
    bpc = BYTES_PER_CELL[mode]
    name = max((k for k in kt if k in bpc), key=lambda k: kt[k][0])
    total_ms, n = kt[name]
    avg_s = total_ms / n / 1e3
    bytes_per_launch = bpc[name] * ncells
    achieved = bytes_per_launch / avg_s / 1e9
    return {"kernel": name, "bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": measured_traffic(mode, name, ncells),
            "bytes_per_launch": bytes_per_launch, "avg_launch_ms": round(avg_s * 1e3, 4)}


def _short_kernel(name):
    return name.split("(")[0].replace("void ", "").replace("fsei::dev::", "").strip()


def summarize_profiles(d, cmd_trace, cmd_pmc):
    """Turn the rocprofv3 outputs under `d` (prof/, pmc_FETCH_SIZE/,
    pmc_WRITE_SIZE/) into the committed summaries under profiles/."""
    import csv
    out = os.path.join(ROOT, "profiles")
    rows = list(csv.DictReader(open(os.path.join(d, "prof", "c3_kernel_stats.csv"))))
    md = ["# Kernel trace: projection (FP32+refine and FP64 modes) and implicit viscous step, "
          "512x512x768 walls tanh 2.5", "",
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


def mode_summary(mode, res, ncells):
    kt = res["kernels"]
    bpc = BYTES_PER_CELL[mode]
    sec = res["ms_per_step"] / 1e3
    # algorithmic bytes per step from the launches actually made
    ks = res["kernel_steps"]   # steps of the instrumented pass the kernel times cover
    bytes_step = sum(bpc.get(k, 0) * ncells * n for k, (ms, n) in kt.items()) / ks
    out = {
        "solves_per_s": round(1.0 / sec, 3),
        "gpts_per_s": round(ncells / sec / 1e9, 3),
        "ms_per_step": round(res["ms_per_step"], 4),
        "model_bytes_per_step_GB": round(bytes_step / 1e9, 3),
        "hbm_frac_of_peak": round(bytes_step / sec / 1e9 / PEAK_HBM_GBS, 4),
        "kernel_ms_per_step": {k: round(ms / ks, 4) for k, (ms, n) in kt.items()},
        "max_abs_div_after": res["div_check"],
    }
    if res["last_info"]:
        out["iterations"] = res["last_info"]["iterations"]
        out["rel_residual"] = res["last_info"]["rel_residual"]
    return out


def cpu_baseline(spec):
    """The FP64 CPU oracle, timed on a bounded sample of the same workload:
    the full projection of the bottom 96 of the 768 z-planes of the same grid
    (same x,y lengths and stretched faces, 1/8 of the cells), scaled to
    solves/s of the whole grid."""
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
    oracle.project(u, v, w, g)
    dt = time.perf_counter() - t0
    frac = nzs / spec.nz
    return {"value": round(frac / dt, 6), "unit": "solves/s", "cores": threads or len(os.sched_getaffinity(0)),
            "kind": "oracle", "sample": f"full FP64 oracle projection of the bottom {nzs} of {spec.nz} z-planes "
            f"({spec.nx}x{spec.ny}x{nzs}, same grid), {dt:.2f} s, scaled by {spec.nz // nzs}",
            "seconds_for_sample": round(dt, 3), "host_cores": len(os.sched_getaffinity(0))}


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
    ap.add_argument("--calib", action="store_true",
                    help="also run torch.neg over one field (a plain streaming kernel of known size: "
                         "reads and writes 8 B per cell) to calibrate hardware byte counters")
    ap.add_argument("--summarize", metavar="DIR",
                    help="write profiles/ summaries from the rocprofv3 outputs under DIR and exit")
    args = ap.parse_args()
    if args.summarize:
        summarize_profiles(
            args.summarize,
            "rocprofv3 --kernel-trace --stats -d gpurun_out/prof -o c3 --output-format csv -- "
            "python3 bench.py --steps 3 --warmup 1 --no-cpu-baseline",
            "rocprofv3 --pmc FETCH_SIZE -d gpurun_out/pmc_FETCH_SIZE -o c3 --output-format csv -- "
            "python3 bench.py --steps 1 --warmup 0 --no-cpu-baseline --calib\n"
            "rocprofv3 --pmc WRITE_SIZE -d gpurun_out/pmc_WRITE_SIZE -o c3 --output-format csv -- "
            "python3 bench.py --steps 1 --warmup 0 --no-cpu-baseline --calib\n"
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
    spec = W.CONFIGS[args.config]
    log(f"[bench] generating {args.config} input {spec.shape}")
    if args.config == "C3":
        u, v, w = W.c3_velocity(spec, W.SEEDS["C3"])
    else:
        u, v, w = W.random_velocity(spec, W.SEEDS.get(args.config, 1))
    dev = torch.device("cuda:0")
    u0, v0, w0 = (torch.from_numpy(a).to(dev) for a in (u, v, w))
    del u, v, w
    ncells = spec.ncells
    if args.calib:
        tmp = torch.empty_like(u0)
        torch.neg(u0, out=tmp)
        torch.cuda.synchronize()
        del tmp
    modes = [m for m in args.modes.split(",") if m]
    results = {}
    for m in modes:
        log(f"[bench] mode {m}: warmup {args.warmup}, steps {args.steps}")
        res, _ = gpu_mode(m, spec, u0, v0, w0, args.steps, args.warmup, torch, fsei)
        results[m] = res
        log(f"[bench] mode {m}: {res['ms_per_step']:.3f} ms/step")
    head = modes[0]
    hres = results[head]
    line = {
        "metric": "Poisson-projection solves/s & Gpts/s at 512^2x768; FP32+refine vs FP64, %HBM peak",
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
        "config": {"workload": f"{args.config}: {spec.nx}x{spec.ny}x{spec.nz} cells, bc x/y "
                   f"{'wall' if spec.bcx else 'periodic'}/{'wall' if spec.bcy else 'periodic'}, z walls "
                   f"tanh {spec.stretch}, u* N(0,1) + Gaussian jet, dt=1; value = {head}",
                   "grid": [spec.nx, spec.ny, spec.nz], "mode": head},
        "roofline": roofline_for(head, hres, ncells),
        "modes": {m: mode_summary(m, results[m], ncells) for m in modes},
        "gpts_per_s": round(ncells * 1e3 / hres["ms_per_step"] / 1e9, 3),
    }
    for m in modes:
        line["modes"][m]["roofline"] = roofline_for(m, results[m], ncells)
    if not args.no_viscous:
        log(f"[bench] viscous step: warmup {args.warmup}, steps {args.steps}")
        vres = gpu_viscous(spec, u0, v0, w0, args.steps, args.warmup, torch, fsei)
        log(f"[bench] viscous step: {vres['ms_per_step']:.3f} ms/step")
        vs = mode_summary("viscous_fp64", vres, ncells)
        vs.pop("max_abs_div_after", None)
        vs["steps_per_s"] = vs.pop("solves_per_s")
        vs["beta"] = vres["beta"]
        vs["roofline"] = roofline_for("viscous_fp64", vres, ncells)
        if not args.no_cpu_baseline:
            vs["cpu_baseline"] = cpu_baseline_viscous(spec, vres["beta"])
        line["modes"]["viscous_fp64"] = vs
        log(f"[bench] momentum right-hand side: warmup {args.warmup}, steps {args.steps}")
        mres = gpu_momentum(spec, u0, v0, w0, args.steps, args.warmup, torch, fsei)
        log(f"[bench] momentum right-hand side: {mres['ms_per_step']:.3f} ms/step")
        ms = mode_summary("momentum_fp64", mres, ncells)
        ms.pop("max_abs_div_after", None)
        ms["steps_per_s"] = ms.pop("solves_per_s")
        ms["roofline"] = roofline_for("momentum_fp64", mres, ncells)
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
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle on a bounded sample)")
        line["cpu_baseline"] = cpu_baseline(spec)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
