"""Benchmark: grid points per second for one E_c^nl + v_c^nl evaluation (N_alpha = 20) on one GPU.

    python bench.py [--steps K] [--warmup W] [--workload nanoparticle_512] [--precision fp64|fp32]

A step is one potential evaluation (theta + forward FFTs, contraction, inverse FFTs, derivative
assembly, spectral divergence, energy) of the workload's seeded synthetic density, with its
analytic gradient, inputs already resident in HBM.  The headline is the 512^3 / 48 Angstrom
nanoparticle (the largest workload; its 23.8 / 47 GB of work buffers fit one GPU) in FP64, the
paper's arithmetic; the FP32_MIXED form on the same workload is reported under "fp32_mixed",
with its difference to the FP64 result.  Prints one JSON line.

The K timed steps run twice per form: without instrumentation (value, ms_per_step), then with
the library's HIP events around every kernel on its stream; the roofline figure is the dominant
kernel's algorithmic bytes per launch over its average event-timed duration.  The CPU baseline is
the FP64 oracle on the host cores, on the bounded workload named in its "sample" field.  The
serving measurement replays a Poisson stream of requests through the continuous-batching server
in the FP32_MIXED form.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
M = 20
METRIC = "grid pts/s for E_c^nl+v_c^nl (Nalpha=20) at stated rel. error; p50/p99 serve latency"


def say(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    from paper_1703_06999_amd.profiling import source_hash
    return source_hash()


def profiled_traffic(workload: str, precision: str, stage: str):
    """HBM bytes per launch of `stage` from the committed rocprofv3 counter summary
    (profiles/traffic_<workload>_<precision>.md: FETCH_SIZE and WRITE_SIZE scaled by a plain
    streaming kernel of known size), or None if there is none or the kernel sources changed since
    the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}_{precision}.md")
    if not os.path.exists(path):
        return None
    src_hash, rows = None, {}
    for line in open(path):
        if line.startswith("source_sha256:"):
            src_hash = line.split(":", 1)[1].strip()
        elif line.startswith("| `") and "|" in line[3:]:
            cells = [c.strip().strip("`") for c in line.strip().strip("|").split("|")]
            try:
                rows[cells[0]] = float(cells[-1])
            except ValueError:
                pass
    if src_hash != kernel_source_hash() or stage not in rows:
        return None
    return rows[stage]


def stage_bytes(stage: str, grid, precision: str, m: int = M) -> float:
    """Algorithmic HBM bytes one launch of a stage must move (reads + writes)."""
    n1, n2, n3 = grid
    N = n1 * n2 * n3
    Nk = n1 * n2 * (n3 // 2 + 1)
    c = 16 if precision == "fp64" else 8          # complex element
    r = c // 2                                    # real element
    st = 32 if precision == "fp64" else 16        # per-point spline state, theta pass -> assembly
    return {
        "theta_zfwd": 32 * N + m * Nk * c + st * N,   # n + grad in, theta(kz) and state out
        "y_fwd": 2 * m * Nk * c,
        "x_contract": 2 * m * Nk * c,
        "y_inv": 2 * m * Nk * c,
        "z_assemble": m * Nk * c + st * N + 16 * N,   # F(kz), state in; v, dE/dsigma out
        "div_z": 32 * N + 3 * r * N,                  # S + grad in; A, B1, B2 out
        "div_y": 5 * r * N,                            # A, B1, B2 in; A', B1' out
        "div_x": 2 * r * N + 16 * N,                   # A', B1' and v in; v out
        "lda": 16 * N,                                 # n in, v_c^LDA out (FP64 in both forms)
    }.get(stage, 0.0)


def host_description() -> dict:
    """CPU model, logical CPUs usable by this process and RAM of the host."""
    model = platform.processor() or "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    ram_gb = None
    try:
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal:"):
                ram_gb = round(int(line.split()[1]) / 2 ** 20, 1)
                break
    except OSError:
        pass
    try:
        cpus = len(os.sched_getaffinity(0))
    except AttributeError:
        cpus = os.cpu_count()
    return {"cpu_model": model, "logical_cpus": cpus, "ram_GiB": ram_gb}


def cpu_baseline(workload_name: str, n_cpu, g_cpu, w, kt):
    """Time the FP64 oracle on the host for one evaluation, stage by stage."""
    from oracle import vdwdf
    stages = {}

    def progress(step, dt):
        stages[step] = round(stages.get(step, 0.0) + dt, 3)
    t0 = time.perf_counter()
    vdwdf.potential(n_cpu, w.cell, kt, grad=g_cpu, progress=progress)
    dt = time.perf_counter() - t0
    host = host_description()
    return {"value": w.npoints / dt, "unit": "grid pts/s", "cores": int(vdwdf.WORKERS), "kind": "oracle",
            "sample": f"one FP64 E+v evaluation (analytic gradient) of {workload_name} "
                      f"({w.grid[0]}x{w.grid[1]}x{w.grid[2]}, {w.npoints} points), {dt:.1f} s; scipy.fft "
                      f"with {vdwdf.WORKERS} worker threads, the other stages numpy on one thread",
            "workload": workload_name, "seconds": round(dt, 3), "stage_seconds": stages, **host}


def time_form(f, n, g, steps: int, warmup: int, grid, precision: str, m: int = M):
    """Warm up, then time `steps` evaluations twice (plain, then with per-kernel HIP events).
    Returns (ms_per_step, stages, roofline, v, E)."""
    import torch
    dev = n.device
    v = torch.empty_like(n)
    e = torch.zeros(1, dtype=torch.float64, device=dev)
    for _ in range(warmup):
        f.potential_async(n, g, v, e)
    torch.cuda.synchronize()
    # timed region 1: throughput, no instrumentation
    t0 = time.perf_counter()
    for _ in range(steps):
        f.potential_async(n, g, v, e)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # timed region 2: the same steps with the library's per-kernel HIP events (recorded on the
    # stream the kernels run on), for the per-kernel durations behind the roofline figure
    f.enable_timing(True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(steps):
        f.potential_async(n, g, v, e)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    stages = f.read_timing()
    f.enable_timing(False)
    ms_per_step = 1e3 * (t1 - t0) / steps
    per_stage = {k: {"ms_avg": round(ms / cnt, 4), "launches": cnt,
                     "GBps": round(stage_bytes(k, grid, precision, m) / (ms / cnt * 1e-3) / 1e9, 1),
                     "frac_hbm": round(stage_bytes(k, grid, precision, m) / (ms / cnt * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
                 for k, (ms, cnt) in stages.items()}
    dom = max(stages, key=lambda k: stages[k][0])
    avg_s = stages[dom][0] / stages[dom][1] * 1e-3
    achieved = stage_bytes(dom, grid, precision, m) / avg_s / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "algorithmic_bytes_per_launch": stage_bytes(dom, grid, precision, m),
                "avg_launch_ms": round(avg_s * 1e3, 4),
                "timing": "HIP events around each kernel over a second timed region of the same steps "
                          f"({1e3 * (t3 - t2) / steps:.4f} ms/step with the events)"}
    return ms_per_step, per_stage, roofline, v, float(e.item())


def time_lda(f, n, steps: int, npoints: int):
    """The LDA correlation pass (E_c^LDA, v_c^LDA; FP64 in both precisions) on the same density:
    per-launch time from the library's HIP events, against its 16 bytes per point."""
    import torch
    v = torch.empty_like(n)
    e = torch.zeros(1, dtype=torch.float64, device=n.device)
    for _ in range(2):
        f.lda_async(n, v, e)
    f.enable_timing(True)
    for _ in range(steps):
        f.lda_async(n, v, e)
    ms, cnt = f.read_timing()["lda"]
    f.enable_timing(False)
    avg = ms / cnt
    gbs = 16.0 * npoints / (avg * 1e-3) / 1e9
    return {"ms_avg": round(avg, 4), "launches": cnt, "GBps": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBS, 4),
            "bytes_per_point": 16, "E_c_lda": float(e.item())}


def time_spin(f, n, g, steps: int):
    """The spin-polarised potential entry on the same density split n_up = 0.6 n, n_dn = 0.4 n
    (zeta = 0.2, gradients split alike), against the spin-paired potential entry on n: wall time per
    evaluation, and the two spin conversion passes from the library's HIP events."""
    import torch
    ins = (0.6 * n, 0.4 * n, 0.6 * g, 0.4 * g)
    vu, vd, v = torch.empty_like(n), torch.empty_like(n), torch.empty_like(n)
    e = torch.zeros(1, dtype=torch.float64, device=n.device)
    res = {"zeta": 0.2, "entry": "vdwxc_calculate_spin_potential_async against vdwxc_calculate_potential_async"}
    for label, call in (("spin_paired", lambda: f.potential_async(n, g, v, e)),
                        ("spin", lambda: f.spin_potential_async(*ins, vu, vd, e))):
        call()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            call()
        torch.cuda.synchronize()
        res[f"{label}_ms_per_eval"] = round((time.perf_counter() - t0) * 1e3 / steps, 4)
    f.enable_timing(True)
    for _ in range(steps):
        f.spin_potential_async(*ins, vu, vd, e)
    st = f.read_timing()
    f.enable_timing(False)
    ms, cnt = st["spin"]
    res["conversion_ms_per_eval"] = round(ms / steps, 4)
    res["conversion_launches"] = cnt
    res["divergence_ms_per_eval"] = round(sum(st[k][0] for k in ("div_z", "div_y", "div_x")) / steps, 4)
    res["E"] = float(e.item())
    del ins, vu, vd, v
    torch.cuda.empty_cache()
    return res


def serving_measurement(kt, count, rate, precision):
    """Poisson stream of `count` energy+potential requests (grids 48..160^3) through the
    continuous-batching server: once with a 64 GB HBM budget, once with the budget capped at 1.25x
    the largest request's workspace, so that admission queues.  Densities are generated, and the
    slots' handles for the five shapes created (as far as the budget allows), before the clock
    starts."""
    import torch

    from paper_1703_06999_amd import serving, vdwxc
    say(f"serving: generating {count} requests")
    reqs = serving.poisson_requests(count, rate, seed=0)
    grids = [48, 64, 96, 128, 160]
    small = 1.25 * vdwxc.workspace_bytes((160, 160, 160), precision)
    res = {"requests": count, "rate_per_s": rate, "grids": grids, "precision": precision}
    for label, budget in (("budget_64GB", 64e9), (f"budget_{small / 1e9:.2f}GB", small)):
        for r in reqs:
            r.admitted = r.finished = r.energy = r.v = None
        srv = serving.Server(kt, slots=4, precision=precision, hbm_budget=budget)
        warmed = srv.warm(serving.serving_shapes())
        summary = srv.run(reqs)
        summary["handles_prewarmed"] = warmed
        srv.close()
        torch.cuda.empty_cache()
        res[label] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in summary.items()}
        say(f"serving {label}: {res[label]}")
    return res


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="nanoparticle_512")
    ap.add_argument("--precision", default="fp64", choices=["fp32", "fp64"],
                    help="arithmetic of the headline value (the other form is reported beside it)")
    ap.add_argument("--no-second-form", action="store_true", help="time only the headline precision")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-workload", default="nanoparticle_slab_64x512x512",
                    help="workload of the oracle timing: a slab of the 512^3 nanoparticle cell (same spacing "
                         "and blob mix; the whole cell is beyond a bounded host run), or any named workload")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--no-qmesh", action="store_true",
                    help="skip the timing of the headline form with a 10-point q-mesh")
    ap.add_argument("--no-spin", action="store_true", help="skip the spin-polarised entry timing")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--serve-rate", type=float, default=40.0)
    ap.add_argument("--density-cache", default=None,
                    help="file holding the workload's density and gradient: read if it exists, else written "
                         "after generating them (saves regenerating them under a profiler)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="after the timed steps, run one plain device copy of this many MiB (a "
                         "kernel of known traffic for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the library runs on one GPU and has no multi-GPU path (the slab decomposition "
              "with all-to-all exchanges is a design only)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1703_06999_amd import inputs, vdwxc

    dev = torch.device("cuda:0")
    kt = inputs.synthetic_kernel_table()
    w = inputs.workload(args.workload)
    say(f"workload {args.workload} grid {w.grid}, headline precision {args.precision}")
    t_in = time.perf_counter()
    if args.density_cache and os.path.exists(args.density_cache):
        cached = torch.load(args.density_cache, map_location="cuda", weights_only=True)
        if cached.get("workload") != args.workload:
            raise SystemExit(f"{args.density_cache} holds {cached.get('workload')}, not {args.workload}")
        n, g = cached["n"], cached["g"]
    else:
        n, g = w.density(device="cuda", progress=lambda done, total: say(f"density: {done}/{total} blobs"))
        if args.density_cache:
            torch.save({"workload": args.workload, "n": n, "g": g}, args.density_cache)
    torch.cuda.synchronize()
    say(f"density ready in {time.perf_counter() - t_in:.1f} s")

    forms = [args.precision] + ([] if args.no_second_form else [p for p in ("fp64", "fp32") if p != args.precision])
    results = {}
    lda = spin = None
    for prec in forms:
        f = vdwxc.Functional(w.grid, w.cell, flavour="DF1", precision=prec, table=kt)
        ms, stages, roof, v, E = time_form(f, n, g, args.steps, args.warmup, w.grid, prec)
        roof["traffic"] = profiled_traffic(args.workload, prec, roof["kernel"])
        if prec == args.precision:
            lda = time_lda(f, n, args.steps, w.npoints)
            say(f"lda correlation: {lda['ms_avg']:.3f} ms, {lda['GBps']:.0f} GB/s")
            if not args.no_spin:
                spin = time_spin(f, n, g, max(2, args.steps // 4))
                say(f"spin: {spin}")
        f.close()
        results[prec] = dict(ms=ms, stages=stages, roofline=roof, v=v, E=E)
        say(f"{prec}: {ms:.3f} ms/step, {w.npoints / ms * 1e3:.4e} pts/s, E = {E:.12e}, "
            f"dominant {roof['kernel']} {roof['frac']:.3f} of HBM")
        if prec == args.precision:
            torch.cuda.synchronize()
        del f
    qmesh = None
    if not args.no_qmesh:
        # the same workload and form with a 10-point q-mesh: the FFT passes scale with M, the
        # contraction with its pair count M(M+1)/2 (bucket 10: 55 pairs against 210)
        m10 = 10
        kt10 = inputs.synthetic_kernel_table(qmesh=inputs.log_qmesh(m10))
        f = vdwxc.Functional(w.grid, w.cell, flavour="DF1", precision=args.precision, table=kt10)
        steps10 = max(2, args.steps // 2)
        ms10, st10, _, v10, E10 = time_form(f, n, g, steps10, max(1, args.warmup // 2), w.grid, args.precision, m10)
        f.close()
        del f, v10
        x20 = results[args.precision]["stages"]["x_contract"]["ms_avg"]
        qmesh = {"n_alpha": m10, "steps": steps10, "ms_per_step": round(ms10, 4),
                 "ms_per_step_n_alpha_20": round(results[args.precision]["ms"], 4),
                 "x_contract_ms": st10["x_contract"]["ms_avg"], "x_contract_ms_n_alpha_20": x20,
                 "x_contract_ratio": round(st10["x_contract"]["ms_avg"] / x20, 4),
                 "stages": st10}
        say(f"q-mesh {m10}: {ms10:.3f} ms/step, x_contract {st10['x_contract']['ms_avg']:.3f} ms (M=20: {x20:.3f})")
    if args.copy_calibration_mb:
        # one streaming elementwise kernel (negation) reading and writing N bytes each
        nel = args.copy_calibration_mb * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst

    head = results[args.precision]
    second = None
    if len(forms) > 1:
        other = forms[1]
        r = results[other]
        ref64 = results["fp64"]
        r32 = results["fp32"]
        d = torch.abs(r32["v"] - ref64["v"])
        vmax = float(torch.max(torch.abs(ref64["v"])))
        core = n >= 1e-6
        second = {"precision": "fp32_mixed" if other == "fp32" else "fp64",
                  "value": w.npoints / r["ms"] * 1e3, "unit": "grid pts/s", "ms_per_step": r["ms"],
                  "roofline": r["roofline"], "stages": r["stages"],
                  "fp32_vs_fp64": {"E_rel": abs(r32["E"] - ref64["E"]) / abs(ref64["E"]),
                                   "v_maxnorm_rel_n_ge_1e-6": float(torch.max(torch.where(core, d, torch.zeros_like(d)))) / vmax,
                                   "v_maxnorm_rel_all": float(torch.max(d)) / vmax,
                                   "v_density_weighted_l1": float(torch.sum(n * d) / torch.sum(n * torch.abs(ref64["v"])))}}
    for r in results.values():
        r["v"] = None
    torch.cuda.empty_cache()

    cpu = None
    accuracy = None
    if not args.no_cpu_baseline:
        m = re.fullmatch(r"nanoparticle_slab_(\d+)x(\d+)x(\d+)", args.cpu_workload)
        bw = (inputs.workload("nanoparticle_slab", grid=tuple(int(x) for x in m.groups())) if m
              else inputs.workload(args.cpu_workload))
        bn, bg = bw.density(device="cuda")
        nc, gc = bn.cpu().numpy(), bg.cpu().numpy()
        say(f"oracle CPU baseline on {args.cpu_workload}")
        cpu = cpu_baseline(args.cpu_workload, nc, gc, bw, kt)
        say(f"oracle: {cpu['seconds']} s, stages {cpu['stage_seconds']}")
        del bn, bg

    serve = None
    if not args.no_serve:
        serve = serving_measurement(kt, args.serve_requests, args.serve_rate, "fp32")

    prec = args.precision
    out = {
        "metric": METRIC,
        "value": w.npoints / head["ms"] * 1e3,
        "unit": "grid pts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "grid": list(w.grid), "cell_bohr": float(w.cell[0, 0]),
                   "n_alpha": M,
                   "precision": ("fp32_mixed (q0 and its derivatives, energy and derivative sums, spectral "
                                 "gradient in fp64; theta, FFTs, table, contraction in fp32)")
                   if prec == "fp32" else "fp64 throughout",
                   "entry": "vdwxc_calculate_potential_async, analytic gradient", "parallelism": "1 GPU"},
        "roofline": head["roofline"],
        "cpu_baseline": cpu,
        "accuracy": accuracy,
        "stages": head["stages"],
        "fp32_mixed" if prec == "fp64" else "fp64": second,
        "serving": serve,
        "q_mesh_10": qmesh,
        "lda_correlation": lda,
        "spin_polarised": spin,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
