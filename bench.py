"""Benchmark: grid points per second for one E_c^nl + v_c^nl evaluation (N_alpha = 20) on one GPU.

    python bench.py [--steps K] [--warmup W] [--workload slater_128] [--precision fp32|fp64]

A step is one potential evaluation (theta + forward FFTs, contraction, inverse FFTs, derivative
assembly, spectral divergence, energy) of the workload's seeded synthetic density, with its
analytic gradient, inputs already resident in HBM.  Prints one JSON line.  The K timed steps run
twice: without instrumentation (value, ms_per_step), then with the library's HIP events around
every kernel on its stream; the roofline figure is the dominant kernel's algorithmic bytes per
launch over its average event-timed duration.  The CPU baseline is the FP64 oracle on the host
cores, on the workload named in its "sample" field.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
M = 20
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
    }.get(stage, 0.0)


def cpu_baseline(workload_name: str, n_cpu, g_cpu, w, kt):
    """Time the FP64 oracle on the host for one evaluation; returns (record, oracle E, oracle v)."""
    from oracle import vdwdf
    t0 = time.perf_counter()
    E, v, _, _ = vdwdf.potential(n_cpu, w.cell, kt, grad=g_cpu)
    dt = time.perf_counter() - t0
    rec = {"value": w.npoints / dt, "unit": "grid pts/s", "cores": int(vdwdf.WORKERS), "kind": "oracle",
           "sample": f"one FP64 E+v evaluation of {workload_name} ({w.grid[0]}x{w.grid[1]}x{w.grid[2]}), "
                     f"{dt:.1f} s, scipy.fft with {vdwdf.WORKERS} workers"}
    return rec, E, v


def serving_measurement(kt, count, rate, precision):
    """Poisson stream of `count` energy+potential requests (grids 48..160^3) through the
    continuous-batching server: once with a 64 GB HBM budget, once capped at 1 GB so admission
    queues.  Densities are generated, and the slots' handles for the five shapes created (as far
    as the budget allows), before the clock starts."""
    import torch

    from paper_1703_06999_amd import serving
    print(f"[bench] serving: generating {count} requests", file=sys.stderr, flush=True)
    reqs = serving.poisson_requests(count, rate, seed=0)
    res = {"requests": count, "rate_per_s": rate, "grids": [48, 64, 96, 128, 160], "precision": precision}
    for label, budget in (("budget_64GB", 64e9), ("budget_1GB", 1e9)):
        for r in reqs:
            r.admitted = r.finished = r.energy = r.v = None
        srv = serving.Server(kt, slots=4, precision=precision, hbm_budget=budget)
        warmed = srv.warm(serving.serving_shapes())
        summary = srv.run(reqs)
        summary["handles_prewarmed"] = warmed
        srv.close()
        torch.cuda.empty_cache()
        res[label] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in summary.items()}
        print(f"[bench] serving {label}: {res[label]}", file=sys.stderr, flush=True)
    return res


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="slater_128")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--serve-rate", type=float, default=40.0)
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
    print(f"[bench] workload {args.workload} grid {w.grid} precision {args.precision}", file=sys.stderr, flush=True)
    t_in = time.perf_counter()
    n, g = w.density(device="cuda", progress=lambda done, total: print(
        f"[bench] density: {done}/{total} blobs", file=sys.stderr, flush=True))
    torch.cuda.synchronize()
    print(f"[bench] density ready in {time.perf_counter() - t_in:.1f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    f = vdwxc.Functional(w.grid, w.cell, flavour="DF1", precision=args.precision, table=kt)
    v = torch.empty_like(n)
    e = torch.zeros(1, dtype=torch.float64, device=dev)

    for _ in range(args.warmup):
        f.potential_async(n, g, v, e)
    torch.cuda.synchronize()
    # timed region 1: throughput, no instrumentation
    t0 = time.perf_counter()
    for _ in range(args.steps):
        f.potential_async(n, g, v, e)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # timed region 2: the same steps with the library's per-kernel HIP events (recorded on the
    # stream the kernels run on), for the per-kernel durations behind the roofline figure
    f.enable_timing(True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(args.steps):
        f.potential_async(n, g, v, e)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    stages = f.read_timing()
    f.enable_timing(False)
    if args.copy_calibration_mb:
        # one streaming elementwise kernel (negation) reading and writing N bytes each
        nel = args.copy_calibration_mb * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    elapsed = t1 - t0
    ms_per_step = 1e3 * elapsed / args.steps
    ms_per_step_instrumented = 1e3 * (t3 - t2) / args.steps
    value = w.npoints * args.steps / elapsed
    E_gpu = float(e.item())
    print(f"[bench] {ms_per_step:.3f} ms/step, {value:.4e} pts/s, E = {E_gpu:.12e}", file=sys.stderr, flush=True)

    # roofline of the dominant kernel
    per_stage = {k: {"ms_avg": ms / cnt, "launches": cnt,
                     "GBps": stage_bytes(k, w.grid, args.precision) / (ms / cnt * 1e-3) / 1e9}
                 for k, (ms, cnt) in stages.items()}
    dom = max(stages, key=lambda k: stages[k][0])
    avg_s = stages[dom][0] / stages[dom][1] * 1e-3
    achieved = stage_bytes(dom, w.grid, args.precision) / avg_s / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": profiled_traffic(args.workload, args.precision, dom),
                "algorithmic_bytes_per_launch": stage_bytes(dom, w.grid, args.precision),
                "avg_launch_ms": round(avg_s * 1e3, 4),
                "timing": "HIP events around each kernel over a second timed region of the same steps "
                          f"({ms_per_step_instrumented:.4f} ms/step with the events)"}

    cpu = None
    accuracy = None
    if not args.no_cpu_baseline:
        bw = w if w.npoints <= 128 ** 3 else inputs.workload("slater_128")
        bname = args.workload if bw is w else "slater_128"
        if bw is w:
            nc, gc = n.cpu().numpy(), g.cpu().numpy()
        else:
            bn, bg = bw.density(device="cuda")
            nc, gc = bn.cpu().numpy(), bg.cpu().numpy()
        print(f"[bench] oracle CPU baseline on {bname}", file=sys.stderr, flush=True)
        cpu, E_ref, v_ref = cpu_baseline(bname, nc, gc, bw, kt)
        if bw is w:
            vv = v.cpu().numpy()
            accuracy = {"E_rel_err_vs_oracle": abs(E_gpu - E_ref) / abs(E_ref),
                        "v_maxnorm_rel_err_vs_oracle": float(np.max(np.abs(vv - v_ref)) / np.max(np.abs(v_ref))),
                        "v_density_weighted_l1": float(np.sum(nc * np.abs(vv - v_ref)) / np.sum(nc * np.abs(v_ref)))}

    serve = None
    if not args.no_serve:
        serve = serving_measurement(kt, args.serve_requests, args.serve_rate, args.precision)

    out = {
        "metric": "grid pts/s for E_c^nl+v_c^nl (Nalpha=20) at stated rel. error; p50/p99 serve latency",
        "value": value,
        "unit": "grid pts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "grid": list(w.grid), "cell_bohr": float(w.cell[0, 0]),
                   "n_alpha": M, "precision": "fp32_mixed (fp64 q0/splines/sums)" if args.precision == "fp32" else "fp64",
                   "entry": "vdwxc_calculate_potential_async, analytic gradient", "parallelism": "1 GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "accuracy": accuracy,
        "stages": {k: {kk: round(vv, 4) for kk, vv in d.items()} for k, d in per_stage.items()},
        "serving": serve,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
