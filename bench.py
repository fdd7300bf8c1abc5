#!/usr/bin/env python3
"""Throughput of the fused pseudopotential LB step on one MI355X.

Headline workload: D2Q9 MRT, 2048 x 2048, FP32, periodic porous medium of
400 cylinders (radii U[8, 32], dart throwing), a prescribed contact angle
per cylinder U[30, 150] deg through the improved virtual-density scheme,
50/50 liquid/gas blobs, Carnahan-Starling at 0.75 Tc.  A step is one launch
of the fused kernel over the whole lattice (density, psi, wall virtual
density, force, MRT collision, streaming with halfway bounce-back).

Prints one JSON line: MLUPS over all nodes (whole job), the HBM roofline of
the step kernel (algorithmic bytes 2*Q*sizeof(real) per fluid node per
step, divided by the HIP-event kernel time), the CPU oracle on a bounded
sample of the same workload, and secondary lines (D3Q19 256^3).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "MLUPS and % HBM roofline (FP32 D2Q9/D3Q19); batched vs single; adjoint/forward time"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("lbm_device.hpp", "lbm_kernels.hpp", "tile2d.hpp", "step2d.hip", "step_march.hip"):
        with open(os.path.join(ROOT, "paper_1908_04443_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """Per-launch HBM bytes from the committed rocprofv3 counter summary,
    if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    if not os.path.exists(path):
        return None
    want = kernel_source_hash()
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        kv = dict(tok.split("=", 1) for tok in line.split() if "=" in tok)
        if kv.get("kernel") == kernel and kv.get("workload") == workload and kv.get("src") == want:
            return float(kv["bytes_per_launch"])
    return None


def setup_solver(L, W, params, data, n_wall_max):
    import torch
    s = L.Solver(params, n_wall_max)
    s.set_geometry(data["solid"])
    walls = s.wall_nodes()
    phi = torch.as_tensor(data["phi"].ravel()[walls], dtype=s.dtype, device=s.device)
    drho = torch.as_tensor(data["drho"].ravel()[walls], dtype=s.dtype, device=s.device)
    s.set_wetting(L.LBM_WET_IVD, 0.0, phi if len(walls) else None, drho if len(walls) else None)
    s.set_fields(data["rho"].ravel())
    return s, len(walls)


def time_steps(s, warmup, steps, runs=5):
    """Warm up, then time exactly `steps` steps: one call with HIP events on
    the solver's stream around its launches, bracketed by host
    synchronisations for the wall clock.  After the timed region, `runs`
    more event-timed runs of max(200, min(steps, 2000)) steps give the
    median time per step.  Returns (wall seconds of the timed region, event
    ms per step over it, median event ms per step of the runs, the runs)."""
    import numpy as np
    import torch
    s.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms = s.step_timed(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n = max(200, min(steps, 2000))
    per_run = [s.step_timed(n) / n for _ in range(runs)]
    return wall, ms / steps, float(np.median(per_run)), [round(x, 5) for x in per_run]


def run_c1(L, W, steps, warmup):
    import numpy as np
    p = L.make_params(lattice=9, precision=4, nx=2048, ny=2048, T_ratio=0.75,
                      sigma=W.SIGMA[("cs", 0.75, 9)], tau=1.0)
    data = W.c1_porous(p.rho_g, p.rho_l)
    solid = data["solid"]
    s, nw = setup_solver(L, W, p, data, int(solid.sum()))
    rc, d0 = s.diagnostics()
    variant = s.variant
    wall, ms_step, ms_med, runs = time_steps(s, warmup, steps)
    # diagnostics (field-mode pass over f, per-tile partials, fixed-order
    # final reduction, copy to the host and a stream synchronisation)
    s.diagnostics()
    t0 = time.perf_counter()
    for _ in range(20):
        rc, d1 = s.diagnostics()
    diag_ms = (time.perf_counter() - t0) * 1e3 / 20
    if rc != 0:
        raise RuntimeError("C1 run left the psi domain")
    N = 2048 * 2048
    nf = int((solid == 0).sum())
    s.close()
    return dict(N=N, n_fluid=nf, n_wall=nw, wall=wall, ms_step=ms_step, ms_median=ms_med, runs=runs,
                variant=variant, diag_ms=diag_ms,
                mass_drift=abs(d1["mass"] - d0["mass"]) / d0["mass"], max_u=d1["max_u"],
                rho=(d1["rho_min"], d1["rho_max"]), data=data, params=p)


def run_c2(L, W, steps, warmup):
    p = L.make_params(lattice=19, precision=4, nx=256, ny=256, nz=256, T_ratio=0.8,
                      sigma=W.SIGMA[("cs", 0.8, 19)], tau=1.0)
    data = W.c2_sphere(p.rho_g, p.rho_l)
    solid = data["solid"]
    s, nw = setup_solver(L, W, p, data, int(solid.sum()))
    wall, ms_step, ms_med, runs = time_steps(s, warmup, steps)
    rc, d1 = s.diagnostics()
    if rc != 0:
        raise RuntimeError("C2 run left the psi domain")
    N = 256 ** 3
    nf = int((solid == 0).sum())
    s.close()
    return dict(N=N, n_fluid=nf, n_wall=nw, wall=wall, ms_step=ms_step, ms_median=ms_med, runs=runs,
                params=p)


def run_c3(L, W, steps, warmup, graph_steps=50):
    """96 D2Q9 FP32 cases of uneven size: one multi-case context (tile shape
    picked by the autotuner) replaying a graph of `graph_steps` steps,
    against one context per case stepped in turn on the same stream, both
    with its default tile shape and plain launches and tuned (autotuned tile
    shape, graph replay)."""
    import numpy as np
    import torch
    p = L.make_params(lattice=9, precision=4, nx=1, ny=1, T_ratio=0.75,
                      sigma=W.SIGMA[("cs", 0.75, 9)], tau=1.0)
    cases = W.c3_cases(p.rho_g, p.rho_l)
    sizes = [(c["n"], c["n"]) for c in cases]
    nwm = [int(c["solid"].sum()) for c in cases]
    total = sum(a * b for a, b in sizes)

    b = L.BatchSolver(p, sizes, nwm)
    b.set_scheme(L.LBM_WET_IVD)
    for i, c in enumerate(cases):
        b.set_geometry(i, c["solid"])
        w = b.wall_nodes(i)
        b.set_wetting(i, torch.as_tensor(c["phi"].ravel()[w], dtype=b.dtype, device="cuda"),
                      torch.as_tensor(c["drho"].ravel()[w], dtype=b.dtype, device="cuda"))
        b.set_fields(i, c["rho"].ravel())
    tuned = b.autotune(steps=20)  # tile shape of the multi-case launch
    b.set_graph_steps(graph_steps)
    b.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    rc, d = b.diagnostics()
    if rc != 0:
        raise RuntimeError("batched run left the psi domain")
    # the multi-case kernel alone: HIP events around `steps` graph-replayed
    # steps, median of 5 runs
    kern_ms = float(np.median([b.step_timed(steps) / steps for _ in range(5)]))
    nf_total = sum(int((c["solid"] == 0).sum()) for c in cases)
    b.close()

    def singles(tune, graphs):
        sols = []
        for c in cases:
            q = L.make_params(lattice=9, precision=4, nx=c["n"], ny=c["n"], T=p.eos_T,
                              sigma=p.sigma, tau=1.0, rho_g=p.rho_g, rho_l=p.rho_l)
            s1, _ = setup_solver(L, W, q, c, int(c["solid"].sum()))
            if tune:
                s1.autotune(steps=10)
            if graphs:
                s1.set_graph_steps(graph_steps)
            sols.append(s1)
        for s1 in sols:
            s1.step(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s1 in sols:
            s1.step(steps)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        for s1 in sols:
            s1.close()
        return t

    # one context per case, launched in turn on one stream: as configured by
    # default (the tile preferred for large lattices, plain launches), and
    # tuned (each case's fastest tile shape, graph replay)
    t_single = singles(False, False)
    t_tuned = singles(True, True)
    b_alg = 2 * 9 * 4 * nf_total
    return dict(total_nodes=total, cases=len(cases), steps=steps,
                batched_mlups=total * steps / t_batch / 1e6,
                single_mlups=total * steps / t_single / 1e6,
                single_tuned_mlups=total * steps / t_tuned / 1e6,
                ratio=t_single / t_batch, ratio_vs_tuned_single=t_tuned / t_batch,
                graph_steps=graph_steps, batch_tile_variant=tuned,
                batch_kernel=dict(kernel="k_step_d2q9_batch", kernel_ms=round(kern_ms, 5),
                                  bytes_per_launch_alg=b_alg,
                                  achieved_GBs=round(b_alg / (kern_ms * 1e-3) / 1e9, 1),
                                  frac=round(b_alg / (kern_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)))


def run_c4(L, W, T=1000, K=50):
    """Adjoint workload: D2Q9 FP32 256^2, cylinder R = 40, droplet r = 32 on
    top, per-wall parameters at phi = 1, drho = 0.  Times the forward step,
    the checkpointed forward, and the full adjoint (recompute included); the
    adjoint step time is the adjoint total minus the recomputed forward
    steps, per step."""
    import numpy as np
    import torch
    p = L.make_params(lattice=9, precision=4, nx=256, ny=256, T_ratio=0.75,
                      sigma=W.SIGMA[("cs", 0.75, 9)], tau=1.0)
    d = W.c4_adjoint(p.rho_g, p.rho_l)
    s, nw = setup_solver(L, W, p, d, int(d["solid"].sum()))
    s.step(50)
    # medians of 5 runs: the 256^2 step is short enough for launch jitter to show
    fwd_ms_default = float(np.median([s.step_timed(T) / T for _ in range(5)]))
    # the forward at its fastest tile shape on this lattice (the adjoint's
    # own tiles fill the chip; the default forward tile leaves most CUs idle)
    fwd_variant = s.autotune(steps=50)
    fwd_ms = float(np.median([s.step_timed(T) / T for _ in range(5)]))
    s.set_fields(d["rho"].ravel())
    ckpt = s.ckpt_buffer(T, K)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step_ckpt(T, K, ckpt)
    torch.cuda.synchronize()
    ckpt_ms = (time.perf_counter() - t0) * 1e3
    rho_T = s.get_fields(rho=True, u=False)["rho"]
    fluid = torch.as_tensor(d["solid"].ravel() == 0, device="cuda")
    seed = torch.where(fluid, 2.0 * (rho_T - 0.5 * (p.rho_g + p.rho_l)), torch.zeros_like(rho_T))
    s.adjoint(seed, T, K, ckpt)  # warm
    runs = []
    for _ in range(5):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gp, gd = s.adjoint(seed, T, K, ckpt)
        torch.cuda.synchronize()
        runs.append((time.perf_counter() - t0) * 1e3)
    adj_ms = float(np.median(runs))
    nseg = (T + K - 1) // K
    recompute = T - nseg
    adj_step_ms = (adj_ms - recompute * fwd_ms) / T  # the recompute runs the tuned forward
    s.close()
    return dict(T=T, K=K, wall_nodes=nw, forward_step_ms=round(fwd_ms, 5),
                forward_tile_variant=fwd_variant,
                forward_step_ms_default_tile=round(fwd_ms_default, 5),
                adjoint_step_ms=round(adj_step_ms, 5),
                adjoint_step_over_forward=round(adj_step_ms / fwd_ms, 3),
                adjoint_step_over_forward_default_tile=round(adj_step_ms / fwd_ms_default, 3),
                backward_total_ms=round(adj_ms, 3), checkpointed_forward_ms=round(ckpt_ms, 3),
                backward_over_forward=round(adj_ms / (fwd_ms * T), 3),
                grad_finite=bool(torch.isfinite(gp).all() and torch.isfinite(gd).all()))


def cpu_baseline(data, lbm_params, steps):
    """The CPU oracle (FP64) on the same 2048^2 lattice and initial state,
    `steps` steps."""
    import numpy as np
    import oracle as O
    op = O.make_params(lattice=9, nx=2048, ny=2048, tau=1.0, T=lbm_params.eos_T,
                       sigma=lbm_params.sigma, rho_g=lbm_params.rho_g, rho_l=lbm_params.rho_l)
    solid = data["solid"]
    walls = O.wall_nodes(op, solid)
    phi = data["phi"].ravel()[walls]
    drho = data["drho"].ravel()[walls]
    f0 = O.init_eq(op, solid, data["rho"])
    t0 = time.perf_counter()
    O.run(op, solid, f0, steps, phi, drho)
    dt = time.perf_counter() - t0
    N = 2048 * 2048
    threads = O.get_threads()
    # the same oracle on one thread, a shorter sample
    s1 = max(1, steps // 20)
    O.set_threads(1)
    try:
        t0 = time.perf_counter()
        O.run(op, solid, f0, s1, phi, drho)
        dt1 = time.perf_counter() - t0
    finally:
        O.set_threads(threads)
    return dict(value=N * steps / dt / 1e6, unit="MLUPS", cores=threads, kind="oracle",
                cpu_model=cpu_model(),
                sample=f"D2Q9 2048x2048 porous workload, same initial state, {steps} FP64 "
                       f"oracle steps ({dt:.1f} s)",
                value_1thread=N * s1 / dt1 / 1e6,
                sample_1thread=f"{s1} steps on one thread ({dt1:.1f} s)")


def cpu_model():
    """The host CPU's model name (Linux /proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_oracle_c2(W, lbm_params, steps=4):
    """The CPU oracle (FP64) on the 256^3 D3Q19 sphere workload, `steps` steps
    from its initial state (a bounded sample: a step is a few seconds)."""
    import oracle as O
    op = O.make_params(lattice=19, nx=256, ny=256, nz=256, tau=1.0, T=lbm_params.eos_T,
                       sigma=lbm_params.sigma, rho_g=lbm_params.rho_g, rho_l=lbm_params.rho_l)
    data = W.c2_sphere(op.rho_g, op.rho_l)
    solid = data["solid"]
    walls = O.wall_nodes(op, solid)
    f0 = O.init_eq(op, solid, data["rho"])
    t0 = time.perf_counter()
    O.run(op, solid, f0, steps, data["phi"].ravel()[walls], data["drho"].ravel()[walls])
    dt = time.perf_counter() - t0
    return dict(value=round(256 ** 3 * steps / dt / 1e6, 3), unit="MLUPS",
                cores=O.get_threads(), kind="oracle",
                sample=f"D3Q19 256^3 sphere workload, {steps} FP64 oracle step(s) ({dt:.1f} s)")


def copy_calibration(nbytes, reps):
    """A plain device-to-device copy of known size, the reference point that
    converts the HBM counters of the profiler into bytes."""
    import torch
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "reps": reps}),
          flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--cpu-steps", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--c2-steps", type=int, default=500)
    ap.add_argument("--c3-steps", type=int, default=500)
    ap.add_argument("--secondary", default="c2,c3,c4",
                    help="secondary workloads to run: any of c2 (D3Q19 256^3), c3 (96 cases), "
                         "c4 (adjoint)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device to device 5 times (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the step is measured on one device "
              "(multi-GPU domain decomposition is not part of this library)", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        copy_calibration(args.copy_calibration << 20, 5)
        return
    from paper_1908_04443_amd import lbm as L
    from paper_1908_04443_amd import workloads as W
    if not os.path.exists(L.LIB_PATH):
        from paper_1908_04443_amd import build
        build.build()
    L.lib()
    torch.cuda.init()

    log(f"C1: D2Q9 2048^2 FP32 porous workload, warmup {args.warmup}, steps {args.steps}")
    c1 = run_c1(L, W, args.steps, args.warmup)
    N, nf = c1["N"], c1["n_fluid"]
    ms_step = 1e3 * c1["wall"] / args.steps
    mlups = N * args.steps / c1["wall"] / 1e6
    kern_s = c1["ms_step"] / 1e3  # HIP-event time per step over the timed region
    b_alg = 2 * 9 * 4 * nf  # one read + one write of every fluid population
    achieved = b_alg / kern_s / 1e9
    traffic = measured_traffic("k_step_d2q9", "c1")
    log(f"C1: {mlups:.1f} MLUPS, {achieved:.0f} GB/s algorithmic, "
        f"mass drift {c1['mass_drift']:.2e}, max|u| {c1['max_u']:.3e}")

    out = {
        "metric": METRIC,
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "D2Q9 MRT pseudopotential 2048x2048 FP32, 400-cylinder "
                               "porous medium, improved virtual density, CS 0.75 Tc",
                   "nx": 2048, "ny": 2048, "lattice": "D2Q9", "fluid_nodes": nf,
                   "wall_nodes": c1["n_wall"], "tile_variant": c1["variant"]},
        "mflups": round(nf * args.steps / c1["wall"] / 1e6, 2),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "kernel": "k_step_d2q9", "bytes_per_launch_alg": b_alg,
                     "kernel_ms": round(kern_s * 1e3, 5),
                     "kernel_ms_median5": round(c1["ms_median"], 5),
                     "kernel_ms_runs": c1["runs"]},
        "check": {"mass_rel_drift": c1["mass_drift"], "max_u": c1["max_u"],
                  "rho_min_max": c1["rho"]},
        # one read of every fluid population per diagnostics call
        "diagnostics": {"ms_per_call": round(c1["diag_ms"], 4),
                        "achieved_read_GBs": round(9 * 4 * nf / c1["diag_ms"] / 1e6, 1)},
        "env": {"device": torch.cuda.get_device_name(0),
                "arch": getattr(torch.cuda.get_device_properties(0), "gcnArchName", ""),
                "cus": torch.cuda.get_device_properties(0).multi_processor_count,
                "hip": torch.version.hip, "torch": torch.__version__},
    }

    want = set() if args.no_secondary else set(x for x in args.secondary.split(",") if x)
    out["secondary"] = {}
    if "c2" in want:
        log(f"C2: D3Q19 256^3 FP32 sphere, {args.c2_steps} steps")
        c2 = run_c2(L, W, args.c2_steps, 20)
        c2_params = c2.pop("params")
        k2 = c2["ms_step"] / 1e3
        b2 = 2 * 19 * 4 * c2["n_fluid"]
        out["secondary"]["d3q19_256cubed_fp32"] = {
            "mlups": round(c2["N"] * args.c2_steps / c2["wall"] / 1e6, 2),
            "achieved_GBs": round(b2 / k2 / 1e9, 1),
            "frac": round(b2 / k2 / 1e9 / HBM_PEAK_GBS, 4),
            "kernel_ms": round(k2 * 1e3, 5), "kernel_ms_median5": round(c2["ms_median"], 5),
            "kernel_ms_runs": c2["runs"],
            "steps": args.c2_steps,
            "traffic": measured_traffic("d3q19_step", "c2")}
        log(f"C2: {out['secondary']['d3q19_256cubed_fp32']}")
    if "c3" in want:
        log(f"C3: 96 uneven D2Q9 FP32 cases, {args.c3_steps} steps, batched vs one per launch")
        c3 = run_c3(L, W, args.c3_steps, 100)  # warm-up of two graph replays (captured there)
        out["secondary"]["batched_96_cases_fp32"] = {k: (round(v, 3) if isinstance(v, float) else v)
                                                     for k, v in c3.items()}
        log(f"C3: {out['secondary']['batched_96_cases_fp32']}")
    if "c4" in want:
        log("C4: adjoint of the 256^2 D2Q9 FP32 workload, T = 1000, K = 50")
        out["secondary"]["adjoint_256_fp32"] = run_c4(L, W)
        log(f"C4: {out['secondary']['adjoint_256_fp32']}")

    if not args.no_cpu_baseline:
        log(f"CPU oracle: {args.cpu_steps} steps of the 2048^2 workload")
        out["cpu_baseline"] = cpu_baseline(c1["data"], c1["params"], args.cpu_steps)
        if "c2" in want:
            log("CPU oracle: 4 steps of the 256^3 D3Q19 workload")
            out["secondary"]["d3q19_256cubed_fp32"]["cpu_oracle"] = cpu_oracle_c2(W, c2_params)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
