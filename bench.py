#!/usr/bin/env python3
"""Throughput of the D3Q19 lattice-Boltzmann step on one MI355X.

A step is one full update of every site: for the binary fluid the
order-parameter kernel and the fused pull-stream + collision kernel.  The
default workload is the binary fluid on a 128^3 periodic lattice in FP64
(spinodal quench, rho = 1, u = 0, phi ~ U(-0.05, 0.05), seed 0), whose
100-step run is the benchmark configuration.

Prints one JSON line on stdout.  Progress goes to stderr.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu]
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "LB site-updates/s (MLUPS) + % HBM peak; FP64 vs FP32 at stated err; adjoint"
HBM_PEAK_GBS = 8000.0          # MI355X published HBM3E bandwidth

WORKLOADS = {
    # name: (model, storage, n, description)
    "binary128_f64": ("binary", "f64", 128, "D3Q19 binary fluid 128^3 periodic, FP64, spinodal quench"),
    "binary256_f64": ("binary", "f64", 256, "D3Q19 binary fluid 256^3 periodic, FP64, spinodal quench"),
    "binary256_f32": ("binary", "f32", 256, "D3Q19 binary fluid 256^3 periodic, FP32 deviation storage"),
    "binary384_f16": ("binary", "f16", 384, "D3Q19 binary fluid 384^3 periodic, FP16 deviation storage"),
    "binary384_f32": ("binary", "f32", 384, "D3Q19 binary fluid 384^3 periodic, FP32 deviation storage"),
    "single256_f64": ("single", "f64", 256, "D3Q19 single-fluid BGK 256^3 periodic, FP64, tau = 1"),
    "single256_f32": ("single", "f32", 256, "D3Q19 single-fluid BGK 256^3 periodic, FP32 deviation storage"),
    "adjoint64_f64": ("adjoint", "f64", 64, "D3Q19 single-fluid BGK 64^3 shear wave, FP64, 200-step rollout "
                                            "+ adjoint with checkpoints every 20 steps"),
    "adjoint128_f64": ("adjoint", "f64", 128, "D3Q19 single-fluid BGK 128^3 shear wave, FP64, 200-step rollout "
                                              "+ adjoint with checkpoints every 20 steps"),
}

ES = {"f64": 8, "f32": 4, "f16": 2}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(model, storage):
    """Bytes per site the method must move, per kernel: every distribution
    value read once and written once; phi written once by its kernel and
    read once by the collision (compute precision: 8 B for FP64, else 4);
    the adjoint step reads f^n and lambda^{n+1} and writes lambda^n."""
    es = ES[storage]
    ps = 8 if storage == "f64" else 4
    if model == "single":
        return {"collide": 2 * 19 * es, "phi": 0}
    if model == "adjoint":
        return {"collide": 2 * 19 * es, "phi": 0, "adjoint": 3 * 19 * es, "stream": 2 * 19 * es}
    return {"collide": 2 * 38 * es + ps, "phi": 19 * es + ps}


def traffic_from_profile(workload):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary, or None when there is none or the kernel
    sources changed since it was taken."""
    from paper_1405_6162_amd import profsummary
    info = profsummary.read_traffic(os.path.join(ROOT, "profiles", "pmc_%s.txt" % workload))
    if not info or info.get("source_digest") != profsummary.kernel_source_digest():
        return None
    return int(float(info["traffic_bytes_per_launch"]))


def cpu_baseline(model, n, seconds_target=12.0):
    """The FP64 oracle on the host, on the same workload's initial state, for
    as many whole steps as fit in about `seconds_target` (at least one)."""
    import numpy as np
    from oracle import lb_oracle as O
    from paper_1405_6162_amd import inputs
    prm = O.Params()
    if model == "binary":
        rho, u, phi = inputs.spinodal_quench(n, n, n, seed=0)
        f, g = O.init_binary(rho, u, phi, prm)
    else:
        rho, u = inputs.single_fluid_random(n, n, n, seed=0)
        f, g = O.init_single(rho, u), None
    steps, t_total = 0, 0.0
    while steps == 0 or (t_total < seconds_target and steps < 50):
        t0 = time.perf_counter()
        if model == "binary":
            f, g = O.step_binary(f, g, prm, 1)
        else:
            f = O.step_single(f, prm.tau_f, 1)
        t_total += time.perf_counter() - t0
        steps += 1
    assert np.isfinite(f).all()
    mlups = n ** 3 * steps / t_total / 1e6
    return {"value": round(mlups, 4), "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": "%d step(s) of the same %d^3 %s-fluid workload from its initial state, %.1f s wall; "
                      "numpy elementwise kernels, one thread" % (steps, n, model, t_total)}


def copy_probe(torch, nbytes=2 << 30, reps=10):
    """Plain device-to-device copy of `nbytes`: the achievable HBM rate, and
    the reference kernel for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    n = nbytes // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return {"bytes_per_launch": 2 * nbytes, "GB/s": round(2 * nbytes / (ms * 1e-3) / 1e9, 1)}


def bench_adjoint(args, n, desc, T=200, K=20):
    """Forward rollout + backward (recompute + adjoint kernel) per timed
    iteration; a step here is one forward step plus one adjoint step."""
    import torch
    from paper_1405_6162_amd import inputs, lb
    from paper_1405_6162_amd.adjoint import rollout, velocity_loss
    log("bench: %s" % desc)
    rho, u = inputs.shear_wave(n, n, n, amplitude=0.01, noise=1e-4, seed=0)
    lat = lb.Lattice(n, n, n, tau_f=0.8)
    lat.init_equilibrium(rho, u)
    f0 = lat.get_state()[0].clone()

    def once():
        f = f0.clone().requires_grad_(True)
        tau = torch.tensor(0.8, dtype=torch.float64, device="cuda", requires_grad=True)
        loss = velocity_loss(rollout(f, tau, lat, T, K))
        loss.backward()
        return f.grad, tau.grad

    for _ in range(max(args.warmup // 10, 1)):
        once()
    torch.cuda.synchronize()
    iters = max(args.steps // 100, 1)
    lb.lb_profile(lat.ctx, True)
    t0 = time.perf_counter()
    for _ in range(iters):
        g, gt = once()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lb.lb_profile(lat.ctx, False)
    adj_ms, adj_n = lb.lb_kernel_times(lat.ctx, lb.LB_K_ADJOINT)
    finite = bool(torch.isfinite(g).all()) and bool(torch.isfinite(gt))
    lat.close()
    if not finite:
        print("non-finite gradient", file=sys.stderr)
        sys.exit(1)
    nsite = n ** 3
    alg = algorithmic_bytes("adjoint", "f64")
    avg = adj_ms / max(adj_n, 1)
    achieved = alg["adjoint"] * nsite / (avg * 1e-3) / 1e9
    out = {
        "metric": METRIC, "value": round(nsite * T * iters / wall / 1e6, 2), "unit": "MLUPS",
        "n_gpus": 1, "steps": T * iters, "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / (T * iters), 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": desc, "nx": n, "ny": n, "nz": n, "tau": 0.8, "rollout_steps": T,
                   "checkpoint_every": K, "seed": 0},
        "roofline": {"bound": "hbm", "kernel": "k_adjoint (adjoint of the fused step)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_from_profile(args.workload),
                     "bytes_per_site": alg["adjoint"], "avg_launch_ms": round(avg, 5), "launches": adj_n},
    }
    if not args.no_copy:
        out["copy_probe"] = copy_probe(torch)
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="binary128_f64", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-copy", action="store_true", help="skip the copy-bandwidth probe")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0:
        print("--steps must be >= 1 and --warmup >= 0", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1405_6162_amd import inputs, lb

    model, storage, n, desc = WORKLOADS[args.workload]
    lb.load()
    torch.cuda.set_device(0)
    if model == "adjoint":
        return bench_adjoint(args, n, desc)
    mcode = lb.LB_BINARY if model == "binary" else lb.LB_SINGLE
    scode = {"f64": lb.LB_F64, "f32": lb.LB_F32, "f16": lb.LB_F16}[storage]
    log("bench: %s, %d warmup + %d timed steps" % (desc, args.warmup, args.steps))

    lat = lb.Lattice(n, n, n, model=mcode, storage=scode)
    if model == "binary":
        rho, u, phi = inputs.spinodal_quench(n, n, n, seed=0)
        lat.init_equilibrium(rho, u, phi)
    else:
        rho, u = inputs.single_fluid_random(n, n, n, seed=0)
        lat.init_equilibrium(rho, u)
    del rho, u
    lat.step(args.warmup)
    torch.cuda.synchronize()
    log("bench: warmup done")

    lb.lb_profile(lat.ctx, True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    lat.step(args.steps)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lb.lb_profile(lat.ctx, False)
    gpu_ms = e0.elapsed_time(e1)
    col_ms, col_n = lb.lb_kernel_times(lat.ctx, lb.LB_K_COLLIDE)
    phi_ms, phi_n = lb.lb_kernel_times(lat.ctx, lb.LB_K_PHI)
    log("bench: timed region %.3f ms (events), %.3f s wall" % (gpu_ms, wall))

    nsite = n ** 3
    sums = lat.conserved_sums().cpu()
    finite = bool(torch.isfinite(sums).all())
    lat.close()
    if not finite:
        print("non-finite state after the timed steps", file=sys.stderr)
        sys.exit(1)

    seconds = wall
    mlups = nsite * args.steps / seconds / 1e6
    alg = algorithmic_bytes(model, storage)
    col_avg_ms = col_ms / max(col_n, 1)
    achieved = alg["collide"] * nsite / (col_avg_ms * 1e-3) / 1e9
    step_bytes = alg["collide"] + alg["phi"]

    out = {
        "metric": METRIC,
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(seconds * 1e3 / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": storage,
        "data": "synthetic",
        "config": {"workload": desc, "nx": n, "ny": n, "nz": n, "fluid": model,
                   "storage": storage, "seed": 0},
        "roofline": {
            "bound": "hbm",
            "kernel": "k_collide (fused pull-stream + collision)",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic_from_profile(args.workload),
            "bytes_per_site": alg["collide"],
            "avg_launch_ms": round(col_avg_ms, 5),
            "launches": col_n,
        },
        "step_roofline": {
            "bytes_per_site": step_bytes,
            "GB/s": round(step_bytes * nsite * args.steps / seconds / 1e9, 1),
            "frac": round(step_bytes * nsite * args.steps / seconds / 1e9 / HBM_PEAK_GBS, 4),
            "phi_kernel_avg_ms": round(phi_ms / phi_n, 5) if phi_n else None,
        },
    }
    if not args.no_copy:
        out["copy_probe"] = copy_probe(torch)
        log("bench: copy probe %s GB/s" % out["copy_probe"]["GB/s"])
    if not args.no_cpu:
        log("bench: timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(model, n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
