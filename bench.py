#!/usr/bin/env python3
"""Throughput of the D3Q19 lattice-Boltzmann step on one MI355X.

A step is one full update of every site: one launch of the fused
pull-stream + collision kernel (for the binary fluid the single-pass kernel
that also computes phi and its stencils).  The default workload is the
binary fluid on a 256^3 periodic lattice in FP64 (spinodal quench, rho = 1,
u = 0, phi ~ U(-0.05, 0.05), seed 0): the largest FP64 configuration on one
GPU, the one the FP64-against-FP32 comparison is quoted on.

The timed region runs the steps as plain launches (no per-launch events);
`value` and `ms_per_step` come from it.  A second, separate pass of the same
number of steps brackets every launch with HIP events on the library's
stream to give the kernel's own average duration, from which `roofline` is
computed.

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
    "binary128_trt_f64": ("binary", "f64", 128, "D3Q19 binary fluid 128^3 periodic, FP64, spinodal quench, "
                          "f by TRT (tau+ = 1, tau- = 1.25)"),
    "binary128_mrt_f64": ("binary", "f64", 128, "D3Q19 binary fluid 128^3 periodic, FP64, spinodal quench, "
                          "f by MRT (tau_shear = 1, tau_flux = 1.25, tau_bulk = 1.4, tau_ghost_even = 0.9, "
                          "tau_ghost_odd = 1.2)"),
    "binary256_f64": ("binary", "f64", 256, "D3Q19 binary fluid 256^3 periodic, FP64, spinodal quench"),
    "binary256_f32": ("binary", "f32", 256, "D3Q19 binary fluid 256^3 periodic, FP32 deviation storage"),
    "binary384_f16": ("binary", "f16", 384, "D3Q19 binary fluid 384^3 periodic, FP16 deviation storage"),
    "binary384_f32": ("binary", "f32", 384, "D3Q19 binary fluid 384^3 periodic, FP32 deviation storage"),
    "single256_f64": ("single", "f64", 256, "D3Q19 single-fluid BGK 256^3 periodic, FP64, tau = 1"),
    "single256_f32": ("single", "f32", 256, "D3Q19 single-fluid BGK 256^3 periodic, FP32 deviation storage"),
    "single256_trt_f64": ("single", "f64", 256, "D3Q19 single-fluid TRT 256^3 periodic, FP64, tau+ = 1, "
                          "tau- = 1.25"),
    "single256_mrt_f64": ("single", "f64", 256, "D3Q19 single-fluid MRT 256^3 periodic, FP64, tau_shear = 1, "
                          "tau_flux = 1.25, tau_bulk = 1.4, tau_ghost_even = 0.9, tau_ghost_odd = 1.2"),
    "adjoint64_f64": ("adjoint", "f64", 64, "D3Q19 single-fluid BGK 64^3 shear wave, FP64, 200-step rollout "
                                            "+ adjoint with checkpoints every 20 steps"),
    "adjoint128_f64": ("adjoint", "f64", 128, "D3Q19 single-fluid BGK 128^3 shear wave, FP64, 200-step rollout "
                                              "+ adjoint with checkpoints every 20 steps"),
    "adjoint64_mrt_f64": ("adjoint", "f64", 64, "D3Q19 single-fluid MRT 64^3 shear wave, FP64, 200-step rollout "
                          "+ adjoint with checkpoints every 20 steps, gradients w.r.t. f0 and the five relaxation "
                          "times (0.8, 1.1, 1.3, 0.9, 1.2)"),
    "adjoint_binary64_f64": ("adjoint_binary", "f64", 64, "D3Q19 binary fluid 64^3 spinodal quench, FP64, "
                             "200-step rollout + adjoint (gradients w.r.t. phi0, rho0, u0, kappa, M, tau_f) "
                             "with checkpoints every 20 steps"),
    "adjoint_binary128_f64": ("adjoint_binary", "f64", 128, "D3Q19 binary fluid 128^3 spinodal quench, FP64, "
                              "200-step rollout + adjoint (gradients w.r.t. phi0, rho0, u0, kappa, M, tau_f) "
                              "with checkpoints every 20 steps"),
    "adjoint_binary128_trt_f64": ("adjoint_binary", "f64", 128, "D3Q19 binary fluid 128^3 spinodal quench, FP64, "
                                  "f by TRT (tau+ = 1, tau- = 1.25), 200-step rollout + adjoint (gradients "
                                  "w.r.t. phi0, rho0, u0, kappa, M, tau+, tau-) with checkpoints every 20 steps"),
    "adjoint_binary128_mrt_f64": ("adjoint_binary", "f64", 128, "D3Q19 binary fluid 128^3 spinodal quench, FP64, "
                                  "f by MRT (tau_shear = 1, tau_flux = 1.25, tau_bulk = 1.4, tau_ghost_even = 0.9, "
                                  "tau_ghost_odd = 1.2), 200-step rollout + adjoint (gradients w.r.t. phi0, rho0, "
                                  "u0, kappa, M and the five times) with checkpoints every 20 steps"),
    "precision256_f32": ("precision", "f32", 256, "D3Q19 binary fluid 256^3 spinodal quench, 500 steps: FP32 "
                                                  "deviation storage against FP64"),
    "precision384_f16": ("precision", "f16", 384, "D3Q19 binary fluid 384^3 spinodal quench, 1000 steps: FP16 "
                                                  "deviation storage against FP32, and a 96^3 run against FP64"),
    "precision256_single_f32": ("precision_single", "f32", 256, "D3Q19 single-fluid BGK 256^3, rho = 1 + "
                                "0.01 N(0,1), u ~ U(-0.01, 0.01), 500 steps: FP32 deviation storage against FP64"),
}

ES = {"f64": 8, "f32": 4, "f16": 2}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(model, storage):
    """Bytes per site the method must move in one step: every distribution
    value read once and written once (the binary step is a single kernel
    that computes phi and its stencils on chip, so phi adds nothing); the
    adjoint step reads f^n and lambda^{n+1} and writes lambda^n."""
    es = ES[storage]
    if model == "single":
        return {"collide": 2 * 19 * es}
    if model == "adjoint":
        return {"collide": 2 * 19 * es, "adjoint": 3 * 19 * es}
    if model == "adjoint_binary":
        # reads f^n, g^n, lambda_f^{n+1}, lambda_g^{n+1}; writes lambda_f^n, lambda_g^n
        return {"collide": 2 * 38 * es, "adjoint": 6 * 19 * es}
    return {"collide": 2 * 38 * es}


def traffic_from_profile(workload):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary, or None when there is none or the kernel
    sources changed since it was taken."""
    from paper_1405_6162_amd import profsummary
    info = profsummary.read_traffic(os.path.join(ROOT, "profiles", "pmc_%s.txt" % workload))
    if not info or info.get("source_digest") != profsummary.kernel_source_digest():
        return None
    return int(float(info["traffic_bytes_per_launch"]))


def cpu_baseline(model, n, slab_div=8, steps=8):
    """The FP64 oracle timed on the host: the C reference (oracle/lb_oracle.c,
    plain loops, OpenMP over sites; its results do not depend on the thread
    count) from the workload's initial state.  All cores: `steps` steps of
    the whole n^3 lattice.  One thread: `steps` steps of an n x n x
    n/slab_div slab of the same workload (periodic, the same per-site work),
    so the sample stays bounded (about 5-10 s of wall time each at 256^3).
    MLUPS = site updates / wall time of the steps (initialisation not
    timed)."""
    import numpy as np
    from oracle import c_backend as C
    from paper_1405_6162_amd import inputs

    def one_step(nz, threads):
        used = C.set_threads(threads)
        if model == "binary":
            rho, u, phi = inputs.spinodal_quench(n, n, nz, seed=0)
            lat = C.CLattice(n, n, nz, model=1)
            lat.init_equilibrium(rho, u, phi)
        else:
            rho, u = inputs.single_fluid_random(n, n, nz, seed=0)
            lat = C.CLattice(n, n, nz, model=0)
            lat.init_equilibrium(rho, u)
        del rho, u
        t0 = time.perf_counter()
        lat.step(steps)
        dt = time.perf_counter() - t0
        ok = bool(np.isfinite(lat.sums()).all())
        lat.close()
        assert ok
        return n * n * nz * steps / dt / 1e6, dt, used

    v_all, t_all, cores = one_step(n, 0)
    nz1 = max(n // slab_div, 1)
    v_one, t_one, _ = one_step(nz1, 1)
    return {"value": round(v_all, 4), "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "value_1_thread": round(v_one, 4),
            "sample": "C reference (plain FP64 loops, OpenMP over sites): %d steps of the %d^3 %s-fluid workload "
                      "on %d threads, %.1f s wall; %d steps of a %dx%dx%d slab of it on 1 thread, %.1f s wall"
                      % (steps, n, model, cores, t_all, steps, n, n, nz1, t_one)}


def fp32_vs_fp64(torch, lb, inputs, n, steps, warmup, fp64_mlups):
    """The metric's comparison on its own configuration: the binary lattice
    in FP32 storage, timed like the FP64 line (plain launches between two
    synchronizations), and its moments after 1 and 10 steps against an FP64
    run from the same seeded state.  The FP64 path is itself held to the
    FP64 oracle within 1e-12 by the GPU tests, so its moments stand in for
    the oracle's here; the error is max |q - q64| / max |q64| per moment."""
    rho, u, phi = inputs.spinodal_quench(n, n, n, seed=0)

    def lattice(storage):
        lat = lb.Lattice(n, n, n, model=lb.LB_BINARY, storage=storage, rho0=1.0, phi0=float(phi.mean()))
        lat.init_equilibrium(rho, u, phi)
        return lat

    lat = lattice(lb.LB_F32)
    lat.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.step(steps)
    torch.cuda.synchronize()
    mlups = n ** 3 * steps / (time.perf_counter() - t0) / 1e6
    lat.close()
    a, b = lattice(lb.LB_F64), lattice(lb.LB_F32)
    errors, done = {}, 0
    for k in (1, 10):
        a.step(k - done)
        b.step(k - done)
        done = k
        errors[str(k)] = {name: float((y - x).abs().max() / x.abs().max())
                          for name, x, y in zip(("rho", "u", "phi"), a.moments(), b.moments())}
    a.close()
    b.close()
    return {"storage": "f32", "MLUPS": round(mlups, 2), "speedup": round(mlups / fp64_mlups, 3),
            "errors_vs_fp64_after_steps": errors, "stated_err": {"u": 1e-6, "after_steps": 10},
            "met": errors["10"]["u"] <= 1e-6}


def copy_probe(torch, nbytes=2 << 30, reps=10):
    """The library's streaming copy (lb_stream_copy: 16-byte loads, nontemporal
    16-byte stores) of `nbytes` device bytes, timed with events on the
    current stream: the HBM rate of a plain read-once / write-once copy, and
    the reference kernel for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    from paper_1405_6162_amd import lb
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    lb.lb_stream_copy(b, a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        lb.lb_stream_copy(b, a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    ok = bool(torch.equal(a, b))
    del a, b
    if not ok:
        raise RuntimeError("lb_stream_copy produced a wrong copy")
    return {"kernel": "k_stream_copy (lb_stream_copy)", "bytes_per_launch": 2 * nbytes,
            "GB/s": round(2 * nbytes / (ms * 1e-3) / 1e9, 1), "frac_of_peak": round(
                2 * nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def pull_copy_ceiling(lb, lat, bytes_per_launch, launches=10):
    """What the step's memory access pattern reaches with no arithmetic:
    lb_propagate on the same lattice (the same 19 pulls and 19 nontemporal
    stores per distribution and site as the step, the same tiles, strides and
    launch shape; both distributions of the binary fluid in one launch),
    timed with the same events.  It changes the lattice state."""
    lb.lb_set_stream(lat.ctx, lb._stream())
    lb.lb_propagate(lat.ctx)          # after lb_step the state is pending: from here every call launches
    lb.lb_profile(lat.ctx, True)
    for _ in range(launches):
        lb.lb_propagate(lat.ctx)
    lb.lb_profile(lat.ctx, False)
    ms, n = lb.lb_kernel_times(lat.ctx, lb.LB_K_STREAM)
    avg = ms / max(n, 1)
    gbs = bytes_per_launch / (avg * 1e-3) / 1e9 if n else 0.0
    kernel = "k_stream2 (f and g)" if lat.model == lb.LB_BINARY else "k_stream"
    return {"kernel": kernel + ": the step's pulls and stores without its arithmetic (lb_propagate)",
            "GB/s": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4), "avg_launch_ms": round(avg, 5),
            "launches": n}


def bench_adjoint(args, n, desc, T=200, K=20):
    """Forward rollout + backward (recompute + adjoint kernel) per timed
    iteration; a step here is one forward step plus one adjoint step."""
    import torch
    from paper_1405_6162_amd import inputs, lb
    from paper_1405_6162_amd.adjoint import rollout, velocity_loss
    log("bench: %s" % desc)
    rho, u = inputs.shear_wave(n, n, n, amplitude=0.01, noise=1e-4, seed=0)
    mrt = "_mrt_" in args.workload
    taus = (0.8, 1.1, 1.3, 0.9, 1.2) if mrt else 0.8
    if mrt:
        lat = lb.Lattice(n, n, n, collision=lb.LB_MRT, tau_f=taus[0], tau_minus=taus[1], tau_bulk=taus[2],
                         tau_ghost_even=taus[3], tau_ghost_odd=taus[4])
    else:
        lat = lb.Lattice(n, n, n, tau_f=taus)
    lat.init_equilibrium(rho, u)
    f0 = lat.get_state()[0].clone()

    def once():
        f = f0.clone().requires_grad_(True)
        tau = torch.tensor(taus, dtype=torch.float64, device="cuda", requires_grad=True)
        loss = velocity_loss(rollout(f, tau, lat, T, K))
        loss.backward()
        return f.grad, tau.grad

    n_warm = max(args.warmup // 10, 1)          # whole rollouts: forward + backward
    for _ in range(n_warm):
        once()
    torch.cuda.synchronize()
    iters = max(args.steps // 100, 1)
    lb.lb_profile_mask(lat.ctx, [lb.LB_K_ADJOINT])      # events on the adjoint kernels only
    t0 = time.perf_counter()
    for _ in range(iters):
        g, gt = once()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lb.lb_profile(lat.ctx, False)
    adj_ms, adj_n = lb.lb_kernel_times(lat.ctx, lb.LB_K_ADJOINT)
    finite = bool(torch.isfinite(g).all()) and bool(torch.isfinite(gt).all())
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
        "n_gpus": 1, "steps": T * iters, "warmup": T * n_warm,
        "ms_per_step": round(wall * 1e3 / (T * iters), 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": desc, "nx": n, "ny": n, "nz": n, "tau": taus, "rollout_steps": T,
                   "checkpoint_every": K, "store_all": K == 0, "seed": 0},
        "roofline": {"bound": "hbm", "kernel": "k_adjoint%s (adjoint of the fused step)" % (" (MRT)" if mrt else ""),
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_from_profile(args.workload),
                     "bytes_per_site": alg["adjoint"], "avg_launch_ms": round(avg, 5), "launches": adj_n},
        "gradients": {"dL/dtau": [float(x) for x in gt.reshape(-1)], "max_abs_df0": float(g.abs().max())},
    }
    if not args.no_copy:
        out["copy_probe"] = copy_probe(torch)
    print(json.dumps(out), flush=True)


def bench_adjoint_binary(args, n, desc, T=200, K=20):
    """Binary fluid: forward rollout from the spinodal fields + backward
    (recorded recompute, the three adjoint kernels per step, the reverse of
    the initialisation) per timed iteration; a step is one forward step plus
    one adjoint step."""
    import torch
    from paper_1405_6162_amd import inputs, lb
    from paper_1405_6162_amd.adjoint import binary_loss, rollout_binary
    log("bench: %s" % desc)
    rho, u, phi = (torch.as_tensor(a, device="cuda") for a in inputs.spinodal_quench(n, n, n, seed=0))
    trt, mrt = "_trt_" in args.workload, "_mrt_" in args.workload
    times = [1.0, 1.25, 1.4, 0.9, 1.2] if mrt else ([1.0, 1.25] if trt else 1.0)
    kw = {}
    if trt:
        kw = dict(collision=lb.LB_TRT, tau_minus=1.25)
    elif mrt:
        kw = dict(collision=lb.LB_MRT, tau_minus=1.25, tau_bulk=1.4, tau_ghost_even=0.9, tau_ghost_odd=1.2)
    lat = lb.Lattice(n, n, n, model=lb.LB_BINARY, **kw)
    par = lambda v: torch.tensor(v, dtype=torch.float64, device="cuda", requires_grad=True)

    def once():
        p0 = phi.clone().requires_grad_(True)
        kap, mob, tau = par(0.04), par(0.45), par(times)
        loss = binary_loss(*rollout_binary(rho, u, p0, lat, T, K, kap, mob, tau), 1.0)
        loss.backward()
        return p0.grad, torch.cat([kap.grad.reshape(1), mob.grad.reshape(1), tau.grad.reshape(-1)])

    n_warm = max(args.warmup // 10, 1)          # whole rollouts: forward + backward
    for _ in range(n_warm):
        once()
    torch.cuda.synchronize()
    iters = max(args.steps // 100, 1)
    lb.lb_profile_mask(lat.ctx, [lb.LB_K_ADJOINT])      # events on the adjoint kernels only
    t0 = time.perf_counter()
    for _ in range(iters):
        gphi, gpar = once()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lb.lb_profile(lat.ctx, False)
    adj_ms, adj_n = lb.lb_kernel_times(lat.ctx, lb.LB_K_ADJOINT)
    finite = bool(torch.isfinite(gphi).all()) and bool(torch.isfinite(gpar).all())
    lat.close()
    if not finite:
        print("non-finite gradient", file=sys.stderr)
        sys.exit(1)
    nsite = n ** 3
    alg = algorithmic_bytes("adjoint_binary", "f64")
    # an adjoint step is the local and the stencil kernel (plus a phi pass for
    # the last step of each segment, and the reverse initialisation once per
    # rollout, both included in this time)
    per_step_ms = adj_ms / (iters * T) if adj_n else 0.0
    achieved = alg["adjoint"] * nsite / (per_step_ms * 1e-3) / 1e9 if per_step_ms else 0.0
    out = {
        "metric": METRIC, "value": round(nsite * T * iters / wall / 1e6, 2), "unit": "MLUPS",
        "n_gpus": 1, "steps": T * iters, "warmup": T * n_warm,
        "ms_per_step": round(wall * 1e3 / (T * iters), 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": desc, "nx": n, "ny": n, "nz": n, "rollout_steps": T, "checkpoint_every": K,
                   "store_all": K == 0, "seed": 0},
        "roofline": {"bound": "hbm",
                     "kernel": "adjoint step: k_adjoint_binary%s + k_adjoint_binary_stencil" % (
                         " (TRT)" if trt else (" (MRT)" if mrt else "")),
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_from_profile(args.workload),
                     "traffic_unit": "bytes per adjoint step (local + stencil kernel)",
                     "bytes_per_site": alg["adjoint"], "bytes_per_site_moved": 1016,
                     "avg_step_ms": round(per_step_ms, 5), "launches": adj_n},
        "gradients": dict({"kappa": float(gpar[0]), "mobility": float(gpar[1]), "tau_f": float(gpar[2]),
                           "max_abs_dphi0": float(gphi.abs().max())},
                          **{k: float(v) for k, v in zip(("tau_minus", "tau_bulk", "tau_ghost_even",
                                                          "tau_ghost_odd"), gpar[3:])}),
    }
    if not args.no_copy:
        out["copy_probe"] = copy_probe(torch)
    print(json.dumps(out), flush=True)


def relative_errors(name, a, ref):
    """{name: max|a - ref| / max|ref|, name_l2: ||a - ref||_2 / ||ref||_2}, the
    two per-moment metrics (a vector moment is one array of all components)."""
    d = a - ref
    return {name: float(d.abs().max() / ref.abs().max()), name + "_l2": float(d.norm() / ref.norm())}


def _moment_errors(lb, ref, other):
    """Per-moment relative errors (max norm, and L2 as name_l2) of `other`
    against `ref` (Lattice objects on the same lattice), and both phi fields."""
    r0, u0, p0 = ref.moments()
    r1, u1, p1 = other.moments()
    err = dict(relative_errors("rho", r1, r0), **relative_errors("u", u1, u0))
    if p0 is not None:
        err.update(relative_errors("phi", p1, p0))
    return err, p0, p1


def _error_history(lb, make, checkpoints):
    """Step three lattices in lock-step and record, at each checkpoint, the
    per-moment errors against the FP64 one ("ref") of the reduced-precision
    one ("low") and of an FP64 run whose initial fields were rounded to FP32
    once ("perturbed": how far a single FP32 rounding of the initial state
    moves the trajectory, the flow's own sensitivity)."""
    lats = {k: make(k) for k in ("ref", "low", "perturbed")}
    hist, done = [], 0
    for c in checkpoints:
        for lat in lats.values():
            lat.step(c - done)
        done = c
        e_low, _, _ = _moment_errors(lb, lats["ref"], lats["low"])
        e_pert, _, _ = _moment_errors(lb, lats["ref"], lats["perturbed"])
        hist.append({"step": c, "low": e_low, "perturbed": e_pert})
    for lat in lats.values():
        lat.close()
    return hist


def _rounded(*a):
    return tuple(x.astype("float32").astype("float64") for x in a)


def interface_density(phi):
    """Fraction of nearest-neighbour bonds (all three axes, periodic) across
    which phi changes sign: interface area per unit volume in lattice units."""
    import torch
    p = phi.to(torch.float64)
    cut = [(p * torch.roll(p, 1, dims=d) < 0).to(torch.float64).mean() for d in range(3)]
    return float(sum(cut) / 3)


def coarsening_length(phi):
    """L = 2 pi sum S(k) / sum |k| S(k) over k != 0, S = |FFT(phi)|^2."""
    import torch
    n = phi.shape
    S = torch.fft.fftn(phi.to(torch.float64)).abs() ** 2
    ks = [2 * torch.pi * torch.fft.fftfreq(m, device=phi.device, dtype=torch.float64) for m in n]
    kz, ky, kx = torch.meshgrid(*ks, indexing="ij")
    k = torch.sqrt(kx * kx + ky * ky + kz * kz)
    S[0, 0, 0] = 0
    return float(2 * torch.pi * S.sum() / (k * S).sum())


def bench_precision(args, storage, n, desc):
    """Run the reduced-precision lattice and its reference from the same
    spinodal initial state and report per-moment errors, drift and MLUPS."""
    import torch
    from paper_1405_6162_amd import inputs, lb
    code = {"f64": lb.LB_F64, "f32": lb.LB_F32, "f16": lb.LB_F16}
    ref_storage = "f64" if storage == "f32" else "f32"
    steps = 500 if storage == "f32" else 1000
    log("bench: %s" % desc)

    def run(sto, nn, nsteps):
        rho, u, phi = inputs.spinodal_quench(nn, nn, nn, seed=0)
        lat = lb.Lattice(nn, nn, nn, model=lb.LB_BINARY, storage=code[sto], rho0=1.0, phi0=float(phi.mean()))
        lat.init_equilibrium(rho, u, phi)
        s0 = lat.conserved_sums().cpu()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.step(nsteps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        s1 = lat.conserved_sums().cpu()
        drift = {"mass_rel": float(abs(s1[0] - s0[0]) / abs(s0[0])),
                 "phi_per_site": float(abs(s1[4] - s0[4]) / nn ** 3)}
        return lat, nn ** 3 * nsteps / dt / 1e6, drift

    ref, ref_mlups, ref_drift = run(ref_storage, n, steps)
    low, mlups, drift = run(storage, n, steps)
    err, p_ref, p_low = _moment_errors(lb, ref, low)
    out = {"metric": METRIC, "value": round(mlups, 2), "unit": "MLUPS", "n_gpus": 1, "steps": steps,
           "warmup": 0, "ms_per_step": round(n ** 3 / mlups / 1e3, 5), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": storage, "data": "synthetic",
           "config": {"workload": desc, "nx": n, "ny": n, "nz": n, "seed": 0},
           "reference": {"storage": ref_storage, "MLUPS": round(ref_mlups, 2),
                         "speedup": round(mlups / ref_mlups, 3)},
           "errors_vs_reference": err, "drift": drift, "reference_drift": ref_drift,
           "coarsening_length": {storage: coarsening_length(p_low), ref_storage: coarsening_length(p_ref)},
           "interface_density": {storage: interface_density(p_low), ref_storage: interface_density(p_ref)}}
    ref.close()
    low.close()
    if storage == "f32":
        def make(kind):
            rho, u, phi = inputs.spinodal_quench(n, n, n, seed=0)
            if kind == "perturbed":
                rho, u, phi = _rounded(rho, u, phi)
            lat = lb.Lattice(n, n, n, model=lb.LB_BINARY, storage=code["f32" if kind == "low" else "f64"],
                             rho0=1.0, phi0=float(phi.mean()))
            lat.init_equilibrium(rho, u, phi)
            return lat
        out["error_history"] = _error_history(lb, make, [1, 10, 100, steps])
    if storage == "f16":
        # 96^3 run of all three storages, errors against the FP64 one
        sub = {}
        r64, _, d64 = run("f64", 96, steps)
        for sto in ("f32", "f16"):
            lat, _, d = run(sto, 96, steps)
            e, p64, pl = _moment_errors(lb, r64, lat)
            sub[sto] = {"errors_vs_f64": e, "drift": d, "coarsening_length": coarsening_length(pl),
                        "interface_density": interface_density(pl)}
            lat.close()
        sub["f64"] = {"drift": d64, "coarsening_length": coarsening_length(p64),
                      "interface_density": interface_density(p64)}
        r64.close()
        out["sub_run_96"] = sub
    print(json.dumps(out), flush=True)


def bench_precision_single(args, n, desc, steps=500):
    """Single fluid from the same random state in FP64 and FP32 storage;
    per-moment errors of FP32 against FP64 after `steps` steps."""
    import torch
    from paper_1405_6162_amd import inputs, lb
    log("bench: %s" % desc)
    rho, u = inputs.single_fluid_random(n, n, n, seed=0)
    res = {}
    lats = {}
    for sto, code in (("f64", lb.LB_F64), ("f32", lb.LB_F32)):
        lat = lb.Lattice(n, n, n, storage=code, rho0=1.0)
        lat.init_equilibrium(rho, u)
        s0 = lat.conserved_sums().cpu()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        s1 = lat.conserved_sums().cpu()
        res[sto] = {"MLUPS": n ** 3 * steps / dt / 1e6, "mass_drift": float(abs(s1[0] - s0[0]) / abs(s0[0]))}
        lats[sto] = lat
    err, _, _ = _moment_errors(lb, lats["f64"], lats["f32"])
    u0 = lats["f64"].moments()[1]
    out = {"metric": METRIC, "value": round(res["f32"]["MLUPS"], 2), "unit": "MLUPS", "n_gpus": 1,
           "steps": steps, "warmup": 0, "ms_per_step": round(n ** 3 / res["f32"]["MLUPS"] / 1e3, 5),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic", "config": {"workload": desc, "nx": n, "ny": n, "nz": n, "seed": 0},
           "reference": {"storage": "f64", "MLUPS": round(res["f64"]["MLUPS"], 2),
                         "speedup": round(res["f32"]["MLUPS"] / res["f64"]["MLUPS"], 3)},
           "errors_vs_reference": err,
           "drift": {"f32_mass_rel": res["f32"]["mass_drift"], "f64_mass_rel": res["f64"]["mass_drift"]}}
    out["final_max_abs_u"] = {"f64": float(u0.abs().max())}
    for lat in lats.values():
        lat.close()

    def make(kind):
        r, v = (rho, u) if kind != "perturbed" else _rounded(rho, u)
        lat = lb.Lattice(n, n, n, storage=lb.LB_F32 if kind == "low" else lb.LB_F64, rho0=1.0)
        lat.init_equilibrium(r, v)
        return lat
    out["error_history"] = _error_history(lb, make, [1, 10, 100, steps])
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="binary256_f64", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-copy", action="store_true", help="skip the copy-bandwidth probe")
    ap.add_argument("--store-all", action="store_true",
                    help="adjoint workloads: record every step in the forward (no recompute) instead of "
                         "checkpoints every 20 steps")
    ap.add_argument("--no-fp32", action="store_true",
                    help="skip the FP32 comparison of the binary 256^3 FP64 workload")
    ap.add_argument("--vvl", type=int, default=1, choices=(1, 2, 4),
                    help="sites per lane of the fused single-fluid kernel (the paper's VVL)")
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
        return bench_adjoint(args, n, desc, K=0 if args.store_all else 20)
    if model == "adjoint_binary":
        return bench_adjoint_binary(args, n, desc, K=0 if args.store_all else 20)
    if model == "precision":
        return bench_precision(args, storage, n, desc)
    if model == "precision_single":
        return bench_precision_single(args, n, desc)
    mcode = lb.LB_BINARY if model == "binary" else lb.LB_SINGLE
    scode = {"f64": lb.LB_F64, "f32": lb.LB_F32, "f16": lb.LB_F16}[storage]
    log("bench: %s, %d warmup + %d timed steps" % (desc, args.warmup, args.steps))

    coll = {}
    if "_trt_" in args.workload:
        coll = dict(collision=lb.LB_TRT, tau_minus=1.25)
    elif "_mrt_" in args.workload:
        coll = dict(collision=lb.LB_MRT, tau_minus=1.25, tau_bulk=1.4, tau_ghost_even=0.9, tau_ghost_odd=1.2)
    lat = lb.Lattice(n, n, n, model=mcode, storage=scode, vvl=args.vvl, **coll)
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

    # timed region: plain launches only
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    lat.step(args.steps)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1)
    log("bench: timed region %.3f ms (events), %.3f s wall" % (gpu_ms, wall))
    # kernel timing pass: the same number of steps, every launch between two
    # HIP events on the library's stream
    lb.lb_profile(lat.ctx, True)
    lat.step(args.steps)
    torch.cuda.synchronize()
    lb.lb_profile(lat.ctx, False)
    col_ms, col_n = lb.lb_kernel_times(lat.ctx, lb.LB_K_COLLIDE)
    log("bench: kernel pass %.3f ms in %d launches" % (col_ms, col_n))

    nsite = n ** 3
    sums = lat.conserved_sums().cpu()
    finite = bool(torch.isfinite(sums).all())
    alg = algorithmic_bytes(model, storage)
    ceiling = pull_copy_ceiling(lb, lat, alg["collide"] * nsite)
    log("bench: pull-copy ceiling %s GB/s" % ceiling["GB/s"])
    lat.close()
    if not finite:
        print("non-finite state after the timed steps", file=sys.stderr)
        sys.exit(1)

    seconds = wall
    mlups = nsite * args.steps / seconds / 1e6
    col_avg_ms = col_ms / max(col_n, 1)
    achieved = alg["collide"] * nsite / (col_avg_ms * 1e-3) / 1e9
    step_bytes = alg["collide"]

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
                   "storage": storage, "seed": 0, "sites_per_lane": args.vvl},
        "roofline": {
            "bound": "hbm",
            "kernel": ("k_binary_march (single-pass pull-stream + phi + collision)" if model == "binary"
                       else "k_collide (fused pull-stream + collision)"),
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic_from_profile(args.workload),
            "bytes_per_site": alg["collide"],
            "avg_launch_ms": round(col_avg_ms, 5),
            "launches": col_n,
            "timing": "HIP events around each launch, in a pass of its own after the timed region",
            "frac_of_pull_copy": round(achieved / ceiling["GB/s"], 4) if ceiling["GB/s"] else None,
        },
        "pull_copy_ceiling": ceiling,
        "step_roofline": {
            "bytes_per_site": step_bytes,
            "GB/s": round(step_bytes * nsite * args.steps / seconds / 1e9, 1),
            "frac": round(step_bytes * nsite * args.steps / seconds / 1e9 / HBM_PEAK_GBS, 4),
            "timing": "wall clock of the whole timed region",
            "event_ms_per_step": round(gpu_ms / args.steps, 5),
        },
    }
    if args.workload == "binary256_f64" and not args.no_fp32:
        log("bench: FP32 comparison")
        out["fp32_vs_fp64"] = fp32_vs_fp64(torch, lb, inputs, n, args.steps, args.warmup, mlups)
    if not args.no_copy:
        out["copy_probe"] = copy_probe(torch)
        out["roofline"]["frac_of_copy_probe"] = round(achieved / out["copy_probe"]["GB/s"], 4)
        log("bench: copy probe %s GB/s" % out["copy_probe"]["GB/s"])
    if not args.no_cpu:
        log("bench: timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(model, n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
