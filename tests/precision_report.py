"""Per-moment errors of the GPU binary fluid in FP64 and FP32 storage
against the FP64 oracle on the 256^3 spinodal quench, over 500 steps.

    python tests/precision_report.py [--n 256] [--steps 500]

The oracle is the plain C reference (oracle/lb_oracle.c) on all host cores;
the three runs start from the same seeded fields (rho = 1, u = 0,
phi ~ U(-0.05, 0.05), seed 0) and are compared at checkpoints.  Also
reported: an FP64 GPU run whose initial fields were rounded to FP32 once
("perturbed"), the flow's own sensitivity to one FP32 rounding.  Prints one
progress line per checkpoint and a JSON line at the end.  Needs a GPU; at
256^3 the oracle takes about five minutes on 16 cores.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def relerr(a, ref):
    return float(np.abs(np.asarray(a) - ref).max() / np.abs(ref).max())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--steps", type=int, default=500)
    args = ap.parse_args()
    import torch
    from oracle import c_backend as C
    from paper_1405_6162_amd import inputs, lb

    lb.load()
    n, T = args.n, args.steps
    checkpoints = [k for k in (1, 10, 50, 100, 200, 300, 400, 500, 1000) if k < T] + [T]
    cores = C.set_threads(0)
    rho, u, phi = inputs.spinodal_quench(n, n, n, seed=0)
    ref = C.CLattice(n, n, n, model=1)
    ref.init_equilibrium(rho, u, phi)
    runs = {}
    for name, code, fields in (("f64", lb.LB_F64, (rho, u, phi)), ("f32", lb.LB_F32, (rho, u, phi)),
                               ("f64_perturbed", lb.LB_F64,
                                tuple(a.astype(np.float32).astype(np.float64) for a in (rho, u, phi)))):
        lat = lb.Lattice(n, n, n, model=lb.LB_BINARY, storage=code, rho0=1.0, phi0=float(fields[2].mean()))
        lat.init_equilibrium(*fields)
        runs[name] = lat
    hist = []
    done = 0
    t_oracle = 0.0
    for k in checkpoints:
        t0 = time.perf_counter()
        ref.step(k - done)
        t_oracle += time.perf_counter() - t0
        r0, u0, p0 = ref.moments()
        row = {"step": k}
        for name, lat in runs.items():
            lat.step(k - done)
            r, v, p = (a.cpu().numpy() for a in lat.moments())
            row[name] = {"rho": relerr(r, r0), "u": relerr(v, u0), "phi": relerr(p, p0)}
        done = k
        row["max_abs_u"] = float(np.abs(u0).max())
        hist.append(row)
        print("step %d: %s" % (k, "; ".join("%s rho %.2e u %.2e phi %.2e" % (nm, e["rho"], e["u"], e["phi"])
                                            for nm, e in row.items() if isinstance(e, dict))), flush=True)
    for lat in runs.values():
        lat.close()
    ref.close()
    print(json.dumps({"workload": "D3Q19 binary fluid %d^3 spinodal quench, %d steps" % (n, T),
                      "oracle": "C reference, FP64, %d threads, %.0f s" % (cores, t_oracle),
                      "metric": "max |q - q_oracle| / max |q_oracle|", "history": hist}), flush=True)
    torch.cuda.synchronize()


if __name__ == "__main__":
    main()
