"""The headline configurations at their full size against the FP64 oracle.

The binary spinodal quench on a 256^3 periodic lattice, seeded as the
benchmark seeds it, run by the library in the launch configuration the
benchmark times (`Lattice` defaults: the single-pass march for the step) and
by the plain C reference (oracle/lb_oracle.c) on all host cores:

- FP64 storage, 3 steps: every site's rho and phi within 1e-12 of the
  oracle's (relative to their largest value), u within 1e-14 in lattice
  units (u starts at zero, so its relative error only measures how small it
  still is), and f and g at sampled sites (corners, a face, seeded random
  sites) within 1e-12;
- FP32 storage, 1 and 10 steps: u within 1e-6 of the oracle relative to
  max |u|, rho and phi within 1e-6.
"""

import numpy as np
import pytest
import torch

from oracle import c_backend as C
from paper_1405_6162_amd import inputs

pytestmark = pytest.mark.gpu

N = 256


def relerr(a, ref):
    return float(np.abs(np.asarray(a) - ref).max() / np.abs(ref).max())


def _sample_sites(n, k, seed):
    rng = np.random.default_rng(seed)
    pts = [(0, 0, 0), (n - 1, n - 1, n - 1), (n - 1, 0, n // 2), (0, n - 1, 1), (n // 2, n // 2, n - 1)]
    pts += [tuple(int(v) for v in rng.integers(0, n, 3)) for _ in range(k)]
    return np.array([x + n * (y + n * z) for (x, y, z) in pts], dtype=np.int64)


def _oracle(fields, steps):
    """{step: (rho, u, phi)} of the C reference, and its f, g after the last."""
    C.set_threads(0)
    rho, u, phi = fields
    ref = C.CLattice(N, N, N, model=1)
    ref.init_equilibrium(rho, u, phi)
    out, done = {}, 0
    for k in sorted(steps):
        ref.step(k - done)
        done = k
        out[k] = ref.moments()
    f, g = ref.state()
    ref.close()
    return out, f, g


def test_binary_256_fp64_headline_config(lbgpu):
    print("case binary 256^3 FP64 x3 vs C oracle", flush=True)
    fields = inputs.spinodal_quench(N, N, N, seed=0)
    ref, fo, go = _oracle(fields, [3])
    r0, u0, p0 = ref[3]
    lat = lbgpu.Lattice(N, N, N, model=lbgpu.LB_BINARY)
    lat.init_equilibrium(*fields)
    lat.step(3)
    r, u, p = (a.cpu().numpy() for a in lat.moments())
    idx = _sample_sites(N, 2000, seed=3)
    fs, gs = lat.get_sites(torch.as_tensor(idx.astype(np.int32), device="cuda"))
    fs, gs = fs.cpu().numpy(), gs.cpu().numpy()
    lat.close()
    er, ep, du = relerr(r, r0), relerr(p, p0), float(np.abs(u - u0).max())
    fo, go = fo.reshape(19, -1)[:, idx], go.reshape(19, -1)[:, idx]
    ef, eg = relerr(fs, fo), relerr(gs, go)
    print("binary 256^3 FP64 x3 vs oracle: rho %.2e phi %.2e u %.2e (absolute; max |u| %.2e) | f %.2e g %.2e at %d "
          "sampled sites" % (er, ep, du, np.abs(u0).max(), ef, eg, idx.size), flush=True)
    assert max(er, ep, ef, eg) <= 1e-12
    assert du <= 1e-14


def test_binary_256_fp32_short_horizon(lbgpu):
    print("case binary 256^3 FP32 x1, x10 vs C oracle", flush=True)
    fields = inputs.spinodal_quench(N, N, N, seed=0)
    ref, _f, _g = _oracle(fields, [1, 10])
    lat = lbgpu.Lattice(N, N, N, model=lbgpu.LB_BINARY, storage=lbgpu.LB_F32, rho0=1.0,
                        phi0=float(fields[2].mean()))
    lat.init_equilibrium(*fields)
    errs, done = {}, 0
    for k in (1, 10):
        lat.step(k - done)
        done = k
        r, u, p = (a.cpu().numpy() for a in lat.moments())
        r0, u0, p0 = ref[k]
        errs[k] = (relerr(r, r0), relerr(u, u0), relerr(p, p0))
        print("binary 256^3 FP32 x%d vs oracle: rho %.2e u %.2e phi %.2e" % ((k,) + errs[k]), flush=True)
    lat.close()
    for k, (er, eu, ep) in errs.items():
        assert eu <= 1e-6 and er <= 1e-6 and ep <= 1e-6, k
