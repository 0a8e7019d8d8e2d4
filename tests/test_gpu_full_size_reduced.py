"""The 384^3 reduced-precision workloads at their full size.

The binary spinodal quench on a 384^3 periodic lattice in FP16-deviation
storage and in FP32 storage (4.3 GB per distribution, beyond 32-bit byte
offsets: 4-byte elements are addressed by element), both in the blocked
layout and in the launch configuration the benchmark times, two steps.  No
FP64 oracle run is sensible at this size in reduced precision, so the
checks are properties that hold at any size:

- the single-pass march (the benchmark's kernel: 128 x 4 tiles, 64-plane
  chunks here) and
  the two-pass step give the same bits (they sum phi in the same order and
  share the collision; both are compared with the oracle at smaller sizes);
- total mass and total phi after two steps equal their initial values
  within the storage's rounding (FP16: 1e-6 relative, FP32: 1e-9);
- FP32: f and g at sampled sites after one step against the C oracle.
"""

import pytest
import torch

from paper_1405_6162_amd import inputs

pytestmark = pytest.mark.gpu

N = 384


@pytest.mark.parametrize("storage,tol", [("f16", 1e-6), ("f32", 1e-9)])
def test_binary_384_march_equals_two_pass(lbgpu, storage, tol):
    print("case binary 384^3 %s x2: march vs two-pass, conservation" % storage, flush=True)
    code = {"f16": lbgpu.LB_F16, "f32": lbgpu.LB_F32}[storage]
    rho, u, phi = inputs.spinodal_quench(N, N, N, seed=0)
    states, sums = {}, {}
    for path, step in (("march", lbgpu.LB_STEP_MARCH), ("two_pass", lbgpu.LB_STEP_TWO_PASS)):
        lat = lbgpu.Lattice(N, N, N, model=lbgpu.LB_BINARY, storage=code, rho0=1.0, phi0=float(phi.mean()),
                            binary_step=step)
        lat.init_equilibrium(rho, u, phi)
        s0 = lat.conserved_sums().cpu()
        lat.step(2)
        s1 = lat.conserved_sums().cpu()
        states[path] = lat.get_state()
        sums[path] = (s0, s1)
        lat.close()
        torch.cuda.synchronize()
    for a, b in zip(states["march"], states["two_pass"]):
        assert torch.equal(a, b)
    s0, s1 = sums["march"]
    mass = abs(float(s1[0] - s0[0])) / abs(float(s0[0]))
    dphi = abs(float(s1[4] - s0[4])) / float(N ** 3)       # total phi starts near 0: per site
    print("384^3 %s x2: mass drift %.2e, phi drift per site %.2e" % (storage, mass, dphi), flush=True)
    assert mass <= tol and dphi <= tol


def test_binary_384_fp32_sampled_sites_against_oracle(lbgpu):
    """FP32 at 384^3, whose blocked state passes 4 GiB per buffer (4-byte
    elements are addressed by element): f and g at sampled sites after one
    step, the lattice corners (the largest offsets and every wrap) among
    them, against the C oracle's FP64 values, within 1e-6 of their largest."""
    import numpy as np
    from oracle import c_backend as C
    from oracle import lb_oracle as O
    print("case binary 384^3 FP32 x1, sampled sites vs C oracle", flush=True)
    rho, u, phi = inputs.spinodal_quench(N, N, N, seed=0)
    rng = np.random.default_rng(7)
    pts = [(x, y, z) for x in (0, N - 1) for y in (0, N - 1) for z in (0, N - 1)]
    pts += [tuple(int(v) for v in rng.integers(0, N, 3)) for _ in range(2000)]
    idx = np.array([x + N * (y + N * z) for (x, y, z) in pts], dtype=np.int64)
    C.set_threads(0)
    ref = C.CLattice(N, N, N, model=1)
    ref.init_equilibrium(rho, u, phi)
    ref.step(1)
    fo, go = ref.state()
    ref.close()
    fo, go = fo.reshape(19, -1)[:, idx].copy(), go.reshape(19, -1)[:, idx].copy()
    phi0 = float(phi.mean())
    lat = lbgpu.Lattice(N, N, N, model=lbgpu.LB_BINARY, storage=lbgpu.LB_F32, rho0=1.0, phi0=phi0)
    lat.init_equilibrium(rho, u, phi)
    lat.step(1)
    fs, gs = lat.get_sites(torch.as_tensor(idx.astype(np.int32), device="cuda"))
    lat.close()
    f = fs.double().cpu().numpy() + O.W[:, None] * 1.0          # stored as deviations from w_i rho0, w_i phi0
    g = gs.double().cpu().numpy() + O.W[:, None] * phi0
    ef = float(np.abs(f - fo).max() / np.abs(fo).max())
    eg = float(np.abs(g - go).max() / np.abs(go).max())
    print("384^3 FP32 x1 vs oracle at %d sites: f %.2e g %.2e" % (idx.size, ef, eg), flush=True)
    assert ef <= 1e-6 and eg <= 1e-6
