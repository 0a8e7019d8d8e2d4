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
  within the storage's rounding (FP16: 1e-6 relative, FP32: 1e-9).
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
