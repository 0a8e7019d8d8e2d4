"""Differentiable rollouts that record every step in the forward (every = 0:
one segment, no recompute in the backward) against the same rollouts with
checkpoints every K steps: the recorded post-collision fields are the same
bits either way (lb_step_record leaves the state that lb_step would), so
every gradient agrees to the rounding of the parameter sums' order.  The
checkpointed rollouts themselves are held to the oracle by the other
adjoint tests."""

import numpy as np
import pytest
import torch

from paper_1405_6162_amd import inputs

pytestmark = pytest.mark.gpu


def test_binary_store_all_equals_checkpointed(lbgpu):
    from paper_1405_6162_amd.adjoint import binary_loss, rollout_binary
    print("case binary rollout 24x20x16 x13: store-all vs K=5", flush=True)
    rho, _u, phi = inputs.spinodal_quench(24, 20, 16, seed=61, phi_max=0.3)
    _r, u = inputs.single_fluid_random(24, 20, 16, seed=62, u_max=0.02)
    lat = lbgpu.Lattice(24, 20, 16, model=lbgpu.LB_BINARY, kappa=0.05, mobility=0.3)
    out = {}
    for every in (5, 0):
        r0, u0, p0 = (torch.as_tensor(a, device="cuda").requires_grad_(True) for a in (rho, u, phi))
        pars = [torch.tensor(v, dtype=torch.float64, device="cuda", requires_grad=True) for v in (0.05, 0.3, 0.9)]
        loss = binary_loss(*rollout_binary(r0, u0, p0, lat, 13, every, *pars), 0.5)
        loss.backward()
        out[every] = [loss.detach()] + [t.grad.detach().clone() for t in (p0, r0, u0)] + [t.grad for t in pars]
    lat.close()
    assert torch.equal(out[5][0], out[0][0])
    for a, b in zip(out[5][1:4], out[0][1:4]):             # dL/dphi0, dL/drho0, dL/du0: same arithmetic
        assert torch.equal(a, b)
    for a, b in zip(out[5][4:], out[0][4:]):               # kappa, mobility, tau_f: sums over steps
        assert abs(float(a) - float(b)) <= 1e-13 * abs(float(b))


def test_single_store_all_equals_checkpointed(lbgpu):
    from paper_1405_6162_amd.adjoint import rollout, velocity_loss
    from oracle import lb_oracle as O
    print("case single rollout 20x16x12 x17: store-all vs K=4", flush=True)
    rho, u = inputs.shear_wave(20, 16, 12, amplitude=0.01, noise=1e-3, seed=63)
    f0 = torch.as_tensor(O.init_single(rho, u), device="cuda")
    lat = lbgpu.Lattice(20, 16, 12, tau_f=0.8)
    out = {}
    for every in (4, 0):
        f = f0.clone().requires_grad_(True)
        t = torch.tensor(0.8, dtype=torch.float64, device="cuda", requires_grad=True)
        loss = velocity_loss(rollout(f, t, lat, 17, every))
        loss.backward()
        out[every] = (loss.detach(), f.grad.detach().clone(), t.grad.detach().clone())
    lat.close()
    assert torch.equal(out[4][0], out[0][0])
    assert torch.equal(out[4][1], out[0][1])
    assert abs(float(out[4][2]) - float(out[0][2])) <= 1e-13 * abs(float(out[0][2]))
