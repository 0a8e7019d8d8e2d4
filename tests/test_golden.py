"""The stored fixtures under tests/golden/ (written by make_golden.py from
the oracle alone): the oracle must still produce them (CPU), and the GPU
library must match them to 1e-12 (gpu)."""

import importlib.util
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
_spec = importlib.util.spec_from_file_location("make_golden", os.path.join(HERE, "golden", "make_golden.py"))
G = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(G)


def _stored(name):
    model, shape, steps, seed = G.CASES[name]
    nx, ny, nz = shape
    k = 1 if model == "single" else 2
    return np.loadtxt(G.path(name)).reshape(k, 19, nz, ny, nx)


@pytest.mark.parametrize("name", sorted(G.CASES))
def test_oracle_reproduces_stored_values(name):
    want = _stored(name)
    got = G.compute(*G.CASES[name])
    assert np.abs(got - want).max() <= 1e-14 * np.abs(want).max()


def test_oracle_reproduces_stored_adjoint_sums():
    for name, (model, shape, steps, seed) in G.CASES.items():
        if model != "binary_mrt_adjoint":
            continue
        want = np.loadtxt(G.grads_path(name))
        got = G.adjoint_grads(shape, steps, seed)
        assert np.abs(got - want).max() <= 1e-14 * np.abs(want).max()


@pytest.mark.gpu
@pytest.mark.parametrize("name", sorted(G.CASES))
def test_gpu_matches_stored_values(lbgpu, name):
    from paper_1405_6162_amd import inputs
    model, (nx, ny, nz), steps, seed = G.CASES[name]
    want = _stored(name)
    if model == "binary_mrt_adjoint":
        import torch
        t = G.MRT_TAUS
        lat = lbgpu.Lattice(nx, ny, nz, model=lbgpu.LB_BINARY, collision=lbgpu.LB_MRT, tau_f=t[0], tau_minus=t[1],
                            tau_bulk=t[2], tau_ghost_even=t[3], tau_ghost_odd=t[4])
        f, g, lf, lg = (torch.as_tensor(a, device="cuda") for a in G.adjoint_inputs((nx, ny, nz), steps, seed))
        lf_n, lg_n = torch.empty_like(lf), torch.empty_like(lg)
        grads = torch.zeros(7, dtype=torch.float64, device="cuda")
        lbgpu.lb_set_stream(lat.ctx, lbgpu._stream())
        lbgpu.lb_adjoint_step_binary(lat.ctx, f, g, lf, lg, lf_n, lg_n, grads)
        got = np.stack([lf_n.cpu().numpy(), lg_n.cpu().numpy()])
        got_sums = grads.cpu().numpy()
        lat.close()
        assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
        want_sums = np.loadtxt(G.grads_path(name))
        for k, w in enumerate(want_sums):
            assert abs(got_sums[k] - w) <= 1e-12 * max(abs(w), 1.0), G.MRT_GRAD_NAMES[k]
        return
    if model == "single":
        rho, u = inputs.single_fluid_random(nx, ny, nz, seed=seed)
        lat = lbgpu.Lattice(nx, ny, nz)
        lat.init_equilibrium(rho, u)
    else:
        rho, u, phi = inputs.spinodal_quench(nx, ny, nz, seed=seed, phi_max=0.3)
        lat = lbgpu.Lattice(nx, ny, nz, model=lbgpu.LB_BINARY)
        lat.init_equilibrium(rho, u, phi)
    lat.step(steps)
    got = np.stack([t.cpu().numpy() for t in lat.get_state() if t is not None])
    lat.close()
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
