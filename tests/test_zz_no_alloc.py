"""The allocation-free entry point lb_conserved_sums_noalloc (partial sums
in the library's fixed device array, no context, no workspace) against
lb_conserved_sums of a context holding the same state: identical bits, on
two calls in a row with the second on a smaller lattice (the fixed array
keeps the first call's partials), for every storage and both models; and
LB_ERANGE beyond the array's size."""

import ctypes

import numpy as np
import pytest
import torch

from paper_1405_6162_amd import inputs

pytestmark = pytest.mark.gpu


def _lattice_state(lb, n, model, storage, seed):
    nx, ny, nz = n
    kw = dict(model=model, storage=storage)
    if storage != lb.LB_F64:
        kw.update(rho0=1.0, phi0=0.0)
    lat = lb.Lattice(nx, ny, nz, **kw)
    if model == lb.LB_BINARY:
        rho, u, phi = inputs.spinodal_quench(nx, ny, nz, seed=seed, phi_max=0.3)
        lat.init_equilibrium(rho, u, phi)
    else:
        rho, u = inputs.single_fluid_random(nx, ny, nz, seed=seed)
        lat.init_equilibrium(rho, u)
    lat.step(3)
    f, g = lat.get_state()
    lat.set_state(f, g)                 # a direct (unpropagated) state: the same summation order
    return lat, f, g


def _sums_both(lb, lat, f, g):
    ref = torch.empty(5, dtype=torch.float64, device="cuda")
    lb.lb_set_stream(lat.ctx, lb._stream())
    lb.lb_conserved_sums(lat.ctx, ref)
    out = torch.full((5,), float("nan"), dtype=torch.float64, device="cuda")
    lb.lb_conserved_sums_noalloc(lat.params, f, g, out)
    torch.cuda.synchronize()
    return out.cpu().numpy(), ref.cpu().numpy()


@pytest.mark.parametrize("storage", [0, 1, 2])
@pytest.mark.parametrize("model", [0, 1])
def test_noalloc_sums_equal_context_sums(lbgpu, model, storage):
    lb = lbgpu
    for n, seed in (((70, 37, 23), 1), ((9, 5, 4), 2)):      # second call smaller than the first
        print("case noalloc sums", model, storage, n, flush=True)
        lat, f, g = _lattice_state(lb, n, model, storage, seed)
        got, want = _sums_both(lb, lat, f, g if model == lb.LB_BINARY else None)
        lat.close()
        assert np.isfinite(want).all()
        assert np.array_equal(got, want), (got, want)
        assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_noalloc_rejects_lattice_beyond_scratch(lbgpu):
    lb = lbgpu
    nz = lb.LB_NOALLOC_MAX_BLOCKS // (2 * 2) + 1            # ceil(128/64) * ceil(8/4) * nz blocks
    prm = lb.make_params(128, 8, nz)
    dummy = torch.zeros(16, dtype=torch.float64, device="cuda")
    out = torch.zeros(5, dtype=torch.float64, device="cuda")
    rc = lb.load().lb_conserved_sums_noalloc(ctypes.byref(prm), lb._ptr(dummy), None, lb._ptr(out), lb._stream())
    assert rc == lb.LB_ERANGE
    assert "too large" in lb.lb_strerror(rc)
