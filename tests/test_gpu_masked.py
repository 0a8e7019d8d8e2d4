"""Masked transfer (pack the selected sites on the device, move only them):
compaction order against numpy, gathered and scattered values against the
oracle's state, in both state representations (direct and pending)."""

import numpy as np
import pytest
import torch

from oracle import lb_oracle as O
from paper_1405_6162_amd import inputs

pytestmark = pytest.mark.gpu


def _mask(shape, density, seed):
    rng = np.random.default_rng(seed)
    return rng.random(shape) < density


@pytest.mark.parametrize("nx,ny,nz,density", [(67, 9, 5, 0.3), (16, 16, 16, 0.0), (16, 16, 16, 1.0),
                                              (5, 6, 37, 0.5), (128, 8, 8, 0.01)])
def test_mask_index_order(lbgpu, nx, ny, nz, density):
    lat = lbgpu.Lattice(nx, ny, nz)
    mask = _mask((nz, ny, nx), density, seed=1)
    idx = lat.mask_index(mask).cpu().numpy()
    assert np.array_equal(idx, np.flatnonzero(mask.ravel()))


@pytest.mark.parametrize("model", ["single", "binary"])
@pytest.mark.parametrize("pending", [False, True])
def test_get_and_set_sites(lbgpu, model, pending):
    nx, ny, nz = 19, 7, 6
    prm = O.Params()
    if model == "single":
        rho, u = inputs.single_fluid_random(nx, ny, nz, seed=2)
        lat = lbgpu.Lattice(nx, ny, nz)
        lat.init_equilibrium(rho, u)
        ref = [O.init_single(rho, u)]
        step = lambda s: [O.step_single(s[0], prm.tau_f, 1)]
    else:
        rho, u, phi = inputs.spinodal_quench(nx, ny, nz, seed=2, phi_max=0.4)
        lat = lbgpu.Lattice(nx, ny, nz, model=lbgpu.LB_BINARY)
        lat.init_equilibrium(rho, u, phi)
        ref = list(O.init_binary(rho, u, phi, prm))
        step = lambda s: list(O.step_binary(s[0], s[1], prm, 1))
    if pending:                       # after a step the library holds a pending buffer
        lat.step(1)
        ref = step(ref)
    mask = _mask((nz, ny, nx), 0.35, seed=3)
    index = lat.mask_index(mask)
    idx = index.cpu().numpy()
    full = [a.cpu().numpy() for a in lat.get_state() if a is not None]     # the logical state
    for a, r in zip(full, ref):
        assert np.abs(a - r).max() <= 1e-12 * np.abs(r).max()
    got = [a for a in lat.get_sites(index) if a is not None]
    for a, r in zip(got, full):                                          # gather is exact
        np.testing.assert_array_equal(a.cpu().numpy(), r.reshape(19, -1)[:, idx])
    # overwrite the masked sites with new values and continue stepping
    rng = np.random.default_rng(4)
    new = [r.reshape(19, -1)[:, idx] * (1 + 1e-3 * rng.standard_normal((19, idx.size))) for r in full]
    lat.set_sites(index, *new) if model == "binary" else lat.set_sites(index, new[0])
    for r, v in zip(full, new):
        r.reshape(19, -1)[:, idx] = v
    st = [a for a in lat.get_state() if a is not None]
    for a, r in zip(st, full):                                           # scatter is exact
        np.testing.assert_array_equal(a.cpu().numpy(), r)
    lat.step(2)
    ref = step(step(full))
    st = [a for a in lat.get_state() if a is not None]
    for a, r in zip(st, ref):
        assert np.abs(a.cpu().numpy() - r).max() <= 1e-12 * np.abs(r).max()


def test_host_masked_copies(lbgpu):
    """copy_from_masked updates only the masked sites of a host array;
    copy_to_masked writes only those back."""
    nx, ny, nz = 33, 5, 4
    rho, u = inputs.single_fluid_random(nx, ny, nz, seed=5)
    lat = lbgpu.Lattice(nx, ny, nz)
    lat.init_equilibrium(rho, u)
    full = lat.get_state()[0].cpu().numpy()          # the copies are exact against the GPU state
    assert np.abs(full - O.init_single(rho, u)).max() <= 1e-15
    mask = _mask((nz, ny, nx), 0.2, seed=6)
    host = np.full_like(full, -7.0)
    lat.copy_from_masked(mask, host)
    sel = np.broadcast_to(mask, full.shape)
    np.testing.assert_array_equal(host[sel], full[sel])
    assert (host[~sel] == -7.0).all()
    host2 = full * 2.0
    lat.copy_to_masked(mask, host2)
    want = np.where(sel, host2, full)
    np.testing.assert_array_equal(lat.get_state()[0].cpu().numpy(), want)
