"""Parity at the largest lattices the library accepts (N < 2^29 sites, where
FP64 byte offsets reach 2^32 - 8), on sampled sites.  The initial fields are
smooth analytic functions of the coordinates, so the oracle can rebuild any
site's neighbourhood on the host: a site's state after two single-fluid steps,
or after one binary step (pull plus the phi stencil), depends only on the
initial state within two sites per axis, so the centre of a periodic 5^3 block
cut around it evolves exactly as in the full lattice.  Sampled sites include
the lattice corners (the largest offsets and every wrap) and seeded random
sites.  (The binary initialisation itself reads the phi stencil, so the
binary case needs the inputs within three sites: a 7^3 block.)"""

import gc

import numpy as np
import pytest
import torch

from oracle import lb_oracle as O

pytestmark = pytest.mark.gpu

TWO_PI = 2.0 * np.pi


def _fields(x, y, z, n, lib):
    """rho, u (3 components) and phi at integer coordinates (arrays of any
    shape, broadcastable) on an (nx, ny, nz) lattice; lib is numpy or torch."""
    nx, ny, nz = n
    X, Y, Z = x / nx, y / ny, z / nz
    rho = 1.0 + 0.01 * lib.sin(TWO_PI * (3 * X + 5 * Y + 7 * Z))
    ux = 0.01 * lib.sin(TWO_PI * (2 * Y + Z))
    uy = 0.01 * lib.cos(TWO_PI * (X + 3 * Z))
    uz = 0.005 * lib.sin(TWO_PI * (4 * X + 2 * Y))
    phi = 0.05 * lib.sin(TWO_PI * (X + 2 * Y)) * lib.cos(TWO_PI * 3 * Z)
    return rho, (ux, uy, uz), phi


def _device_fields(n):
    nx, ny, nz = n
    d = dict(dtype=torch.float64, device="cuda")
    z = torch.arange(nz, **d).view(nz, 1, 1)
    y = torch.arange(ny, **d).view(1, ny, 1)
    x = torch.arange(nx, **d).view(1, 1, nx)
    rho, u, phi = _fields(x, y, z, n, torch)
    shape = (nz, ny, nx)
    rho = rho.expand(shape).contiguous()
    u = torch.stack([c.expand(shape) for c in u]).contiguous()
    phi = phi.expand(shape).contiguous()
    return rho, u, phi


def _block(site, n, r=2):
    """Host fields on the periodic (2r+1)^3 block centred on site (x, y, z)."""
    nx, ny, nz = n
    x0, y0, z0 = site
    off = np.arange(-r, r + 1)
    z = ((z0 + off) % nz).astype(np.float64).reshape(-1, 1, 1)
    y = ((y0 + off) % ny).astype(np.float64).reshape(1, -1, 1)
    x = ((x0 + off) % nx).astype(np.float64).reshape(1, 1, -1)
    rho, u, phi = _fields(x, y, z, n, np)
    shape = (2 * r + 1,) * 3
    return (np.broadcast_to(rho, shape).copy(), np.stack([np.broadcast_to(c, shape) for c in u]),
            np.broadcast_to(phi, shape).copy())


def _samples(n, count, seed):
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    pts = [(0, 0, 0), (nx - 1, ny - 1, nz - 1), (nx - 1, 0, nz - 1), (0, ny - 1, 0)]
    pts += [tuple(int(v) for v in (rng.integers(nx), rng.integers(ny), rng.integers(nz))) for _ in range(count)]
    return pts


def _release():
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def _gathered(lat, pts, n):
    nx, ny, _ = n
    idx = torch.tensor([x + nx * (y + ny * z) for (x, y, z) in pts], dtype=torch.int32, device="cuda")
    f, g = lat.get_sites(idx)
    return f.cpu().numpy(), (g.cpu().numpy() if g is not None else None)


def test_single_fluid_fp64_largest_lattice(lbgpu):
    n = (1024, 1024, 511)                           # 535,822,336 sites < 2^29
    assert n[0] * n[1] * n[2] < 2 ** 29
    print("case single FP64 max size", n, flush=True)
    _release()
    try:
        lat = lbgpu.Lattice(*n)
        rho, u, _phi = _device_fields(n)
        lat.init_equilibrium(rho, u)
        del rho, u
        lat.step(2)
        pts = _samples(n, 6, seed=1)
        f, _ = _gathered(lat, pts, n)
        lat.close()
    finally:
        _release()
    for k, p in enumerate(pts):
        rho, u, _phi = _block(p, n)
        want = O.step_single(O.init_single(rho, u), 1.0, 2)[:, 2, 2, 2]
        assert np.abs(f[:, k] - want).max() <= 1e-12 * np.abs(want).max(), p


@pytest.mark.parametrize("step_kernel", [1, 2])          # LB_STEP_MARCH, LB_STEP_TWO_PASS
def test_binary_fp64_largest_offsets(lbgpu, step_kernel):
    """Two steps: the first collides the initial (direct) state in place, the
    second pulls from the pending one through the chosen step kernel; the
    oracle's 11^3 block around each sample is exact at its centre for two
    steps after the initialisation."""
    n = (1024, 512, 511)                            # 267,911,168 sites: FP64 offsets up to 2^31
    print("case binary FP64 max size", n, "step kernel", step_kernel, flush=True)
    prm = O.Params()
    _release()
    try:
        lat = lbgpu.Lattice(*n, model=lbgpu.LB_BINARY, binary_step=step_kernel)
        rho, u, phi = _device_fields(n)
        lat.init_equilibrium(rho, u, phi)
        del rho, u, phi
        lat.step(2)
        pts = _samples(n, 6, seed=2)
        f, g = _gathered(lat, pts, n)
        stats = lat.conserved_sums().cpu().numpy()
        lat.close()
    finally:
        _release()
    for k, p in enumerate(pts):
        rho, u, phi = _block(p, n, r=5)
        wf, wg = O.step_binary(*O.init_binary(rho, u, phi, prm), prm, 2)
        wf, wg = wf[:, 5, 5, 5], wg[:, 5, 5, 5]
        assert np.abs(f[:, k] - wf).max() <= 1e-12 * np.abs(wf).max(), p
        assert np.abs(g[:, k] - wg).max() <= 1e-12 * np.abs(wg).max(), p
    assert np.isfinite(stats).all()
