"""Adjoint parity at the benchmarked sizes on sampled sites: one binary
adjoint step at 128^3 and one single-fluid adjoint step at 64^3, for each
collision, with the state given directly or as the previous step's
post-collision fields (pulled).  Every input field is a smooth analytic
function of the coordinates, so the oracle can rebuild any site's
neighbourhood on the host.  A binary adjoint step at site s reads the adjoint
fields within two sites of s and the state within two sites (three when it is
pulled); the single-fluid step reads one (two).  The centre of a periodic
9^3 block cut around s therefore comes out of the oracle exactly as in the
full lattice.  Sampled sites include the lattice corners (every wrap) and
seeded random sites; the global rate sums are checked to be finite."""

import numpy as np
import pytest
import torch

from oracle import lb_oracle as O

pytestmark = pytest.mark.gpu

TWO_PI = 2.0 * np.pi
R = 4                                             # block radius
TAUS = {"bgk": None, "trt": (0.9, 1.3, 0.9, 0.9, 1.3), "mrt": (0.9, 1.3, 1.4, 0.85, 1.15)}


def _wave(i):
    """Integer wave numbers and a phase for direction i."""
    return (i % 3) + 1, (2 * i) % 5 + 1, (3 * i) % 7 + 1, 0.1 * i


def _fields(x, y, z, n, lib, binary):
    """f, g, lambda_f, lambda_g (each a list of 19 arrays) at integer
    coordinates on an (nx, ny, nz) lattice; lib is numpy or torch."""
    nx, ny, nz = n
    X, Y, Z = x / nx, y / ny, z / nz
    phi = 0.05 * lib.sin(TWO_PI * (X + 2 * Y)) * lib.cos(TWO_PI * 3 * Z)
    f, g, lf, lg = [], [], [], []
    for i in range(19):
        a, b, c, ph = _wave(i)
        w = float(O.W[i])
        f.append(w * (1.0 + 0.01 * lib.sin(TWO_PI * (a * X + b * Y + c * Z) + ph)))
        lf.append(lib.sin(TWO_PI * (b * X + c * Y + a * Z) + 3 * ph))
        if binary:
            g.append(w * phi + 0.001 * w * lib.cos(TWO_PI * (c * X + a * Y + b * Z) + ph))
            lg.append(lib.cos(TWO_PI * (a * X + c * Y + b * Z) + 2 * ph))
    return f, g, lf, lg


def _device(n, binary):
    nx, ny, nz = n
    d = dict(dtype=torch.float64, device="cuda")
    z = torch.arange(nz, **d).view(nz, 1, 1)
    y = torch.arange(ny, **d).view(1, ny, 1)
    x = torch.arange(nx, **d).view(1, 1, nx)
    shape = (nz, ny, nx)
    return [torch.stack([a.expand(shape) for a in arrs]).contiguous() if arrs else None
            for arrs in _fields(x, y, z, n, torch, binary)]


def _block(site, n, binary):
    nx, ny, nz = n
    x0, y0, z0 = site
    off = np.arange(-R, R + 1)
    z = ((z0 + off) % nz).astype(np.float64).reshape(-1, 1, 1)
    y = ((y0 + off) % ny).astype(np.float64).reshape(1, -1, 1)
    x = ((x0 + off) % nx).astype(np.float64).reshape(1, 1, -1)
    shape = (2 * R + 1,) * 3
    return [np.stack([np.broadcast_to(a, shape) for a in arrs]) if arrs else None
            for arrs in _fields(x, y, z, n, np, binary)]


def _samples(n, count, seed):
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    pts = [(0, 0, 0), (nx - 1, ny - 1, nz - 1), (nx - 1, 0, nz - 1), (0, ny - 1, 0)]
    pts += [tuple(int(v) for v in (rng.integers(nx), rng.integers(ny), rng.integers(nz))) for _ in range(count)]
    return pts


def _at(t, pts):
    return np.stack([t[:, z, y, x].cpu().numpy() for (x, y, z) in pts], axis=1)


def _times(lbgpu, coll):
    t = TAUS[coll]
    if t is None:
        return dict(tau_f=0.9)
    kw = dict(collision=lbgpu.LB_TRT if coll == "trt" else lbgpu.LB_MRT, tau_f=t[0], tau_minus=t[1])
    if coll == "mrt":
        kw.update(tau_bulk=t[2], tau_ghost_even=t[3], tau_ghost_odd=t[4])
    return kw


@pytest.mark.parametrize("pending", [False, True])
@pytest.mark.parametrize("coll", ["bgk", "trt", "mrt"])
def test_binary_adjoint_step_128(lbgpu, coll, pending):
    n = (128, 128, 128)
    print("case binary adjoint 128^3", coll, "pending" if pending else "direct", flush=True)
    prm = O.Params(tau_f=0.9, kappa=0.05, mobility=0.3)
    lat = lbgpu.Lattice(*n, model=lbgpu.LB_BINARY, kappa=prm.kappa, mobility=prm.mobility, **_times(lbgpu, coll))
    f, g, lf, lg = _device(n, True)
    lf_n, lg_n = torch.empty_like(lf), torch.empty_like(lg)
    grads = torch.zeros({"bgk": 3, "trt": 4, "mrt": 7}[coll], dtype=torch.float64, device="cuda")
    lbgpu.lb_set_stream(lat.ctx, lbgpu._stream())
    lbgpu.lb_adjoint_step_binary(lat.ctx, f, g, lf, lg, lf_n, lg_n, grads, pending=pending)
    pts = _samples(n, 8, seed=31)
    got_f, got_g = _at(lf_n, pts), _at(lg_n, pts)
    assert torch.isfinite(grads).all()
    lat.close()
    for k, p in enumerate(pts):
        bf, bg, blf, blg = _block(p, n, True)
        if pending:
            bf, bg = O.propagate(bf), O.propagate(bg)
        wf, wg, _gr = O.adjoint_step_binary(bf, bg, blf, blg, prm, TAUS[coll])
        wf, wg = wf[:, R, R, R], wg[:, R, R, R]
        assert np.abs(got_f[:, k] - wf).max() <= 1e-12 * np.abs(wf).max(), p
        assert np.abs(got_g[:, k] - wg).max() <= 1e-12 * np.abs(wg).max(), p


@pytest.mark.parametrize("pending", [False, True])
@pytest.mark.parametrize("coll", ["bgk", "trt", "mrt"])
def test_single_adjoint_step_64(lbgpu, coll, pending):
    n = (64, 64, 64)
    print("case single adjoint 64^3", coll, "pending" if pending else "direct", flush=True)
    lat = lbgpu.Lattice(*n, **_times(lbgpu, coll))
    f, _g, lam, _lg = _device(n, False)
    lam_n = torch.empty_like(lam)
    domega = torch.zeros({"bgk": 1, "trt": 2, "mrt": 5}[coll], dtype=torch.float64, device="cuda")
    lbgpu.lb_set_stream(lat.ctx, lbgpu._stream())
    lbgpu.lb_adjoint_step(lat.ctx, f, lam, lam_n, domega, f_pending=pending)
    pts = _samples(n, 8, seed=32)
    got = _at(lam_n, pts)
    assert torch.isfinite(domega).all()
    lat.close()
    for k, p in enumerate(pts):
        bf, _bg, bl, _blg = _block(p, n, False)
        if pending:
            bf = O.propagate(bf)
        if coll == "bgk":
            want, _dw = O.adjoint_step_single(bf, bl, 0.9)
        else:
            want, _dw = O.adjoint_step_single_mrt(bf, bl, TAUS[coll])
        want = want[:, R, R, R]
        assert np.abs(got[:, k] - want).max() <= 1e-12 * np.abs(want).max(), p
