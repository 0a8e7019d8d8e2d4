"""The GPU binary-fluid adjoint against the definition of the reverse step.

lambda^n = J^T lambda^{n+1}, J the Jacobian of one whole step, is built by
the oracle column by column from its plain forward
(`adjoint_step_binary_plain`), with none of the hand-derived sums the
kernels use.  The local and stencil adjoint kernels (BGK, TRT and MRT
relaxation of f, state given directly or pulled from the previous step's
post-collision fields) and the reverse of the initialisation are compared
with it on every component and every parameter gradient."""

import numpy as np
import pytest
import torch

from oracle import lb_oracle as O
from paper_1405_6162_amd import inputs

pytestmark = pytest.mark.gpu

NX, NY, NZ = 5, 4, 3
TRT_TAUS = (0.9, 1.3, 0.9, 0.9, 1.3)           # even groups at tau+, odd (flux, odd ghosts) at tau-
MRT_TAUS = (0.9, 1.3, 1.4, 0.85, 1.15)
TAUS = {"bgk": None, "trt": TRT_TAUS, "mrt": MRT_TAUS}
EVEN, ODD = ("shear", "bulk", "ghost_even"), ("flux", "ghost_odd")


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def relerr(a, ref):
    return float(np.abs(np.asarray(a) - ref).max() / np.abs(ref).max())


def _prm(coll):
    t = TAUS[coll]
    return O.Params(tau_f=0.9 if t is None else t[0], kappa=0.05, mobility=0.3)


def _state(coll):
    rho, u, phi = inputs.spinodal_quench(NX, NY, NZ, seed=21, phi_max=0.3)
    _r, u = inputs.single_fluid_random(NX, NY, NZ, seed=22, u_max=0.02)
    rho = rho + 0.01 * np.cos(2 * np.pi * np.arange(NX) / NX)
    prm, t = _prm(coll), TAUS[coll]
    f, g = O.init_binary(rho, u, phi, prm)
    return O.step_binary(f, g, prm, 1) if t is None else O.step_binary_mrt(f, g, prm, t, 1)


def _lattice(lbgpu, coll):
    prm, t = _prm(coll), TAUS[coll]
    kw = dict(A=prm.A, B=prm.B, kappa=prm.kappa, mobility=prm.mobility, gamma=prm.gamma, tau_f=prm.tau_f)
    if coll == "trt":
        kw.update(collision=lbgpu.LB_TRT, tau_minus=t[1])
    elif coll == "mrt":
        kw.update(collision=lbgpu.LB_MRT, tau_minus=t[1], tau_bulk=t[2], tau_ghost_even=t[3], tau_ghost_odd=t[4])
    return lbgpu.Lattice(NX, NY, NZ, model=lbgpu.LB_BINARY, **kw)


def _tau_grads(lib, coll, prm):
    """The library's rate sums (d/d omega, in its order) as derivatives with
    respect to the times the definition perturbs: tau_f or the groups' taus,
    and the mobility (tau_g = M / Gamma + 1/2)."""
    t = TAUS[coll]
    out = {"kappa": lib[2], "mobility": -lib[1] / prm.tau_g ** 2 / prm.gamma}
    if coll == "bgk":
        out["tau_f"] = -lib[0] / prm.tau_f ** 2
    elif coll == "trt":                 # d/d tau+ and d/d tau-: the sums over the tied groups
        out["tau_plus"] = -lib[0] / t[0] ** 2
        out["tau_minus"] = -lib[3] / t[1] ** 2
    else:
        out["tau_shear"] = -lib[0] / t[0] ** 2
        for k, name in enumerate(O.MRT_RATES[1:]):
            out["tau_" + name] = -lib[3 + k] / t[1 + k] ** 2
    return out


def _definition_grads(gr, coll):
    if coll != "trt":
        return gr
    out = {"kappa": gr["kappa"], "mobility": gr["mobility"]}
    out["tau_plus"] = sum(gr["tau_" + k] for k in EVEN)
    out["tau_minus"] = sum(gr["tau_" + k] for k in ODD)
    return out


@pytest.mark.parametrize("pending", [False, True])
@pytest.mark.parametrize("coll", ["bgk", "trt", "mrt"])
def test_binary_adjoint_step_equals_definition(lbgpu, coll, pending):
    print("case binary adjoint step vs definition", coll, "pending" if pending else "direct", flush=True)
    prm, t = _prm(coll), TAUS[coll]
    f, g = _state(coll)
    if pending:                         # the kernel pulls f^n, g^n from the post-collision fields
        pf, pg = O.collide_binary(f, g, prm) if t is None else O.collide_binary_mrt(f, g, prm, t)
        fn, gn = O.propagate(pf), O.propagate(pg)
        given = (pf, pg)
    else:
        fn, gn = f, g
        given = (f, g)
    rng = np.random.default_rng(23)
    lf1, lg1 = rng.standard_normal(f.shape), rng.standard_normal(g.shape)
    want_f, want_g, want = O.adjoint_step_binary_plain(fn, gn, lf1, lg1, prm, t)
    lat = _lattice(lbgpu, coll)
    lf, lg = torch.empty_like(dev(lf1)), torch.empty_like(dev(lg1))
    ng = {"bgk": 3, "trt": 4, "mrt": 7}[coll]
    grads = torch.zeros(ng, dtype=torch.float64, device="cuda")
    lbgpu.lb_set_stream(lat.ctx, lbgpu._stream())
    lbgpu.lb_adjoint_step_binary(lat.ctx, dev(given[0]), dev(given[1]), dev(lf1), dev(lg1), lf, lg, grads,
                                 pending=pending)
    got_f, got_g = lf.cpu().numpy(), lg.cpu().numpy()
    lat.close()
    assert relerr(got_f, want_f) < 1e-12
    assert relerr(got_g, want_g) < 1e-12
    got = _tau_grads(grads.cpu().numpy(), coll, prm)
    want = _definition_grads(want, coll)
    assert set(got) == set(want)
    for name, w in want.items():
        assert abs(got[name] - w) <= 1e-12 * max(abs(w), 1e-3), name


def test_binary_adjoint_init_equals_definition(lbgpu):
    nx, ny, nz = 4, 3, 5
    prm = O.Params(kappa=0.03)
    rho, u, phi = inputs.spinodal_quench(nx, ny, nz, seed=24, phi_max=0.3)
    _r, u = inputs.single_fluid_random(nx, ny, nz, seed=25, u_max=0.02)
    rho = rho + 0.01 * np.sin(2 * np.pi * np.arange(nx) / nx)
    rng = np.random.default_rng(26)
    lf0, lg0 = rng.standard_normal((19, nz, ny, nx)), rng.standard_normal((19, nz, ny, nx))
    want_phi, want_rho, want_u, want_k = O.adjoint_init_binary_plain(rho, u, phi, lf0, lg0, prm)
    lat = lbgpu.Lattice(nx, ny, nz, model=lbgpu.LB_BINARY, kappa=prm.kappa)
    dphi, drho, du = (torch.empty(s, dtype=torch.float64, device="cuda") for s in (phi.shape, rho.shape, u.shape))
    dk = torch.zeros(1, dtype=torch.float64, device="cuda")
    lbgpu.lb_set_stream(lat.ctx, lbgpu._stream())
    lbgpu.lb_adjoint_init_binary(lat.ctx, dev(rho), dev(u), dev(phi), dev(lf0), dev(lg0), dphi, drho, du, dk)
    got = [a.cpu().numpy() for a in (dphi, drho, du)]
    lat.close()
    for name, c, w in zip(("phi", "rho", "u"), got, (want_phi, want_rho, want_u)):
        assert relerr(c, w) < 1e-12, name
    assert abs(dk.item() - want_k) <= 1e-12 * abs(want_k)
