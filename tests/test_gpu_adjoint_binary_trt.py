"""Adjoint of the binary-fluid FP64 step with f relaxing by two times (TRT):
the local adjoint kernel with mu = Omega lambda*_f, the recorded TRT
recompute, the segment sweep and the checkpointed rollout against the
oracle's moment-space reverse sweep (TRT as the MRT case with the even
groups at tau_plus and the odd at tau_minus; pinned by complex-step
derivatives), and central differences of the GPU forward in the two times."""

import numpy as np
import pytest
import torch

from oracle import lb_oracle as O
from paper_1405_6162_amd import inputs

pytestmark = pytest.mark.gpu

TP, TM = 0.9, 1.3
EVEN, ODD = ("shear", "bulk", "ghost_even"), ("flux", "ghost_odd")


def relerr(a, ref):
    return float(np.abs(np.asarray(a) - ref).max() / np.abs(ref).max())


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def _taus(tp=TP, tm=TM):
    return (tp, tm, tp, tp, tm)


def _fields(nx, ny, nz, seed, phi_max=0.3):
    rho, u, phi = inputs.spinodal_quench(nx, ny, nz, seed=seed, phi_max=phi_max)
    _r, u = inputs.single_fluid_random(nx, ny, nz, seed=seed + 1, u_max=0.02)
    rho = rho + 0.01 * np.cos(2 * np.pi * np.arange(nx) / nx)
    return rho, u, phi


def _state(nx, ny, nz, seed, prm):
    f, g = O.init_binary(*_fields(nx, ny, nz, seed), prm)
    return O.step_binary_mrt(f, g, prm, _taus(), 1)


def _lattice(lbgpu, nx, ny, nz, prm, **kw):
    return lbgpu.Lattice(nx, ny, nz, model=lbgpu.LB_BINARY, collision=lbgpu.LB_TRT, tau_f=TP, tau_minus=TM,
                         A=prm.A, B=prm.B, kappa=prm.kappa, mobility=prm.mobility, gamma=prm.gamma, **kw)


def _lib_grads(want):
    """The oracle's group sums as the library's (omega_f, omega_g, kappa, omega_minus)."""
    return [sum(want["omega_" + k] for k in EVEN), want["omega_g"], want["kappa"],
            sum(want["omega_" + k] for k in ODD)]


@pytest.mark.parametrize("given_phi", [False, True])
@pytest.mark.parametrize("pending", [False, True])
@pytest.mark.parametrize("nx,ny,nz", [(5, 6, 7), (67, 9, 5)])
def test_binary_trt_adjoint_step_kernels(lbgpu, nx, ny, nz, pending, given_phi):
    print("case binary trt adjoint step", nx, ny, nz, pending, given_phi, flush=True)
    prm = O.Params(tau_f=TP, kappa=0.05, mobility=0.3)
    f, g = _state(nx, ny, nz, 1, prm)
    rng = np.random.default_rng(2)
    lf1, lg1 = rng.standard_normal(f.shape), rng.standard_normal(g.shape)
    if pending:                    # the kernel pulls f^n, g^n from the previous post-collision fields
        pf, pg = O.collide_binary_mrt(f, g, prm, _taus())
        fn, gn = O.propagate(pf), O.propagate(pg)
        given_f, given_g = pf, pg
    else:
        fn, gn = f, g
        given_f, given_g = f, g
    want_f, want_g, want = O.adjoint_step_binary(fn, gn, lf1, lg1, prm, _taus())
    lat = _lattice(lbgpu, nx, ny, nz, prm)
    lf, lg = torch.empty_like(dev(lf1)), torch.empty_like(dev(lg1))
    grads = torch.full((4,), 0.5, dtype=torch.float64, device="cuda")     # the call increments it
    lbgpu.lb_set_stream(lat.ctx, lbgpu._stream())
    phi = dev(O.order_parameter(gn)) if given_phi else None
    lbgpu.lb_adjoint_step_binary(lat.ctx, dev(given_f), dev(given_g), dev(lf1), dev(lg1), lf, lg, grads,
                                 pending=pending, phi=phi)
    assert relerr(lf.cpu().numpy(), want_f) < 1e-12
    assert relerr(lg.cpu().numpy(), want_g) < 1e-12
    got = grads.cpu().numpy() - 0.5
    for k, w in enumerate(_lib_grads(want)):
        assert abs(got[k] - w) <= 1e-12 * max(abs(w), 1.0), k


@pytest.mark.parametrize("step_kernel", [1, 2])          # LB_STEP_MARCH, LB_STEP_TWO_PASS
def test_binary_trt_step_record(lbgpu, step_kernel):
    nx, ny, nz, n = 7, 5, 6, 3
    prm = O.Params(tau_f=TP)
    f, g = _state(nx, ny, nz, 5, prm)
    lat = _lattice(lbgpu, nx, ny, nz, prm, binary_step=step_kernel)
    lat.set_state(f, g)
    post = torch.empty((n, 38, nz, ny, nx), dtype=torch.float64, device="cuda")
    phi = torch.empty((n, nz, ny, nx), dtype=torch.float64, device="cuda")
    lbgpu.lb_set_stream(lat.ctx, lbgpu._stream())
    lbgpu.lb_step_record(lat.ctx, n, post, phi)
    p, ph = post.cpu().numpy(), phi.cpu().numpy()
    for k in range(n):
        assert relerr(ph[k], O.order_parameter(g)) < 1e-13
        pf, pg = O.collide_binary_mrt(f, g, prm, _taus())
        assert relerr(p[k, :19], pf) < 1e-12 and relerr(p[k, 19:], pg) < 1e-12
        f, g = O.propagate(pf), O.propagate(pg)
    sf, sg = (a.cpu().numpy() for a in lat.get_state())
    assert relerr(sf, f) < 1e-12 and relerr(sg, g) < 1e-12


def test_binary_trt_segment(lbgpu):
    """lb_adjoint_segment_binary on a recorded TRT segment against the
    oracle's reverse sweep over the same states."""
    nx, ny, nz, length = 67, 9, 5, 4
    prm = O.Params(tau_f=TP, kappa=0.05, mobility=0.3)
    f0, g0 = _state(nx, ny, nz, 23, prm)
    rng = np.random.default_rng(24)
    lf_T, lg_T = rng.standard_normal(f0.shape), rng.standard_normal(g0.shape)
    lat = _lattice(lbgpu, nx, ny, nz, prm)
    lat.set_state(f0, g0)
    lbgpu.lb_set_stream(lat.ctx, lbgpu._stream())
    post = torch.empty((length - 1, 38, nz, ny, nx), dtype=torch.float64, device="cuda")
    phi = torch.empty((length - 1, nz, ny, nx), dtype=torch.float64, device="cuda")
    lbgpu.lb_step_record(lat.ctx, length - 1, post, phi)
    lf, lg = dev(lf_T), dev(lg_T)
    work = torch.empty((38, nz, ny, nx), dtype=torch.float64, device="cuda")
    grads = torch.full((4,), 0.25, dtype=torch.float64, device="cuda")
    lbgpu.lb_adjoint_segment_binary(lat.ctx, dev(f0), dev(g0), post, phi, length, lf, lg, work, grads)
    states = [(f0, g0)]
    for _ in range(length - 1):
        states.append(O.step_binary_mrt(*states[-1], prm, _taus(), 1))
    a, b = lf_T, lg_T
    tot = np.zeros(4)
    for n in range(length - 1, -1, -1):
        a, b, gr = O.adjoint_step_binary(states[n][0], states[n][1], a, b, prm, _taus())
        tot = tot + np.array(_lib_grads(gr))
    assert relerr(lf.cpu().numpy(), a) < 1e-12
    assert relerr(lg.cpu().numpy(), b) < 1e-12
    got = grads.cpu().numpy() - 0.25
    for k in range(4):
        assert abs(got[k] - tot[k]) <= 1e-12 * max(abs(tot[k]), 1.0), k


@pytest.mark.parametrize("T,K", [(5, 2), (4, 4)])
def test_binary_trt_rollout_matches_oracle(lbgpu, T, K):
    """The checkpointed rollout with tau_f = (tau_plus, tau_minus) against
    the oracle's full reverse sweep: dL/dphi0, dL/drho0, dL/du0, kappa, M
    and the two times."""
    from paper_1405_6162_amd.adjoint import binary_loss, rollout_binary
    print("case binary trt rollout T=%d K=%d" % (T, K), flush=True)
    nx, ny, nz = 12, 10, 8
    prm = O.Params(tau_f=TP, kappa=0.04, mobility=0.45)
    rho, u, phi = _fields(nx, ny, nz, seed=8)
    beta = 0.5
    loss_o, dphi_o, drho_o, du_o, g_o = O.rollout_gradient_binary(rho, u, phi, prm, T, beta, taus=_taus())
    lat = _lattice(lbgpu, nx, ny, nz, prm)
    r0, u0, p0 = (dev(a).requires_grad_(True) for a in (rho, u, phi))
    kap, mob = (torch.tensor(v, dtype=torch.float64, device="cuda", requires_grad=True)
                for v in (prm.kappa, prm.mobility))
    tau = torch.tensor([TP, TM], dtype=torch.float64, device="cuda", requires_grad=True)
    fT, gT = rollout_binary(r0, u0, p0, lat, T, K, kap, mob, tau)
    loss = binary_loss(fT, gT, beta)
    assert abs(loss.item() - loss_o) <= 1e-12 * abs(loss_o)
    loss.backward()
    assert relerr(p0.grad.cpu().numpy(), dphi_o) < 1e-11
    assert relerr(r0.grad.cpu().numpy(), drho_o) < 1e-11
    assert relerr(u0.grad.cpu().numpy(), du_o) < 1e-11
    assert abs(kap.grad.item() - g_o["kappa"]) <= 1e-11 * abs(g_o["kappa"])
    assert abs(mob.grad.item() - g_o["mobility"]) <= 1e-11 * abs(g_o["mobility"])
    want = [sum(g_o["tau_" + k] for k in EVEN), sum(g_o["tau_" + k] for k in ODD)]
    got = tau.grad.cpu().numpy()
    for k in range(2):
        assert abs(got[k] - want[k]) <= 1e-11 * abs(want[k]), k


def test_binary_trt_rollout_central_differences_24(lbgpu):
    """24^3 spinodal quench, 12 steps, checkpoints every 5: the two TRT time
    gradients and sampled phi0 components against central differences
    (eps 1e-6) of the GPU forward."""
    from paper_1405_6162_amd.adjoint import binary_loss, rollout_binary
    n, T, K, eps = 24, 12, 5, 1e-6
    prm = O.Params(tau_f=TP)
    rho, u, phi = inputs.spinodal_quench(n, n, n, seed=9, phi_max=0.1)
    _r, u = inputs.single_fluid_random(n, n, n, seed=10, u_max=0.02)
    lat = _lattice(lbgpu, n, n, n, prm)
    p0 = dev(phi).requires_grad_(True)
    tau = torch.tensor([TP, TM], dtype=torch.float64, device="cuda", requires_grad=True)
    loss = binary_loss(*rollout_binary(dev(rho), dev(u), p0, lat, T, K, tau_f=tau), 1.0)
    loss.backward()
    grad, gt = p0.grad.cpu().numpy(), tau.grad.cpu().numpy()

    def L(ph, tp=TP, tm=TM):
        with torch.no_grad():
            t = torch.tensor([tp, tm], dtype=torch.float64, device="cuda")
            return binary_loss(*rollout_binary(dev(rho), dev(u), dev(ph), lat, T, K, tau_f=t), 1.0).item()
    floor = 1e-3 * np.abs(grad).max()
    for (_i, s) in inputs.sample_components(n ** 3, 4, seed=11):
        idx = np.unravel_index(s, phi.shape)
        pp, pm = phi.copy(), phi.copy()
        pp[idx] += eps
        pm[idx] -= eps
        fd = (L(pp) - L(pm)) / (2 * eps)
        assert abs(fd - grad[idx]) <= 1e-6 * max(abs(grad[idx]), floor), (fd, grad[idx])
    fd_p = (L(phi, tp=TP + eps) - L(phi, tp=TP - eps)) / (2 * eps)
    fd_m = (L(phi, tm=TM + eps) - L(phi, tm=TM - eps)) / (2 * eps)
    assert abs(fd_p - gt[0]) <= 1e-6 * abs(gt[0]), (fd_p, gt[0])
    assert abs(fd_m - gt[1]) <= 1e-6 * abs(gt[1]), (fd_m, gt[1])
