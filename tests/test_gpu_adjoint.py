"""Adjoint (reverse) of the single-fluid FP64 step on the GPU, against the
oracle's hand-derived adjoint (itself pinned by complex-step derivatives)
and against central finite differences of the GPU forward."""

import numpy as np
import pytest
import torch

from oracle import lb_oracle as O
from paper_1405_6162_amd import inputs

pytestmark = pytest.mark.gpu


def relerr(a, ref):
    return float(np.abs(np.asarray(a) - ref).max() / np.abs(ref).max())


def _state(nx, ny, nz, seed, noise=1e-3):
    rho, u = inputs.shear_wave(nx, ny, nz, amplitude=0.01, noise=noise, seed=seed)
    f = O.init_single(rho, u)
    rng = np.random.default_rng(seed + 50)
    return f + 1e-4 * rng.standard_normal(f.shape) * O.W[:, None, None, None]


@pytest.mark.parametrize("nx,ny,nz", [(4, 4, 4), (5, 6, 7), (67, 9, 5), (16, 16, 16)])
def test_adjoint_step_kernel(lbgpu, nx, ny, nz):
    print("case adjoint step", nx, ny, nz, flush=True)
    tau = 0.8
    f = _state(nx, ny, nz, seed=1)
    rng = np.random.default_rng(2)
    lam_next = rng.standard_normal(f.shape)
    want, want_dw = O.adjoint_step_single(f, lam_next, tau)
    lat = lbgpu.Lattice(nx, ny, nz, tau_f=tau)
    dev = lambda a: torch.as_tensor(a, device="cuda").contiguous()
    ft, lt = dev(f), dev(lam_next)
    out = torch.empty_like(lt)
    dw = torch.full((1,), 0.25, dtype=torch.float64, device="cuda")   # the call increments it
    lbgpu.lb_set_stream(lat.ctx, lbgpu._stream())
    lbgpu.lb_adjoint_step(lat.ctx, ft, lt, out, dw)
    assert relerr(out.cpu().numpy(), want) < 1e-12
    assert abs(dw.item() - 0.25 - want_dw) <= 1e-12 * max(abs(want_dw), np.abs(want).max())


def test_adjoint_step_from_pending_field(lbgpu):
    """f_pending: the kernel pulls f^n from the previous step's post-collision
    field; same result as giving f^n itself."""
    nx, ny, nz, tau = 9, 6, 5, 0.85
    f = _state(nx, ny, nz, seed=7)
    post = O.collide_single(f, tau)                  # f^{n} = propagate(post)
    fn = O.propagate(post)
    rng = np.random.default_rng(8)
    lam_next = rng.standard_normal(f.shape)
    want, want_dw = O.adjoint_step_single(fn, lam_next, tau)
    lat = lbgpu.Lattice(nx, ny, nz, tau_f=tau)
    dev = lambda a: torch.as_tensor(a, device="cuda").contiguous()
    out = torch.empty_like(dev(lam_next))
    dw = torch.zeros(1, dtype=torch.float64, device="cuda")
    lbgpu.lb_set_stream(lat.ctx, lbgpu._stream())
    lbgpu.lb_adjoint_step(lat.ctx, dev(post), dev(lam_next), out, dw, f_pending=True)
    assert relerr(out.cpu().numpy(), want) < 1e-12
    assert abs(dw.item() - want_dw) <= 1e-12 * max(abs(want_dw), np.abs(want).max())


@pytest.mark.parametrize("pending_start", [False, True])
def test_step_record(lbgpu, pending_start):
    """lb_step_record leaves the state of lb_step and records, per step, the
    post-collision field whose propagation is the next state."""
    nx, ny, nz, tau, n = 7, 5, 6, 0.9, 4
    f0 = _state(nx, ny, nz, seed=9)
    lat = lbgpu.Lattice(nx, ny, nz, tau_f=tau)
    lat.set_state(f0)
    ref = f0
    if pending_start:
        lat.step(1)
        ref = O.step_single(ref, tau, 1)
    post = torch.empty((n, 19, nz, ny, nx), dtype=torch.float64, device="cuda")
    lbgpu.lb_set_stream(lat.ctx, lbgpu._stream())
    lbgpu.lb_step_record(lat.ctx, n, post)
    p = post.cpu().numpy()
    for k in range(n):
        c = O.collide_single(ref, tau)
        assert relerr(p[k], c) < 1e-12
        ref = O.propagate(c)
    assert relerr(lat.get_state()[0].cpu().numpy(), ref) < 1e-12
    lat.step(2)
    assert relerr(lat.get_state()[0].cpu().numpy(), O.step_single(ref, tau, 2)) < 1e-12


@pytest.mark.parametrize("nsteps,every", [(7, 3), (7, 7), (7, 1), (6, 2), (0, 4)])
def test_rollout_gradient_vs_oracle(lbgpu, nsteps, every):
    from paper_1405_6162_amd.adjoint import rollout, velocity_loss
    nx, ny, nz, tau = 8, 8, 8, 0.8
    f0 = _state(nx, ny, nz, seed=3)
    loss_o, g_o, dtau_o = O.rollout_gradient(f0, tau, nsteps)
    lat = lbgpu.Lattice(nx, ny, nz, tau_f=tau)
    f0t = torch.tensor(f0, device="cuda", requires_grad=True)
    taut = torch.tensor(tau, dtype=torch.float64, device="cuda", requires_grad=True)
    loss = velocity_loss(rollout(f0t, taut, lat, nsteps, every))
    loss.backward()
    assert abs(loss.item() - loss_o) <= 1e-12 * loss_o
    assert relerr(f0t.grad.cpu().numpy(), g_o) < 1e-10
    if nsteps > 0:
        assert abs(taut.grad.item() - dtau_o) <= 1e-10 * abs(dtau_o)
    else:
        assert taut.grad.item() == 0.0


def test_shear_wave_64_adjoint_vs_finite_differences(lbgpu):
    """64^3, u_x = 0.01 sin(2 pi y / 64) + U(-1e-4, 1e-4) noise on each
    component, rho = 1, f = f^eq, tau = 0.8 (learnable), 200 steps, loss =
    mean u.u at the final step, checkpoints every 20 steps.  Gradients with
    respect to 20 random components of f0 and tau against central
    differences (eps = 1e-6) of the GPU forward."""
    from paper_1405_6162_amd.adjoint import rollout, velocity_loss
    n, tau, T, K, eps = 64, 0.8, 200, 20, 1e-6
    rho, u = inputs.shear_wave(n, n, n, amplitude=0.01, noise=1e-4, seed=0)
    lat = lbgpu.Lattice(n, n, n, tau_f=tau)
    lat.init_equilibrium(rho, u)
    f0 = lat.get_state()[0].clone()
    f0t = f0.clone().requires_grad_(True)
    taut = torch.tensor(tau, dtype=torch.float64, device="cuda", requires_grad=True)
    loss = velocity_loss(rollout(f0t, taut, lat, T, K))
    loss.backward()
    g = f0t.grad.reshape(19, -1)
    # closed-form estimate: viscous decay exp(-2 nu k^2 T), nu = (tau - 1/2)/3
    k = 2 * np.pi / n
    est = 0.5 * 0.01 ** 2 * np.exp(-2 * (tau - 0.5) / 3 * k * k * T)
    assert abs(loss.item() / est - 1) < 0.05

    def L(f, t):
        lat.set_tau(t)
        lat.set_state(f)
        lat.step(T)
        return velocity_loss(lat.get_state()[0]).item()

    comps = inputs.sample_components(n ** 3, 20, seed=1)
    gmax = g.abs().max().item()
    worst = 0.0
    for (i, s) in comps:
        fp, fm = f0.clone(), f0.clone()
        fp.view(19, -1)[i, s] += eps
        fm.view(19, -1)[i, s] -= eps
        fd = (L(fp, tau) - L(fm, tau)) / (2 * eps)
        err = abs(fd - g[i, s].item())
        worst = max(worst, err / (abs(fd) + 1e-5 * gmax))
        # 1e-6 relative, with a floor of 1e-5 max|g| for components near zero
        assert err <= 1e-6 * abs(fd) + 1e-5 * gmax, (i, s, fd, g[i, s].item())
    fd_tau = (L(f0, tau + eps) - L(f0, tau - eps)) / (2 * eps)
    print("adjoint vs FD: worst component %.2e, tau rel %.2e (dL/dtau %.4e)"
          % (worst, abs(fd_tau - taut.grad.item()) / abs(fd_tau), taut.grad.item()), flush=True)
    assert abs(fd_tau - taut.grad.item()) <= 1e-6 * abs(fd_tau)


@pytest.mark.parametrize("length", [1, 2, 5])
def test_segment_sweep_equals_per_step_calls(lbgpu, length):
    """lb_adjoint_segment over a recorded segment: the same kernels in the
    same order as `length` per-step calls, so equal bit for bit (lambda and
    the accumulated dL/domega), whichever buffer the last step lands in; and
    the oracle's reverse sweep over the same states."""
    nx, ny, nz, tau = 67, 9, 5, 0.85
    print("case single segment length=%d" % length, flush=True)
    f0 = _state(nx, ny, nz, seed=21)
    rng = np.random.default_rng(22)
    lam_T = rng.standard_normal(f0.shape)
    lat = lbgpu.Lattice(nx, ny, nz, tau_f=tau)
    lat.set_state(f0)
    dev = lambda a: torch.as_tensor(a, device="cuda").contiguous()
    f0t = dev(f0)
    post = None
    if length > 1:
        post = torch.empty((length - 1, 19, nz, ny, nx), dtype=torch.float64, device="cuda")
        lbgpu.lb_set_stream(lat.ctx, lbgpu._stream())
        lbgpu.lb_step_record(lat.ctx, length - 1, post)
    # per-step calls
    lam = dev(lam_T)
    dw_steps = torch.full((1,), 0.125, dtype=torch.float64, device="cuda")
    for n in range(length - 1, -1, -1):
        out = torch.empty_like(lam)
        if n == 0:
            lbgpu.lb_adjoint_step(lat.ctx, f0t, lam, out, dw_steps)
        else:
            lbgpu.lb_adjoint_step(lat.ctx, post[n - 1], lam, out, dw_steps, f_pending=True)
        lam = out
    # one segment call
    lam_seg = dev(lam_T)
    work = torch.empty_like(lam_seg)
    dw_seg = torch.full((1,), 0.125, dtype=torch.float64, device="cuda")
    lbgpu.lb_adjoint_segment(lat.ctx, f0t, post, length, lam_seg, work, dw_seg)
    assert torch.equal(lam_seg, lam)
    assert torch.equal(dw_seg, dw_steps)
    # the oracle over the same states
    states = [f0]
    for _ in range(length - 1):
        states.append(O.step_single(states[-1], tau, 1))
    lam_o, dw_o = lam_T, 0.0
    for n in range(length - 1, -1, -1):
        lam_o, d = O.adjoint_step_single(states[n], lam_o, tau)
        dw_o += d
    assert relerr(lam_seg.cpu().numpy(), lam_o) < 1e-12
    assert abs(dw_seg.item() - 0.125 - dw_o) <= 1e-12 * max(abs(dw_o), np.abs(lam_o).max())


# ---------------------------------------------------------------------------
# TRT and MRT: the same kernel with mu = Omega lambda* in place of
# omega lambda*, and one rate sum per relaxation time
# ---------------------------------------------------------------------------

MRT_TAUS = (0.8, 1.1, 1.3, 0.9, 1.2)        # tau_f (shear), tau_minus (flux), tau_bulk, ghost even, ghost odd
TRT_TAUS = (0.85, 1.15)


def _collision_lattice(lbgpu, nx, ny, nz, coll):
    if coll == "trt":
        return lbgpu.Lattice(nx, ny, nz, collision=lbgpu.LB_TRT, tau_f=TRT_TAUS[0], tau_minus=TRT_TAUS[1])
    t = MRT_TAUS
    return lbgpu.Lattice(nx, ny, nz, collision=lbgpu.LB_MRT, tau_f=t[0], tau_minus=t[1], tau_bulk=t[2],
                         tau_ghost_even=t[3], tau_ghost_odd=t[4])


def _oracle_taus(coll):
    """The five MRT times of the collision (TRT: the even ones tied to tau_f,
    the odd ones to tau_minus) and how the oracle's group sums add up to the
    library's rate sums."""
    if coll == "trt":
        tp, tm = TRT_TAUS
        return (tp, tm, tp, tp, tm), [("shear", "bulk", "ghost_even"), ("flux", "ghost_odd")]
    return MRT_TAUS, [(k,) for k in O.MRT_RATES]


@pytest.mark.parametrize("pending", [False, True])
@pytest.mark.parametrize("coll", ["trt", "mrt"])
@pytest.mark.parametrize("nx,ny,nz", [(5, 6, 7), (67, 9, 5)])
def test_adjoint_step_kernel_trt_mrt(lbgpu, nx, ny, nz, coll, pending):
    print("case adjoint step", coll, nx, ny, nz, "pending" if pending else "direct", flush=True)
    taus, groups = _oracle_taus(coll)
    f = _state(nx, ny, nz, seed=31)
    src = O.collide_single_mrt(f, taus) if pending else f     # pending: f^n = propagate(src)
    fn = O.propagate(src) if pending else f
    lam_next = np.random.default_rng(32).standard_normal(f.shape)
    want, g = O.adjoint_step_single_mrt(fn, lam_next, taus)
    want_dw = [sum(g[k] for k in grp) for grp in groups]
    lat = _collision_lattice(lbgpu, nx, ny, nz, coll)
    dev = lambda a: torch.as_tensor(a, device="cuda").contiguous()
    out = torch.empty_like(dev(lam_next))
    dw = torch.full((len(groups),), 0.5, dtype=torch.float64, device="cuda")      # incremented
    lbgpu.lb_set_stream(lat.ctx, lbgpu._stream())
    lbgpu.lb_adjoint_step(lat.ctx, dev(src), dev(lam_next), out, dw, f_pending=pending)
    assert relerr(out.cpu().numpy(), want) < 1e-12
    got = dw.cpu().numpy() - 0.5
    for k in range(len(groups)):
        assert abs(got[k] - want_dw[k]) <= 1e-12 * max(abs(want_dw[k]), np.abs(want).max()), (coll, k)


@pytest.mark.parametrize("coll", ["trt", "mrt"])
def test_segment_sweep_trt_mrt_equals_per_step_calls(lbgpu, coll):
    nx, ny, nz, length = 13, 7, 6, 4
    f0 = _state(nx, ny, nz, seed=33)
    lam_T = np.random.default_rng(34).standard_normal(f0.shape)
    lat = _collision_lattice(lbgpu, nx, ny, nz, coll)
    lat.set_state(f0)
    dev = lambda a: torch.as_tensor(a, device="cuda").contiguous()
    f0t = dev(f0)
    post = torch.empty((length - 1, 19, nz, ny, nx), dtype=torch.float64, device="cuda")
    lbgpu.lb_set_stream(lat.ctx, lbgpu._stream())
    lbgpu.lb_step_record(lat.ctx, length - 1, post)
    K = 2 if coll == "trt" else 5
    lam, dw = dev(lam_T), torch.zeros(K, dtype=torch.float64, device="cuda")
    for n in range(length - 1, -1, -1):
        out = torch.empty_like(lam)
        if n == 0:
            lbgpu.lb_adjoint_step(lat.ctx, f0t, lam, out, dw)
        else:
            lbgpu.lb_adjoint_step(lat.ctx, post[n - 1], lam, out, dw, f_pending=True)
        lam = out
    lam_s, dw_s = dev(lam_T), torch.zeros(K, dtype=torch.float64, device="cuda")
    lbgpu.lb_adjoint_segment(lat.ctx, f0t, post, length, lam_s, torch.empty_like(lam_s), dw_s)
    assert torch.equal(lam_s, lam) and torch.equal(dw_s, dw)


@pytest.mark.parametrize("coll", ["trt", "mrt"])
def test_rollout_gradient_trt_mrt_vs_oracle(lbgpu, coll):
    """The checkpointed rollout on a TRT / MRT lattice against the oracle's
    plain reverse sweep: dL/df0 and dL/dtau for every relaxation time."""
    from paper_1405_6162_amd.adjoint import rollout, velocity_loss
    nx, ny, nz, T, K = 8, 8, 8, 7, 3
    taus, groups = _oracle_taus(coll)
    f0 = _state(nx, ny, nz, seed=35)
    loss_o, g_o, dtau_o = O.rollout_gradient_mrt(f0, taus, T)
    # d/dtau_f of a TRT lattice moves the three even groups together: sum of
    # their dL/domega, converted with the shared tau
    lib_taus = TRT_TAUS if coll == "trt" else MRT_TAUS
    want_tau = []
    for grp, t in zip(groups, lib_taus):
        dom = sum(-dtau_o[k] * taus[O.MRT_RATES.index(k)] ** 2 for k in grp)   # dL/domega of the group
        want_tau.append(-dom / (t * t))
    lat = _collision_lattice(lbgpu, nx, ny, nz, coll)
    f0t = torch.tensor(f0, device="cuda", requires_grad=True)
    taut = torch.tensor(lib_taus, dtype=torch.float64, device="cuda", requires_grad=True)
    loss = velocity_loss(rollout(f0t, taut, lat, T, K))
    loss.backward()
    assert abs(loss.item() - loss_o) <= 1e-12 * loss_o
    assert relerr(f0t.grad.cpu().numpy(), g_o) < 1e-10
    got = taut.grad.cpu().numpy()
    for k in range(len(groups)):
        assert abs(got[k] - want_tau[k]) <= 1e-10 * abs(want_tau[k]), (coll, k)


def test_mrt_shear_wave_32_adjoint_vs_finite_differences(lbgpu):
    """MRT at 32^3: a shear wave with noise, 60 steps, checkpoints every 20;
    dL/df0 on sampled components and dL/dtau for all five relaxation times
    against central differences (eps 1e-6) of the GPU forward."""
    from paper_1405_6162_amd.adjoint import rollout, velocity_loss
    n, T, K, eps = 32, 60, 20, 1e-6
    rho, u = inputs.shear_wave(n, n, n, amplitude=0.01, noise=1e-3, seed=36)
    lat = _collision_lattice(lbgpu, n, n, n, "mrt")
    lat.init_equilibrium(rho, u)
    f0 = lat.get_state()[0].clone()
    f0t = f0.clone().requires_grad_(True)
    taut = torch.tensor(MRT_TAUS, dtype=torch.float64, device="cuda", requires_grad=True)
    loss = velocity_loss(rollout(f0t, taut, lat, T, K))
    loss.backward()
    g = f0t.grad.reshape(19, -1)
    names = ("tau_f", "tau_minus", "tau_bulk", "tau_ghost_even", "tau_ghost_odd")

    def L(f, taus):
        lat.set_params(**dict(zip(names, taus)))
        lat.set_state(f)
        lat.step(T)
        return velocity_loss(lat.get_state()[0]).item()

    # 1e-6 relative, with a floor at the rounding of a central difference in
    # FP64: each loss carries a few ulp, divided by 2 eps
    floor = 4 * np.finfo(np.float64).eps * abs(loss.item()) / eps
    for (i, s) in inputs.sample_components(n ** 3, 6, seed=37):
        fp, fm = f0.clone(), f0.clone()
        fp.reshape(19, -1)[i, s] += eps
        fm.reshape(19, -1)[i, s] -= eps
        fd = (L(fp, MRT_TAUS) - L(fm, MRT_TAUS)) / (2 * eps)
        assert abs(fd - g[i, s].item()) <= 1e-6 * abs(g[i, s].item()) + floor, (i, s, fd, g[i, s].item())
    for k in range(5):
        tp, tm = list(MRT_TAUS), list(MRT_TAUS)
        tp[k] += eps
        tm[k] -= eps
        fd = (L(f0, tp) - L(f0, tm)) / (2 * eps)
        gk = taut.grad[k].item()
        print("  dL/d%s adjoint %.9e fd %.9e" % (names[k], gk, fd), flush=True)
        assert abs(fd - gk) <= 1e-6 * abs(gk) + floor, names[k]


def test_bindings_refuse_wrong_dtypes(lbgpu):
    """The FP64-only calls check their tensors' dtype before passing raw
    device addresses to the library."""
    lat = lbgpu.Lattice(4, 4, 4)
    f = torch.zeros((19, 4, 4, 4), dtype=torch.float32, device="cuda")
    lam = torch.zeros((19, 4, 4, 4), dtype=torch.float64, device="cuda")
    dw = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(TypeError):
        lbgpu.lb_adjoint_step(lat.ctx, f, lam, torch.empty_like(lam), dw)
    with pytest.raises(TypeError):
        lbgpu.lb_moments(lat.ctx, torch.empty((4, 4, 4), dtype=torch.float32, device="cuda"), None)
    lat.close()
