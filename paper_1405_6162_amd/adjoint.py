"""Differentiable rollouts: the single fluid, f_T = step^T(f_0; tau), and the
binary fluid, (f_T, g_T) from the equilibrium on (rho0, u0, phi0) with
kappa, mobility and tau_f, as torch.autograd.Functions whose backward runs
the hand-written adjoint kernels of the fused collide-stream step, one
library call per checkpoint segment (lb_adjoint_segment,
lb_adjoint_segment_binary; for the binary fluid then lb_adjoint_init_binary).

Memory: the forward keeps only the states at steps 0, K, 2K, ...; the
backward recomputes each segment of at most K steps on the GPU, recording
every step's post-collision field (lb_step_record), and walks it in reverse;
the adjoint kernel pulls f^n from the recorded field, so the recompute costs
one fused step per step and nothing else.  A T-step rollout holds T/K + K
states instead of T.  With every = 0 the forward records every step itself
(one segment, no recompute): T - 1 recorded states (single fluid 19 N
doubles each, binary fluid 39 N with phi; 130 GB for 200 binary steps at
128^3), for a GPU whose memory holds them.

The loss is ordinary torch code on the returned f_T (for instance the mean
of u.u over the lattice); its gradient arrives as grad_output.
"""

import torch

from . import lb


# Relaxation times of f per collision, in the order of the rate sums
# lb_adjoint_step accumulates (and lb_adjoint_step_binary after its omega_g
# and kappa sums).
RATE_NAMES = {lb.LB_BGK: ("tau_f",), lb.LB_TRT: ("tau_f", "tau_minus"),
              lb.LB_MRT: ("tau_f", "tau_minus", "tau_bulk", "tau_ghost_even", "tau_ghost_odd")}


def _relaxation_times(tau, lattice):
    """The rollout's relaxation times as floats, checked against the
    lattice's collision: a 0-d (or one-element) tensor for BGK, two values
    (tau_f, tau_minus) for TRT, five (tau_f, tau_minus, tau_bulk,
    tau_ghost_even, tau_ghost_odd) for MRT."""
    names = RATE_NAMES[lattice.params.collision]
    vals = [float(v) for v in tau.detach().reshape(-1).cpu()]
    if len(vals) != len(names):
        raise ValueError("this lattice's collision takes %d relaxation time(s) (%s), got %d"
                         % (len(names), ", ".join(names), len(vals)))
    return dict(zip(names, vals))


class LBRollout(torch.autograd.Function):
    """f_T = LBRollout.apply(f0, tau, lattice, nsteps, every).

    f0: (19, nz, ny, nx) float64 device tensor (pre-collision state);
    tau: float64 tensor of relaxation times (each > 1/2): 0-d for a BGK
    lattice, (tau_f, tau_minus) for TRT, (tau_f, tau_minus, tau_bulk,
    tau_ghost_even, tau_ghost_odd) for MRT;
    lattice: an lb.Lattice with model LB_SINGLE and storage LB_F64, whose
    state and relaxation times this call overwrites; nsteps: T >= 0; every:
    checkpoint interval K >= 1, or 0 to record every step in the forward
    (no recompute in the backward).  Gradients flow to f0 and tau.
    """

    @staticmethod
    def forward(ctx, f0, tau, lattice, nsteps, every):
        if lattice.model != lb.LB_SINGLE or lattice.storage != lb.LB_F64:
            raise ValueError("the adjoint is implemented for the single fluid in FP64")
        if nsteps < 0 or every < 0:
            raise ValueError("nsteps must be >= 0 and every >= 0")
        taus = _relaxation_times(tau, lattice)
        lattice.set_params(**taus)
        lattice.set_state(f0.detach())
        ckpts = [f0.detach().clone()]
        records = None
        if every == 0:
            # one segment, recorded as the forward runs
            post = None
            if nsteps > 1:
                post = torch.empty((nsteps - 1,) + tuple(f0.shape), dtype=torch.float64, device=f0.device)
                lb.lb_set_stream(lattice.ctx, lb._stream())
                lb.lb_step_record(lattice.ctx, nsteps - 1, post)
            if nsteps > 0:
                lattice.step(1)
            records, every = [post], max(nsteps, 1)
        else:
            done = 0
            while done < nsteps:
                k = min(every, nsteps - done)
                lattice.step(k)
                done += k
                if done < nsteps:
                    ckpts.append(lattice.get_state()[0])
        fT = lattice.get_state()[0] if nsteps > 0 else f0.detach().clone()
        ctx.lattice, ctx.nsteps, ctx.every, ctx.taus = lattice, nsteps, every, taus
        ctx.tau_shape = tau.shape
        ctx.ckpts, ctx.records = ckpts, records
        return fT

    @staticmethod
    def backward(ctx, grad_fT):
        lat, T, K, taus = ctx.lattice, ctx.nsteps, ctx.every, ctx.taus
        lam = grad_fT.detach().to(torch.float64).contiguous().clone()     # updated in place below
        work = torch.empty_like(lam)
        domega = torch.zeros(len(taus), dtype=torch.float64, device=lam.device)
        lat.set_params(**taus)
        nseg = len(ctx.ckpts)
        for seg in range(nseg - 1, -1, -1):
            start = seg * K
            length = min(K, T - start)
            if length <= 0:
                continue
            # recompute the segment: the checkpoint is f^start; the recorded
            # post-collision fields post[k] give f^{start+k+1} in pull form;
            # then one library call walks the segment backwards
            ckpt = ctx.ckpts[seg]
            lb.lb_set_stream(lat.ctx, lb._stream())
            if ctx.records is not None:
                post = ctx.records[seg]                     # recorded by the forward
            else:
                lat.set_state(ckpt)
                post = None
                if length > 1:
                    post = torch.empty((length - 1,) + tuple(ckpt.shape), dtype=torch.float64,
                                       device=ckpt.device)
                    lb.lb_step_record(lat.ctx, length - 1, post)
            lb.lb_adjoint_segment(lat.ctx, ckpt, post, length, lam, work, domega)
            del post
        tv = torch.tensor(list(taus.values()), dtype=torch.float64, device=lam.device)
        grad_tau = (-domega / (tv * tv)).reshape(ctx.tau_shape)
        ctx.ckpts = ctx.records = None
        return lam, grad_tau, None, None, None


class LBBinaryRollout(torch.autograd.Function):
    """(f_T, g_T) = LBBinaryRollout.apply(rho0, u0, phi0, kappa, mobility,
    tau_f, lattice, nsteps, every).

    Binary-fluid rollout from the equilibrium built on (rho0, u0, phi0)
    (float64 device tensors of shapes (nz, ny, nx), (3, nz, ny, nx),
    (nz, ny, nx)), with kappa and mobility as 0-d float64 tensors and tau_f
    0-d (BGK) or the tensor of the lattice's relaxation times of f: on a TRT
    lattice (tau_f, tau_minus), the even and odd times; on an MRT lattice
    (tau_f, tau_minus, tau_bulk, tau_ghost_even, tau_ghost_odd).  lattice:
    an lb.Lattice with model LB_BINARY and storage LB_F64, whose state and
    parameters this call overwrites.  Gradients flow to rho0, u0,
    phi0, kappa, mobility and tau_f.  The backward recomputes each segment of
    at most `every` steps from its checkpoint (every = 0: the forward records
    every step itself, one segment, no recompute), recording every step's
    post-collision f and g, and reverses it in one call
    (lb_adjoint_segment_binary: the local and the stencil adjoint kernel per
    step), then the reverse of the initialisation (lb_adjoint_init_binary).
    """

    @staticmethod
    def forward(ctx, rho0, u0, phi0, kappa, mobility, tau_f, lattice, nsteps, every):
        if lattice.model != lb.LB_BINARY or lattice.storage != lb.LB_F64:
            raise ValueError("the binary adjoint is implemented for the binary fluid in FP64")
        if nsteps < 0 or every < 0:
            raise ValueError("nsteps must be >= 0 and every >= 0")
        names = RATE_NAMES[lattice.params.collision]
        if tuple(tau_f.shape) != ((len(names),) if len(names) > 1 else ()):
            raise ValueError("tau_f must be %s on this lattice" % ("(%s)" % ", ".join(names) if len(names) > 1
                                                                   else "0-d"))
        times = dict(zip(names, (float(t) for t in tau_f.reshape(-1))))
        lattice.set_params(kappa=float(kappa), mobility=float(mobility), **times)
        fields = tuple(t.detach().to(torch.float64).contiguous() for t in (rho0, u0, phi0))
        lattice.init_equilibrium(*fields)
        ckpts = [lattice.get_state()]
        records = None
        if every == 0:
            # one segment, recorded as the forward runs
            post = phi = None
            if nsteps > 1:
                shape = ckpts[0][0].shape
                dev = ckpts[0][0].device
                post = torch.empty((nsteps - 1, 2 * lb.Q) + tuple(shape[1:]), dtype=torch.float64, device=dev)
                phi = torch.empty((nsteps - 1,) + tuple(shape[1:]), dtype=torch.float64, device=dev)
                lb.lb_set_stream(lattice.ctx, lb._stream())
                lb.lb_step_record(lattice.ctx, nsteps - 1, post, phi)
            if nsteps > 0:
                lattice.step(1)
            records, every = [(post, phi)], max(nsteps, 1)
        else:
            done = 0
            while done < nsteps:
                k = min(every, nsteps - done)
                lattice.step(k)
                done += k
                if done < nsteps:
                    ckpts.append(lattice.get_state())
        fT, gT = lattice.get_state() if nsteps > 0 else (ckpts[0][0].clone(), ckpts[0][1].clone())
        ctx.lattice, ctx.nsteps, ctx.every = lattice, nsteps, every
        ctx.ckpts, ctx.fields, ctx.records = ckpts, fields, records
        ctx.params = (float(kappa), float(mobility), times)
        return fT, gT

    @staticmethod
    def backward(ctx, grad_f, grad_g):
        lat, T, K = ctx.lattice, ctx.nsteps, ctx.every
        kappa, mobility, times = ctx.params
        lat.set_params(kappa=kappa, mobility=mobility, **times)
        shape = ctx.ckpts[0][0].shape
        dev = ctx.ckpts[0][0].device
        zero = lambda: torch.zeros(shape, dtype=torch.float64, device=dev)
        # lf, lg are updated in place below: never the caller's gradient tensors
        lf = grad_f.detach().to(torch.float64).contiguous().clone() if grad_f is not None else zero()
        lg = grad_g.detach().to(torch.float64).contiguous().clone() if grad_g is not None else zero()
        work = torch.empty((2 * lb.Q,) + tuple(shape[1:]), dtype=torch.float64, device=dev)
        # dL/domega_f, dL/domega_g, dL/dkappa, then the other times of f (lb.h)
        grads = torch.zeros(3 + len(times) - 1, dtype=torch.float64, device=dev)
        for seg in range(len(ctx.ckpts) - 1, -1, -1):
            start = seg * K
            length = min(K, T - start)
            if length <= 0:
                continue
            f_ck, g_ck = ctx.ckpts[seg]
            lb.lb_set_stream(lat.ctx, lb._stream())
            if ctx.records is not None:
                post, phi = ctx.records[seg]                # recorded by the forward
            else:
                lat.set_state(f_ck, g_ck)
                post = phi = None
                if length > 1:
                    # post[k] and phi[k] (phi of the state step k collides) for k < length - 1;
                    # the last step's phi is computed by the sweep itself
                    post = torch.empty((length - 1, 2 * lb.Q) + tuple(shape[1:]), dtype=torch.float64,
                                       device=dev)
                    phi = torch.empty((length - 1,) + tuple(shape[1:]), dtype=torch.float64, device=dev)
                    lb.lb_step_record(lat.ctx, length - 1, post, phi)
            lb.lb_adjoint_segment_binary(lat.ctx, f_ck, g_ck, post, phi, length, lf, lg, work, grads)
            del post, phi
        rho0, u0, phi0 = ctx.fields
        dphi, drho, du = torch.empty_like(phi0), torch.empty_like(rho0), torch.empty_like(u0)
        dkappa0 = torch.zeros(1, dtype=torch.float64, device=dev)
        lb.lb_set_stream(lat.ctx, lb._stream())
        lb.lb_adjoint_init_binary(lat.ctx, rho0, u0, phi0, lf, lg, dphi, drho, du, dkappa0)
        tau_g = mobility / lat.params.gamma + 0.5
        g_kappa = (grads[2] + dkappa0[0]).reshape(())
        g_mob = (-grads[1] / (tau_g * tau_g) / lat.params.gamma).reshape(())
        # tau_f's sum is grads[0], the further times' are grads[3:]
        rate_sums = torch.cat([grads[:1], grads[3:]])
        tv = torch.tensor(list(times.values()), dtype=torch.float64, device=dev)
        g_tau = (-rate_sums / (tv * tv)).reshape(() if len(times) == 1 else (len(times),))
        ctx.ckpts = ctx.fields = ctx.records = None
        return drho, du, dphi, g_kappa, g_mob, g_tau, None, None, None


def rollout_binary(rho0, u0, phi0, lattice, nsteps, every=20, kappa=None, mobility=None, tau_f=None):
    """Convenience wrapper: LBBinaryRollout.apply with tensor parameters
    (defaults: the lattice's current values; on a TRT or MRT lattice tau_f
    is the tensor of its relaxation times of f)."""
    dev = phi0.device
    as_t = lambda v, d: v if torch.is_tensor(v) else torch.tensor(float(d if v is None else v),
                                                                   dtype=torch.float64, device=dev)
    names = RATE_NAMES[lattice.params.collision]
    if len(names) > 1 and not torch.is_tensor(tau_f):
        vals = [getattr(lattice.params, k) for k in names] if tau_f is None else tau_f
        tau_f = torch.tensor([float(t) for t in vals], dtype=torch.float64, device=dev)
    return LBBinaryRollout.apply(rho0, u0, phi0, as_t(kappa, lattice.params.kappa),
                                 as_t(mobility, lattice.params.mobility), as_t(tau_f, lattice.params.tau_f),
                                 lattice, int(nsteps), int(every))


def binary_loss(f, g, beta=1.0):
    """Mean over the lattice of u.u + beta phi^2, as torch ops."""
    c = velocity_table(f.device, f.dtype)
    rho = f.sum(0)
    u = torch.tensordot(c.t(), f, dims=1) / rho
    phi = g.sum(0)
    return ((u * u).sum(0) + beta * phi * phi).mean()


def rollout(f0, tau, lattice, nsteps, every=20):
    """Convenience wrapper: LBRollout.apply with tau as a tensor (a number,
    or a sequence of the lattice's relaxation times, is converted)."""
    if not torch.is_tensor(tau):
        tau = torch.tensor([float(t) for t in tau] if isinstance(tau, (list, tuple)) else float(tau),
                           dtype=torch.float64, device=f0.device)
    return LBRollout.apply(f0, tau, lattice, int(nsteps), int(every))


def velocity_loss(f):
    """Mean of u.u over the lattice for a (19, nz, ny, nx) distribution, as
    torch ops (differentiable); the D3Q19 velocities come from the library's
    ordering."""
    c = velocity_table(f.device, f.dtype)
    rho = f.sum(0)
    j = torch.tensordot(c.t(), f, dims=1)          # (3, nz, ny, nx)
    u = j / rho
    return (u * u).sum(0).mean()


def velocity_table(device, dtype=torch.float64):
    """(19, 3) D3Q19 velocities in the library's order: rest first, then the
    18 velocities with |c|^2 in {1, 2} in lexicographic order of (cx, cy, cz)."""
    vel = [(0, 0, 0)]
    for cx in (-1, 0, 1):
        for cy in (-1, 0, 1):
            for cz in (-1, 0, 1):
                if cx * cx + cy * cy + cz * cz in (1, 2):
                    vel.append((cx, cy, cz))
    return torch.tensor(vel, dtype=dtype, device=device)
