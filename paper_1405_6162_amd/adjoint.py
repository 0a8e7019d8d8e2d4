"""Differentiable single-fluid rollout: f_T = step^T(f_0; tau) as a
torch.autograd.Function whose backward runs the hand-written adjoint kernel
(lb_adjoint_step) of the fused collide-stream step.

Memory: the forward keeps only the states at steps 0, K, 2K, ...; the
backward recomputes each segment of at most K steps on the GPU, recording
every step's post-collision field (lb_step_record), and walks it in reverse;
the adjoint kernel pulls f^n from the recorded field, so the recompute costs
one fused step per step and nothing else.  A T-step rollout holds T/K + K
states instead of T.

The loss is ordinary torch code on the returned f_T (for instance the mean
of u.u over the lattice); its gradient arrives as grad_output.
"""

import torch

from . import lb


class LBRollout(torch.autograd.Function):
    """f_T = LBRollout.apply(f0, tau, lattice, nsteps, every).

    f0: (19, nz, ny, nx) float64 device tensor (pre-collision state);
    tau: 0-d float64 tensor (BGK relaxation time, > 1/2);
    lattice: an lb.Lattice with model LB_SINGLE and storage LB_F64, whose
    state this call overwrites; nsteps: T >= 0; every: checkpoint interval
    K >= 1.  Gradients flow to f0 and tau.
    """

    @staticmethod
    def forward(ctx, f0, tau, lattice, nsteps, every):
        if lattice.model != lb.LB_SINGLE or lattice.storage != lb.LB_F64:
            raise ValueError("the adjoint is implemented for the single fluid in FP64")
        if nsteps < 0 or every < 1:
            raise ValueError("nsteps must be >= 0 and every >= 1")
        tau_v = float(tau)
        lattice.set_tau(tau_v)
        lattice.set_state(f0.detach())
        ckpts = [f0.detach().clone()]
        done = 0
        while done < nsteps:
            k = min(every, nsteps - done)
            lattice.step(k)
            done += k
            if done < nsteps:
                ckpts.append(lattice.get_state()[0])
        fT = lattice.get_state()[0] if nsteps > 0 else f0.detach().clone()
        ctx.lattice, ctx.nsteps, ctx.every, ctx.tau = lattice, nsteps, every, tau_v
        ctx.ckpts = ckpts
        return fT

    @staticmethod
    def backward(ctx, grad_fT):
        lat, T, K, tau = ctx.lattice, ctx.nsteps, ctx.every, ctx.tau
        lam = grad_fT.detach().to(torch.float64).contiguous()
        domega = torch.zeros(1, dtype=torch.float64, device=lam.device)
        lat.set_tau(tau)
        nseg = len(ctx.ckpts)
        for seg in range(nseg - 1, -1, -1):
            start = seg * K
            length = min(K, T - start)
            if length <= 0:
                continue
            # recompute the segment: the checkpoint is f^start; the recorded
            # post-collision fields post[k] give f^{start+k+1} in pull form
            ckpt = ctx.ckpts[seg]
            lat.set_state(ckpt)
            post = None
            if length > 1:
                post = torch.empty((length - 1,) + tuple(ckpt.shape), dtype=torch.float64, device=ckpt.device)
                lb.lb_set_stream(lat.ctx, lb._stream())
                lb.lb_step_record(lat.ctx, length - 1, post)
            for n in range(length - 1, -1, -1):
                lam_prev = torch.empty_like(lam)
                lb.lb_set_stream(lat.ctx, lb._stream())
                if n == 0:
                    lb.lb_adjoint_step(lat.ctx, ckpt, lam, lam_prev, domega)
                else:
                    lb.lb_adjoint_step(lat.ctx, post[n - 1], lam, lam_prev, domega, f_pending=True)
                lam = lam_prev
            del post
        grad_tau = (-domega[0] / (tau * tau)).reshape(())
        ctx.ckpts = None
        return lam, grad_tau, None, None, None


def rollout(f0, tau, lattice, nsteps, every=20):
    """Convenience wrapper: LBRollout.apply with a tensor tau."""
    if not torch.is_tensor(tau):
        tau = torch.tensor(float(tau), dtype=torch.float64, device=f0.device)
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
