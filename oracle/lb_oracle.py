"""Plain FP64 reference implementation of the D3Q19 lattice-Boltzmann update.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
module: only the tests, the smoke check and the CPU baseline leg of the
benchmark use it.  It shares no code, tables or constants with the HIP
library; the two meet only on the seeded inputs they are both given.  A
second, independent reference of the core step in plain C behind the
library's C ABI (lb_oracle.c) is checked against this one by the tests.

What the paper fixes and what is a reading
------------------------------------------
The paper's benchmark (Section IV, "Application Benchmark Results") is a
lattice-Boltzmann collision for a mixture of two fluids, taken from a
code that couples LB hydrodynamics to a free-energy order parameter whose
gradients are computed by finite differences (Section II-A).  Lattice
fields are double precision, stored structure-of-arrays with consecutive
sites contiguous (Section III-B), and the innermost loops run over the 19
discrete momenta or the 3 spatial dimensions (Section IV).  The paper
prints no equation for any of this, so every formula below is a stated
textbook reading:

* D3Q19 velocity set and weights with c_s^2 = 1/3, and the second-order
  equilibrium of the BGK model (Qian, d'Humieres & Lallemand 1992).
* Symmetric phi^4 free energy F = A/2 phi^2 + B/4 phi^4 + kappa/2 |grad phi|^2,
  chemical potential mu = A phi + B phi^3 - kappa lap(phi) and the chemical
  (thermodynamic) stress P_ab entering the second moment of f^eq, with a
  second distribution g carrying phi (Swift, Osborn & Yeomans 1995;
  Swift, Orlandini, Osborn & Yeomans 1996).
* Second-order 7-point central differences for grad(phi) and lap(phi).
* Collide, then propagate; periodic in x, y and z; the state the user sees
  is the post-propagation (pre-collision) distribution.

Layout: every distribution is an array of shape (19, nz, ny, nx), so the
site index s = x + nx*(y + ny*z) runs fastest in x (Section III-B's
structure-of-arrays field[i*N + s]).  Scalar fields are (nz, ny, nx).

The arithmetic is written so that it also runs on complex128 arrays; the
tests use that for complex-step derivatives of the whole rollout.
"""

from dataclasses import dataclass

import numpy as np

# ---------------------------------------------------------------------------
# D3Q19 velocity set
# ---------------------------------------------------------------------------


def _velocity_set():
    """Rest velocity first, then the 18 velocities with |c|^2 in {1, 2} in
    lexicographic order of (c_x, c_y, c_z).  The paper only says there are
    19 momenta (Section IV); this ordering is a reading, and it is part of
    the interface because gradients with respect to f expose it."""
    vel = [(0, 0, 0)]
    for cx in (-1, 0, 1):
        for cy in (-1, 0, 1):
            for cz in (-1, 0, 1):
                if cx * cx + cy * cy + cz * cz in (1, 2):
                    vel.append((cx, cy, cz))
    return np.array(vel, dtype=np.int64)


C = _velocity_set()                       # (19, 3) integer velocities
NQ = C.shape[0]                           # 19
_C2 = (C * C).sum(axis=1)                 # |c_i|^2
W = np.where(_C2 == 0, 1.0 / 3.0, np.where(_C2 == 1, 1.0 / 18.0, 1.0 / 36.0))
OPP = np.array([int(np.flatnonzero((C == -C[i]).all(axis=1))[0]) for i in range(NQ)])
CS2 = 1.0 / 3.0

# Axis of a (nz, ny, nx) scalar field that each velocity component moves along.
_AXIS_OF_COMPONENT = (2, 1, 0)            # c_x -> axis 2, c_y -> axis 1, c_z -> axis 0


@dataclass
class Params:
    """Physical parameters of one run (plain numbers, no derived state)."""
    tau_f: float = 1.0
    A: float = -0.0625
    B: float = 0.0625
    kappa: float = 0.04
    mobility: float = 0.45
    gamma: float = 1.0

    @property
    def tau_g(self):
        # Cahn-Hilliard mobility M = Gamma (tau_g - 1/2)  =>  tau_g = M/Gamma + 1/2.
        return self.mobility / self.gamma + 0.5


# ---------------------------------------------------------------------------
# Small helpers on periodic scalar fields
# ---------------------------------------------------------------------------


def shift(field, c):
    """Return h with h(s) = field(s - c) on the periodic lattice, i.e. every
    value moved by +c.  `field` is (nz, ny, nx); c = (cx, cy, cz)."""
    out = field
    for comp in range(3):
        if c[comp] != 0:
            out = np.roll(out, int(c[comp]), axis=_AXIS_OF_COMPONENT[comp])
    return out


def neighbour(field, c):
    """Return h with h(s) = field(s + c)."""
    return shift(field, (-int(c[0]), -int(c[1]), -int(c[2])))


# ---------------------------------------------------------------------------
# Moments
# ---------------------------------------------------------------------------


def density(f):
    """rho(s) = sum_i f_i(s)."""
    rho = np.zeros_like(f[0])
    for i in range(NQ):
        rho = rho + f[i]
    return rho


def momentum(f):
    """j_a(s) = sum_i f_i(s) c_ia, returned as a (3, nz, ny, nx) array."""
    j = np.zeros((3,) + f.shape[1:], dtype=f.dtype)
    for i in range(NQ):
        for a in range(3):
            if C[i, a] != 0:
                j[a] = j[a] + C[i, a] * f[i]
    return j


def velocity(f):
    """u = j / rho (no forcing correction: the fluids couple through the
    chemical stress in the equilibrium, not through a body force)."""
    rho = density(f)
    return momentum(f) / rho, rho


def order_parameter(g):
    """phi(s) = sum_i g_i(s)."""
    return density(g)


# ---------------------------------------------------------------------------
# Finite differences and free energy (binary fluid)
# ---------------------------------------------------------------------------


def gradient(phi):
    """Second-order central difference d_a phi = [phi(s+e_a) - phi(s-e_a)] / 2,
    periodic.  Returns (3, nz, ny, nx) ordered (x, y, z)."""
    out = np.zeros((3,) + phi.shape, dtype=phi.dtype)
    for a in range(3):
        e = [0, 0, 0]
        e[a] = 1
        out[a] = 0.5 * (neighbour(phi, e) - neighbour(phi, [-v for v in e]))
    return out


def laplacian(phi):
    """Second-order 7-point Laplacian sum_a [phi(s+e_a) + phi(s-e_a)] - 6 phi(s)."""
    out = -6.0 * phi
    for a in range(3):
        e = [0, 0, 0]
        e[a] = 1
        out = out + neighbour(phi, e) + neighbour(phi, [-v for v in e])
    return out


def chemical_potential(phi, lap, prm):
    """mu = dF/dphi = A phi + B phi^3 - kappa lap(phi)."""
    return prm.A * phi + prm.B * phi ** 3 - prm.kappa * lap


def chemical_stress(phi, grad, lap, prm):
    """Thermodynamic stress of the phi^4 free energy (without the ideal-gas
    rho c_s^2 part, which the equilibrium carries itself):

        P_ab = [A/2 phi^2 + 3B/4 phi^4 - kappa phi lap(phi) - kappa/2 |grad phi|^2] delta_ab
               + kappa d_a phi d_b phi.

    Returned as a (3, 3, nz, ny, nx) array."""
    iso = (0.5 * prm.A * phi ** 2 + 0.75 * prm.B * phi ** 4
           - prm.kappa * phi * lap
           - 0.5 * prm.kappa * (grad[0] ** 2 + grad[1] ** 2 + grad[2] ** 2))
    P = np.zeros((3, 3) + phi.shape, dtype=np.result_type(phi, grad))
    for a in range(3):
        for b in range(3):
            P[a, b] = prm.kappa * grad[a] * grad[b]
        P[a, a] = P[a, a] + iso
    return P


# ---------------------------------------------------------------------------
# Equilibria
# ---------------------------------------------------------------------------


def equilibrium_f(rho, u, P=None):
    """Second-order equilibrium whose moments are rho, rho u and
    rho c_s^2 delta + rho u u + P:

        f^eq_i = w_i { rho [1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u]
                       + 9/2 [c_i.P.c_i - tr(P)/3] }.
    P = None is the single fluid."""
    uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2]
    if P is not None:
        trP = P[0, 0] + P[1, 1] + P[2, 2]
    feq = np.zeros((NQ,) + rho.shape, dtype=np.result_type(rho, u))
    for i in range(NQ):
        cu = C[i, 0] * u[0] + C[i, 1] * u[1] + C[i, 2] * u[2]
        val = rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu)
        if P is not None:
            cPc = np.zeros_like(trP)
            for a in range(3):
                for b in range(3):
                    if C[i, a] != 0 and C[i, b] != 0:
                        cPc = cPc + C[i, a] * C[i, b] * P[a, b]
            val = val + 4.5 * (cPc - trP / 3.0)
        feq[i] = W[i] * val
    return feq


def equilibrium_g(phi, u, mu, prm):
    """Equilibrium of the order-parameter distribution with moments phi,
    phi u and Gamma mu delta + phi u u:

        g^eq_i = w_i { phi [1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u]
                       + 9/2 (Gamma mu - phi/3)(|c_i|^2 - 1) }."""
    uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2]
    geq = np.zeros((NQ,) + phi.shape, dtype=np.result_type(phi, u, mu))
    for i in range(NQ):
        cu = C[i, 0] * u[0] + C[i, 1] * u[1] + C[i, 2] * u[2]
        val = phi * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu)
        val = val + 4.5 * (prm.gamma * mu - phi / 3.0) * (_C2[i] - 1)
        geq[i] = W[i] * val
    return geq


# ---------------------------------------------------------------------------
# Collision, propagation, step
# ---------------------------------------------------------------------------


def bgk(f, feq, tau):
    """BGK relaxation f* = f - (f - f^eq) / tau."""
    return f - (f - feq) / tau


def collide_single(f, tau):
    """Single-fluid BGK collision of every site."""
    u, rho = velocity(f)
    return bgk(f, equilibrium_f(rho, u), tau)


def trt(f, feq, tau_plus, tau_minus):
    """Two-relaxation-time collision (Ginzburg): the parts of f - f^eq even
    and odd under c -> -c relax with 1/tau_plus and 1/tau_minus,
        f^{+-}_i = (f_i +- f_opp(i)) / 2,
        f*_i = f_i - (f^+_i - f^eq+_i)/tau_plus - (f^-_i - f^eq-_i)/tau_minus.
    tau_minus = tau_plus is BGK."""
    fo, eo = f[OPP], feq[OPP]
    fp, fm = 0.5 * (f + fo), 0.5 * (f - fo)
    ep, em = 0.5 * (feq + eo), 0.5 * (feq - eo)
    return f - (fp - ep) / tau_plus - (fm - em) / tau_minus


def collide_single_trt(f, tau_plus, tau_minus):
    """Single-fluid TRT collision of every site."""
    u, rho = velocity(f)
    return trt(f, equilibrium_f(rho, u), tau_plus, tau_minus)


def step_single_trt(f, tau_plus, tau_minus, nsteps=1):
    for _ in range(nsteps):
        f = propagate(collide_single_trt(f, tau_plus, tau_minus))
    return f


# Multiple-relaxation-time collision in moment space (d'Humieres, Ginzburg,
# Krafczyk, Lallemand & Luo 2002): f* = f - M^-1 S M (f - f^eq) with an
# orthogonal moment basis M of the D3Q19 velocities and a diagonal S.


def mrt_basis():
    """(19, 19) integer matrix whose rows are the moment polynomials at the
    19 velocities, in the order rho, e, eps, j_x, q_x, j_y, q_y, j_z, q_z,
    3p_xx, 3pi_xx, p_ww, pi_ww, p_xy, p_yz, p_xz, m_x, m_y, m_z:
        1, 19c^2 - 30, (21c^4 - 53c^2 + 24)/2, c_x, (5c^2 - 9)c_x, c_y,
        (5c^2 - 9)c_y, c_z, (5c^2 - 9)c_z, 3c_x^2 - c^2,
        (3c^2 - 5)(3c_x^2 - c^2), c_y^2 - c_z^2, (3c^2 - 5)(c_y^2 - c_z^2),
        c_x c_y, c_y c_z, c_x c_z, (c_y^2 - c_z^2)c_x, (c_z^2 - c_x^2)c_y,
        (c_x^2 - c_y^2)c_z.
    The rows are mutually orthogonal (plain dot product over the velocities)."""
    M = np.zeros((NQ, NQ))
    for i in range(NQ):
        x, y, z = (int(v) for v in C[i])
        c2 = x * x + y * y + z * z
        M[:, i] = [1, 19 * c2 - 30, (21 * c2 * c2 - 53 * c2 + 24) // 2,
                   x, (5 * c2 - 9) * x, y, (5 * c2 - 9) * y, z, (5 * c2 - 9) * z,
                   3 * x * x - c2, (3 * c2 - 5) * (3 * x * x - c2),
                   y * y - z * z, (3 * c2 - 5) * (y * y - z * z),
                   x * y, y * z, x * z,
                   (y * y - z * z) * x, (z * z - x * x) * y, (x * x - y * y) * z]
    return M


# Rate group of each moment: conserved (rate irrelevant: f^eq carries them
# exactly), 'bulk' (e), 'ghost_even' (eps, pi_xx, pi_ww), 'flux' (q),
# 'shear' (the five traceless stresses), 'ghost_odd' (m).
MRT_GROUP = ("conserved", "bulk", "ghost_even", "conserved", "flux", "conserved", "flux", "conserved", "flux",
             "shear", "ghost_even", "shear", "ghost_even", "shear", "shear", "shear",
             "ghost_odd", "ghost_odd", "ghost_odd")


def mrt(f, feq, tau_shear, tau_flux, tau_bulk, tau_ghost_even, tau_ghost_odd):
    """f* = f - M^-1 S M (f - f^eq), S = diag of the inverse relaxation
    times by group (M^-1 = M^T diag(1/|row|^2) for the orthogonal basis).
    The even moments relax with tau_shear, tau_bulk or tau_ghost_even and the
    odd ones with tau_flux or tau_ghost_odd, so tau_bulk = tau_ghost_even =
    tau_shear and tau_ghost_odd = tau_flux is the TRT collision, and all
    five equal is BGK."""
    M = mrt_basis()
    norm = (M * M).sum(axis=1)
    tau = {"shear": tau_shear, "flux": tau_flux, "bulk": tau_bulk, "ghost_even": tau_ghost_even,
           "ghost_odd": tau_ghost_odd}
    rate = np.array([0.0 if g == "conserved" else 1.0 / tau[g] for g in MRT_GROUP])
    neq = f - feq
    m = np.tensordot(M, neq, axes=1)                      # moments of the non-equilibrium part
    back = np.tensordot(M.T, (rate / norm)[:, None, None, None] * m, axes=1)
    return f - back


def collide_single_mrt(f, taus):
    """Single-fluid MRT collision; taus = (shear, flux, bulk, ghost_even, ghost_odd)."""
    u, rho = velocity(f)
    return mrt(f, equilibrium_f(rho, u), *taus)


def step_single_mrt(f, taus, nsteps=1):
    for _ in range(nsteps):
        f = propagate(collide_single_mrt(f, taus))
    return f


def binary_fields(g, prm):
    """phi, grad phi, lap phi, mu and P of the current g (whole lattice first,
    because the stencils need phi at the neighbours)."""
    phi = order_parameter(g)
    grad = gradient(phi)
    lap = laplacian(phi)
    mu = chemical_potential(phi, lap, prm)
    P = chemical_stress(phi, grad, lap, prm)
    return phi, grad, lap, mu, P


def collide_binary(f, g, prm):
    """Binary-fluid collision: f relaxes to f^eq(rho, u, P) with tau_f and g
    relaxes to g^eq(phi, u, mu) with tau_g; u comes from f."""
    phi, _grad, _lap, mu, P = binary_fields(g, prm)
    u, rho = velocity(f)
    f_new = bgk(f, equilibrium_f(rho, u, P), prm.tau_f)
    g_new = bgk(g, equilibrium_g(phi, u, mu, prm), prm.tau_g)
    return f_new, g_new


def collide_binary_mrt(f, g, prm, taus):
    """Binary-fluid collision with f relaxing by the multiple-relaxation-time
    collision (mrt, taus = (shear, flux, bulk, ghost_even, ghost_odd)) around
    the same equilibrium f^eq(rho, u, P) as collide_binary; g relaxes as in
    collide_binary."""
    phi, _grad, _lap, mu, P = binary_fields(g, prm)
    u, rho = velocity(f)
    f_new = mrt(f, equilibrium_f(rho, u, P), *taus)
    g_new = bgk(g, equilibrium_g(phi, u, mu, prm), prm.tau_g)
    return f_new, g_new


def step_binary_mrt(f, g, prm, taus, nsteps=1):
    for _ in range(nsteps):
        f, g = collide_binary_mrt(f, g, prm, taus)
        f, g = propagate(f), propagate(g)
    return f, g


def propagate(f):
    """Periodic streaming f_i(s + c_i) <- f_i(s): a pure permutation."""
    out = np.empty_like(f)
    for i in range(NQ):
        out[i] = shift(f[i], C[i])
    return out


def step_single(f, tau, nsteps=1):
    for _ in range(nsteps):
        f = propagate(collide_single(f, tau))
    return f


def step_binary(f, g, prm, nsteps=1):
    for _ in range(nsteps):
        f, g = collide_binary(f, g, prm)
        f, g = propagate(f), propagate(g)
    return f, g


# ---------------------------------------------------------------------------
# Initial state
# ---------------------------------------------------------------------------


def init_single(rho, u):
    """f = f^eq(rho, u)."""
    return equilibrium_f(rho, u)


def init_binary(rho, u, phi, prm):
    """f = f^eq(rho, u, P(phi)) and g = g^eq(phi, u, mu(phi)), with the same
    stencils the collision uses applied to the given phi."""
    grad = gradient(phi)
    lap = laplacian(phi)
    mu = chemical_potential(phi, lap, prm)
    P = chemical_stress(phi, grad, lap, prm)
    return equilibrium_f(rho, u, P), equilibrium_g(phi, u, mu, prm)


# ---------------------------------------------------------------------------
# Conserved sums
# ---------------------------------------------------------------------------


def conserved_sums(f, g=None):
    """(sum rho, sum j_x, sum j_y, sum j_z, sum phi) over the lattice."""
    rho = density(f)
    j = momentum(f)
    phi_sum = order_parameter(g).sum() if g is not None else 0.0
    return np.array([rho.sum(), j[0].sum(), j[1].sum(), j[2].sum(), phi_sum])


# ---------------------------------------------------------------------------
# Adjoint of the single-fluid BGK step
# ---------------------------------------------------------------------------


def velocity_loss(f):
    """L = (1/N) sum_s u(s).u(s), written with u*u (not |u|^2) so that it is
    analytic for complex-step differentiation."""
    u, _rho = velocity(f)
    return (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]).mean()


def velocity_loss_seed(f):
    """dL/df_j(s) = (2/N) u.(c_j - u) / rho, the adjoint at the final step."""
    u, rho = velocity(f)
    n = rho.size
    lam = np.zeros_like(f)
    for j in range(NQ):
        acc = np.zeros_like(rho)
        for a in range(3):
            acc = acc + u[a] * (C[j, a] - u[a])
        lam[j] = 2.0 / n * acc / rho
    return lam


def adjoint_step_single(f_n, lam_next, tau):
    """Reverse of one step f^{n+1} = propagate(collide(f^n)).

    With lambda*_i(s) = lambda^{n+1}_i(s + c_i) (the transpose of the
    streaming permutation) and omega = 1/tau, the transpose of the local
    collision Jacobian gives

        lambda^n_j = (1 - omega) lambda*_j
                     + omega [ S + sum_a T_a (c_ja - u_a) / rho ],
        S   = sum_i lambda*_i f^eq_i / rho,
        T_a = sum_i lambda*_i w_i rho (3 c_ia + 9 (c_i.u) c_ia - 3 u_a),

    from d f^eq_i / d f_j = f^eq_i/rho + w_i rho dE_i/du_a (c_ja - u_a)/rho.
    The relaxation-rate sensitivity is dL/domega = sum_s sum_i
    lambda*_i (f^eq_i - f_i).  Returns (lambda^n, dL/domega)."""
    omega = 1.0 / tau
    lam_star = np.empty_like(lam_next)
    for i in range(NQ):
        lam_star[i] = neighbour(lam_next[i], C[i])
    u, rho = velocity(f_n)
    feq = equilibrium_f(rho, u)
    S = np.zeros_like(rho)
    T = np.zeros((3,) + rho.shape, dtype=np.result_type(rho, lam_star))
    for i in range(NQ):
        S = S + lam_star[i] * feq[i] / rho
        cu = C[i, 0] * u[0] + C[i, 1] * u[1] + C[i, 2] * u[2]
        for a in range(3):
            T[a] = T[a] + lam_star[i] * W[i] * rho * (3.0 * C[i, a] + 9.0 * cu * C[i, a] - 3.0 * u[a])
    lam_n = np.empty_like(lam_star)
    for j in range(NQ):
        acc = S.copy()
        for a in range(3):
            acc = acc + T[a] * (C[j, a] - u[a]) / rho
        lam_n[j] = (1.0 - omega) * lam_star[j] + omega * acc
    domega = (lam_star * (feq - f_n)).sum()
    return lam_n, domega


def rollout_gradient(f0, tau, nsteps, seed=velocity_loss_seed):
    """Gradient of L(f^T) with respect to f^0 and tau by a plain reverse
    sweep over every stored state (small lattices only).  Returns
    (L, dL/df0, dL/dtau)."""
    states = [f0]
    f = f0
    for _ in range(nsteps):
        f = step_single(f, tau)
        states.append(f)
    loss = velocity_loss(f)
    lam = seed(f)
    domega = 0.0
    for n in range(nsteps - 1, -1, -1):
        lam, dw = adjoint_step_single(states[n], lam, tau)
        domega = domega + dw
    dtau = -domega / (tau * tau)           # omega = 1/tau
    return loss, lam, dtau


# ---------------------------------------------------------------------------
# Adjoint of the single-fluid TRT and MRT steps
# ---------------------------------------------------------------------------
#
# Every collision here is f* = f - Omega (f - f^eq(f)) with a constant 19x19
# relaxation matrix Omega (omega I for BGK).  Its Jacobian is
# I - Omega (I - J), J = d f^eq / d f, so the adjoint of the collision is
# lambda -> lambda - (I - J)^T Omega^T lambda, and
# dL/domega_k = sum_s lambda*^T (d f*/d omega_k) = sum_s (P_k^T lambda*).(f^eq - f)
# where Omega = sum_k omega_k P_k over the rate groups.  These functions
# build Omega, P_k and J as explicit matrices per site and apply their
# transposes: slow, and free of the reductions the kernels use.

MRT_RATES = ("shear", "flux", "bulk", "ghost_even", "ghost_odd")


def relaxation_projectors():
    """{group: P_k (19x19)} with Omega = sum_k P_k / tau_k for the MRT groups:
    P_k = M^-1 E_k M, E_k selecting the moments of group k (conserved
    moments belong to no group: f - f^eq has none of them)."""
    M = mrt_basis()
    Minv = np.linalg.inv(M)
    out = {}
    for k in MRT_RATES:
        E = np.diag([1.0 if g == k else 0.0 for g in MRT_GROUP])
        out[k] = Minv @ E @ M
    return out


def relaxation_matrix(taus):
    """Omega for taus = (shear, flux, bulk, ghost_even, ghost_odd)."""
    P = relaxation_projectors()
    return sum(P[k] / t for k, t in zip(MRT_RATES, taus))


def equilibrium_jacobian(f):
    """J[i, j] = d f^eq_i / d f_j at every site, (19, 19, nz, ny, nx), from
    f^eq_i = w_i rho E_i(u), rho = sum f, u = sum f c / rho:
    d rho / d f_j = 1, d u_a / d f_j = (c_ja - u_a) / rho."""
    u, rho = velocity(f)
    feq = equilibrium_f(rho, u)
    J = np.empty((NQ, NQ) + rho.shape, dtype=np.result_type(f, rho))
    for i in range(NQ):
        cu = C[i, 0] * u[0] + C[i, 1] * u[1] + C[i, 2] * u[2]
        dEdu = [W[i] * rho * (3.0 * C[i, a] + 9.0 * cu * C[i, a] - 3.0 * u[a]) for a in range(3)]
        for j in range(NQ):
            acc = feq[i] / rho
            for a in range(3):
                acc = acc + dEdu[a] * (C[j, a] - u[a]) / rho
            J[i, j] = acc
    return J


def adjoint_step_single_mrt(f_n, lam_next, taus):
    """Reverse of one MRT step f^{n+1} = propagate(collide_single_mrt(f^n))
    (TRT and BGK are the special cases of tied times).  lambda*_i(s) =
    lambda^{n+1}_i(s + c_i); lambda^n = A^T lambda* per site with
    A = I - Omega (I - J).  Returns (lambda^n, {group: dL/domega_group})."""
    lam_star = np.empty_like(lam_next)
    for i in range(NQ):
        lam_star[i] = neighbour(lam_next[i], C[i])
    Om = relaxation_matrix(taus)
    J = equilibrium_jacobian(f_n)
    eye = np.eye(NQ)
    # A_ij(s) = delta_ij - sum_k Om_ik (delta_kj - J_kj(s))
    A = eye[:, :, None, None, None] - np.einsum("ik,kj...->ij...", Om, eye[:, :, None, None, None] - J)
    lam_n = np.einsum("i...,ij...->j...", lam_star, A)
    u, rho = velocity(f_n)
    neq_neg = equilibrium_f(rho, u) - f_n
    P = relaxation_projectors()
    grads = {k: np.einsum("i...,ij,j...->...", lam_star, P[k], neq_neg).sum() for k in MRT_RATES}
    return lam_n, grads


def rollout_gradient_mrt(f0, taus, nsteps, seed=velocity_loss_seed):
    """Gradient of L(f^T) under MRT steps with respect to f^0 and the five
    relaxation times, by a plain reverse sweep over every stored state.
    Returns (L, dL/df0, {group: dL/dtau_group})."""
    states = [f0]
    f = f0
    for _ in range(nsteps):
        f = step_single_mrt(f, taus)
        states.append(f)
    loss = velocity_loss(f)
    lam = seed(f)
    dw = {k: 0.0 for k in MRT_RATES}
    for n in range(nsteps - 1, -1, -1):
        lam, g = adjoint_step_single_mrt(states[n], lam, taus)
        for k in MRT_RATES:
            dw[k] = dw[k] + g[k]
    dtau = {k: -dw[k] / (t * t) for k, t in zip(MRT_RATES, taus)}
    return loss, lam, dtau


# ---------------------------------------------------------------------------
# Adjoint of the binary-fluid step
# ---------------------------------------------------------------------------
#
# The step is f^{n+1} = propagate(f*), g^{n+1} = propagate(g*) with
#   f*_i = f_i - omega_f (f_i - f^eq_i(rho, u, P)),
#   g*_i = g_i - omega_g (g_i - g^eq_i(phi, u, mu)),
# where rho, u come from f at the site, phi = sum_i g_i at the site, and P and
# mu also read grad(phi) and lap(phi), i.e. phi at the six neighbours.  The
# reverse sweep therefore has a local part (the transpose of the site's
# Jacobian with respect to f, g and the three stencil inputs phi, grad phi,
# lap phi) and a non-local part (the transpose of the two finite-difference
# stencils, which scatters the stencil sensitivities back to the sites whose
# phi they read, and then to every g_i there because phi = sum_i g_i).


def binary_adjoint_sums(lf, lg, u, G):
    """Weighted sums of the post-collision adjoints at every site that the
    transpose of the local Jacobian is built from:
        Lf = sum_i lf_i w_i,          Sf = sum_i lf_i w_i E_i,
        Sg = sum_i lg_i w_i E_i,      Xf = 9/2 sum_i lf_i w_i (|c_i|^2 - 1),
        Xg = 9/2 sum_i lg_i w_i (|c_i|^2 - 1),
        Tf_a = sum_i lf_i w_i dE_i/du_a,  Tg_a = sum_i lg_i w_i dE_i/du_a,
        YG_a = sum_i lf_i w_i c_ia (c_i.G)
    with E_i = 1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u and
    dE_i/du_a = 3 c_ia + 9 (c_i.u) c_ia - 3 u_a."""
    uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2]
    z = np.zeros_like(uu * lf[0])
    Lf, Sf, Sg, Xf, Xg = z.copy(), z.copy(), z.copy(), z.copy(), z.copy()
    Tf = [z.copy() for _ in range(3)]
    Tg = [z.copy() for _ in range(3)]
    YG = [z.copy() for _ in range(3)]
    for i in range(NQ):
        cu = C[i, 0] * u[0] + C[i, 1] * u[1] + C[i, 2] * u[2]
        cG = C[i, 0] * G[0] + C[i, 1] * G[1] + C[i, 2] * G[2]
        E = 1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu
        a, b = lf[i] * W[i], lg[i] * W[i]
        Lf = Lf + a
        Sf = Sf + a * E
        Sg = Sg + b * E
        Xf = Xf + 4.5 * a * (_C2[i] - 1)
        Xg = Xg + 4.5 * b * (_C2[i] - 1)
        for k in range(3):
            dE = 3.0 * C[i, k] + 9.0 * cu * C[i, k] - 3.0 * u[k]
            Tf[k] = Tf[k] + a * dE
            Tg[k] = Tg[k] + b * dE
            YG[k] = YG[k] + a * C[i, k] * cG
    return Lf, Sf, Sg, Xf, Xg, Tf, Tg, YG


def binary_stencil_sensitivities(lf, lg, phi, G, lap, u, prm, omega_f, omega_g):
    """Sensitivities of sum_i (lf_i f*_i + lg_i g*_i) at each site to the
    site's own stencil inputs, at fixed f, g (hence fixed rho, u):
        a_phi = omega_f Xf dIso/dphi + omega_g [Sg + Xg (Gamma dmu/dphi - 1/3)],
        a_G_a = omega_f kappa [9 (YG_a - Lf G_a / 3) - Xf G_a],
        a_lap = -kappa (omega_f phi Xf + omega_g Gamma Xg),
    with Iso = A/2 phi^2 + 3B/4 phi^4 - kappa phi lap - kappa/2 |G|^2 the
    isotropic part of P (dIso/dphi = A phi + 3 B phi^3 - kappa lap) and
    dmu/dphi = A + 3 B phi^2.  f^eq carries P as
    9/2 w_i [kappa ((c.G)^2 - |G|^2/3) + Iso (|c|^2 - 1)], g^eq carries mu as
    9/2 w_i Gamma mu (|c|^2 - 1).  Also returns the sensitivity to kappa at
    fixed phi, G, lap (summed over the lattice)."""
    Lf, Sf, Sg, Xf, Xg, Tf, Tg, YG = binary_adjoint_sums(lf, lg, u, G)
    k = prm.kappa
    GG = G[0] * G[0] + G[1] * G[1] + G[2] * G[2]
    diso = prm.A * phi + 3.0 * prm.B * phi ** 3 - k * lap
    dmu = prm.A + 3.0 * prm.B * phi ** 2
    a_phi = omega_f * Xf * diso + omega_g * (Sg + Xg * (prm.gamma * dmu - 1.0 / 3.0))
    a_G = np.array([omega_f * k * (9.0 * (YG[a] - Lf * G[a] / 3.0) - Xf * G[a]) for a in range(3)])
    a_lap = -k * (omega_f * phi * Xf + omega_g * prm.gamma * Xg)
    # kappa: the anisotropic stress 9/2 kappa sum_i lf_i w_i ((c.G)^2 - |G|^2/3),
    # Iso's -phi lap - |G|^2/2, and mu's -lap
    GYG = G[0] * YG[0] + G[1] * YG[1] + G[2] * YG[2]
    d_kappa = (omega_f * (4.5 * (GYG - Lf * GG / 3.0) + Xf * (-phi * lap - 0.5 * GG))
               + omega_g * prm.gamma * Xg * (-lap)).sum()
    return a_phi, a_G, a_lap, d_kappa, (Sf, Tf, Tg)


def stencil_transpose(a_phi, a_G, a_lap):
    """dL/dphi(s') from per-site sensitivities to phi(s), G(s) = grad phi(s)
    and lap phi(s): the transposes of the central difference
    G_a(s) = [phi(s+e_a) - phi(s-e_a)]/2 and of the 7-point Laplacian,
        b(s') = a_phi(s') + sum_a [a_G_a(s'-e_a) - a_G_a(s'+e_a)] / 2
                + sum_a [a_lap(s'+e_a) + a_lap(s'-e_a)] - 6 a_lap(s')."""
    b = a_phi - 6.0 * a_lap
    for a in range(3):
        e = [0, 0, 0]
        e[a] = 1
        m = [-v for v in e]
        b = b + 0.5 * (neighbour(a_G[a], m) - neighbour(a_G[a], e))
        b = b + neighbour(a_lap, e) + neighbour(a_lap, m)
    return b


def adjoint_step_binary(f_n, g_n, lf_next, lg_next, prm, taus=None):
    """Reverse of one binary step.  With lambda*_i(s) = lambda^{n+1}_i(s + c_i)
    for both distributions,
        lf^n_j = (1 - omega_f) lf*_j + omega_f Sf
                 + sum_a [omega_f Tf_a + omega_g (phi/rho) Tg_a] (c_ja - u_a),
        lg^n_j = (1 - omega_g) lg*_j + b,
    where the f-row comes from d rho/d f_j = 1 and d u_a/d f_j = (c_ja - u_a)/rho
    (f^eq_i = w_i rho E_i + stress, g^eq_i = w_i phi E_i + ...), and b is the
    transposed stencil of the sensitivities (stencil_transpose), the same for
    every j because phi = sum_j g_j.  Also returns the parameter sensitivities
    dL/domega_f = sum lf* (f^eq - f), dL/domega_g = sum lg* (g^eq - g) and
    dL/dkappa (at fixed omega).

    taus: None for the BGK step above, else the five times of f's
    moment-space collision (collide_binary_mrt; TRT is the case of even
    groups at one time and odd groups at another).  Omega is symmetric and
    f^eq depends on f only through rho and u, so every omega_f lf* above
    becomes mu = Omega lf* (and (1 - omega_f) lf* becomes lf* - mu); the rate
    sensitivities are then dL/domega_k = sum (P_k lf*) (f^eq - f) for the
    group projectors P_k, returned as grads["omega_<group>"]."""
    omega_f, omega_g = 1.0 / prm.tau_f, 1.0 / prm.tau_g
    lf = np.empty_like(lf_next)
    lg = np.empty_like(lg_next)
    for i in range(NQ):
        lf[i] = neighbour(lf_next[i], C[i])
        lg[i] = neighbour(lg_next[i], C[i])
    phi, G, lap, mu, P = binary_fields(g_n, prm)
    u, rho = velocity(f_n)
    if taus is None:
        mu_f = omega_f * lf
    else:
        mu_f = np.einsum("ij,j...->i...", relaxation_matrix(taus), lf)
    a_phi, a_G, a_lap, d_kappa, (Sf, Tf, Tg) = binary_stencil_sensitivities(
        mu_f, lg, phi, G, lap, u, prm, 1.0, omega_g)
    b = stencil_transpose(a_phi, a_G, a_lap)
    lf_n = np.empty_like(lf)
    lg_n = np.empty_like(lg)
    for j in range(NQ):
        acc = Sf
        for a in range(3):
            acc = acc + (Tf[a] + omega_g * phi / rho * Tg[a]) * (C[j, a] - u[a])
        lf_n[j] = lf[j] - mu_f[j] + acc
        lg_n[j] = (1.0 - omega_g) * lg[j] + b
    feq = equilibrium_f(rho, u, P)
    geq = equilibrium_g(phi, u, mu, prm)
    grads = {"omega_g": (lg * (geq - g_n)).sum(), "kappa": d_kappa}
    if taus is None:
        grads["omega_f"] = (lf * (feq - f_n)).sum()
    else:
        proj = relaxation_projectors()
        for k in MRT_RATES:
            grads["omega_" + k] = np.einsum("i...,ij,j...->...", lf, proj[k], feq - f_n).sum()
    return lf_n, lg_n, grads


def adjoint_init_binary(rho, u, phi, lf0, lg0, prm):
    """Reverse of init_binary: f^0 = f^eq(rho, u, P(phi)), g^0 = g^eq(phi, u,
    mu(phi)).  Given dL/df^0 and dL/dg^0 (no streaming here, so no shift),
    returns dL/dphi (stencil sensitivities with unit relaxation, transposed),
    dL/drho = Sf, dL/du_a = rho Tf_a + phi Tg_a, and dL/dkappa through the
    initial state."""
    G = gradient(phi)
    lap = laplacian(phi)
    a_phi, a_G, a_lap, d_kappa, (Sf, Tf, Tg) = binary_stencil_sensitivities(
        lf0, lg0, phi, G, lap, u, prm, 1.0, 1.0)
    dphi = stencil_transpose(a_phi, a_G, a_lap)
    du = np.array([rho * Tf[a] + phi * Tg[a] for a in range(3)])
    return dphi, Sf, du, d_kappa


def binary_loss(f, g, beta=1.0):
    """L = (1/N) sum_s [u.u + beta phi^2] (analytic, for complex steps)."""
    u, _rho = velocity(f)
    phi = order_parameter(g)
    return (u[0] * u[0] + u[1] * u[1] + u[2] * u[2] + beta * phi * phi).mean()


def binary_loss_seed(f, g, beta=1.0):
    """(dL/df, dL/dg) of binary_loss: the velocity part as in
    velocity_loss_seed, and 2 beta phi / N for every g_j."""
    phi = order_parameter(g)
    lg = np.empty_like(g)
    for j in range(NQ):
        lg[j] = 2.0 * beta * phi / phi.size
    return velocity_loss_seed(f), lg


def rollout_gradient_binary(rho, u, phi, prm, nsteps, beta=1.0, taus=None):
    """Gradient of binary_loss after nsteps binary steps from
    init_binary(rho, u, phi) by a plain reverse sweep over every stored
    state (small lattices only).  Returns (L, dL/dphi0, dL/drho0, dL/du0,
    {tau_f, mobility, kappa}); with taus (the five moment-space times of f,
    step_binary_mrt) the f times are returned as tau_<group> instead of
    tau_f."""
    f, g = init_binary(rho, u, phi, prm)
    states = [(f, g)]
    for _ in range(nsteps):
        f, g = step_binary(f, g, prm) if taus is None else step_binary_mrt(f, g, prm, taus)
        states.append((f, g))
    loss = binary_loss(f, g, beta)
    lf, lg = binary_loss_seed(f, g, beta)
    fkeys = ["omega_f"] if taus is None else ["omega_" + k for k in MRT_RATES]
    dw = {k: 0.0 for k in fkeys + ["omega_g", "kappa"]}
    for n in range(nsteps - 1, -1, -1):
        lf, lg, gr = adjoint_step_binary(states[n][0], states[n][1], lf, lg, prm, taus)
        for k in dw:
            dw[k] = dw[k] + gr[k]
    dphi, drho, du, dk0 = adjoint_init_binary(rho, u, phi, lf, lg, prm)
    # omega = 1/tau; tau_g = M/Gamma + 1/2
    grads = {"mobility": -dw["omega_g"] / prm.tau_g ** 2 / prm.gamma, "kappa": dw["kappa"] + dk0}
    if taus is None:
        grads["tau_f"] = -dw["omega_f"] / prm.tau_f ** 2
    else:
        for k, t in zip(MRT_RATES, taus):
            grads["tau_" + k] = -dw["omega_" + k] / (t * t)
    return loss, dphi, drho, du, grads


# ---------------------------------------------------------------------------
# The binary adjoint by its definition
# ---------------------------------------------------------------------------
#
# The reverse of one step is, by definition, lambda^n = J^T lambda^{n+1} with
# J the Jacobian of the whole step (collide, then propagate) with respect to
# the state (f^n, g^n).  The functions below build J one column at a time
# from the plain forward above by complex-step differentiation: column k is
# Im step(x + i h e_k) / h.  Every operation of the forward (+, -, *, /,
# integer powers, periodic shifts) is analytic and nothing is subtracted to
# form the derivative, so each column is exact to rounding (Squire & Trapp
# 1998).  Parameters are differentiated the same way.  This uses none of
# the hand-derived sums above (binary_adjoint_sums and what builds on it):
# one forward step per state component, so small lattices only.

CSTEP = 1e-30          # complex step; far below any rounding of the real part


def _binary_step_once(f, g, prm, taus):
    if taus is None:
        return step_binary(f, g, prm, 1)
    return step_binary_mrt(f, g, prm, taus, 1)


def _flat_state(f, g):
    return np.concatenate([f.ravel(), g.ravel()])


def binary_step_jacobian(f, g, prm, taus=None):
    """J[m, k] = d x'_m / d x_k for one binary step x' = step(x), x the state
    (f, g) flattened as concatenate(f.ravel(), g.ravel()) (f first, each in
    the (19, nz, ny, nx) layout).  taus: None for BGK, else f's five
    moment-space times (step_binary_mrt).  Returns a (2*19*N, 2*19*N) array."""
    x = _flat_state(f, g).astype(np.complex128)
    n = x.size
    half = n // 2
    J = np.empty((n, n))
    for k in range(n):
        xk = x.copy()
        xk[k] += 1j * CSTEP
        fo, go = _binary_step_once(xk[:half].reshape(f.shape), xk[half:].reshape(g.shape), prm, taus)
        J[:, k] = _flat_state(fo, go).imag / CSTEP
    return J


def _parameter_derivative(fun, prm, name, taus=None, k=None):
    """d fun / d parameter by one complex step: `name` is a field of Params,
    or "taus" with k the index of f's moment-space time."""
    import dataclasses
    if name == "taus":
        t = [complex(v) for v in taus]
        t[k] += 1j * CSTEP
        return fun(prm, tuple(t)).imag / CSTEP
    p = dataclasses.replace(prm, **{name: getattr(prm, name) + 1j * CSTEP})
    return fun(p, taus).imag / CSTEP


def adjoint_step_binary_plain(f_n, g_n, lf_next, lg_next, prm, taus=None):
    """Reverse of one binary step from its definition: (lf^n, lg^n) =
    J^T (lf^{n+1}, lg^{n+1}) with J = binary_step_jacobian, and the
    parameter gradients d/dp <lambda^{n+1}, step(f^n, g^n; p)> for
    p = kappa, mobility and tau_f (BGK), or kappa, mobility and
    tau_<group> for the five groups of MRT_RATES (taus given).  Returns
    (lf^n, lg^n, grads)."""
    J = binary_step_jacobian(f_n, g_n, prm, taus)
    lam = J.T @ _flat_state(lf_next, lg_next)
    half = lam.size // 2
    lf_n, lg_n = lam[:half].reshape(f_n.shape), lam[half:].reshape(g_n.shape)
    fc, gc = f_n.astype(np.complex128), g_n.astype(np.complex128)

    def projected(p, t):
        a, b = _binary_step_once(fc, gc, p, t)
        return (lf_next * a).sum() + (lg_next * b).sum()
    grads = {"kappa": _parameter_derivative(projected, prm, "kappa", taus),
             "mobility": _parameter_derivative(projected, prm, "mobility", taus)}
    if taus is None:
        grads["tau_f"] = _parameter_derivative(projected, prm, "tau_f")
    else:
        for k, name in enumerate(MRT_RATES):
            grads["tau_" + name] = _parameter_derivative(projected, prm, "taus", taus, k)
    return lf_n, lg_n, grads


def adjoint_init_binary_plain(rho, u, phi, lf0, lg0, prm):
    """Reverse of init_binary from its definition: for every component of
    phi, rho and u, the complex-step derivative of <(lf0, lg0), init_binary>,
    and d/dkappa of the same.  Returns (dL/dphi, dL/drho, dL/du, dL/dkappa)."""
    cx = lambda a: np.asarray(a).astype(np.complex128)

    def projected(r, v, p, q=prm):
        a, b = init_binary(r, v, p, q)
        return (lf0 * a).sum() + (lg0 * b).sum()
    out = []
    for which, arr in (("phi", phi), ("rho", rho), ("u", u)):
        d = np.empty(arr.shape)
        for idx in np.ndindex(arr.shape):
            args = {"rho": cx(rho), "u": cx(u), "phi": cx(phi)}
            args[which][idx] += 1j * CSTEP
            d[idx] = projected(args["rho"], args["u"], args["phi"]).imag / CSTEP
        out.append(d)
    dk = _parameter_derivative(lambda p, _t: projected(cx(rho), cx(u), cx(phi), p), prm, "kappa")
    return out[0], out[1], out[2], dk
