"""The pins must catch plausible mistakes: each case plants one slip in the
CPU reference (on the CPU, through monkeypatching) and checks that at least
one pin of tests/test_oracle_pins.py then fails."""

import numpy as np
import pytest

from oracle import lb_oracle as O
import tests.test_oracle_pins as pins


def _fails(*checks):
    """True if at least one pin check raises AssertionError."""
    for check in checks:
        try:
            check()
        except AssertionError:
            return True
    return False


def _mut_feq_square(rho, u, P=None):
    # 9/2 (c.u)^2 written as 3 (c.u)^2
    uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2]
    feq = np.zeros((O.NQ,) + rho.shape, dtype=np.result_type(rho, u))
    for i in range(O.NQ):
        cu = O.C[i, 0] * u[0] + O.C[i, 1] * u[1] + O.C[i, 2] * u[2]
        feq[i] = O.W[i] * rho * (1.0 + 3.0 * cu + 3.0 * cu * cu - 1.5 * uu)
    return feq


def _mut_feq_no_trace(rho, u, P=None):
    # stress term without the - tr(P)/3 part
    feq = O.equilibrium_f.__wrapped__(rho, u, None)
    if P is not None:
        for i in range(O.NQ):
            cPc = sum(O.C[i, a] * O.C[i, b] * P[a, b] for a in range(3) for b in range(3))
            feq[i] = feq[i] + O.W[i] * 4.5 * cPc
    return feq


def _mut_geq_sign(phi, u, mu, prm):
    geq = O.equilibrium_g.__wrapped__(phi, u, mu, prm)
    for i in range(O.NQ):
        geq[i] = geq[i] - 2 * O.W[i] * 4.5 * (prm.gamma * mu - phi / 3.0) * ((O.C[i] ** 2).sum() - 1)
    return geq


def _mut_mu_sign(phi, lap, prm):
    return prm.A * phi + prm.B * phi ** 3 + prm.kappa * lap


def _mut_stress_gsq(phi, grad, lap, prm):
    P = O.chemical_stress.__wrapped__(phi, grad, lap, prm)
    for a in range(3):
        P[a, a] = P[a, a] + prm.kappa * (grad[0] ** 2 + grad[1] ** 2 + grad[2] ** 2)
    return P


def _mut_gradient_sign(phi):
    return -O.gradient.__wrapped__(phi)


def _mut_laplacian_centre(phi):
    return O.laplacian.__wrapped__(phi) + 2.0 * phi


def _mut_propagate_back(f):
    out = np.empty_like(f)
    for i in range(O.NQ):
        out[i] = O.shift(f[i], -O.C[i])
    return out


def _mut_bgk_tau(f, feq, tau):
    return f - (f - feq) * tau


def _mut_momentum_axes(f):
    j = O.momentum.__wrapped__(f)
    return j[[1, 0, 2]]


def _mut_seed_factor(f):
    return 0.5 * O.velocity_loss_seed.__wrapped__(f)


def _mut_adjoint_T(f_n, lam_next, tau):
    # T_a with the sign of the -3 u_a term flipped
    omega = 1.0 / tau
    lam_star = np.empty_like(lam_next)
    for i in range(O.NQ):
        lam_star[i] = O.neighbour(lam_next[i], O.C[i])
    u, rho = O.velocity(f_n)
    feq = O.equilibrium_f(rho, u)
    S = sum(lam_star[i] * feq[i] / rho for i in range(O.NQ))
    T = np.zeros((3,) + rho.shape)
    for i in range(O.NQ):
        cu = O.C[i, 0] * u[0] + O.C[i, 1] * u[1] + O.C[i, 2] * u[2]
        for a in range(3):
            T[a] += lam_star[i] * O.W[i] * rho * (3.0 * O.C[i, a] + 9.0 * cu * O.C[i, a] + 3.0 * u[a])
    lam_n = np.empty_like(lam_star)
    for j in range(O.NQ):
        acc = S + sum(T[a] * (O.C[j, a] - u[a]) / rho for a in range(3))
        lam_n[j] = (1.0 - omega) * lam_star[j] + omega * acc
    return lam_n, (lam_star * (feq - f_n)).sum()


def _mut_stencil_transpose_sign(a_phi, a_G, a_lap):
    # the central difference transposed without its sign flip
    return O.stencil_transpose.__wrapped__(a_phi, -a_G, a_lap)


def _mut_alap_sign(lf, lg, phi, G, lap, u, prm, omega_f, omega_g):
    a_phi, a_G, a_lap, d_kappa, rest = O.binary_stencil_sensitivities.__wrapped__(
        lf, lg, phi, G, lap, u, prm, omega_f, omega_g)
    return a_phi, a_G, -a_lap, d_kappa, rest


def _mut_no_geq_velocity(lf, lg, u, G):
    # g^eq's dependence on u forgotten in the reverse sweep
    Lf, Sf, Sg, Xf, Xg, Tf, Tg, YG = O.binary_adjoint_sums.__wrapped__(lf, lg, u, G)
    return Lf, Sf, Sg, Xf, Xg, Tf, [0.0 * t for t in Tg], YG


def _mut_phi_seed_factor(f, g, beta=1.0):
    lf, lg = O.binary_loss_seed.__wrapped__(f, g, beta)
    return lf, 0.5 * lg


def _mut_mrt_flux_polynomial():
    # (5c^2 - 8) c_x for the x energy flux
    M = O.mrt_basis.__wrapped__()
    M[4] = M[4] + O.C[:, 0]
    return M


def _mut_mrt_bulk_group():
    # the bulk rate applied to eps, the ghost rate to e
    g = list(O.MRT_GROUP)
    g[1], g[2] = g[2], g[1]
    return tuple(g)


def _mut_jacobian_transposed(f):
    return np.swapaxes(O.equilibrium_jacobian.__wrapped__(f), 0, 1)


def _mut_projectors_swapped():
    P = O.relaxation_projectors.__wrapped__()
    P["bulk"], P["ghost_even"] = P["ghost_even"], P["bulk"]
    return P


def _mut_relaxation_odd_times_swapped(taus):
    t = list(taus)
    t[1], t[4] = t[4], t[1]
    return O.relaxation_matrix.__wrapped__(tuple(t))


def _swap_weights():
    w = O.W.copy()
    c2 = (O.C * O.C).sum(1)
    w[c2 == 1], w[c2 == 2] = 1.0 / 36.0, 1.0 / 18.0
    return w


MUTATIONS = {
    "weights 1/18 <-> 1/36": ("W", _swap_weights, [pins.test_weights_exact_isotropy,
                                                   pins.test_equilibrium_f_moments_single_fluid]),
    "f^eq (c.u)^2 coefficient": ("equilibrium_f", _mut_feq_square,
                                 [pins.test_equilibrium_f_moments_single_fluid]),
    "f^eq stress without trace": ("equilibrium_f", _mut_feq_no_trace,
                                  [pins.test_equilibrium_f_moments_with_stress]),
    "g^eq mobility term sign": ("equilibrium_g", _mut_geq_sign, [pins.test_equilibrium_g_moments]),
    "mu with +kappa lap": ("chemical_potential", _mut_mu_sign,
                           [pins.test_flat_interface_mu_stress_and_tension, pins.test_gibbs_duhem]),
    "stress +kappa/2 |grad|^2": ("chemical_stress", _mut_stress_gsq,
                                 [pins.test_flat_interface_mu_stress_and_tension, pins.test_gibbs_duhem]),
    "gradient sign": ("gradient", _mut_gradient_sign, [lambda: pins.test_stencils_on_sine_waves(2)]),
    "laplacian centre weight": ("laplacian", _mut_laplacian_centre,
                                [lambda: pins.test_stencils_on_sine_waves(1)]),
    "propagation against c": ("propagate", _mut_propagate_back,
                               [pins.test_propagate_one_hot_exhaustive_4cubed]),
    "BGK with tau for 1/tau": ("bgk", _mut_bgk_tau, [pins.test_shear_wave_viscous_decay]),
    "momentum axes swapped": ("momentum", _mut_momentum_axes, [pins.test_moments_one_hot]),
    "loss seed factor": ("velocity_loss_seed", _mut_seed_factor, [pins.test_velocity_loss_seed_complex_step]),
    "adjoint T sign": ("adjoint_step_single", _mut_adjoint_T, [pins.test_adjoint_rollout_matches_complex_step]),
    "binary adjoint: gradient stencil not negated": ("stencil_transpose", _mut_stencil_transpose_sign,
                                                     [pins.test_binary_adjoint_rollout_matches_complex_step]),
    "binary adjoint: Laplacian sensitivity sign": ("binary_stencil_sensitivities", _mut_alap_sign,
                                                   [pins.test_binary_adjoint_step_matches_complex_step]),
    "binary adjoint: g^eq velocity term dropped": ("binary_adjoint_sums", _mut_no_geq_velocity,
                                                   [pins.test_binary_adjoint_step_matches_complex_step]),
    "binary loss seed phi factor": ("binary_loss_seed", _mut_phi_seed_factor,
                                    [pins.test_binary_loss_seed_complex_step]),
    "MRT energy-flux polynomial": ("mrt_basis", lambda: _mut_mrt_flux_polynomial(),
                                   [pins.test_mrt_basis_orthogonal_full_rank_and_parity]),
    "MRT adjoint: equilibrium Jacobian transposed": ("equilibrium_jacobian", _mut_jacobian_transposed,
                                                     [pins.test_mrt_adjoint_step_matches_complex_step]),
    "MRT adjoint: bulk and even-ghost projectors swapped": ("relaxation_projectors", _mut_projectors_swapped,
                                                            [pins.test_mrt_adjoint_step_matches_complex_step]),
    "binary MRT adjoint: flux and odd-ghost times swapped in Omega": (
        "relaxation_matrix", _mut_relaxation_odd_times_swapped,
        [pins.test_binary_mrt_adjoint_step_matches_complex_step]),
}

# non-callable attributes replaced by a value
VALUE_MUTATIONS = {
    "MRT bulk rate on the wrong moment": ("MRT_GROUP", _mut_mrt_bulk_group,
                                          [lambda: pins.test_mrt_sound_damping_follows_bulk_viscosity(1.4)]),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_planted_mistake(monkeypatch, name):
    attr, mutant, checks = MUTATIONS[name]
    original = getattr(O, attr)
    if callable(original):
        mutant.__wrapped__ = original          # mutants that extend the original call it here
        monkeypatch.setattr(O, attr, mutant)
    else:
        monkeypatch.setattr(O, attr, mutant())
    assert _fails(*checks), "no pin caught: %s" % name


@pytest.mark.parametrize("name", sorted(VALUE_MUTATIONS))
def test_pins_catch_planted_value(monkeypatch, name):
    attr, make, checks = VALUE_MUTATIONS[name]
    monkeypatch.setattr(O, attr, make())
    assert _fails(*checks), "no pin caught: %s" % name


def test_unmutated_pins_pass():
    for check in (pins.test_weights_exact_isotropy, pins.test_equilibrium_f_moments_single_fluid,
                  pins.test_gibbs_duhem, pins.test_adjoint_rollout_matches_complex_step):
        check()
