"""Seeded synthetic inputs for the lattice-Boltzmann workloads.

This module only draws random numbers and lays them out; it holds none of
the method's arithmetic, so both the HIP path and the CPU reference can be
fed from it.  Every field is float64, shaped (nz, ny, nx) for scalars and
(3, nz, ny, nx) for vectors (x component first), with x fastest in memory.

Draw order for a given seed: rho (N normals) then u_x, u_y, u_z (N uniforms
each), or phi (N uniforms).
"""

import numpy as np


def single_fluid_random(nx, ny, nz, seed=0, rho_sigma=0.01, u_max=0.01):
    """rho = 1 + rho_sigma*N(0,1) per site, u components uniform in
    [-u_max, u_max]."""
    rng = np.random.default_rng(seed)
    shape = (nz, ny, nx)
    rho = 1.0 + rho_sigma * rng.standard_normal(shape)
    u = np.stack([rng.uniform(-u_max, u_max, shape) for _ in range(3)])
    return rho, u


def spinodal_quench(nx, ny, nz, seed=0, phi_max=0.05):
    """rho = 1, u = 0, phi uniform in [-phi_max, phi_max]."""
    rng = np.random.default_rng(seed)
    shape = (nz, ny, nx)
    phi = rng.uniform(-phi_max, phi_max, shape)
    rho = np.ones(shape)
    u = np.zeros((3,) + shape)
    return rho, u, phi


def shear_wave(nx, ny, nz, amplitude=0.01, noise=1e-4, seed=0):
    """rho = 1, u_x = amplitude*sin(2 pi y / ny) plus independent uniform
    noise in [-noise, noise] on each velocity component."""
    rng = np.random.default_rng(seed)
    shape = (nz, ny, nx)
    y = np.arange(ny, dtype=np.float64).reshape(1, ny, 1)
    u = np.stack([rng.uniform(-noise, noise, shape) for _ in range(3)]) if noise > 0 \
        else np.zeros((3,) + shape)
    u[0] += amplitude * np.sin(2.0 * np.pi * y / ny)
    rho = np.ones(shape)
    return rho, u


def sample_components(n_sites, count, seed=1, nq=19):
    """`count` distinct (direction, site) pairs drawn without replacement."""
    rng = np.random.default_rng(seed)
    flat = rng.choice(nq * n_sites, size=count, replace=False)
    return [(int(k // n_sites), int(k % n_sites)) for k in flat]
