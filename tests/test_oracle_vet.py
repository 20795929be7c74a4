"""Pins of the oracle's VET hand-off update (oracle/vet.py) against closed
forms of its scheme: equilibrium, a Fourier mode (the discrete dispersion of
central differences), the placement of the off-diagonal Eddington components,
one-sided z differences on a linear field, local absorption, and exact energy
conservation with the gas exchange on a periodic grid."""
import math

import numpy as np

from oracle.vet import vet_step


def _iso(P, v=1.0 / 3.0):
    f = np.zeros((P, 6))
    f[:, :3] = v
    return f


def test_equilibrium_is_kept():
    grid = (6, 5, 4, 1.0, 0.8, 1.2)
    P = 6 * 5 * 4
    rs = np.random.default_rng(0)
    f = np.tile(rs.uniform(-0.2, 0.5, 6), (P, 1))
    J, H, G = vet_step(grid, f, np.full(P, 2.0), np.full(P, 3.0), np.full(P, 1.5), np.full(P, 1.5),
                       np.zeros((P, 3)), 0.01, nsteps=5)
    assert np.allclose(J, 1.5, rtol=0, atol=1e-15) and np.abs(H).max() < 1e-15 and np.abs(G).max() < 1e-15


def test_fourier_mode_in_x():
    nx, lx = 16, 2.0
    grid = (nx, 1, 2, lx, 1.0, 1.0)
    P = nx * 2
    dx, dt, a, m = lx / nx, 0.03, 0.7, 3
    k = 2 * math.pi * m / lx
    x = np.tile(np.arange(nx) * dx, 2)
    kp = math.sin(k * dx) / dx                        # the central difference's wavenumber
    H0 = np.zeros((P, 3))
    H0[:, 0] = a * np.sin(k * x)
    J, H, G = vet_step(grid, _iso(P), np.zeros(P), np.zeros(P), np.zeros(P), np.cos(k * x), H0, dt)
    h1 = a + dt * kp / 3.0
    assert np.allclose(H[:, 0], h1 * np.sin(k * x), rtol=0, atol=1e-14)
    assert np.allclose(J, (1.0 - dt * kp * h1) * np.cos(k * x), rtol=0, atol=1e-14)
    assert np.abs(H[:, 1:]).max() == 0.0 and np.abs(G).max() == 0.0


def test_off_diagonal_components_act_in_their_own_equations():
    ny, ly, dt, c = 12, 1.5, 0.02, 0.25
    grid = (3, ny, 2, 0.9, ly, 1.0)
    P = 3 * ny * 2
    k = 2 * math.pi / ly
    y = np.tile(np.repeat(np.arange(ny) * (ly / ny), 3), 2)
    kp = math.sin(k * ly / ny) / (ly / ny)
    f = np.zeros((P, 6))
    f[:, 3] = c                                        # f_xy only
    J, H, G = vet_step(grid, f, np.zeros(P), np.zeros(P), np.zeros(P), np.cos(k * y), np.zeros((P, 3)), dt)
    # x equation: d_y (f_xy J); y equation: d_x (f_xy J) = 0 (J uniform in x)
    assert np.allclose(H[:, 0], dt * c * kp * np.sin(k * y), rtol=0, atol=1e-14)
    assert np.abs(H[:, 1]).max() < 1e-15 and np.abs(H[:, 2]).max() == 0.0


def test_one_sided_z_differences_are_exact_on_a_linear_field():
    nz, lz, dt, c = 7, 1.3, 0.05, 0.4
    grid = (2, 3, nz, 1.0, 1.0, lz)
    P = 2 * 3 * nz
    z = np.repeat(np.arange(nz) * (lz / (nz - 1)), 6)
    f = np.zeros((P, 6))
    f[:, 4] = c                                        # f_xz
    f[:, 2] = 0.5                                      # f_zz
    J, H, G = vet_step(grid, f, np.zeros(P), np.zeros(P), np.zeros(P), 2.0 * z + 1.0, np.zeros((P, 3)), dt)
    assert np.allclose(H[:, 0], -dt * c * 2.0, rtol=0, atol=1e-14)
    assert np.allclose(H[:, 2], -dt * 0.5 * 2.0, rtol=0, atol=1e-14)
    # div H = d_z H_z = 0 (H_z uniform): J keeps its values
    assert np.allclose(J, 2.0 * z + 1.0, rtol=0, atol=1e-14)


def test_local_absorption_closed_form():
    grid = (4, 4, 3, 1.0, 1.0, 1.0)
    P = 48
    dt, ka, ch, b, j0 = 0.1, 3.0, 5.0, 2.0, 0.5
    h0 = np.array([0.3, -0.2, 0.1])
    J, H, G = vet_step(grid, _iso(P), np.full(P, ka), np.full(P, ch), np.full(P, b), np.full(P, j0),
                       np.tile(h0, (P, 1)), dt)
    j1 = (j0 + dt * ka * b) / (1 + dt * ka)
    h1 = h0 / (1 + dt * ch)
    assert np.allclose(J, j1, rtol=1e-15) and np.allclose(H, h1, rtol=1e-15)
    assert np.allclose(G[:, 0], dt * ka * (j1 - b), rtol=1e-15) and np.allclose(G[:, 1:], dt * ch * h1, rtol=1e-15)


def test_energy_with_the_gas_exchange_is_conserved_on_a_periodic_grid():
    nx, ny = 9, 7
    grid = (nx, ny, 2, 1.0, 0.7, 1.0)
    rs = np.random.default_rng(3)
    Q = nx * ny
    tile = lambda a: np.concatenate([a, a])           # uniform in z: no z derivatives
    f = tile(rs.uniform(0.0, 0.4, (Q, 6)))
    ka, ch, b = tile(rs.uniform(0, 2, Q)), tile(rs.uniform(0, 2, Q)), tile(rs.uniform(0, 1, Q))
    J0, H0 = tile(rs.uniform(0, 1, Q)), tile(rs.uniform(-0.3, 0.3, (Q, 3)))
    J, H, G = vet_step(grid, f, ka, ch, b, J0, H0, 0.01, nsteps=20)
    assert abs((J.sum() - J0.sum()) + G[:, 0].sum()) < 1e-12 * J0.sum()
