"""Oracle of the variable-Eddington-tensor (VET) hand-off: the frequency-
integrated radiation moment equations closed with the Eddington tensor that
the transport solution provides (Sec. 4: the tensor from the transfer
solution replaces an approximate closure in a radiation-hydrodynamics update).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain NumPy, FP64.

With c = 1 and the moments J = <I>, H = <n I>, K = <n n I> (angle averages,
the library's normalisation), the angle integrals of the time-dependent
transfer equation give

    dJ/dt + div H = kappa_E (B - J),      dH/dt + div (f J) = -chi_F H,

with the closure K = f J.  The caller (the hydrodynamics side) supplies the
energy-exchange coefficient kappa_E, the flux extinction chi_F and the
emission B per point; the library supplies f.  The update is not in the paper
(it only states the goal); it is the plain forward-backward scheme below:

    H^{n+1} = (H^n - dt div(f J^n)) / (1 + dt chi_F)
    J^{n+1} = (J^n - dt div H^{n+1} + dt kappa_E B) / (1 + dt kappa_E)

on the library's grid (x, y periodic, spacings lx/nx, ly/ny; z points
0 .. lz with spacing lz/(nz - 1)), derivatives by central differences, one-
sided (first order) on the two z faces; a direction with one point has no
derivative.  The exchange with the gas over the steps is returned as
G = (sum dt kappa_E (J^{n+1} - B), sum dt chi_F H^{n+1}): the energy and
momentum the radiation gave the gas, per unit volume (in the units of J, H).
"""
import numpy as np


def _derivs(nx, ny, nz, lx, ly, lz):
    dx, dy = lx / nx, ly / ny
    dz = lz / (nz - 1) if nz > 1 else 1.0

    def Dx(u):
        return (np.roll(u, -1, axis=2) - np.roll(u, 1, axis=2)) / (2.0 * dx)

    def Dy(u):
        return (np.roll(u, -1, axis=1) - np.roll(u, 1, axis=1)) / (2.0 * dy)

    def Dz(u):
        d = np.zeros_like(u)
        if nz == 1:
            return d
        d[1:-1] = (u[2:] - u[:-2]) / (2.0 * dz)
        d[0] = (u[1] - u[0]) / dz
        d[-1] = (u[-1] - u[-2]) / dz
        return d

    return Dx, Dy, Dz


def vet_step(grid, f, kappa_E, chi_F, B, J, H, dt, nsteps=1):
    """nsteps steps of length dt.  grid = (nx, ny, nz, lx, ly, lz); f [P][6]
    (xx, yy, zz, xy, xz, yz), kappa_E, chi_F, B, J [P], H [P][3] with point
    index p = (z ny + y) nx + x.  Returns (J, H, G [P][4])."""
    nx, ny, nz, lx, ly, lz = grid
    sh = (nz, ny, nx)
    Dx, Dy, Dz = _derivs(nx, ny, nz, lx, ly, lz)
    D = (Dx, Dy, Dz)
    f = np.asarray(f, dtype=np.float64).reshape(sh + (6,))
    comp = ((0, 3, 4), (3, 1, 5), (4, 5, 2))          # f_ab as (xx, yy, zz, xy, xz, yz) columns
    ka = np.asarray(kappa_E, dtype=np.float64).reshape(sh)
    ch = np.asarray(chi_F, dtype=np.float64).reshape(sh)
    b = np.asarray(B, dtype=np.float64).reshape(sh)
    J = np.array(J, dtype=np.float64).reshape(sh)
    H = np.array(H, dtype=np.float64).reshape(sh + (3,))
    G = np.zeros(sh + (4,))
    for _ in range(nsteps):
        Hn = np.empty_like(H)
        for a in range(3):
            div = sum(D[c](f[..., comp[a][c]] * J) for c in range(3))
            Hn[..., a] = (H[..., a] - dt * div) / (1.0 + dt * ch)
        H = Hn
        divH = Dx(H[..., 0]) + Dy(H[..., 1]) + Dz(H[..., 2])
        J = (J - dt * divH + dt * ka * b) / (1.0 + dt * ka)
        G[..., 0] += dt * ka * (J - b)
        for a in range(3):
            G[..., 1 + a] += dt * ch * H[..., a]
    P = nx * ny * nz
    return J.reshape(P), H.reshape(P, 3), G.reshape(P, 4)
