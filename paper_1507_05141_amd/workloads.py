"""Seeded synthetic inputs for the radiative-transfer problems.

This module only *describes inputs*: grid sizes, group edges, and the fields
(absorption, scattering, thermal source, velocity, electron temperature) drawn
from a seeded NumPy ``Generator(PCG64(seed))``.  It holds none of the solver's
arithmetic and is shared by the HIP library's tests/benchmark and by the
oracle.

A problem description is a plain dict:
  nx, ny, nz, lx, ly, lz     grid (x, y periodic; z has nz points on [0, lz])
  nmu, nphi, lmax            Gauss-Legendre polar x uniform azimuth mesh, SH order
  edges                      group edges (G+1,), or None for one grey group
  log_centres                geometric (True) or arithmetic (False) group centres
  scatter                    "thomson" or "compton"
  mec2                       electron rest energy in the units of the edges
  kappa  (P, G)              comoving absorption coefficient per unit length
  sigma  (P,)                n_e sigma_T per unit length
  bnu    (P, G)              comoving thermal source function B_nu at the centres
  beta   (P, 3) or None      flow velocity v/c
  kte    (P,) or None        electron temperature (same units as the edges)
  bc_bot, bc_top             incoming lab intensity on z = 0 / z = lz,
                             (K, ny, nx, G) or None for vacuum
with the point index p = (z*ny + y)*nx + x.

Workloads (the paper's own test problems are two-dimensional; these are the
three-dimensional workloads the benchmark and the tests are quoted on):
  uniform_slab      16^3 grey slab, kappa = sigma = B = 1, L = 3, 8x16 ordinates
  thomson_jet       32^3, 16 log groups, relativistic jet (Gamma_max = 10),
                    log-uniform sigma in [0.1, 10], L = 7, 16x32 ordinates
  compton_jet       64^3, 32 log groups over [1e-3, 1e3] keV, electron
                    temperature field 10-100 keV, Thomson depth 1-5, L = 15
"""
import numpy as np

MEC2_KEV = 510.99895


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def grid_coords(n, nz=None):
    """Point coordinates on the unit cube: x_i = i/n (periodic), z_m = m/(nz-1)."""
    nz = n if nz is None else nz
    x = np.arange(n) / n
    z = np.arange(nz) / (nz - 1)
    Z, Yc, X = np.meshgrid(z, x, x, indexing="ij")
    return X.ravel(), Yc.ravel(), Z.ravel()


def gaussian_random_field(n, nz, ell, gen):
    """White noise on an n x n x nz periodic box, smoothed in Fourier space by
    exp(-|k|^2 ell^2 / 4) and standardised to zero mean and unit variance."""
    w = gen.standard_normal((nz, n, n))
    kx = 2 * np.pi * np.fft.fftfreq(n, d=1.0 / n)
    kz = 2 * np.pi * np.fft.fftfreq(nz, d=1.0 / nz)
    KZ, KY, KX = np.meshgrid(kz, kx, kx, indexing="ij")
    f = np.fft.ifftn(np.fft.fftn(w) * np.exp(-(KX ** 2 + KY ** 2 + KZ ** 2) * ell ** 2 / 4)).real
    f = (f - f.mean()) / f.std()
    return f.ravel()


def normal_cdf(x):
    from scipy.special import ndtr
    return ndtr(x)


def jet_beta(n, nz, gamma_max, r_jet=0.5, width2=0.02):
    """Cylindrical jet along +z on the axis x = y = 1/2:
    Gamma(r) = 1 + (Gamma_max - 1) exp(-r^2 / width2) for r <= r_jet, beta = 0 beyond."""
    X, Yc, Z = grid_coords(n, nz)
    r2 = (X - 0.5) ** 2 + (Yc - 0.5) ** 2
    gam = 1.0 + (gamma_max - 1.0) * np.exp(-r2 / width2)
    b = np.sqrt(np.maximum(0.0, 1.0 - 1.0 / gam ** 2))
    b[r2 > r_jet ** 2] = 0.0
    beta = np.zeros((X.size, 3))
    beta[:, 2] = b
    return beta


def planck(nu, kt):
    """2 nu^3 / (exp(nu/kT) - 1) in units h = c = 1 (0 where exp overflows)."""
    x = np.asarray(nu, dtype=np.float64) / kt
    out = np.zeros_like(x)
    ok = x < 700.0
    out[ok] = 2.0 * np.asarray(nu, dtype=np.float64)[ok] ** 3 / np.expm1(x[ok])
    return out


def _centres_for_input(edges, log_centres):
    e = np.asarray(edges, dtype=np.float64)
    return np.sqrt(e[:-1] * e[1:]) if log_centres else 0.5 * (e[:-1] + e[1:])


def uniform_slab(n=16, lmax=3, nmu=8, nphi=16, kappa=1.0, sigma=1.0, B=1.0, beta=None):
    """Plain method, grey: uniform absorption, Thomson scattering and emission."""
    P = n * n * n
    return dict(nx=n, ny=n, nz=n, lx=1.0, ly=1.0, lz=1.0, nmu=nmu, nphi=nphi, lmax=lmax,
                edges=None, log_centres=True, scatter="thomson", mec2=MEC2_KEV,
                kappa=np.full((P, 1), kappa), sigma=np.full(P, sigma), bnu=np.full((P, 1), B),
                beta=None if beta is None else np.tile(np.asarray(beta, float), (P, 1)),
                kte=None, bc_bot=None, bc_top=None)


def thomson_jet(n=32, ng=16, lmax=7, nmu=16, nphi=32, gamma_max=10.0, seed=2, nz=None):
    """Relativistic Thomson flow: kappa = 0.5, sigma log-uniform in [0.1, 10]
    per point, comoving blackbody (T = 1) in ng log groups over h nu / kT in
    [0.01, 100], jet with Gamma_max."""
    nz = n if nz is None else nz
    P = n * n * nz
    gen = rng(seed)
    sigma = 10.0 ** gen.uniform(-1.0, 1.0, P)
    edges = 10.0 ** (-2.0 + 4.0 * np.arange(ng + 1) / ng)
    nu = _centres_for_input(edges, True)
    bnu = np.tile(planck(nu, 1.0), (P, 1))
    return dict(nx=n, ny=n, nz=nz, lx=1.0, ly=1.0, lz=1.0, nmu=nmu, nphi=nphi, lmax=lmax,
                edges=edges, log_centres=True, scatter="thomson", mec2=MEC2_KEV,
                kappa=np.full((P, ng), 0.5), sigma=sigma, bnu=bnu,
                beta=jet_beta(n, nz, gamma_max), kte=None, bc_bot=None, bc_top=None)


def compton_jet(n=64, ng=32, lmax=15, nmu=16, nphi=32, gamma_max=10.0, seed=3, nz=None,
                e_lo=1e-3, e_hi=1e3, kt_seed=1.0):
    """Compton scattering in a jet: ng log groups over [e_lo, e_hi] keV,
    kT_e = 10^(1 + Phi(g1)) keV and n_e sigma_T = 1 + 4 Phi(g2) from two smooth
    Gaussian random fields (correlation length 0.1; g1 from the first stream of
    the seed, g2 from the second), kappa = 0.1 with a blackbody seed at 1 keV."""
    nz = n if nz is None else nz
    P = n * n * nz
    g1 = gaussian_random_field(n, nz, 0.1, rng([seed, 0]))
    g2 = gaussian_random_field(n, nz, 0.1, rng([seed, 1]))
    kte = 10.0 ** (1.0 + normal_cdf(g1))
    sigma = 1.0 + 4.0 * normal_cdf(g2)
    edges = np.exp(np.linspace(np.log(e_lo), np.log(e_hi), ng + 1))
    nu = _centres_for_input(edges, True)
    bnu = np.tile(planck(nu, kt_seed), (P, 1))
    return dict(nx=n, ny=n, nz=nz, lx=1.0, ly=1.0, lz=1.0, nmu=nmu, nphi=nphi, lmax=lmax,
                edges=edges, log_centres=True, scatter="compton", mec2=MEC2_KEV,
                kappa=np.full((P, ng), 0.1), sigma=sigma, bnu=bnu,
                beta=jet_beta(n, nz, gamma_max), kte=kte, bc_bot=None, bc_top=None)


def random_medium(n=8, nz=None, ng=4, lmax=3, nmu=4, nphi=8, seed=11, scatter="thomson",
                  gamma_max=5.0, edges=None, log_centres=True, with_bc=True, grey=False):
    """Small random problem for parity tests: every field drawn i.i.d. from the seed,
    with a random velocity field (|beta| up to that of gamma_max) and random
    z-boundary inflow."""
    nz = n if nz is None else nz
    P = n * n * nz
    gen = rng(seed)
    if grey:
        ng = 1
        edges = None
    elif edges is None:
        edges = 10.0 ** np.linspace(-1.0, 1.0, ng + 1) if log_centres else np.linspace(0.0, 1.1, ng + 1)
    else:
        ng = len(edges) - 1
    K = nmu * nphi
    bmax = np.sqrt(1.0 - 1.0 / gamma_max ** 2)
    d = gen.standard_normal((P, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    beta = d * (bmax * gen.uniform(0.0, 1.0, (P, 1)) ** 0.5)
    spec = dict(nx=n, ny=n, nz=nz, lx=1.0, ly=1.0, lz=1.0, nmu=nmu, nphi=nphi, lmax=lmax,
                edges=edges, log_centres=log_centres, scatter=scatter,
                mec2=1.0 if not log_centres else MEC2_KEV,
                kappa=gen.uniform(0.2, 2.0, (P, ng)), sigma=10.0 ** gen.uniform(-1, 1, P),
                bnu=gen.uniform(0.5, 2.0, (P, ng)), beta=beta, kte=None,
                bc_bot=gen.uniform(0.0, 1.0, (K, n, n, ng)) if with_bc else None,
                bc_top=gen.uniform(0.0, 1.0, (K, n, n, ng)) if with_bc else None)
    return spec


# ---------------------------------------------------------------------------
# The paper's validation problems (Sec. 3), two-dimensional: ny = 1, symmetry
# in y.  Lengths are in units of the paper's 1e10 cm domain side, so with c = 1
# one time unit is 1/3 s; x is periodic and z has nz points on [0, 1].  Each
# generator returns the problem description and the initial lab intensity
# (K, P, 1).  Where light enters through the bottom face, the initial field
# already holds the inflow on that face (the beam is on from t = 0): the
# inflow-face values are prescribed data that no time step changes.
# ---------------------------------------------------------------------------

DOMAIN_CM = 1.0e10
SECOND = 3.0            # c t for t = 1 s, in domain sides (c = 3e10 cm/s)


def _plane(n, nz):
    x = np.arange(n) / n
    z = np.arange(nz) / (nz - 1)
    Z, X = np.meshgrid(z, x, indexing="ij")
    return X.ravel(), Z.ravel()


def _two_d(n, nz, nmu, nphi, lmax, kappa, sigma, bnu, beta=None, bc_bot=None):
    return dict(nx=n, ny=1, nz=nz, lx=1.0, ly=1.0 / n, lz=1.0, nmu=nmu, nphi=nphi, lmax=lmax,
                edges=None, log_centres=True, scatter="thomson", mec2=MEC2_KEV,
                kappa=np.asarray(kappa, float).reshape(-1, 1), sigma=np.asarray(sigma, float).ravel(),
                bnu=np.asarray(bnu, float).reshape(-1, 1), beta=beta, kte=None, bc_bot=bc_bot, bc_top=None)


def _inflow_start(spec):
    """Zero field except the bottom-face inflow (K, P, 1)."""
    K, n = spec["nmu"] * spec["nphi"], spec["nx"]
    I0 = np.zeros((K, n * spec["nz"], 1))
    I0[:, :n, 0] = spec["bc_bot"][:, 0, :, 0]
    return I0


def beam_ordinate(nmu, nphi, phi_index=0):
    """Index k = a nphi + b of the upward ordinate with the largest mu (the
    paper's 0.17 pi zenith angle for nmu = 4) and azimuth 2 pi b / nphi."""
    return (nmu - 1) * nphi + phi_index


def searchlight(n=512, nz=None, alpha_cm=0.0, nmu=4, nphi=8, lmax=1):
    """Searchlight beam (Sec. 3.1): unit intensity enters through the bottom
    face for 0.15 < x < 0.45 along the ordinate (0.17 pi, 0); uniform
    absorption alpha (1e-10 / cm in the paper's second case), no scattering."""
    nz = n if nz is None else nz
    X, Z = _plane(n, nz)
    P, K = X.size, nmu * nphi
    bc = np.zeros((K, 1, n, 1))
    x = np.arange(n) / n
    bc[beam_ordinate(nmu, nphi), 0, (x > 0.15) & (x < 0.45), 0] = 1.0
    spec = _two_d(n, nz, nmu, nphi, lmax, np.full(P, alpha_cm * DOMAIN_CM), np.zeros(P), np.zeros(P), bc_bot=bc)
    return spec, _inflow_start(spec)


def two_beam_shadow(n=512, nz=None, nmu=4, nphi=8, lmax=1, beams=(0, 1)):
    """Two beams and a shadow (Sec. 3.2): plane-parallel unit intensity enters
    through the whole bottom face along (0.17 pi, 0) and (0.17 pi, pi); an
    absorbing cylinder of radius 0.15 about (x, z) = (0.5, 0.33), optical depth
    100 across its diameter, in vacuum.  `beams` selects which of the two enter."""
    nz = n if nz is None else nz
    X, Z = _plane(n, nz)
    P, K = X.size, nmu * nphi
    kap = np.where((X - 0.5) ** 2 + (Z - 0.33) ** 2 <= 0.15 ** 2, 3.3e-8 * DOMAIN_CM, 0.0)
    bc = np.zeros((K, 1, n, 1))
    for b in beams:
        bc[beam_ordinate(nmu, nphi, b * nphi // 2), 0, :, 0] = 1.0
    spec = _two_d(n, nz, nmu, nphi, lmax, kap, np.zeros(P), np.zeros(P), bc_bot=bc)
    return spec, _inflow_start(spec)


def radiative_pulse(n=128, nz=None, nmu=64, nphi=128, lmax=1, thick=False, w_cm=9.0e8):
    """Radiative pulse (Sec. 3.3): an isotropic initial intensity
    100 exp(-(r/w)^2) about the domain centre in vacuum (thin), or
    100 exp(-(x/w)^2) in a purely scattering medium of Thomson depth 300 across
    the domain (thick, isotropic scattering: the Thomson kernel with L = 0).
    Returns (problem, initial lab intensity)."""
    nz = (n + 1) if nz is None else nz
    X, Z = _plane(n, nz)
    P, K = X.size, nmu * nphi
    w = w_cm / DOMAIN_CM
    dx, dz = X - 0.5, Z - 0.5
    prof = 100.0 * np.exp(-(dx / w) ** 2) if thick else 100.0 * np.exp(-(dx ** 2 + dz ** 2) / w ** 2)
    sig = np.full(P, 3.0e-8 * DOMAIN_CM if thick else 0.0)
    spec = _two_d(n, nz, nmu, nphi, 0 if thick else lmax, np.zeros(P), sig, np.zeros(P))
    I0 = np.broadcast_to(prof[None, :, None], (K, P, 1)).copy()
    # vacuum inflow: no light enters through either face (upward ordinates at
    # z = 0, downward ones at z = 1)
    up = np.repeat(np.arange(nmu) >= nmu // 2, nphi)
    I0[up, :n] = 0.0
    I0[~up, P - n:] = 0.0
    return spec, I0


def beaming_cylinder(n=128, nz=None, nmu=32, nphi=64, lmax=1, beta=(0.0, 0.0), radius_cm=5.0e8,
                     kappa=1e-9, emission=1.0):
    """Relativistic beaming (Sec. 3.4): a cylinder of radius 5e8 cm about the
    domain centre whose matter moves with beta = (vx/c, vz/c) and emits
    isotropically in its own frame (emissivity kappa B = `emission`, with an
    absorption coefficient small enough to leave the light unabsorbed); vacuum
    at rest outside.  Returns (problem, zero initial lab intensity)."""
    nz = (n + 1) if nz is None else nz
    X, Z = _plane(n, nz)
    P = X.size
    inside = (X - 0.5) ** 2 + (Z - 0.5) ** 2 <= (radius_cm / DOMAIN_CM) ** 2
    kap = np.where(inside, kappa, 0.0)
    B = np.where(inside, emission / kappa, 0.0)
    b = np.zeros((P, 3))
    b[inside, 0], b[inside, 2] = beta[0], beta[1]
    spec = _two_d(n, nz, nmu, nphi, lmax, kap, np.zeros(P), B, beta=b)
    return spec, np.zeros((nmu * nphi, P, 1))
