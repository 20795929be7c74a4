"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every check here compares the oracle with something other than itself: a
library routine, a closed form, an exact discrete invariant, an independent
brute-force computation written in this file, or a value the paper prints
(``tests/golden/paper_values.json``).  None of them needs a GPU.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate, special

import oracle
from paper_1507_05141_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def spec_uniform(n=4, nz=None, nmu=4, nphi=8, lmax=3, kappa=1.0, sigma=0.0, B=0.0, edges=None,
                 lx=1.0, ly=1.0, lz=1.0, beta=None, bc_bot=None, bc_top=None, scatter="thomson", mec2=1.0,
                 log_centres=True):
    nz = n if nz is None else nz
    P = n * n * nz
    G = 1 if edges is None else len(edges) - 1
    kap = np.broadcast_to(np.asarray(kappa, float), (P, G)).copy()
    return dict(nx=n, ny=n, nz=nz, lx=lx, ly=ly, lz=lz, nmu=nmu, nphi=nphi, lmax=lmax,
                edges=edges, log_centres=log_centres, scatter=scatter, mec2=mec2,
                kappa=kap, sigma=np.full(P, float(sigma)), bnu=np.broadcast_to(np.asarray(B, float), (P, G)).copy(),
                beta=None if beta is None else np.broadcast_to(np.asarray(beta, float), (P, 3)).copy(),
                kte=None, bc_bot=bc_bot, bc_top=bc_top)


def ordinate_dirs(o):
    mu = np.repeat(o.mu, o.nphi)
    phi = np.tile(2 * np.pi * np.arange(o.nphi) / o.nphi, o.nmu)
    st = np.sqrt(1 - mu ** 2)
    return np.stack([st * np.cos(phi), st * np.sin(phi), mu], axis=1), mu, phi


# ---------------------------------------------------------------------------
# quadrature and spherical harmonics (Eq. 9)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 3, 4, 8, 16, 32])
def test_gauss_legendre_matches_library(n):
    x, w = oracle.gauss_legendre(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    assert np.allclose(x, xr, atol=1e-14, rtol=0)
    assert np.allclose(w, wr, atol=1e-14, rtol=0)


def test_searchlight_angle_is_a_four_point_gauss_node():
    g = json.load(open(GOLDEN))["searchlight_beam_angle"]
    x, _ = oracle.gauss_legendre(g["n_theta"])
    assert abs(math.acos(x[-1]) / math.pi - g["theta_over_pi"]) < 5e-3


def test_real_sh_against_scipy():
    rs = np.random.default_rng(0)
    L = 15
    for _ in range(20):
        mu = rs.uniform(-1, 1)
        phi = rs.uniform(0, 2 * np.pi)
        Y = oracle.sh_eval(L, mu, phi)
        theta = math.acos(mu)
        for l in range(L + 1):
            for m in range(-l, l + 1):
                c = special.sph_harm_y(l, abs(m), theta, phi)   # includes the (-1)^m phase
                if m == 0:
                    ref = c.real
                elif m > 0:
                    ref = math.sqrt(2) * (-1) ** m * c.real
                else:
                    ref = math.sqrt(2) * (-1) ** m * c.imag
                assert abs(Y[l * l + l + m] - ref) < 1e-12 * max(1.0, abs(ref)), (l, m)


@pytest.mark.parametrize("nmu,nphi,L", [(8, 16, 3), (16, 32, 7), (16, 32, 15), (4, 8, 3)])
def test_sh_discrete_orthonormality(nmu, nphi, L):
    o = oracle.Oracle(spec_uniform(n=2, nz=2, nmu=nmu, nphi=nphi, lmax=L))
    w = np.repeat(o.wmu, nphi) * 2 * np.pi / nphi
    assert abs(w.sum() - 4 * np.pi) < 1e-13
    dirs, mu, _ = ordinate_dirs(o)
    assert abs((w * mu ** 2).sum() - 4 * np.pi / 3) < 1e-13
    M = (o.Y * w[:, None]).T @ o.Y
    assert np.abs(M - np.eye(o.NL)).max() < 1e-12


def test_sh_addition_theorem():
    rs = np.random.default_rng(1)
    L = 7
    for _ in range(10):
        a = rs.normal(size=3); a /= np.linalg.norm(a)
        b = rs.normal(size=3); b /= np.linalg.norm(b)
        Ya = oracle.sh_eval(L, a[2], math.atan2(a[1], a[0]))
        Yb = oracle.sh_eval(L, b[2], math.atan2(b[1], b[0]))
        for l in range(L + 1):
            s = sum(Ya[l * l + l + m] * Yb[l * l + l + m] for m in range(-l, l + 1))
            assert abs(s - (2 * l + 1) / (4 * np.pi) * special.eval_legendre(l, a @ b)) < 1e-12


# ---------------------------------------------------------------------------
# source function (Eqs. 10-12): brute-force angular integral of the phase function
# ---------------------------------------------------------------------------

def _fine_sphere(nm=40, nf=80):
    x, w = np.polynomial.legendre.leggauss(nm)
    phi = 2 * np.pi * np.arange(nf) / nf
    MU, PH = np.meshgrid(x, phi, indexing="ij")
    st = np.sqrt(1 - MU ** 2)
    dirs = np.stack([st * np.cos(PH), st * np.sin(PH), MU], -1).reshape(-1, 3)
    ww = (w[:, None] * np.full(nf, 2 * np.pi / nf)[None, :]).ravel()
    return dirs, ww


def _sh_at(L, dirs):
    return np.array([oracle.sh_eval(L, d[2], math.atan2(d[1], d[0])) for d in dirs])


def test_thomson_source_equals_phase_function_integral():
    L = 3
    kap, sig, B = 0.7, 1.9, 1.3
    o = oracle.Oracle(spec_uniform(n=2, nz=2, nmu=8, nphi=16, lmax=L, kappa=kap, sigma=sig, B=B))
    rs = np.random.default_rng(2)
    I_lm = np.zeros(o.sh_shape())
    I_lm[:] = rs.normal(size=o.NL)
    S = o.source(I_lm)[0, 0]
    dirs, ww = _fine_sphere()
    Yf = _sh_at(L, dirs)
    I_f = Yf @ I_lm[0, 0]
    rs_dirs = rs.normal(size=(6, 3))
    rs_dirs /= np.linalg.norm(rs_dirs, axis=1, keepdims=True)
    chi = kap + sig
    for n in rs_dirs:
        cos = dirs @ n
        phase = 0.75 * (1 + cos ** 2)                         # Eq. 12, normalised to 4 pi
        ref = sig / chi * np.sum(ww * phase * I_f) / (4 * np.pi) + kap * B / chi
        got = oracle.sh_eval(L, n[2], math.atan2(n[1], n[0])) @ S
        assert abs(got - ref) < 1e-12


def test_thomson_scattering_conserves_photons():
    """kappa = 0: the isotropic part of the source equals that of the intensity."""
    o = oracle.Oracle(spec_uniform(n=2, nz=2, lmax=3, kappa=0.0, sigma=3.0, B=5.0))
    rs = np.random.default_rng(3)
    I_lm = rs.normal(size=o.sh_shape())
    S = o.source(I_lm)
    assert np.allclose(S[..., 0], I_lm[..., 0], rtol=0, atol=1e-14)


# ---------------------------------------------------------------------------
# Klein-Nishina tables (Eqs. 13-14)
# ---------------------------------------------------------------------------

def kn_total_closed_form(x):
    """Klein-Nishina total cross-section / sigma_T (Rybicki & Lightman Eq. 7.5),
    evaluated in 60-digit decimal arithmetic (the formula cancels badly at small x)."""
    from decimal import Decimal, getcontext
    getcontext().prec = 60
    X = Decimal(repr(float(x)))
    one, two = Decimal(1), Decimal(2)
    lg = (one + two * X).ln()
    v = Decimal("0.75") * ((one + X) / X ** 3 * (two * X * (one + X) / (one + two * X) - lg)
                           + lg / (two * X) - (one + 3 * X) / (one + two * X) ** 2)
    return float(v)


def test_compton_total_cross_section_closed_form():
    xs = np.array([1e-3, 0.01, 0.1, 0.5, 1.0, 1.05, 2.0, 5.0])
    edges = np.concatenate([[0.0], np.sort(np.concatenate([xs * 0.99, xs * 1.01]))])
    centres = xs                           # evaluate at exactly these energies
    s, _ = oracle.compton_cold(np.linspace(0, 6, 9), centres, 1.0, 2)
    for x, v in zip(xs, s):
        assert abs(v - kn_total_closed_form(x)) < 1e-12 * kn_total_closed_form(x)


def test_compton_tables_match_direct_quadrature():
    """Each Legendre moment p_l^{i->j} against an adaptive integral of the
    Klein-Nishina cross-section written independently here."""
    g = json.load(open(GOLDEN))["compton_injection"]
    edges = np.linspace(0.0, g["e_max_mec2"], g["n_bins"] + 1)
    centres = 0.5 * (edges[:-1] + edges[1:])
    L = 4
    s, p = oracle.compton_cold(edges, centres, 1.0, L)
    for i in (3, 9):
        x = centres[i]

        def dsdo(mu):
            e = 1.0 / (1.0 + x * (1.0 - mu))
            return 0.5 * e * e * (1.0 / e + e - (1.0 - mu * mu))

        tot = 2 * np.pi * integrate.quad(dsdo, -1, 1, epsabs=1e-15, epsrel=1e-14)[0]
        for j in range(len(centres)):
            for l in range(L + 1):
                def f(mu):
                    nu1 = x / (1 + x * (1 - mu))
                    inside = edges[j] <= nu1 < edges[j + 1]
                    return dsdo(mu) * special.eval_legendre(l, mu) if inside else 0.0
                pts = [1 - (x / e - 1) / x for e in edges if e > 0 and -1 < 1 - (x / e - 1) / x < 1]
                ref = (2 * l + 1) / 2 * 4 * np.pi / tot * integrate.quad(
                    f, -1, 1, points=pts or None, limit=200, epsabs=1e-14, epsrel=1e-12)[0]
                assert abs(p[l, i, j] - ref) < 1e-9, (i, j, l)


def test_compton_normalisation_downscatter_and_recoil_limit():
    g = json.load(open(GOLDEN))["compton_injection"]
    edges = np.linspace(0.0, g["e_max_mec2"], g["n_bins"] + 1)
    centres = 0.5 * (edges[:-1] + edges[1:])
    s, p = oracle.compton_cold(edges, centres, 1.0, 6)
    # photons scattered from bin i stay inside [0, e_max): number is conserved
    assert np.allclose(p[0].sum(axis=1), 1.0, atol=1e-13)
    # electrons at rest only take energy: no up-scattering
    for i in range(len(centres)):
        assert np.all(p[:, i, i + 1:] == 0.0)
    # minimum scattered energy nu/(1+2x): for the top bin centre 1.045 it is 0.3382,
    # so bins 0-2 receive nothing and bin 3 [0.33, 0.44) does
    i = len(centres) - 1
    x = centres[i]
    numin = x / (1 + 2 * x)
    assert edges[3] < numin < edges[4]
    assert np.all(p[0, i, :3] == 0.0) and p[0, i, 3] > 0.0
    # the paper's injection energy 1.05 m_e c^2 has minimum 0.3387 m_e c^2
    assert abs(g["e_inject_mec2"] / (1 + 2 * g["e_inject_mec2"]) - 0.3387) < 1e-4


def test_compton_thomson_limit():
    edges = 10.0 ** np.linspace(-7, -5, 5)
    centres = np.sqrt(edges[:-1] * edges[1:])
    s, p = oracle.compton_cold(edges, centres, 1.0, 4)
    assert np.allclose(s, 1.0, atol=1e-4)
    for i in range(4):
        assert abs(p[0, i, i] - 1.0) < 1e-4 and abs(p[2, i, i] - 0.5) < 1e-4
        assert abs(p[1, i, i]) < 1e-4 and abs(p[3, i, i]) < 1e-4
    off = p.copy()
    for i in range(4):
        off[:, i, i] = 0
    assert np.abs(off).max() < 1e-4


def test_compton_source_conserves_photon_number():
    """Photons removed by scattering from all groups equal photons re-emitted
    (isotropic part), with the bin-width and centre-frequency weights."""
    edges = np.linspace(0.0, 1.1, 11)
    o = oracle.Oracle(spec_uniform(n=2, nz=2, lmax=3, kappa=0.0, sigma=2.0, B=0.0, edges=edges,
                                   scatter="compton", mec2=1.0, log_centres=False))
    rs = np.random.default_rng(4)
    I_lm = rs.uniform(0.1, 1.0, o.sh_shape())
    S = o.source(I_lm)
    dnu = np.diff(o.edges)
    chi = o.sigma[0] * o.kn_s
    emitted = np.sum(dnu / o.centres * chi * S[0, :, 0])
    absorbed = np.sum(dnu / o.centres * o.sigma[0] * o.kn_s * I_lm[0, :, 0])
    assert abs(emitted - absorbed) < 1e-13 * absorbed


def test_compton_source_reduces_to_thomson_at_low_energy():
    edges = 10.0 ** np.linspace(-8, -7, 5)
    base = dict(n=2, nz=2, lmax=3, kappa=0.3, sigma=1.7, B=0.8, edges=edges, mec2=1.0)
    oc = oracle.Oracle(spec_uniform(scatter="compton", **base))
    ot = oracle.Oracle(spec_uniform(scatter="thomson", **base))
    I_lm = np.random.default_rng(5).normal(size=oc.sh_shape())
    assert np.allclose(oc.source(I_lm), ot.source(I_lm), rtol=0, atol=1e-6)


# ---------------------------------------------------------------------------
# Compton scattering on hot electrons (a Maxwell-Juttner average of the
# Klein-Nishina rate; not in the paper, whose electrons are at rest)
# ---------------------------------------------------------------------------

KEV_EDGES = np.exp(np.linspace(np.log(20.0), np.log(2000.0), 7))


def test_thermal_compton_tables_reduce_to_the_cold_kernel():
    """kT = 0 is the paper's kernel (electrons at rest, Eqs. 13-14) exactly;
    at kT = 1e-12 keV the electrons' motion changes the tables by less than
    1e-10."""
    c = oracle.group_centres(KEV_EDGES, True)
    s0, p0 = oracle.compton_cold(KEV_EDGES, c, W.MEC2_KEV, 3)
    for kT, tol in ((0.0, 1e-14), (1e-12, 1e-10)):
        s, p = oracle.compton_thermal(KEV_EDGES, c, W.MEC2_KEV, 3, kT)
        assert np.abs(s - s0).max() < tol and np.abs(p - p0).max() < tol, kT


def test_thermal_compton_rate_integrates_to_the_invariant_cross_section():
    """Integrating the lab-frame rate of a moving electron over every
    scattered direction gives (1 - beta.n) sigma_KN(nu') (the cross-section is
    invariant; the flux factor counts the electrons met per unit photon path),
    so both totals agree; and in the Thomson limit (h nu -> 0) the flux factor
    averages to 1 over isotropic electrons at any temperature."""
    for nu, kT in ((50.0, 10.0), (500.0, 100.0), (1e-4, 50.0)):
        s, _, tot = oracle.compton_thermal_moments(nu, W.MEC2_KEV, kT)
        assert abs(tot / s - 1) < 1e-7, (nu, kT)
    for theta in (0.01, 0.1):
        s, _, _ = oracle.compton_thermal_moments(1e-9, 1.0, theta)
        assert abs(s - 1) < 1e-7


def test_thermal_compton_mean_energy_exchange_nonrelativistic_limit():
    """Mean fractional energy change per scattering (4 kT - h nu) / m_e c^2
    for kT, h nu << m_e c^2 (Rybicki & Lightman, Eq. 7.36); the corrections are
    of relative order kT/m_e c^2 and h nu/m_e c^2."""
    for x, th in ((1e-4, 1e-4), (1e-4, 3e-4), (3e-4, 1e-4), (2e-5, 1e-5)):
        shift = oracle.compton_thermal_moments(x * W.MEC2_KEV, W.MEC2_KEV, th * W.MEC2_KEV)[1]
        assert abs(shift / (4 * th - x) - 1) < 20 * max(x, th), (x, th, shift)


def test_thermal_compton_tables_conserve_photons_within_the_groups():
    """Every photon scattered from a group whose reachable frequencies stay
    inside the edges lands in some group: sum_j p_0^{i->j} = 1, and at most 1
    near the ends of the range; s > 0."""
    edges = np.exp(np.linspace(np.log(1e-3), np.log(1e3), 17))
    c = oracle.group_centres(edges, True)
    s, p = oracle.compton_thermal(edges, c, W.MEC2_KEV, 3, 10.0)
    tot = p[0].sum(axis=1)
    assert np.all(tot <= 1 + 1e-7) and np.all(s > 0)
    assert np.abs(tot[4:10] - 1).max() < 1e-7


def test_thermal_compton_bin_fractions_by_brute_force():
    """The scattered photons' split among the groups, checked on one incident
    group at 100 keV against a brute-force integration written here: the same
    electron and azimuth nodes, but along the scattering cosine a fine midpoint
    rule that sorts each sample into its group (no band limits), for p_0 and
    p_1 of every target group."""
    edges = np.exp(np.linspace(np.log(1e-3), np.log(1e3), 13))
    c = oracle.group_centres(edges, True)
    mec2, kT, i = W.MEC2_KEV, 100.0, 10
    s, p = oracle.compton_thermal(edges, c, mec2, 1, kT)
    nu, x, th = c[i], c[i] / mec2, kT / mec2
    tx, tw = np.polynomial.legendre.leggauss(16)
    ex, ew = np.polynomial.legendre.leggauss(16)
    fx, fw = np.polynomial.legendre.leggauss(12)
    m = 50000
    mu1 = -1 + (np.arange(m) + 0.5) * (2.0 / m)
    s1 = np.sqrt(1 - mu1 ** 2)
    acc = np.zeros((2, len(c)))
    wsum = tot = 0.0
    for a in range(16):
        t = 3 * (tx[a] + 1)
        gam = 1 + th * t * t
        pm = math.sqrt(gam * gam - 1)
        beta = pm / gam
        wt = 3 * tw[a] * pm * gam * t * math.exp(-t * t)
        wsum += wt
        for b in range(16):
            mue = ex[b]
            for f in range(12):
                cph = math.cos(0.5 * np.pi * (fx[f] + 1))
                w = wt * 0.5 * ew[b] * 0.5 * fw[f]
                # the scattering in the electron's rest frame, seen from the lab
                bo, bo1 = beta * mue, beta * (math.sqrt(1 - mue * mue) * s1 * cph + mue * mu1)
                nu1 = nu * (1 - bo) / (1 - bo1 + x / gam * (1 - mu1))
                nup, nu1p = gam * nu * (1 - bo), gam * nu1 * (1 - bo1)
                cos_r = 1 - nu * nu1 * (1 - mu1) / (nup * nu1p)
                r = nu1p / nup
                rate = (1 - bo) * 0.5 * r * r * (1 / r + r - (1 - cos_r ** 2)) * (nu1 / nu1p) ** 2
                grp = np.searchsorted(edges, nu1, side="right") - 1
                ok = (grp >= 0) & (grp < len(c))
                v = w * rate * (2.0 / m)
                tot += v.sum()
                acc[0] += np.bincount(grp[ok], weights=v[ok], minlength=len(c))
                acc[1] += np.bincount(grp[ok], weights=(v * mu1)[ok], minlength=len(c))
    # normalised by the total over every direction (2 pi int R dmu1 = s sigma_T)
    ref = np.array([0.5, 1.5])[:, None] * acc / (tot / 2.0)
    assert abs(2 * np.pi * tot / wsum / (8 * np.pi / 3) / s[i] - 1) < 1e-6
    assert np.abs(p[:, i, :] - ref).max() < 5e-4, (p[:, i, :], ref)


def test_compton_source_with_a_uniform_node_temperature_uses_that_node():
    """A uniform temperature field on one node temperature gives the source
    of the tables at that temperature, and the extinction sigma s(T)."""
    edges = KEV_EDGES
    kte = 10.0 ** 1.25
    base = dict(n=2, nz=2, lmax=3, kappa=0.3, sigma=1.7, B=0.8, edges=edges, mec2=W.MEC2_KEV, scatter="compton")
    spec = spec_uniform(**base)
    spec["kte"] = np.full(8, kte)
    o = oracle.Oracle(spec)
    assert np.allclose(o.lt_nodes, [1.25])
    c = oracle.group_centres(edges, True)
    s, p = oracle.compton_thermal(edges, c, W.MEC2_KEV, 3, kte)
    I_lm = np.random.default_rng(8).normal(size=o.sh_shape())
    S = o.source(I_lm)
    G = len(c)
    dnu = np.diff(edges)
    chi = 0.3 + 1.7 * s
    for l in range(4):
        A = s[:, None] * (c[None, :] * dnu[:, None]) / (c[:, None] * dnu[None, :]) * p[l] / (2 * l + 1)  # [i][j]
        for m in range(-l, l + 1):
            q = l * l + l + m
            ref = 1.7 / chi[None, :] * np.einsum("ij,pi->pj", A, I_lm[:, :, q])
            if q == 0:
                ref = ref + math.sqrt(4 * np.pi) * 0.3 * 0.8 / chi[None, :]
            assert np.allclose(S[:, :, q], ref, rtol=1e-12, atol=1e-14)


def test_compton_tables_interpolate_linearly_in_log_temperature():
    """Between two node temperatures the source is the log10 T weighted mean
    of the sources at the nodes (the tables enter linearly)."""
    edges = KEV_EDGES
    base = dict(n=2, nz=2, lmax=3, kappa=0.3, sigma=1.7, B=0.0, edges=edges, mec2=W.MEC2_KEV, scatter="compton")
    lo, hi = 10.0 ** 1.25, 10.0 ** 1.375
    spec = spec_uniform(**base)
    spec["kte"] = np.array([lo, hi] + [10.0 ** 1.3] * 6)       # nodes 1.25, 1.375; 1.3 = 40 % of the way
    o = oracle.Oracle(spec)
    assert np.allclose(o.lt_nodes, [1.25, 1.375])
    I_lm = np.random.default_rng(9).normal(size=o.sh_shape())
    I_lm[:] = I_lm[:1]
    S = o.source(I_lm)
    chi = o.kappa + o.sigma[:, None] * (np.stack([o.kn_s[0], o.kn_s[1]]).T @ np.array([[1, 0, 0.6], [0, 1, 0.4]]))[:, [0, 1, 2, 2, 2, 2, 2, 2]].T
    # the scattering part times chi / sigma is linear in the node tables
    Ssc = S * (chi / 1.7)[:, :, None]
    assert np.allclose(Ssc[2], 0.6 * Ssc[0] + 0.4 * Ssc[1], rtol=1e-12, atol=1e-14)


# ---------------------------------------------------------------------------
# Lorentz maps (Eqs. 7-8) and the invariants
# ---------------------------------------------------------------------------

def test_isotropic_boost_is_exact_for_an_invariant_linear_in_log_nu():
    edges = 10.0 ** np.linspace(-1, 1, 9)
    n = 3
    P = n ** 3
    rs = np.random.default_rng(6)
    beta = rs.normal(size=(P, 3))
    beta /= np.linalg.norm(beta, axis=1, keepdims=True)
    beta *= rs.uniform(0, 0.6, (P, 1))
    kap = 0.9
    o = oracle.Oracle(spec_uniform(n=n, nmu=8, nphi=16, lmax=3, kappa=kap, sigma=0.4, B=0.0,
                                   edges=edges, beta=beta))
    a, b = 2.0, 0.7
    nu = o.centres
    S_lm = np.zeros(o.sh_shape())
    S_lm[:, :, 0] = math.sqrt(4 * np.pi) * nu ** 3 * (a + b * np.log(nu))
    S0 = o.sh2do(S_lm)
    I_prev = rs.uniform(0, 1, o.lab_shape())
    icdt = 3.0
    St, Xt = o.boost(S0, I_prev, icdt)
    dirs, _, _ = ordinate_dirs(o)
    chi0 = kap + 0.4
    lo, hi = np.log(nu[0]), np.log(nu[-1])
    checked = 0
    for p in range(P):
        bb = beta[p]
        gam = 1 / math.sqrt(1 - bb @ bb)
        D = 1 / (gam * (1 - dirs @ bb))                    # nu / nu0 from Eq. 7
        for g in range(o.G):
            x = np.log(nu[g] / D)
            ok = (x >= lo) & (x <= hi)
            s_lab = nu[g] ** 3 * (a + b * x)
            chi_lab = chi0 / D
            ref = (chi_lab * s_lab + I_prev[:, p, g] * icdt) / (chi_lab + icdt)
            assert np.allclose(Xt[ok, p, g], (chi_lab + icdt)[ok], rtol=1e-13, atol=0)
            assert np.allclose(St[ok, p, g], ref[ok], rtol=1e-12, atol=0)
            checked += ok.sum()
    assert checked > 1000


def test_grey_boost_direction_map():
    """Comoving source a + b mu0 (exact under bilinear interpolation inside the
    rings) seen from the lab: D^4 (a + b mu0(n)) with the textbook aberration."""
    a, b = 1.5, 0.8
    for axis, bv in ((2, 0.5), (2, -0.8), (0, 0.7), (1, 0.3)):
        beta = np.zeros(3)
        beta[axis] = bv
        o = oracle.Oracle(spec_uniform(n=2, nz=2, nmu=8, nphi=16, lmax=3, kappa=1.0, beta=beta))
        S_lm = np.zeros(o.sh_shape())
        S_lm[..., 0] = math.sqrt(4 * np.pi) * a
        S_lm[..., 2] = math.sqrt(4 * np.pi / 3) * b
        St, Xt = o.boost(o.sh2do(S_lm))
        dirs, mu, _ = ordinate_dirs(o)
        gam = 1 / math.sqrt(1 - bv * bv)
        D = 1 / (gam * (1 - bv * dirs[:, axis]))
        if axis == 2:
            mu0 = (mu - bv) / (1 - bv * mu)
        else:
            mu0 = D * mu
        inside = (mu0 > o.mu[0]) & (mu0 < o.mu[-1])
        ref = D ** 4 * (a + b * mu0)
        assert inside.sum() > 40
        assert np.allclose(St[inside, 0, 0], ref[inside], rtol=1e-12)
        assert np.allclose(Xt[:, 0, 0], 1.0 / D, rtol=1e-13)


def test_grey_unboost_inverse_map():
    a, b = 1.2, -0.5
    bv = 0.6
    o = oracle.Oracle(spec_uniform(n=2, nz=2, nmu=8, nphi=16, lmax=3, beta=[0, 0, bv]))
    dirs, mu, _ = ordinate_dirs(o)
    I_lab = np.zeros(o.lab_shape())
    I_lab[:, :, 0] = (a + b * mu)[:, None]
    I0 = o.unboost(I_lab)
    gam = 1 / math.sqrt(1 - bv * bv)
    mu_lab = (mu + bv) / (1 + bv * mu)             # lab direction of each comoving ordinate
    Dp = gam * (1 + bv * mu)
    inside = (mu_lab > o.mu[0]) & (mu_lab < o.mu[-1])
    ref = (a + b * mu_lab) / Dp ** 4
    assert np.allclose(I0[0, 0, inside], ref[inside], rtol=1e-12)


def test_nongrey_unboost_is_exact_for_an_invariant_linear_in_log_nu_and_mu():
    """Lab intensity nu^3 (a + b ln nu + c n_z): bilinear angle taps and the
    ln-nu interpolation of the invariant are exact for it, so the comoving
    value on ordinate n0 at centre nu is nu^3 (a + b ln(D' nu) + c n_z(n)),
    with D' = Gamma (1 + beta.n0) and n the aberrated lab direction (textbook
    velocity addition for photons).  Evaluating the invariant at nu / D'
    instead fails this check."""
    edges = 10.0 ** np.linspace(-1, 1, 11)
    n = 2
    P = n ** 3
    rs = np.random.default_rng(16)
    beta = rs.normal(size=(P, 3))
    beta /= np.linalg.norm(beta, axis=1, keepdims=True)
    beta *= rs.uniform(0.05, 0.5, (P, 1))
    o = oracle.Oracle(spec_uniform(n=n, nmu=8, nphi=16, lmax=3, kappa=1.0, edges=edges, beta=beta))
    a, b, c = 2.0, 0.45, 0.6
    nu = o.centres
    dirs, _, _ = ordinate_dirs(o)
    I_lab = nu[None, None, :] ** 3 * (a + b * np.log(nu)[None, None, :] + c * dirs[:, 2][:, None, None])
    I_lab = np.broadcast_to(I_lab, o.lab_shape()).copy()
    I0 = o.unboost(I_lab)
    lo, hi = np.log(nu[0]), np.log(nu[-1])
    checked = 0
    for p in range(P):
        bb = beta[p]
        gam = 1 / math.sqrt(1 - bb @ bb)
        for j in range(o.K):
            n0 = dirs[j]
            bn = bb @ n0
            Dp = gam * (1 + bn)
            # lab direction: the component along beta adds relativistically, the
            # transverse part shrinks by 1/(Gamma (1 + beta.n0))
            bh = bb / np.linalg.norm(bb)
            par0 = n0 @ bh
            bv = np.linalg.norm(bb)
            par = (par0 + bv) / (1 + bv * par0)
            perp = (n0 - par0 * bh) / (gam * (1 + bv * par0))
            nl = par * bh + perp
            if not (o.mu[0] < nl[2] < o.mu[-1]):
                continue
            x = np.log(Dp * nu)
            ok = (x >= lo) & (x <= hi)
            ref = nu ** 3 * (a + b * x + c * nl[2])
            assert np.allclose(I0[p, ok, j], ref[ok], rtol=1e-12, atol=0), (p, j)
            checked += ok.sum()
    assert checked > 1000


def test_ghost_taper_is_interpolation_towards_an_empty_neighbour_bin():
    """Beyond the outer group centres the invariant falls linearly in ln nu to
    zero at ghost centres mirrored about the outer edges.  For logarithmic bins
    a ghost centre is the centre of the next bin of the same width, so a boost
    with G groups must equal, frequency for frequency, the boost of the same
    spectrum with one empty bin added on each side (where the frequency stays
    inside the widened set of centres, so that the wider problem interpolates
    between real centres)."""
    G = 6
    dl = 0.25
    edges = 10.0 ** (dl * np.arange(G + 1))
    wide = 10.0 ** (dl * np.arange(-1, G + 2))
    n = 2
    P = n ** 3
    rs = np.random.default_rng(17)
    beta = rs.normal(size=(P, 3))
    beta /= np.linalg.norm(beta, axis=1, keepdims=True)
    beta *= rs.uniform(0.3, 0.7, (P, 1))
    on = oracle.Oracle(spec_uniform(n=n, nmu=8, nphi=16, lmax=3, kappa=0.0, edges=edges, beta=beta))
    ow = oracle.Oracle(spec_uniform(n=n, nmu=8, nphi=16, lmax=3, kappa=0.0, edges=wide, beta=beta))
    assert np.allclose(ow.centres[1:-1], on.centres, rtol=1e-14)
    S_lm = np.zeros(on.sh_shape())
    S_lm[:, :, 0] = math.sqrt(4 * np.pi) * on.centres ** 3 * rs.uniform(0.5, 2.0, G)
    Sw = np.zeros(ow.sh_shape())
    Sw[:, 1:-1, :] = S_lm
    St_n, _ = on.boost(on.sh2do(S_lm), None, 1.0)
    St_w, _ = ow.boost(ow.sh2do(Sw), None, 1.0)
    dirs, _, _ = ordinate_dirs(on)
    lo, hi = np.log(ow.centres[0]), np.log(ow.centres[-1])
    outside = 0
    for p in range(P):
        bb = beta[p]
        gam = 1 / math.sqrt(1 - bb @ bb)
        D = 1 / (gam * (1 - dirs @ bb))
        for g in range(G):
            x = np.log(on.centres[g] / D)
            ok = (x > lo) & (x < hi)
            assert np.allclose(St_n[ok, p, g], St_w[ok, p, g + 1], rtol=1e-12, atol=1e-300)
            outside += np.sum(ok & ((x < np.log(on.centres[0])) | (x > np.log(on.centres[-1]))))
    assert outside > 200            # the taper itself is exercised


def test_residual_closed_form():
    """S_new = (1 + e_g) S_old in group g gives ||S_new - S_old|| / ||S_new|| =
    |e_g| / |1 + e_g|; an all-zero group that did not change has residual 0,
    one that became zero has an infinite residual."""
    o = oracle.Oracle(spec_uniform(n=3, nmu=4, nphi=8, lmax=3, kappa=1.0, edges=10.0 ** np.linspace(-1, 1, 6)))
    rs = np.random.default_rng(18)
    S_old = rs.normal(size=o.sh_shape())
    e = np.array([0.1, -0.3, 2.0, 0.0, -1.0])
    S_new = S_old * (1 + e)[None, :, None]
    S_old[:, 3] = 0.0
    S_new[:, 3] = 0.0
    r = o.residual(S_old, S_new)
    assert np.allclose(r[:3], np.abs(e[:3]) / np.abs(1 + e[:3]), rtol=1e-13)
    assert r[3] == 0.0 and np.isinf(r[4])


def test_frequency_integrated_moments_of_an_isotropic_spectrum():
    """An isotropic field with group values c_g: J_tot = sum dnu_g c_g (the
    group widths), H_tot = 0, K_tot = J_tot / 3 on the diagonal, so the
    frequency-integrated Eddington tensor is 1/3 times the identity."""
    edges = 10.0 ** np.linspace(-1, 1, 6)
    o = oracle.Oracle(spec_uniform(n=2, nz=2, nmu=8, nphi=16, lmax=3, kappa=1.0, edges=edges))
    cg = np.array([0.5, 2.0, 1.5, 0.25, 3.0])
    I_lab = np.broadcast_to(cg[None, None, :], o.lab_shape()).copy()
    Jt, Ht, Kt, f = o.integrated(*o.moments_lab(I_lab))
    assert np.allclose(Jt, np.sum(np.diff(edges) * cg), rtol=1e-13)
    assert np.abs(Ht).max() < 1e-13
    assert np.allclose(f, [1 / 3, 1 / 3, 1 / 3, 0, 0, 0], atol=1e-13)


def test_comoving_moments_of_a_quadratic_field_match_closed_forms():
    """At rest, a field I(n) = a + b.n + n.C.n with a symmetric C (non-zero
    off-diagonal terms) has J = a + tr C / 3, H = b / 3 and
    K_ij = a delta_ij / 3 + (tr C delta_ij + 2 C_ij) / 15 (moments of the unit
    sphere).  The comoving moments read from the SH coefficients (l <= 2) and
    the lab quadrature moments must both give them; a swapped off-diagonal
    coefficient fails."""
    o = oracle.Oracle(spec_uniform(n=2, nz=2, nmu=8, nphi=16, lmax=3, kappa=1.0))
    dirs, _, _ = ordinate_dirs(o)
    a, b = 1.3, np.array([0.2, -0.35, 0.5])
    C = np.array([[0.4, 0.15, -0.25], [0.15, -0.1, 0.32], [-0.25, 0.32, 0.7]])
    I = a + dirs @ b + np.einsum("ki,ij,kj->k", dirs, C, dirs)
    I_lab = np.broadcast_to(I[:, None, None], o.lab_shape()).copy()
    Jr = a + np.trace(C) / 3
    Hr = b / 3
    Kr = a * np.eye(3) / 3 + (np.trace(C) * np.eye(3) + 2 * C) / 15
    k6 = np.array([Kr[0, 0], Kr[1, 1], Kr[2, 2], Kr[0, 1], Kr[0, 2], Kr[1, 2]])
    for J, H, Kt in (o.moments_lab(I_lab), o.moments_comoving(o.do2sh(o.unboost(I_lab)))):
        assert np.allclose(J, Jr, rtol=1e-13)
        assert np.allclose(H, Hr[None, None, :], rtol=0, atol=1e-13)
        assert np.allclose(Kt, k6[None, None, :], rtol=0, atol=1e-13)


def test_paper_lorentz_factors():
    """The Doppler factors used by the boost reproduce the Lorentz factors the
    paper prints for its beaming test (to the printed digits)."""
    gv = json.load(open(GOLDEN))["beaming_lorentz_factors"]
    for bv, gs in zip(gv["beta"], gv["gamma_printed"]):
        gp = float(gs)
        tol = 0.5 * 10.0 ** -(len(gs.split(".")[1]) if "." in gs else 0)
        o = oracle.Oracle(spec_uniform(n=2, nz=2, nmu=8, nphi=16, lmax=3, beta=[bv, 0, 0]))
        S_lm = np.zeros(o.sh_shape())
        S_lm[..., 0] = math.sqrt(4 * np.pi)                 # isotropic, S0 = 1
        St, _ = o.boost(o.sh2do(S_lm))
        D = St[:, 0, 0] ** 0.25
        dirs, _, _ = ordinate_dirs(o)
        g_impl = 1.0 / (D * (1 - bv * dirs[:, 0]))
        assert np.allclose(g_impl, g_impl[0], rtol=1e-12)
        assert abs(g_impl[0] - gp) <= tol


def test_isotropic_boost_high_gamma_matches_paper_bound():
    """Isotropic comoving field, flat invariant: lab I = [Gamma(1 - mu beta)]^-4
    times the comoving value for a grey group, exactly, for the paper's Gamma."""
    g = json.load(open(GOLDEN))["isotropic_boost_accuracy"]
    for cmv in g["c_minus_vz_over_c"]:
        bv = 1.0 - cmv
        o = oracle.Oracle(spec_uniform(n=2, nz=2, nmu=16, nphi=32, lmax=3, beta=[0, 0, bv]))
        S_lm = np.zeros(o.sh_shape())
        S_lm[..., 0] = math.sqrt(4 * np.pi)
        St, _ = o.boost(o.sh2do(S_lm))
        dirs, mu, _ = ordinate_dirs(o)
        gam = 1 / math.sqrt((1 - bv) * (1 + bv))
        ref = (gam * (1 - mu * bv)) ** -4.0
        assert np.max(np.abs(St[:, 0, 0] / ref - 1)) < g["max_rel_deviation"]


# ---------------------------------------------------------------------------
# ray trace and the steady solve
# ---------------------------------------------------------------------------

def test_free_streaming_translates_the_inflow_pattern():
    n, nz = 8, 6
    nmu, nphi = 4, 8
    x, _ = oracle.gauss_legendre(nmu)
    a = nmu - 1                       # most vertical upward ordinate, phi = 0
    tan = math.sqrt(1 - x[a] ** 2) / x[a]
    lz = 1.0
    dz = lz / (nz - 1)
    lx = n * dz * tan                 # one cell of horizontal travel per plane
    K = nmu * nphi
    rs = np.random.default_rng(7)
    bc = np.zeros((K, n, n, 1))
    k = a * nphi
    bc[k, :, :, 0] = rs.uniform(0, 1, (n, n))
    o = oracle.Oracle(spec_uniform(n=n, nz=nz, nmu=nmu, nphi=nphi, lmax=3, kappa=0.0, lx=lx, lz=lz,
                                   bc_bot=bc))
    St = np.zeros(o.lab_shape())
    I = o.trace(St, np.zeros(o.lab_shape()))
    planes = I[k, :, 0].reshape(nz, n, n)
    for m in range(nz):
        assert np.allclose(planes[m], np.roll(bc[k, :, :, 0], m, axis=1), atol=1e-12)
    others = np.delete(I[:, :, 0], k, axis=0)
    assert np.abs(others).max() == 0.0


def test_pure_absorption_attenuation():
    n, nz, alpha = 3, 7, 1.7
    nmu, nphi = 4, 8
    K = nmu * nphi
    bc = np.ones((K, n, n, 1))
    o = oracle.Oracle(spec_uniform(n=n, nz=nz, nmu=nmu, nphi=nphi, kappa=alpha, bc_bot=bc, bc_top=bc))
    res = o.solve(tol=1e-14, max_iter=5)
    I = res["I_lab"].reshape(K, nz, n, n)
    dz = 1.0 / (nz - 1)
    dirs, mu, _ = ordinate_dirs(o)
    for k in range(K):
        depth = np.arange(nz) * dz if mu[k] > 0 else (nz - 1 - np.arange(nz)) * dz
        ref = np.exp(-alpha * depth / abs(mu[k]))
        assert np.allclose(I[k, :, 0, 0], ref, rtol=1e-13)


def _lc_ray_integral(p_xyz, n, S_fun, X_fun, I_bc_fun, lz):
    """Long characteristic from the inflow face to p: I = I_bc e^{-tau} + int S chi e^{-tau'} ds."""
    s_end = (p_xyz[2] / n[2]) if n[2] > 0 else ((p_xyz[2] - lz) / n[2])
    start = p_xyz - s_end * n

    def pos(s):
        return start + s * n

    def tau_between(s0, s1):
        return integrate.quad(lambda s: X_fun(pos(s)), s0, s1, epsabs=1e-14, epsrel=1e-13, limit=200)[0]

    def integrand(s):
        return S_fun(pos(s)) * X_fun(pos(s)) * math.exp(-tau_between(s, s_end))

    src = integrate.quad(integrand, 0.0, s_end, epsabs=1e-13, epsrel=1e-12, limit=200)[0]
    return I_bc_fun(start) * math.exp(-tau_between(0.0, s_end)) + src


def test_short_characteristics_equal_long_characteristics_for_linear_source():
    """S~ linear in z and uniform chi~: the cubic Bezier short-characteristic
    sweep reproduces the brute-force long-characteristic integral on 4^3."""
    n = 4
    o = oracle.Oracle(spec_uniform(n=n, nmu=4, nphi=8, lmax=3))
    a0, a1, chi = 0.3, 1.4, 2.2
    z = np.arange(n) / (n - 1)
    St = np.zeros(o.lab_shape())
    St[:] = np.repeat(a0 + a1 * z, n * n)[None, :, None]
    Xt = np.full(o.lab_shape(), chi)
    I = o.trace(St, Xt)
    dirs, mu, _ = ordinate_dirs(o)
    for k in range(o.K):
        for m in (1, 2, 3):
            p = np.array([0.25, 0.5, z[m] if mu[k] > 0 else z[n - 1 - m]])
            ref = _lc_ray_integral(p, dirs[k], lambda r: a0 + a1 * r[2], lambda r: chi, lambda r: 0.0, 1.0)
            idx = ((m if mu[k] > 0 else n - 1 - m) * n + 2) * n + 1
            assert abs(I[k, idx, 0] - ref) < 1e-11 * max(1.0, abs(ref)), (k, m)


@pytest.mark.slow
def test_short_characteristics_converge_to_long_characteristics_3d():
    """Smooth 3-D fields: the SC error against the exact ray integral falls
    with refinement (4^3, 8^3, 16^3)."""
    def S_fun(r):
        return 1.0 + 0.5 * math.sin(2 * np.pi * r[0]) * math.cos(2 * np.pi * r[1]) + 0.8 * r[2] ** 2

    def X_fun(r):
        return 1.5 + 0.7 * math.cos(2 * np.pi * (r[0] + r[1])) + r[2]

    targets = [(0.5, 0.25, 1.0), (0.0, 0.5, 0.5)]
    errs = []
    for n in (4, 8, 16):
        o = oracle.Oracle(spec_uniform(n=n, nmu=4, nphi=8, lmax=3))
        X, Yc, Z = W.grid_coords(n)
        s_pts = np.array([S_fun(r) for r in zip(X, Yc, Z)])
        x_pts = np.array([X_fun(r) for r in zip(X, Yc, Z)])
        St = np.broadcast_to(s_pts[:, None], o.lab_shape()).copy()
        Xt = np.broadcast_to(x_pts[:, None], o.lab_shape()).copy()
        I = o.trace(St, Xt)
        dirs, mu, _ = ordinate_dirs(o)
        e = 0.0
        for k in (o.nphi * 2 + 1, o.nphi * 3 + 2, o.nphi * 1 + 5):
            for t in targets:
                i, j, m = int(round(t[0] * n)), int(round(t[1] * n)), int(round(t[2] * (n - 1)))
                p = np.array([i / n, j / n, m / (n - 1)])
                ref = _lc_ray_integral(p, dirs[k], S_fun, X_fun, lambda r: 0.0, 1.0)
                e = max(e, abs(I[k, (m * n + j) * n + i, 0] - ref))
        errs.append(e)
    assert errs[1] < 0.7 * errs[0] and errs[2] < 0.7 * errs[1], errs


def test_isotropic_field_has_eddington_factor_one_third():
    n, nmu, nphi = 5, 8, 16
    K = nmu * nphi
    B = 1.7
    bc = np.full((K, n, n, 1), B)
    o = oracle.Oracle(spec_uniform(n=n, nmu=nmu, nphi=nphi, lmax=3, kappa=0.6, sigma=1.3, B=B,
                                   bc_bot=bc, bc_top=bc))
    res = o.solve(tol=1e-14, max_iter=100)
    for J, H, Kt in (o.moments_lab(res["I_lab"]), o.moments_comoving(res["I_lm"])):
        assert np.allclose(J, B, rtol=1e-12)
        assert np.abs(H).max() < 1e-12
        assert np.allclose(Kt[..., :3] / J[..., None], 1.0 / 3.0, rtol=1e-12)
        assert np.abs(Kt[..., 3:]).max() < 1e-12


def _slab_1d(nz, mu, wmu, kappa, sigma, B, dx, tol=1e-15):
    """Independent one-dimensional slab solver for an x,y-uniform medium with
    Thomson scattering and the same cubic-Bezier characteristics: the path
    between neighbouring z planes is cut into the smallest number of equal
    pieces that move a ray of polar cosine mu at most one cell (dx) sideways,
    the source is linear in z along it, and the intensity is carried piece by
    piece from the previous plane."""
    dz = 1.0 / (nz - 1)
    chi = kappa + sigma
    # azimuthal mean of the Thomson phase function 3/4 (1 + cos^2)
    pbar = 0.75 * (1 + np.outer(mu ** 2, mu ** 2) + 0.5 * np.outer(1 - mu ** 2, 1 - mu ** 2))
    I = np.zeros((len(mu), nz))
    S = np.full((len(mu), nz), kappa * B / chi)

    def fb(dl, dr, hl, hr):
        if dl * dr <= 0:
            return 0.0
        al = (1 + hr / (hl + hr)) / 3
        return dl * dr / (al * dr + (1 - al) * dl)

    def weights(h):
        E = np.zeros(4)
        if h < 0.5:
            for nn in range(4):
                E[nn] = sum(h * (-h) ** m / (math.factorial(m) * (nn + m + 1)) for m in range(40))
        else:
            e = math.exp(-h)
            E[0] = 1 - e
            for nn in range(1, 4):
                E[nn] = nn / h * E[nn - 1] - e
        return math.exp(-h), (E[3], 3 * (E[2] - E[3]), 3 * (E[1] - 2 * E[2] + E[3]), E[0] - 3 * E[1] + 3 * E[2] - E[3])

    for _ in range(2000):
        for a, m_ in enumerate(mu):
            order = list(range(nz) if m_ > 0 else range(nz - 1, -1, -1))
            npc = max(1, math.ceil(dz * math.sqrt(1 - m_ * m_) / (abs(m_) * dx) - 1e-9))
            h = dz / abs(m_) / npc * chi
            I[a, order[0]] = 0.0
            for t in range(1, nz):
                p, u = order[t], order[t - 1]
                # source at the path points q_c, c = -1 .. npc + 1 (None where the plane is missing)
                q = {c: (1 - c / npc) * S[a, p] + c / npc * S[a, u] for c in range(npc + 1)}
                q[-1] = (1 - 1 / npc) * S[a, p] + S[a, order[t + 1]] / npc if t + 1 < nz else None
                q[npc + 1] = (1 - 1 / npc) * S[a, u] + S[a, order[t - 2]] / npc if t >= 2 else None
                Iv = I[a, u]
                for c in range(npc - 1, -1, -1):
                    Sp, Su, Sd, Suu = q[c], q[c + 1], q[c - 1], q[c + 2]
                    d1 = (Sp - Su) / h
                    dSp = fb(d1, (Sd - Sp) / h, h, h) if Sd is not None else d1
                    dSu = fb((Su - Suu) / h, d1, h, h) if Suu is not None else d1
                    Cu = min(max(Su + h * dSu / 3, min(Su, Sp)), max(Su, Sp))
                    Cp = min(max(Sp - h * dSp / 3, min(Su, Sp)), max(Su, Sp))
                    ex, w = weights(h)
                    Iv = Iv * ex + w[0] * Su + w[1] * Cu + w[2] * Cp + w[3] * Sp
                I[a, p] = Iv
        Snew = sigma / chi * (pbar * (wmu / 2)[None, :]) @ I + kappa * B / chi
        done = np.max(np.abs(Snew - S)) < tol
        S = Snew
        if done:
            break
    return I


def test_steady_slab_matches_independent_1d_solver():
    n, nmu, nphi = 4, 8, 16
    nz = 9
    kap, sig, B = 1.0, 1.0, 1.0
    o = oracle.Oracle(spec_uniform(n=n, nz=nz, nmu=nmu, nphi=nphi, lmax=3, kappa=kap, sigma=sig, B=B))
    res = o.solve(tol=1e-14, max_iter=400, use_ng=True)
    I1 = _slab_1d(nz, o.mu, o.wmu, kap, sig, B, dx=1.0 / n)
    I3 = res["I_lab"].reshape(nmu, nphi, nz, n * n)
    for a in range(nmu):
        ref = I1[a][None, :, None]
        assert np.allclose(I3[a], ref, rtol=0, atol=1e-12)
    J, H, Kt = o.moments_lab(res["I_lab"])
    Jp = J.reshape(nz, n * n)
    assert np.allclose(Jp, Jp[:, :1], atol=1e-13)                 # x,y independent
    assert np.allclose(Jp, Jp[::-1], atol=1e-12)                   # mirror symmetric in z
    assert np.abs(H[..., :2]).max() < 1e-13                       # no horizontal flux
    assert np.abs(Kt[..., 3]).max() < 1e-13 and np.abs(Kt[..., 4]).max() < 1e-13
    assert np.allclose(Kt[..., 0], Kt[..., 1], atol=1e-13)
    Jc, Hc, Kc = o.moments_comoving(res["I_lm"])
    assert np.allclose(Jc, J, atol=1e-13) and np.allclose(Hc, H, atol=1e-13) and np.allclose(Kc, Kt, atol=1e-13)


def test_moving_slab_pure_absorption_is_the_boosted_static_slab():
    """Grey absorbing slab moving along x: lab I(n) = D^4 B (1 - exp(-kappa z / mu0))
    with mu0 = D mu the comoving direction cosine (the comoving solution is static)."""
    n, nz, nmu, nphi = 3, 6, 8, 16
    kap, B, bv = 1.3, 0.9, 0.6
    o = oracle.Oracle(spec_uniform(n=n, nz=nz, nmu=nmu, nphi=nphi, lmax=3, kappa=kap, B=B, beta=[bv, 0, 0]))
    res = o.solve(tol=1e-14, max_iter=3)
    dirs, mu, _ = ordinate_dirs(o)
    gam = 1 / math.sqrt(1 - bv * bv)
    I = res["I_lab"].reshape(o.K, nz, n * n)
    z = np.arange(nz) / (nz - 1)
    for k in range(o.K):
        D = 1 / (gam * (1 - bv * dirs[k, 0]))
        depth = z if mu[k] > 0 else 1 - z
        ref = D ** 4 * B * (1 - np.exp(-kap * depth / (D * abs(mu[k]))))
        assert np.allclose(I[k, :, 0], ref, rtol=1e-12, atol=1e-14)


# ---------------------------------------------------------------------------
# time dependence (Eqs. 4-6, Appendix A)
# ---------------------------------------------------------------------------

def _stage(Iin, delta, kap, B):
    return (kap * B + Iin / delta) / (kap + 1.0 / delta)


def _rk_scalar(I, dt, kap, B):
    d1 = _stage(I, dt / 6, kap, B) - I
    I1 = I + 3 * d1
    d2 = _stage(I1, dt / 3, kap, B) - I1
    I2 = I + 1.5 * d2
    d3 = _stage(I2, dt / 3, kap, B) - I2
    I3 = I + 3 * d3
    d4 = _stage(I3, dt / 6, kap, B) - I3
    return I + d1 + d2 + d3 + d4


@pytest.mark.parametrize("kap", [0.8, 2560.0], ids=["mild", "stiff"])
@pytest.mark.parametrize("scheme", ["rk4", "euler"])
def test_interior_follows_the_scalar_time_recursion(scheme, kap):
    """Deep inside a uniform medium the implicit solve of each stage reduces to
    I = (kappa B + I_prev/(c dt))/(kappa + 1/(c dt)); boundary influence is
    damped by exp(-dz/(c dt)) per plane.  The stiff case (kappa c dt = 20) pins
    the four-stage scheme's amplification of stiff modes: per step the
    deviation from kappa B grows by G(20) = 3.675 (G -> 9 as kappa c dt grows),
    where the single implicit stage damps it by 1/21."""
    n, nz = 3, 20
    sig, B = 0.5, 2.0
    o = oracle.Oracle(spec_uniform(n=n, nz=nz, nmu=4, nphi=8, lmax=3, kappa=kap, sigma=sig, B=B))
    dt = 0.5 / 64
    I0 = np.full(o.lab_shape(), 0.3)
    I, _ = o.advance(I0, dt, nsteps=3, scheme=scheme, tol=1e-14, max_iter=100)
    s = 0.3
    for _ in range(3):
        s = _rk_scalar(s, dt, kap, B) if scheme == "rk4" else _stage(s, dt, kap, B)
    planes = I.reshape(o.K, nz, n * n)[:, 6:nz - 6]
    assert np.allclose(planes, s, rtol=1e-12)
    if kap > 100:
        z = kap * dt
        g = (s - B) / (0.3 - B)
        expect = (1.0 / (1.0 + z)) ** 3 if scheme == "euler" else _rk_scalar(1.0, dt, kap, 0.0) ** 3
        assert np.isclose(g, expect, rtol=1e-10)
        if scheme == "rk4":
            assert abs(_rk_scalar(1.0, dt, kap, 0.0) - 3.67536) < 1e-4


def test_scattering_pulse_follows_the_diffusion_solution():
    """An isotropic Gaussian pulse (width 0.09) in a purely scattering slab two
    optical depths per cell thick spreads as the diffusion equation's Gaussian
    with D = c/(3 sigma) (the paper's optically thick test, Eq. 16), and keeps
    its photon number (backward Euler steps; the four-stage scheme amplifies
    the stiff modes of such a medium at this step, see the scalar recursion)."""
    n, nz = 2, 64
    sig, w = 2.0 * (nz - 1), 0.09
    z = np.arange(nz) / (nz - 1)
    o = oracle.Oracle(spec_uniform(n=n, nz=nz, nmu=4, nphi=8, lmax=3, kappa=0.0, sigma=sig, B=0.0))
    prof = 100 * np.exp(-((z - 0.5) / w) ** 2)
    I0 = np.zeros(o.lab_shape())
    I0[:] = np.repeat(prof, n * n)[None, :, None]
    dt, nsteps = 0.05, 16
    I, _ = o.advance(I0, dt, nsteps=nsteps, scheme="euler", tol=1e-9, max_iter=400, use_ng=True)
    J = o.moments_lab(I)[0][:, 0].reshape(nz, n * n)
    assert np.allclose(J, J[:, :1], rtol=1e-12)           # x, y independent
    J = J[:, 0]
    D, t = 1.0 / (3 * sig), dt * nsteps
    Jd = 100 * w / np.sqrt(w ** 2 + 4 * D * t) * np.exp(-(z - 0.5) ** 2 / (w ** 2 + 4 * D * t))
    main = Jd > 0.1 * Jd.max()
    assert np.max(np.abs(J - Jd)[main]) < 0.02 * Jd.max()
    assert abs(J.sum() / prof.sum() - 1) < 1e-4


def test_backward_euler_front_moves_at_c():
    """A beam entering a vacuum along one ordinate: after n implicit steps the
    plane-wave profile approaches I_in Q(n, s/(c dt)) (Poisson tail), with the
    same width with and without absorption once exp(-alpha s) is divided out."""
    nmu, nphi = 4, 8
    K = nmu * nphi
    nz, n = 241, 2
    dt = 1.0 / 48
    nsteps = 24
    out = {}
    for alpha in (0.0, 0.8):
        bc = np.zeros((K, n, n, 1))
        bc[(nmu - 1) * nphi] = 1.0
        o = oracle.Oracle(spec_uniform(n=n, nz=nz, nmu=nmu, nphi=nphi, lmax=3, kappa=alpha, bc_bot=bc))
        I, _ = o.advance(None, dt, nsteps=nsteps, scheme="euler", tol=1e-14, max_iter=3)
        k = (nmu - 1) * nphi
        mu = o.mu[-1]
        s = np.arange(nz) / (nz - 1) / mu
        prof = I.reshape(K, nz, n * n)[k, :, 0]
        out[alpha] = (s, prof)
        ref = np.exp(-alpha * s) * special.gammaincc(nsteps, s / dt)
        assert np.max(np.abs(prof - ref)) < 0.03
    s, p0 = out[0.0]
    _, p1 = out[0.8]
    assert np.max(np.abs(p1 * np.exp(0.8 * s) - p0)) < 0.03
    half = s[np.argmin(np.abs(p0 - 0.5))]
    assert abs(half - nsteps * dt) < 0.05 * nsteps * dt


# ---------------------------------------------------------------------------
# Ng acceleration
# ---------------------------------------------------------------------------

def test_ng_is_exact_for_a_rank_two_linear_iteration():
    """Ng2 recovers the fixed point of x -> A x + b exactly when the error lies in
    a two-dimensional invariant subspace, whatever the (per-group) weighting:
    here on [points][groups][terms] arrays whose groups differ by 6 decades."""
    rs = np.random.default_rng(8)
    shape = (5, 3, 2)
    n = int(np.prod(shape))
    scale = np.broadcast_to(np.array([1.0, 1e-3, 1e-6])[None, :, None], shape).ravel()
    U = np.linalg.qr(rs.normal(size=(n, 2)))[0]
    A = np.diag(scale) @ U @ np.diag([0.9, -0.5]) @ U.T @ np.diag(1 / scale)
    b = rs.normal(size=n) * scale
    fixed = np.linalg.solve(np.eye(n) - A, b)
    chain = [A @ (rs.normal(size=n) * scale) + b]    # error already inside the range of A
    for _ in range(3):
        chain.append(A @ chain[-1] + b)
    S = oracle.Oracle.ng_extrapolate([c.reshape(shape) for c in chain])
    assert np.allclose(S.ravel(), fixed, rtol=1e-9, atol=1e-15)


def test_ng_weighting_is_invariant_to_group_scale():
    """Each group enters the Ng dot products by its relative change: rescaling one
    group of every chain member rescales that group of the result and leaves the
    others unchanged."""
    rs = np.random.default_rng(9)
    chain = [rs.normal(size=(6, 3, 4)) + 3.0 for _ in range(4)]
    c = np.array([1.0, 1e-8, 1.0])[None, :, None]
    a = oracle.Oracle.ng_extrapolate(chain)
    b = oracle.Oracle.ng_extrapolate([x * c for x in chain])
    assert np.allclose(b, a * c, rtol=1e-10)


def test_ng_reaches_the_plain_fixed_point():
    spec = W.random_medium(n=4, ng=3, lmax=3, nmu=4, nphi=8, seed=21, gamma_max=3.0)
    o = oracle.Oracle(spec)
    a = o.solve(tol=1e-12, max_iter=400, use_ng=False)
    b = o.solve(tol=1e-12, max_iter=400, use_ng=True)
    assert b["iters"] <= a["iters"]
    assert np.allclose(a["I_lab"], b["I_lab"], rtol=1e-9, atol=1e-11)


def test_floored_residual_only_changes_negligible_groups():
    """The convergence test's per-group norm is floored at 1e-20 of the largest
    group's.  Ordinary groups keep the plain relative residual that the C sweep
    reports; a group 30 decades down, or one that underflowed to zero, is
    measured against the floor."""
    o = oracle.Oracle(W.random_medium(n=4, ng=3, lmax=2, nmu=4, nphi=8, seed=4))
    S = o.initial_source()
    _, _, S_new, r = o.sweep(S)
    assert np.allclose(oracle.Oracle.floored_residual(S, S_new), r, rtol=1e-12)
    rs = np.random.default_rng(3)
    S_new = rs.uniform(0.5, 1.0, (5, 4, 9))
    S_new[:, 2] *= 1e-30
    S_new[:, 3] = 0.0
    S_old = S_new * (1 + 1e-3 * rs.normal(size=S_new.shape))
    S_old[:, 3] = 1e-40
    out = oracle.Oracle.floored_residual(S_old, S_new)
    floor = 1e-20 * np.sqrt(np.sum(S_new[:, :2] ** 2, axis=(0, 2)).max())
    assert np.isclose(out[2], np.sqrt(np.sum((S_new[:, 2] - S_old[:, 2]) ** 2)) / floor, rtol=1e-12)
    assert np.isclose(out[3], np.sqrt(np.sum(S_old[:, 3] ** 2)) / floor, rtol=1e-12)


# ---------------------------------------------------------------------------
# the paper's two-dimensional validation problems (Sec. 3), small grids
# ---------------------------------------------------------------------------

def test_searchlight_attenuation_and_front_in_two_dimensions():
    """Sec. 3.1 on a 48 x 48 plane with (4, 8) ordinates and the four-stage
    scheme, one cell per step: behind the front J is the beam's J times
    exp(-alpha s) (alpha = 1 per domain side), and the front's half point is
    within two cell paths of c t."""
    n = 48
    spec, I0 = W.searchlight(n, alpha_cm=1e-10)
    o = oracle.Oracle(spec)
    dt = 1.0 / (n - 1)
    nsteps = 28
    I, _ = o.advance(I0, dt, nsteps=nsteps, scheme="rk4", tol=1e-12, max_iter=5)
    J = o.moments_lab(I)[0][:, 0].reshape(n, n)
    mu, wmu = np.polynomial.legendre.leggauss(4)
    Jb = wmu[-1] * 2 * np.pi / 8 / (4 * np.pi)
    z = np.arange(n) / (n - 1)
    xi = ((0.3 + z * np.sqrt(1 - mu[-1] ** 2) / mu[-1]) % 1.0) * n
    i0 = np.floor(xi).astype(int)
    f = xi - i0
    Jr = (1 - f) * J[np.arange(n), i0 % n] + f * J[np.arange(n), (i0 + 1) % n]
    s = z / mu[-1]
    rel = Jr / Jb / np.exp(-s)
    ct = nsteps * dt
    assert np.max(np.abs(rel[s < ct - 0.25] - 1)) < 2e-3
    assert abs(s[np.argmin(np.abs(rel - 0.5))] - ct) < 2 * dt / mu[-1]


def _free_streaming_J(spec, t, w=0.09, amp=100.0):
    """Mean intensity of an isotropic Gaussian pulse amp exp(-r^2/w^2) about the
    plane's centre after free streaming for c t = t, exactly for the discrete
    ordinate set: each ordinate's intensity is the initial profile translated
    by t n (periodic in x).  Returns J on the (nz, nx) grid."""
    n, nz = spec["nx"], spec["nz"]
    mu, wmu = np.polynomial.legendre.leggauss(spec["nmu"])
    nphi = spec["nphi"]
    X = (np.arange(n) / n)[None, :] - 0.5
    Z = (np.arange(nz) / (nz - 1))[:, None] - 0.5
    J = np.zeros((nz, n))
    for a in range(spec["nmu"]):
        st = math.sqrt(1 - mu[a] ** 2)
        for b in range(nphi):
            nx_ = st * math.cos(2 * np.pi * b / nphi)
            dx = (X - t * nx_ + 0.5) % 1.0 - 0.5
            J += wmu[a] / (2 * nphi) * amp * np.exp(-(dx ** 2 + (Z - t * mu[a]) ** 2) / w ** 2)
    return J


def test_thin_pulse_spreads_at_c_like_free_streaming():
    """Sec. 3.3.1 on a 48 x 48 plane with (8, 16) ordinates, four-stage steps
    of one cell light-crossing time, to t = 0.1 s (c t = 0.29 of the side):
    in vacuum every ordinate's intensity is the initial pulse translated by
    c t n, so J is known exactly for the ordinate set.  The computed J keeps
    the photon count of that solution (1 %), its J-weighted mean radius to a
    quarter cell, its profile to a quarter of the peak everywhere, and puts the
    peak along the x and z axes within two cells of the exact one, with the
    same height to 5 %."""
    n = 48
    spec, I0 = W.radiative_pulse(n, nmu=8, nphi=16)
    o = oracle.Oracle(spec)
    nz = spec["nz"]
    dt = 1.0 / (nz - 1)
    nsteps = int(round(0.1 * W.SECOND / dt))
    I, _ = o.advance(I0, dt, nsteps=nsteps, scheme="rk4", tol=1e-10, max_iter=5)
    J = o.moments_lab(I)[0][:, 0].reshape(nz, n)
    t = nsteps * dt
    Jx = _free_streaming_J(spec, t)
    X = (np.arange(n) / n)[None, :] - 0.5
    Z = (np.arange(nz) / (nz - 1))[:, None] - 0.5
    R = np.sqrt(X ** 2 + Z ** 2)
    assert abs(J.sum() / Jx.sum() - 1) < 0.01
    assert abs((J * R).sum() / J.sum() - (Jx * R).sum() / Jx.sum()) < 0.25 / n
    assert np.abs(J - Jx).max() < 0.25 * Jx.max()
    mid = (nz - 1) // 2
    for got, ref in ((J[mid, n // 2:], Jx[mid, n // 2:]), (J[mid:mid + n // 2, n // 2], Jx[mid:mid + n // 2, n // 2])):
        assert abs(int(np.argmax(got)) - int(np.argmax(ref))) <= 2
        assert abs(got.max() / ref.max() - 1) < 0.05


def test_inconsistent_inflow_face_grows_ninefold_per_four_stage_step():
    """Inflow-face values are fixed by the boundary in every stage, the z -> inf
    mode of the four-stage combination: an initial field that disagrees with the
    boundary there by d disagrees by d 9^m after m steps (the state is 1 - 9^m for
    a unit beam from zero), while one that agrees
    stays bounded."""
    spec, I0 = W.searchlight(16)
    o = oracle.Oracle(spec)
    I, _ = o.advance(np.zeros_like(I0), 0.05, nsteps=2, scheme="rk4", tol=1e-12, max_iter=5)
    assert np.isclose(np.abs(I).max(), 80.0)
    I, _ = o.advance(I0, 0.05, nsteps=2, scheme="rk4", tol=1e-12, max_iter=5)
    assert np.abs(I).max() <= 1.0 + 1e-12


@pytest.mark.parametrize("bx", [0.0, 0.9, 0.995])
def test_moving_emitter_is_beamed_as_the_cube_of_the_doppler_factor(bx):
    """Sec. 3.4: isotropic comoving emission from matter moving along x has the
    lab emissivity D^3 eta_0 along n; on a grid and ordinate set symmetric under
    x -> -x the intensity along (theta, phi) at x over that along (theta, pi - phi)
    at -x is ((1 + beta sin(theta) cos(phi)) / (1 - beta sin(theta) cos(phi)))^3
    (up to the 1e-9 absorption left in the emitter)."""
    nmu, nphi, n = 8, 16, 24
    spec, _ = W.beaming_cylinder(n, nmu=nmu, nphi=nphi, beta=(bx, 0.0), radius_cm=1.5e9)
    o = oracle.Oracle(spec)
    I = o.solve(tol=1e-12, max_iter=5, use_ng=False)["I_lab"][:, :, 0].reshape(nmu * nphi, spec["nz"], n)
    worst = 0.0
    for a in range(nmu):
        st = np.sqrt(1 - o.mu[a] ** 2)
        for b in range(nphi):
            cph = np.cos(2 * np.pi * b / nphi)
            if cph <= 0:
                continue
            ratio = ((1 + bx * st * cph) / (1 - bx * st * cph)) ** 3
            A, M = I[a * nphi + b], I[a * nphi + (nphi // 2 - b) % nphi][:, (-np.arange(n)) % n]
            lit = A > 1e-6 * A.max()
            worst = max(worst, float(np.max(np.abs(A[lit] / (M[lit] * ratio) - 1))))
    assert worst < 1e-8


def test_single_ordinate_trace_and_extinction_match_the_full_oracle_steps():
    """The oracle's one-ordinate entry points (used to check sampled marches of
    full-size sweeps) give exactly the corresponding slices of its full S3 and
    S4: the extinction chi~ = chi_lab + 1/(c dt) of the boost, and the march of
    one ordinate and group including its inflow boundary (Sec. 2, Eqs. 5-8)."""
    spec = W.random_medium(n=6, nz=5, ng=4, lmax=3, nmu=6, nphi=8, seed=21)
    o = oracle.Oracle(spec)
    gen = np.random.default_rng(5)
    S0 = gen.uniform(0.1, 1.0, o.co_shape())
    Ip = gen.uniform(0.0, 1.0, o.lab_shape())
    St, Xt = o.boost(S0, Ip, 3.0)
    I = o.trace(St, Xt)
    for k, g in [(0, 0), (o.K - 1, o.G - 1), (7, 2), (20, 1), (30, 3)]:
        assert np.array_equal(o.lab_extinction(k, g, 3.0), Xt[k, :, g])
        assert np.array_equal(o.trace_one(k, g, St[k, :, g], Xt[k, :, g]), I[k, :, g])
