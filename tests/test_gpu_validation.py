"""The paper's validation problems (Sec. 3) on the HIP library, through the C ABI.

Each problem runs in its two-dimensional form (ny = 1, lengths in units of the
paper's 1e10 cm domain, c = 1).  On reduced grids the library is compared
element by element with the FP64 oracle; at the resolutions in the tests it is
checked against what the paper compares with: exp(-alpha s) and a front moving
at c (searchlight, Sec. 3.1), independent beams and full shadows (Sec. 3.2),
the diffusion solution of Eq. 16 (optically thick pulse, Sec. 3.3.2) and the
D^3 beaming of isotropic comoving emission (Sec. 3.4).  Every reference value
here is a closed form (Gauss-Legendre weights from NumPy, the Doppler factor)."""
import numpy as np
import pytest

import oracle
from paper_1507_05141_amd import binding as B
from paper_1507_05141_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {B.FP64: 1e-10, B.FP32: 1e-5}
PREC_IDS = {B.FP64: "fp64", B.FP32: "fp32"}


def _problem(spec, I0, prec):
    g = B.Problem.from_spec(spec, precision=prec)
    g.set_intensity(I0)
    return g


def _plane_J(J, spec):
    return J[:, 0].reshape(spec["nz"], spec["nx"])


def _beam_J(nmu, nphi):
    """Mean intensity of unit intensity along one ordinate: its quadrature
    weight (Gauss-Legendre in mu times 2 pi / n_phi) over 4 pi."""
    mu, wmu = np.polynomial.legendre.leggauss(nmu)
    return mu[-1], wmu[-1] * 2 * np.pi / nphi / (4 * np.pi)


def _close(a, b, tol, what):
    scale = max(np.abs(b).max(), 1e-300)
    err = np.abs(a - b).max() / scale
    assert err <= tol, f"{what}: max error {err:.3g} of the maximum (tolerance {tol:g})"


def _parity(spec, I0, prec, run, tol=None):
    """Run the same steps on the library and the oracle; compare the lab
    intensity and the lab mean intensity element by element."""
    tol = tol or TOL[prec]
    o = oracle.Oracle(spec)
    g = _problem(spec, I0, prec)
    I_ref = run(o, I0, None)
    run(None, None, g)
    _close(g.intensity(), I_ref, tol, "lab intensity")
    _close(g.moments(B.FRAME_LAB)[0], o.moments_lab(I_ref)[0], tol, "J")
    g.close()


# ---------------------------------------------------------------------------
# parity with the oracle on reduced grids
# ---------------------------------------------------------------------------

def _advance(dt, nsteps, scheme, tol=1e-12, max_iter=5, use_ng=False, oracle_tol=None):
    def run(o, I0, g):
        if o is not None:
            return o.advance(I0, dt, nsteps=nsteps, scheme=scheme, tol=oracle_tol or tol, max_iter=max_iter,
                             use_ng=use_ng)[0]
        g.advance(dt, nsteps=nsteps, scheme=B.SCHEME_RK4 if scheme == "rk4" else B.SCHEME_EULER,
                  tol=tol, max_iter=max_iter, use_ng=use_ng)
    return run


def _steady(tol=1e-12, max_iter=5):
    def run(o, I0, g):
        if o is not None:
            return o.solve(tol=tol, max_iter=max_iter, use_ng=False)["I_lab"]
        g.solve(tol=tol, max_iter=max_iter, use_ng=False)
    return run


@pytest.mark.parametrize("prec", [B.FP64, B.FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("alpha_cm", [0.0, 1e-10], ids=["vacuum", "absorbing"])
def test_searchlight_parity(alpha_cm, prec):
    print(f"searchlight parity alpha={alpha_cm} {PREC_IDS[prec]}", flush=True)
    spec, I0 = W.searchlight(24, alpha_cm=alpha_cm)
    _parity(spec, I0, prec, _advance(1.0 / 23, 8, "rk4"))


@pytest.mark.parametrize("prec", [B.FP64, B.FP32], ids=["fp64", "fp32"])
def test_two_beam_shadow_parity(prec):
    print(f"two-beam shadow parity {PREC_IDS[prec]}", flush=True)
    spec, I0 = W.two_beam_shadow(24)
    _parity(spec, I0, prec, _steady())


@pytest.mark.parametrize("prec", [B.FP64, B.FP32], ids=["fp64", "fp32"])
def test_thin_pulse_parity(prec):
    print(f"thin pulse parity {PREC_IDS[prec]}", flush=True)
    spec, I0 = W.radiative_pulse(20, nmu=8, nphi=16)
    _parity(spec, I0, prec, _advance(1.0 / 20, 4, "rk4"))


@pytest.mark.parametrize("prec", [B.FP64, B.FP32], ids=["fp64", "fp32"])
def test_thick_pulse_parity(prec):
    """Scattering: each step is a Lambda iteration with stage albedo
    omega = sigma / (sigma + 1/dt) = 0.94, stopped at residual tol, so an
    iterate differs from the fixed point by up to about tol omega / (1 - omega)
    per step.  FP64 stops at 1e-13; FP32 at 1e-6 (near its rounding floor) is
    compared with the oracle's fixed point (1e-13) to 2e-4 over 3 steps."""
    print(f"thick pulse parity {PREC_IDS[prec]}", flush=True)
    spec, I0 = W.radiative_pulse(16, nmu=4, nphi=8, thick=True)
    tol = 1e-13 if prec == B.FP64 else 1e-6
    _parity(spec, I0, prec, _advance(0.05, 3, "euler", tol=tol, max_iter=400, use_ng=True, oracle_tol=1e-13),
            tol=None if prec == B.FP64 else 2e-4)


@pytest.mark.parametrize("prec", [B.FP64, B.FP32], ids=["fp64", "fp32"])
def test_beaming_cylinder_parity(prec):
    print(f"beaming cylinder parity {PREC_IDS[prec]}", flush=True)
    spec, I0 = W.beaming_cylinder(24, nmu=8, nphi=16, beta=(0.9, 0.3), radius_cm=1.5e9)
    _parity(spec, I0, prec, _steady())


# ---------------------------------------------------------------------------
# the paper's closed-form comparisons
# ---------------------------------------------------------------------------

def _ray_J(J, n, nz, mu, x0=0.3):
    """J bilinearly sampled along the beam's centre line x = x0 + z tan(theta)
    (periodic in x), with the path length s = z / mu."""
    z = np.arange(nz) / (nz - 1)
    xi = ((x0 + z * np.sqrt(1 - mu * mu) / mu) % 1.0) * n
    i0 = np.floor(xi).astype(int)
    f = xi - i0
    rows = np.arange(nz)
    return z / mu, (1 - f) * J[rows, i0 % n] + f * J[rows, (i0 + 1) % n]


def test_searchlight_attenuates_as_exp_minus_alpha_s_and_moves_at_c():
    """Sec. 3.1 at 128 x 128 (the paper: 512 x 512), (4, 8) ordinates, one cell
    per time step, to t = 0.25 s: behind the front J equals the beam's J times
    exp(-alpha s); the front's half point lies within two steps of c t; and the
    front has the same shape with and without absorption once exp(-alpha s) is
    divided out."""
    n = 128
    mu, Jb = _beam_J(4, 8)
    dt = 1.0 / (n - 1)
    nsteps = int(round(0.25 * W.SECOND / dt))
    ct = nsteps * dt
    prof = {}
    for alpha_cm in (0.0, 1e-10):
        print(f"searchlight 128^2 alpha={alpha_cm}", flush=True)
        spec, I0 = W.searchlight(n, alpha_cm=alpha_cm)
        g = _problem(spec, I0, B.FP32)
        g.advance(dt, nsteps=nsteps, scheme=B.SCHEME_RK4, tol=1e-10, max_iter=5)
        J = _plane_J(g.moments(B.FRAME_LAB)[0], spec)
        g.close()
        s, Jr = _ray_J(J, n, spec["nz"], mu)
        alpha = alpha_cm * W.DOMAIN_CM
        att = np.exp(-alpha * s)
        behind = s < ct - 0.25
        assert np.max(np.abs(Jr[behind] / Jb - att[behind])) < 2e-3
        rel = Jr / Jb / att
        half = s[np.argmin(np.abs(rel - 0.5))]
        assert abs(half - ct) < 2 * dt / mu, (half, ct)
        prof[alpha_cm] = rel
    assert np.max(np.abs(prof[1e-10] - prof[0.0])) < 0.02


def test_two_beams_cross_without_interaction_and_cast_shadows():
    """Sec. 3.2 at 128 x 128, steady state: the field of both beams is the sum
    of the fields of each; below the cylinder and above the shadows J is both
    beams' J; where one beam is shadowed it is one beam's; in both shadows it
    vanishes."""
    n = 128
    mu, Jb = _beam_J(4, 8)
    J = {}
    for beams in ((0,), (1,), (0, 1)):
        print(f"two-beam shadow 128^2 beams={beams}", flush=True)
        spec, I0 = W.two_beam_shadow(n, beams=beams)
        g = _problem(spec, I0, B.FP32)
        g.solve(tol=1e-10, max_iter=5, use_ng=False)
        J[beams] = _plane_J(g.moments(B.FRAME_LAB)[0], spec) / Jb
        g.close()
    both = J[(0, 1)]
    assert np.max(np.abs(both - J[(0,)] - J[(1,)])) < 1e-5
    nz = spec["nz"]

    def at(x, z):
        return both[int(round(z * (nz - 1))), int(round(x * n)) % n]
    for x, z in ((0.1, 0.05), (0.9, 0.05), (0.5, 0.9)):        # lit by both beams
        assert abs(at(x, z) - 2.0) < 1e-2, (x, z, at(x, z))
    for x, z in ((0.75, 0.7), (0.25, 0.7)):                    # in one beam's shadow
        assert abs(at(x, z) - 1.0) < 1e-2, (x, z, at(x, z))
    assert at(0.5, 0.52) < 1e-3                                # in both shadows


def test_thin_pulse_spreads_at_c_like_free_streaming():
    """Sec. 3.3.1 at the paper's size, 128 x 128 with (64, 128) ordinates,
    four-stage steps of one cell light-crossing time to t = 0.1 s: in vacuum
    each ordinate carries the initial pulse translated by c t n, so J is known
    exactly for the ordinate set.  The computed J keeps that solution's photon
    count (1 %) and J-weighted mean radius (half a cell); the peak along the x
    and z axes lies within two cells of the exact one, 5 % of its height."""
    print("thin pulse 128^2 (64, 128)", flush=True)
    spec, I0 = W.radiative_pulse(128, nmu=64, nphi=128)
    g = _problem(spec, I0, B.FP32)
    n, nz = spec["nx"], spec["nz"]
    dt = 1.0 / (nz - 1)
    nsteps = int(round(0.1 * W.SECOND / dt))
    g.advance(dt, nsteps=nsteps, scheme=B.SCHEME_RK4, tol=1e-10, max_iter=5)
    J = _plane_J(g.moments(B.FRAME_LAB)[0], spec)
    g.close()
    t = nsteps * dt
    mu, wmu = np.polynomial.legendre.leggauss(spec["nmu"])
    nphi = spec["nphi"]
    X = (np.arange(n) / n)[None, :] - 0.5
    Z = (np.arange(nz) / (nz - 1))[:, None] - 0.5
    Jx = np.zeros((nz, n))
    for a in range(spec["nmu"]):
        st = np.sqrt(1 - mu[a] ** 2)
        for b in range(nphi):
            dx = (X - t * st * np.cos(2 * np.pi * b / nphi) + 0.5) % 1.0 - 0.5
            Jx += wmu[a] / (2 * nphi) * 100 * np.exp(-(dx ** 2 + (Z - t * mu[a]) ** 2) / 0.09 ** 2)
    R = np.sqrt(X ** 2 + Z ** 2)
    assert abs(J.sum() / Jx.sum() - 1) < 0.01
    assert abs((J * R).sum() / J.sum() - (Jx * R).sum() / Jx.sum()) < 0.5 / n
    mid = (nz - 1) // 2
    for got, ref in ((J[mid, n // 2:], Jx[mid, n // 2:]), (J[mid:mid + n // 2, n // 2], Jx[mid:mid + n // 2, n // 2])):
        assert abs(int(np.argmax(got)) - int(np.argmax(ref))) <= 2
        assert abs(got.max() / ref.max() - 1) < 0.05


def test_thick_pulse_follows_the_diffusion_solution():
    """Sec. 3.3.2 at the paper's size, 128 x 128 with (32, 64) ordinates (an
    optical depth of 2.3 per cell, as there): an isotropic pulse
    100 exp(-(x/w)^2) in a purely (isotropically) scattering medium of depth
    300 across the domain, backward-Euler steps of 1/20 to t = 1: J along x
    follows Eq. 16's Gaussian with D = c/(3 sigma) to 10 % of the peak and is
    independent of z away from the open faces."""
    print("thick pulse 128^2", flush=True)
    spec, I0 = W.radiative_pulse(128, nmu=32, nphi=64, thick=True)
    g = _problem(spec, I0, B.FP32)
    dt, nsteps = 0.05, 20
    g.advance(dt, nsteps=nsteps, scheme=B.SCHEME_EULER, tol=1e-6, max_iter=400, use_ng=True)
    J = _plane_J(g.moments(B.FRAME_LAB)[0], spec)
    g.close()
    n, nz = spec["nx"], spec["nz"]
    x = np.arange(n) / n - 0.5
    w, D, t = 0.09, 1.0 / (3 * 300.0), dt * nsteps
    Jd = 100 * w / np.sqrt(w ** 2 + 4 * D * t) * np.exp(-x ** 2 / (w ** 2 + 4 * D * t))
    mid = (nz - 1) // 2
    assert np.max(np.abs(J[mid] - Jd)) < 0.10 * Jd.max()
    assert np.max(np.abs(J[nz // 4:3 * nz // 4] - J[mid])) < 1e-3 * Jd.max()


@pytest.mark.parametrize("prec", [B.FP64, B.FP32], ids=["fp64", "fp32"])
def test_beaming_is_the_cube_of_the_doppler_factor(prec):
    """Sec. 3.4: matter moving with beta along x emits isotropically in its own
    frame, so along lab direction n its emissivity is D^3 times the comoving
    one, D = 1/(Gamma (1 - beta.n)).  The grid and the ordinates are symmetric
    under x -> -x, so the lab intensity along (theta, phi) at (x, z) divided by
    that along (theta, pi - phi) at (1 - x, z) is exactly
    ((1 + beta sin(theta) cos(phi)) / (1 - beta sin(theta) cos(phi)))^3; and
    the lab light is carried forward: the domain's total flux along x over its
    total J is zero at rest and grows with the speed."""
    nmu, nphi, n = 8, 16, 48
    mu = np.polynomial.legendre.leggauss(nmu)[0]
    ahead = []
    for bx in (0.0, 0.5, 0.9, 0.995):
        print(f"beaming cylinder beta={bx} {PREC_IDS[prec]}", flush=True)
        spec, I0 = W.beaming_cylinder(n, nmu=nmu, nphi=nphi, beta=(bx, 0.0), radius_cm=1.0e9)
        g = _problem(spec, I0, prec)
        g.solve(tol=1e-12, max_iter=5, use_ng=False)
        nz = spec["nz"]
        I = g.intensity()[:, :, 0].reshape(nmu * nphi, nz, n)
        J, H, _ = g.moments(B.FRAME_LAB)
        g.close()
        worst = 0.0
        for a in range(nmu):
            st = np.sqrt(1 - mu[a] ** 2)
            for b in range(nphi):
                cph = np.cos(2 * np.pi * b / nphi)
                if cph <= 0:
                    continue
                k, km = a * nphi + b, a * nphi + (nphi // 2 - b) % nphi
                ratio = ((1 + bx * st * cph) / (1 - bx * st * cph)) ** 3
                A, M = I[k], I[km][:, (-np.arange(n)) % n]
                lit = A > 1e-6 * A.max()
                worst = max(worst, float(np.max(np.abs(A[lit] / (M[lit] * ratio) - 1))))
        assert worst < (1e-8 if prec == B.FP64 else 1e-4), (bx, worst)
        ahead.append(H[:, 0, 0].sum() / J[:, 0].sum())
    assert abs(ahead[0]) < 1e-6
    assert all(b > a for a, b in zip(ahead, ahead[1:])), ahead


@pytest.mark.parametrize("problem", ["thick_pulse", "beaming_cylinder"])
def test_validation_problems_in_mixed_precision(problem):
    """Mixed precision (FP16 matrix-core SH <-> ordinate products with FP32
    accumulation) against the FP64 oracle: J, H and K of the lab frame within
    1e-3 of each moment's maximum.  The scattering pulse's steps stop at
    residual 1e-5 (stage albedo 0.94: up to ~2e-4 from the fixed point)."""
    print(f"{problem} mixed precision", flush=True)
    if problem == "thick_pulse":
        spec, I0 = W.radiative_pulse(16, nmu=4, nphi=8, thick=True)
        run = _advance(0.05, 3, "euler", tol=1e-5, max_iter=400, use_ng=True, oracle_tol=1e-13)
    else:
        spec, I0 = W.beaming_cylinder(24, nmu=8, nphi=16, beta=(0.9, 0.3), radius_cm=1.5e9)
        run = _steady()
    o = oracle.Oracle(spec)
    g = _problem(spec, I0, B.MIXED)
    I_ref = run(o, I0, None)
    run(None, None, g)
    for name, got, ref in zip("JHK", g.moments(B.FRAME_LAB), o.moments_lab(I_ref)):
        _close(got, ref, 1e-3, name)
    g.close()
