"""Parity of the HIP library (through its C ABI) with the FP64 oracle.

Every case runs the same seeded inputs through both and compares element by
element: 1e-11 relative (to the per-group maximum) for the FP64 device path,
1e-5 for FP32.  Sizes are chosen so the oracle finishes in seconds while the
kernels still see several tiles and ragged edges; the last case runs one full
sweep of the 32^3 x 16-group x 512-ordinate relativistic Thomson jet.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1507_05141_amd import binding as B
from paper_1507_05141_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {B.FP64: 1e-11, B.FP32: 1e-5}
PREC_IDS = {B.FP64: "fp64", B.FP32: "fp32"}


def close_by_group(got, ref, rtol, gaxis, what="", reach=None):
    """Every element within rtol of its group's largest magnitude.

    With `reach`, a group is held instead to rtol of 1/100 of the brightest
    group within `reach` groups of it when that is larger.  The frame
    transforms interpolate the invariant I/nu^3 linearly in ln nu between
    groups up to ln(2 Gamma)/dln(nu) apart, and the Compton source mixes
    groups; in FP32 the interpolation weights carry ~1e-7 of absolute
    rounding, so a group 100 times fainter than a neighbour it is built from
    has an error of ~1e-7 of that neighbour (the deepest groups of a
    35-decade spectrum).  Their errors relative to their own magnitude are
    printed."""
    g = np.moveaxis(got, gaxis, 0).reshape(got.shape[gaxis], -1)
    r = np.moveaxis(ref, gaxis, 0).reshape(ref.shape[gaxis], -1)
    own = np.abs(r).max(axis=1)
    for i in range(r.shape[0]):
        scale = own[i]
        err = np.max(np.abs(g[i] - r[i]))
        if reach is not None:
            nb = 1e-2 * own[max(0, i - reach):i + reach + 1].max()
            if nb > scale:
                print(f"{what} group {i}: error {err / max(own[i], 1e-300):.2e} of its own maximum "
                      f"{own[i]:.2e}, {err / nb * 1e-2:.2e} of its brightest neighbour", flush=True)
                scale = nb
        assert err <= rtol * scale + 1e-300, f"{what} group {i}: max err {err:.3e} vs scale {scale:.3e}"


def custom_spec(nx, ny, nz, G=3, lmax=3, nmu=4, nphi=8, seed=0, scatter="thomson", gamma_max=4.0,
                edges=None, log_centres=True, grey=False, with_bc=True, mec2=None, grey_kappa=False):
    rs = np.random.default_rng(seed)
    P = nx * ny * nz
    if grey:
        edges, G = None, 1
    elif edges is None:
        edges = 10.0 ** np.linspace(-1, 1, G + 1) if log_centres else np.linspace(0.0, 1.1, G + 1)
    else:
        G = len(edges) - 1
    K = nmu * nphi
    bmax = math.sqrt(1 - 1 / gamma_max ** 2)
    d = rs.normal(size=(P, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    beta = d * bmax * rs.uniform(0, 1, (P, 1)) ** 0.5
    beta[rs.uniform(size=P) < 0.25] = 0.0                  # part of the medium at rest
    return dict(nx=nx, ny=ny, nz=nz, lx=1.0, ly=0.8, lz=1.1, nmu=nmu, nphi=nphi, lmax=lmax,
                edges=edges, log_centres=log_centres, scatter=scatter,
                mec2=mec2 if mec2 is not None else (1.0 if scatter == "compton" else W.MEC2_KEV),
                kappa=(np.repeat(rs.uniform(0.1, 2.0, (P, 1)), G, axis=1) if grey_kappa
                       else rs.uniform(0.1, 2.0, (P, G))),
                sigma=10 ** rs.uniform(-1, 1, P),
                bnu=rs.uniform(0.2, 2.0, (P, G)), beta=beta, kte=None,
                bc_bot=rs.uniform(0, 1, (K, ny, nx, G)) if with_bc else None,
                bc_top=rs.uniform(0, 1, (K, ny, nx, G)) if with_bc else None)


CASES = {
    "thomson_log": dict(nx=9, ny=7, nz=6, G=3, seed=1),
    "thomson_grey": dict(nx=6, ny=6, nz=5, grey=True, seed=2, nmu=8, nphi=16),
    "compton_linear_bins": dict(nx=5, ny=4, nz=4, G=6, scatter="compton", log_centres=False, seed=3, lmax=3),
    "compton_log_keV": dict(nx=4, ny=5, nz=5, G=5, scatter="compton", seed=4,
                            edges=np.exp(np.linspace(np.log(20.0), np.log(2000.0), 6)), mec2=W.MEC2_KEV),
    "lmax0_min_z": dict(nx=3, ny=3, nz=2, G=2, lmax=0, nmu=2, nphi=4, seed=5),
    "high_gamma_L7": dict(nx=5, ny=5, nz=4, G=4, lmax=7, nmu=8, nphi=16, gamma_max=20.0, seed=6),
    "vacuum_boundaries": dict(nx=6, ny=6, nz=6, G=2, with_bc=False, seed=7),
    "grey_extinction_8g": dict(nx=7, ny=6, nz=7, G=8, grey_kappa=True, seed=8, gamma_max=10.0),
    # 16 groups (64 bytes per point in FP32: two points per frame-transform workgroup), odd point count
    "thomson_16g_odd_points": dict(nx=5, ny=3, nz=5, G=16, seed=10, gamma_max=6.0),
    # L = 15 Thomson (the fused source and residual on 256-term rows)
    "thomson_L15": dict(nx=4, ny=3, nz=3, G=2, lmax=15, nmu=16, nphi=32, seed=11),
    # two-dimensional (ny = 1, as the paper's own tests) with a per-group extinction, and a
    # single column (nx = ny = 1)
    "two_d_groups": dict(nx=12, ny=1, nz=9, G=4, seed=12, gamma_max=6.0),
    "one_column": dict(nx=1, ny=1, nz=16, G=2, seed=13, nmu=8, nphi=16),
    # SH orders whose term counts are not the matrix-core tiles' widths (25, 81, 144 terms)
    "thomson_L4": dict(nx=4, ny=4, nz=3, G=3, lmax=4, nmu=8, nphi=16, seed=14),
    "thomson_L8": dict(nx=4, ny=3, nz=3, G=2, lmax=8, nmu=10, nphi=18, seed=15),
    "compton_L11": dict(nx=3, ny=3, nz=3, G=4, lmax=11, nmu=12, nphi=24, scatter="compton", seed=16,
                        edges=np.exp(np.linspace(np.log(1.0), np.log(150.0), 5)), mec2=W.MEC2_KEV),
    # 312 ordinates (not a multiple of 32: a partial last table chunk in the products)
    "thomson_L11_312_ordinates": dict(nx=3, ny=3, nz=3, G=3, lmax=11, nmu=12, nphi=26, seed=17),
    # L = 15 (256 SH terms, 16 x 32 ordinates): the widest SH products and Compton source
    "compton_L15": dict(nx=4, ny=4, nz=3, G=4, lmax=15, nmu=16, nphi=32, scatter="compton", seed=9,
                        edges=np.exp(np.linspace(np.log(1.0), np.log(150.0), 5)), mec2=W.MEC2_KEV),
}


def _both(spec, prec):
    o = oracle.Oracle(spec)
    print(f"case nx={spec['nx']} ny={spec['ny']} nz={spec['nz']} G={o.G} L={spec['lmax']} "
          f"K={o.K} {spec['scatter']} prec={PREC_IDS[prec]}", flush=True)
    g = B.Problem.from_spec(spec, precision=prec)
    return o, g


@pytest.mark.parametrize("prec", [B.FP64, B.FP32], ids=["fp64", "fp32"])
def test_ray_trace_parity(prec):
    spec = custom_spec(11, 7, 9, G=3, seed=10)
    o, g = _both(spec, prec)
    rs = np.random.default_rng(11)
    St = rs.uniform(0.0, 2.0, o.lab_shape())
    Xt = 10 ** rs.uniform(-1.5, 1.5, o.lab_shape())
    Xt[:, : spec["nx"], :] = 0.0                            # a vacuum row: h = 0 branches
    ref = o.trace(St, Xt)
    got = g.ray_trace(St, Xt)
    close_by_group(got, ref, TOL[prec], 2, "I")
    g.close()


@pytest.mark.parametrize("prec", [B.FP64, B.FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("case", list(CASES))
def test_sweep_parity(case, prec):
    spec = custom_spec(**CASES[case])
    o, g = _both(spec, prec)
    rs = np.random.default_rng(99)
    S = o.initial_source() + 0.3 * rs.normal(size=o.sh_shape()) * np.abs(o.initial_source()[..., :1]).mean()
    ref_I, ref_Ilm, ref_S, ref_r = o.sweep(S)
    g.set_source_sh(S)
    info = g.sweep()
    close_by_group(g.sweep_intensity(), ref_I, TOL[prec], 2, "I_lab")
    close_by_group(g.intensity_sh(), ref_Ilm, TOL[prec], 1, "I_lm")
    close_by_group(g.source_sh(), ref_S, TOL[prec], 1, "S_new")
    assert abs(info["residual"] - ref_r.max()) <= 10 * TOL[prec] * max(1.0, ref_r.max())
    g.close()


@pytest.mark.parametrize("gc", [1, 2, 4], ids=["gc1", "gc2", "gc4"])
@pytest.mark.parametrize("grey_kappa", [True, False], ids=["grey_chi", "group_chi"])
def test_ray_trace_variants_parity(gc, grey_kappa, monkeypatch):
    """Every ray-trace variant (groups per workgroup; grey, per-group or given
    extinction) on one time-dependent problem."""
    variant = f"gc{gc}"
    monkeypatch.setenv("RRT_TRACE_GC", str(gc))
    spec = custom_spec(9, 5, 7, G=4, seed=21, grey_kappa=grey_kappa, gamma_max=8.0)
    o, g = _both(spec, B.FP32)
    rs = np.random.default_rng(22)
    S = o.initial_source() * (1 + 0.2 * rs.uniform(size=o.sh_shape()))
    Iprev = rs.uniform(0.0, 1.0, o.lab_shape())
    ref_I = o.sweep(S, I_prev=Iprev, inv_cdt=3.0)[0]
    g.set_source_sh(S)
    g.set_intensity(Iprev)
    g.sweep(dt_stage=1.0 / 3.0)
    close_by_group(g.sweep_intensity(), ref_I, TOL[B.FP32], 2, f"I_lab {variant}")
    # the stand-alone entry point: chi~ given per ordinate and group
    St = rs.uniform(0.0, 2.0, o.lab_shape())
    Xt = 10 ** rs.uniform(-1.5, 1.5, o.lab_shape())
    close_by_group(g.ray_trace(St, Xt), o.trace(St, Xt), TOL[B.FP32], 2, f"ray trace {variant}")
    g.close()


@pytest.mark.parametrize("shape", [((9, 5, 7), 4, 4, 8), ((8, 5, 6), 4, 4, 8), ((9, 5, 7), 8, 8, 16)],
                         ids=["odd_points", "points_multiple_of_4", "eight_groups_128_ordinates"])
@pytest.mark.parametrize("prec", [B.FP32, B.FP64], ids=["fp32", "fp64"])
@pytest.mark.parametrize("grey_kappa", [True, False], ids=["grey_chi", "group_chi"])
def test_group_major_trace_parity(grey_kappa, prec, shape):
    """The ray trace on group-major planes (source transposed before, intensity
    after; a per-group extinction kept transposed) on one time-dependent sweep,
    then again after a new medium.  Point counts that are multiples of 4 take
    the 16-byte transposes (here two tiles, the second partial); the third case
    has two 4-group runs per point and 128 ordinates."""
    grid, G, nmu, nphi = shape
    spec = custom_spec(*grid, G=G, nmu=nmu, nphi=nphi, seed=23, grey_kappa=grey_kappa, gamma_max=8.0)
    o, g = _both(spec, prec)
    g.set_variants(trace_groups=-1)
    assert g.variants()["trace_groups"] == -1
    rs = np.random.default_rng(24)
    for rep in range(2):
        S = o.initial_source() * (1 + 0.2 * rs.uniform(size=o.sh_shape()))
        Iprev = rs.uniform(0.0, 1.0, o.lab_shape())
        ref_I, ref_Ilm, ref_S, _ = o.sweep(S, I_prev=Iprev, inv_cdt=3.0)
        g.set_source_sh(S)
        g.set_intensity(Iprev)
        g.sweep(dt_stage=1.0 / 3.0)
        close_by_group(g.sweep_intensity(), ref_I, TOL[prec], 2, f"I_lab group-major {rep}")
        close_by_group(g.source_sh(), ref_S, TOL[prec], 1, f"S_new group-major {rep}")
        # a new medium: the transposed extinction is recomputed
        spec = custom_spec(*grid, G=G, nmu=nmu, nphi=nphi, seed=25 + rep, grey_kappa=grey_kappa, gamma_max=6.0)
        o = oracle.Oracle(spec)
        g.set_medium(spec["kappa"], spec["sigma"], spec["bnu"], spec.get("beta"))
        for face, key in ((0, "bc_bot"), (1, "bc_top")):
            g.set_boundary(face, spec.get(key))
    g.close()


@pytest.mark.parametrize("plane", [(40, 36), (64, 50)], ids=["two_points_per_thread", "four_points_per_thread"])
@pytest.mark.parametrize("grey_kappa", [True, False], ids=["grey_chi", "group_chi"])
def test_large_plane_trace_parity(plane, grey_kappa):
    """Planes of more than 1024 and more than 2048 points (each ray-trace
    thread then owns two or four points, as on the 48^3 and 64^3 grids), on a
    time-dependent FP32 sweep, for every ray-trace variant the LDS holds
    (groups per workgroup, and one group on group-major planes).  nz, the
    ordinates and the groups are few so that the oracle stays fast; lz makes
    the path between planes cross a few cells for the shallow ordinates."""
    nx, ny = plane
    spec = custom_spec(nx, ny, 4, G=4, lmax=1, nmu=4, nphi=8, seed=31, grey_kappa=grey_kappa, gamma_max=5.0)
    spec["lz"] = 0.06
    o, g = _both(spec, B.FP32)
    rs = np.random.default_rng(32)
    S = o.initial_source() * (1 + 0.2 * rs.uniform(size=o.sh_shape()))
    Iprev = rs.uniform(0.0, 1.0, o.lab_shape())
    ref_I = o.sweep(S, I_prev=Iprev, inv_cdt=3.0)[0]
    ran = []
    for gc in (1, 2, 4, -1):
        try:
            g.set_variants(trace_groups=gc)
        except B.RRTError:
            continue
        ran.append(gc)
        print(f"  trace groups {gc}", flush=True)
        g.set_source_sh(S)
        g.set_intensity(Iprev)
        g.sweep(dt_stage=1.0 / 3.0)
        close_by_group(g.sweep_intensity(), ref_I, TOL[B.FP32], 2, f"I_lab {plane} gc {gc}")
    assert 1 in ran and -1 in ran
    g.close()


@pytest.mark.parametrize("prec", [B.FP64, B.FP32], ids=["fp64", "fp32"])
def test_time_dependent_sweep_parity(prec):
    spec = custom_spec(7, 6, 5, G=4, seed=12)
    o, g = _both(spec, prec)
    rs = np.random.default_rng(13)
    I_prev = rs.uniform(0, 1.5, o.lab_shape())
    S = o.initial_source(I_prev)
    dt = 0.5 / 7 / 6
    ref_I, ref_Ilm, ref_S, ref_r = o.sweep(S, I_prev, 1.0 / dt)
    g.set_intensity(I_prev)
    g.set_source_sh(S)
    g.sweep(dt)
    close_by_group(g.sweep_intensity(), ref_I, TOL[prec], 2, "I_lab")
    close_by_group(g.source_sh(), ref_S, TOL[prec], 1, "S_new")
    g.close()


@pytest.mark.parametrize("prec", [B.FP64, B.FP32], ids=["fp64", "fp32"])
def test_depth_cut_with_a_bright_upwind_slab(prec):
    """The multi-piece walk's depth cut at its worst: a short time step (pieces of
    at least ~14 optical depths of the time term, so the FP32 walk starts two or
    three pieces upwind, the FP64 one four) and a stage-start intensity a thousand
    times brighter in the slab x < 0.3 than elsewhere, which the shallow ordinates
    cross before reaching the dim points.  The oracle walks every piece; FP64 is
    held to 1e-9 of each element (down to 1e-6 of its group's maximum), FP32 to
    the usual 1e-5 of the group scale."""
    spec = custom_spec(12, 12, 6, G=2, nmu=8, nphi=16, seed=31, gamma_max=2.0)
    o, g = _both(spec, prec)
    rs = np.random.default_rng(32)
    I_prev = rs.uniform(1e-3, 2e-3, o.lab_shape())
    x = (np.arange(o.P) % spec["nx"] + 0.5) / spec["nx"]
    I_prev[:, x < 0.3, :] *= 1000.0
    S = o.initial_source(I_prev)
    dt = 1.0 / 200.0
    ref_I, _, ref_S, _ = o.sweep(S, I_prev, 1.0 / dt)
    g.set_intensity(I_prev)
    g.set_source_sh(S)
    g.sweep(dt)
    got = g.sweep_intensity()
    close_by_group(got, ref_I, TOL[prec], 2, "I_lab")
    close_by_group(g.source_sh(), ref_S, TOL[prec], 1, "S_new")
    if prec == B.FP64:
        big = np.abs(ref_I) >= 1e-6 * np.abs(ref_I).max(axis=(0, 1), keepdims=True)
        rel = np.abs(got - ref_I)[big] / np.abs(ref_I)[big]
        print(f"worst element error {rel.max():.2e} relative to the element", flush=True)
        assert rel.max() <= 1e-9
    g.close()


def _close_moments(got, ref, rtol, what):
    J, H, K = got
    Jr, Hr, Kr = ref
    for gi in range(Jr.shape[1]):
        jr = Jr[:, gi]
        assert np.all(np.abs(J[:, gi] - jr) <= rtol * np.abs(jr)), f"{what} J group {gi}"
        for arr, ar, nm in ((H, Hr, "H"), (K, Kr, "K")):
            scale = np.max(np.abs(ar[:, gi]))
            assert np.max(np.abs(arr[:, gi] - ar[:, gi])) <= rtol * scale + 1e-300, f"{what} {nm} group {gi}"


def test_uniform_slab_solve_parity_fp64():
    """The plain-method slab at its full size: 16^3, grey, L = 3, 8 x 16, FP64,
    residual < 1e-8; J, H and the Eddington tensor at every point, both frames."""
    spec = W.uniform_slab()
    o, g = _both(spec, B.FP64)
    ref = o.solve(tol=1e-8, max_iter=300, use_ng=True)
    info = g.solve(tol=1e-8, max_iter=300, use_ng=True)
    assert info["iters"] == ref["iters"]
    _close_moments(g.moments(B.FRAME_LAB), o.moments_lab(ref["I_lab"]), 1e-10, "lab")
    _close_moments(g.moments(B.FRAME_COMOVING), o.moments_comoving(ref["I_lm"]), 1e-10, "comoving")
    g.close()


@pytest.mark.parametrize("prec", [B.FP64, B.FP32], ids=["fp64", "fp32"])
def test_small_jet_time_steps_parity(prec):
    """Two four-stage time steps of a reduced relativistic Thomson jet."""
    spec = W.thomson_jet(n=8, ng=4, lmax=3, nmu=4, nphi=8, seed=2)
    o, g = _both(spec, prec)
    dt = 0.5 / 8
    tol = 1e-12 if prec == B.FP64 else 1e-7
    I_ref, last = o.advance(None, dt, nsteps=2, scheme="rk4", tol=1e-12, max_iter=100)
    g.advance(dt, nsteps=2, scheme=B.SCHEME_RK4, tol=tol, max_iter=100)
    rt = 1e-10 if prec == B.FP64 else 1e-5
    close_by_group(g.intensity(), I_ref, rt, 2, "I")
    _close_moments(g.moments(B.FRAME_LAB), o.moments_lab(I_ref), rt, "lab")
    _close_moments(g.moments(B.FRAME_COMOVING), o.moments_comoving(o.fold(I_ref)), rt, "comoving")
    g.close()


def test_full_size_thomson_jet_sweep_fp32():
    """One full sweep of the 32^3, 16-group, L = 7, 16 x 32 relativistic jet
    (the benchmarked workload) against the oracle, every output element."""
    spec = W.thomson_jet()
    o, g = _both(spec, B.FP32)
    S = o.initial_source()
    I_prev = None
    ref_I, ref_Ilm, ref_S, _ = o.sweep(S, I_prev, 0.0)
    g.set_source_sh(S)
    g.sweep()
    close_by_group(g.sweep_intensity(), ref_I, 1e-5, 2, "I_lab")
    close_by_group(g.intensity_sh(), ref_Ilm, 1e-5, 1, "I_lm")
    close_by_group(g.source_sh(), ref_S, 1e-5, 1, "S_new")
    g.close()


@pytest.mark.parametrize("lmax", [3, 5])
def test_products_walking_many_row_blocks(lmax):
    """At L <= 7 with 512 ordinates the SH <-> ordinate products run as one
    persistent workgroup per compute unit that walks row blocks, loading the next
    block's rows during the current one's products (S6 also across blocks).  On
    a 16^3 x 40-group Thomson jet (163840 rows) every workgroup walks several
    blocks: S2 ten of 64 rows (at L = 3 with whole 16-term rows, at L = 5 with
    the guarded loads of 36 terms), S6 one to three of 256 or 512 rows.  One
    FP32 sweep against the oracle, every output element."""
    spec = W.thomson_jet(n=16, ng=40, lmax=lmax)
    o, g = _both(spec, B.FP32)
    S = o.initial_source()
    ref_I, ref_Ilm, ref_S, _ = o.sweep(S, None, 0.0)
    g.set_source_sh(S)
    g.sweep()
    close_by_group(g.sweep_intensity(), ref_I, 1e-5, 2, "I_lab")
    close_by_group(g.intensity_sh(), ref_Ilm, 1e-5, 1, "I_lm")
    close_by_group(g.source_sh(), ref_S, 1e-5, 1, "S_new")
    g.close()


@pytest.mark.parametrize("prec", [B.FP64, B.FP32], ids=["fp64", "fp32"])
def test_frequency_integrated_moments_parity(prec):
    """Frequency-integrated J, H, K and f = K/J, reduced on the device in FP64,
    in both frames, after one time-dependent sweep of a moving multi-group
    medium, against the oracle's integrals of its own moments."""
    spec = custom_spec(6, 5, 4, G=5, seed=51)
    o, g = _both(spec, prec)
    rs = np.random.default_rng(52)
    Iprev = rs.uniform(0.0, 1.0, o.lab_shape())
    S = o.initial_source(Iprev)
    ref_I, ref_Ilm, _, _ = o.sweep(S, Iprev, 4.0)
    g.set_intensity(ref_I)                          # the lab moments read the intensity state
    g.set_source_sh(S)
    g.sweep(0.0)
    tol = 10 * TOL[prec]
    for frame, ref in ((B.FRAME_LAB, o.integrated(*o.moments_lab(ref_I))),
                       (B.FRAME_COMOVING, o.integrated(*o.moments_comoving(g.intensity_sh())))):
        got = g.moments_integrated(frame)
        for a, b, name in zip(got, ref, ("J", "H", "K", "f")):
            assert np.abs(a - b).max() <= tol * np.abs(b).max(), (frame, name)
    g.close()


@pytest.mark.parametrize("thermal", [False, True], ids=["electrons_at_rest", "thermal_electrons"])
def test_compton_tables_built_on_the_gpu_match_the_oracle(thermal):
    """The library builds its group-to-group tables on the GPU (FP64, its own
    code); they equal the oracle's to 1e-11 of each table's largest entry,
    node for node: the electrons at rest of the paper, and the thermal tables
    at the node temperatures of a 10-100 keV field."""
    spec = W.compton_jet(n=4, ng=12, lmax=7, nmu=8, nphi=16, e_hi=1e3)
    if not thermal:
        spec["kte"] = None
    o = oracle.Oracle(spec)
    g = B.Problem.from_spec(spec, precision=B.FP64)
    kT, s, A = g.compton_tables()
    g.close()
    if thermal:
        assert np.allclose(np.log10(kT), o.lt_nodes, rtol=0, atol=1e-12)
        s_ref, p_ref = o.kn_s, o.kn_p
    else:
        assert kT.tolist() == [0.0]
        s_ref, p_ref = o.kn_s[None], o.kn_p[None]
    G, nl = o.G, o.lmax + 1
    dnu = np.diff(o.edges)
    c = o.centres
    for n in range(len(kT)):
        assert np.abs(s[n] - s_ref[n]).max() <= 1e-11 * np.abs(s_ref[n]).max()
        for l in range(nl):
            ref = s_ref[n][None, :] * (c[:, None] * dnu[None, :]) / (c[None, :] * dnu[:, None]) * p_ref[n][l].T / (2 * l + 1)
            assert np.abs(A[n, l] - ref).max() <= 1e-11 * np.abs(ref).max(), (n, l)


def test_standalone_compton_tables_match_the_oracle():
    """rrt_compton_tables at electrons at rest and at 10, 31.6, 100 and 511 keV
    (the last relativistic, Theta = 1) (s and p, FP64) against the oracle's
    tables: 1e-11 of each table's largest entry; an invalid temperature is
    refused."""
    edges = np.exp(np.linspace(np.log(1.0), np.log(1e3), 11))
    kT = np.array([0.0, 10.0, 10 ** 1.5, 100.0, W.MEC2_KEV])
    s, p = B.compton_tables(edges, W.MEC2_KEV, 5, kT)
    c = oracle.group_centres(edges, True)
    for n, t in enumerate(kT):
        so, po = oracle.compton_thermal(edges, c, W.MEC2_KEV, 5, t)
        assert np.abs(s[n] - so).max() <= 1e-11 * np.abs(so).max()
        assert np.abs(p[n] - po).max() <= 1e-11 * np.abs(po).max(), n
    with pytest.raises(B.RRTError):
        B.compton_tables(edges, W.MEC2_KEV, 5, [-1.0])


@pytest.mark.parametrize("prec", [B.FP64, B.FP32], ids=["fp64", "fp32"])
def test_thermal_compton_sweep_parity(prec):
    """One sweep with a smooth 10-100 keV electron temperature field (tables on
    nine nodes, each point between two): the per-point interpolation of the
    source tables and of the scattering extinction, in the vector kernel (FP64)
    and on the matrix cores (FP32)."""
    spec = W.compton_jet(n=8, ng=8, lmax=3, nmu=4, nphi=8, e_hi=200.0)
    o, g = _both(spec, prec)
    assert len(o.lt_nodes) >= 2
    rs = np.random.default_rng(41)
    S = o.initial_source() * (1 + 0.2 * rs.uniform(size=o.sh_shape()))
    ref_I, ref_Ilm, ref_S, ref_r = o.sweep(S)
    g.set_source_sh(S)
    g.sweep()
    close_by_group(g.sweep_intensity(), ref_I, TOL[prec], 2, "I_lab")
    close_by_group(g.intensity_sh(), ref_Ilm, TOL[prec], 1, "I_lm")
    close_by_group(g.source_sh(), ref_S, TOL[prec], 1, "S_new")
    g.close()


def test_compton_jet_reduced_sweep_fp32():
    """The Compton workload's physics (32 log groups over [1e-3, 1e3] keV, L = 15,
    16 x 32 ordinates, jet with Gamma_max = 10, Thomson depth 1-5, electron
    temperature 10-100 keV on nine table nodes) on a 12^3 grid: one FP32 sweep
    against the oracle.  The groups 20-35 decades below the spectral peak are
    held to 1e-5 of 1/100 of their brightest neighbour within 8 groups (the
    Doppler and Compton reach), see close_by_group."""
    spec = W.compton_jet(n=12)
    o, g = _both(spec, B.FP32)
    S = o.initial_source()
    ref_I, ref_Ilm, ref_S, _ = o.sweep(S)
    g.set_source_sh(S)
    g.sweep()
    close_by_group(g.sweep_intensity(), ref_I, 1e-5, 2, "I_lab", reach=8)
    close_by_group(g.intensity_sh(), ref_Ilm, 1e-5, 1, "I_lm", reach=8)
    close_by_group(g.source_sh(), ref_S, 1e-5, 1, "S_new", reach=8)
    g.close()


def test_invalid_inputs_are_rejected():
    spec = custom_spec(3, 3, 3, G=2, seed=20)
    g = B.Problem(spec, precision=B.FP32)
    bad = spec["kappa"].copy()
    bad[0, 0] = -1.0
    with pytest.raises(B.RRTError) as e:
        g.set_medium(bad, spec["sigma"], spec["bnu"], spec["beta"])
    assert e.value.status == B.RRT_E_INVALID
    with pytest.raises(B.RRTError) as e:
        g.sweep()
    assert e.value.status == B.RRT_E_STATE
    b2 = spec["beta"].copy()
    b2[0] = [0.0, 0.0, 1.0]
    with pytest.raises(B.RRTError):
        g.set_medium(spec["kappa"], spec["sigma"], spec["bnu"], b2)
    g.set_medium(spec["kappa"], spec["sigma"], spec["bnu"], spec["beta"])
    info = g.solve(tol=1e-30, max_iter=2, use_ng=False, allow_not_converged=True)
    assert not info["converged"] and info["iters"] == 2
    g.close()
