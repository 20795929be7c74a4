"""Mixed precision (FP16 matrix-core SH <-> ordinate products, FP32 elsewhere)
against the FP64 oracle, through the C ABI.

Target: 1e-3 on J, H and the Eddington tensor of converged solves, with the
error definitions J: per-point relative; H and K: max-norm error relative to
the max-norm of the reference, per group; f = K/J: absolute, over points with
J > 1e-6 max J.  One sweep is compared element by element to the per-group
maximum.  Every test prints the errors it measured.
"""
import numpy as np
import pytest

import oracle
from paper_1507_05141_amd import binding as B
from paper_1507_05141_amd import workloads as W
from test_gpu_parity import CASES, custom_spec

pytestmark = pytest.mark.gpu

TARGET = 1e-3


def _group_err(got, ref, gaxis):
    g = np.moveaxis(got, gaxis, 0).reshape(got.shape[gaxis], -1)
    r = np.moveaxis(ref, gaxis, 0).reshape(ref.shape[gaxis], -1)
    return max(np.max(np.abs(g[i] - r[i])) / max(np.max(np.abs(r[i])), 1e-300) for i in range(r.shape[0]))


def moment_errors(got, ref):
    """Errors of (J, H, K) against the reference, each group's relative to its own
    magnitude, and of the Eddington tensor f = K/J where J is resolved."""
    J, H, K = got
    Jr, Hr, Kr = ref
    e = {"J": float(np.max(np.abs(J - Jr) / np.maximum(np.abs(Jr), 1e-300)))}
    for nm, a, ar in (("H", H, Hr), ("K", K, Kr)):
        e[nm] = max(float(np.max(np.abs(a[:, g] - ar[:, g])) / max(np.max(np.abs(ar[:, g])), 1e-300))
                    for g in range(Jr.shape[1]))
    mask = Jr > 1e-6 * Jr.max(axis=0, keepdims=True)
    f, fr = K / np.where(mask, J, 1.0)[..., None], Kr / np.where(mask, Jr, 1.0)[..., None]
    e["f"] = float(np.max(np.abs(f - fr)[mask]))
    return e


@pytest.mark.parametrize("case", ["thomson_log", "high_gamma_L7", "grey_extinction_8g", "compton_log_keV",
                                  "lmax0_min_z", "compton_L15", "thomson_L4", "thomson_L8", "compton_L11",
                                  "thomson_L11_312_ordinates"])
def test_mixed_sweep_against_oracle(case):
    spec = custom_spec(**CASES[case])
    o = oracle.Oracle(spec)
    print(f"case {case} mixed", flush=True)
    g = B.Problem.from_spec(spec, precision=B.MIXED)
    rs = np.random.default_rng(99)
    S = o.initial_source() + 0.3 * rs.normal(size=o.sh_shape()) * np.abs(o.initial_source()[..., :1]).mean()
    ref_I, ref_Ilm, ref_S, _ = o.sweep(S)
    g.set_source_sh(S)
    g.sweep()
    errs = {"I_lab": _group_err(g.sweep_intensity(), ref_I, 2), "I_lm": _group_err(g.intensity_sh(), ref_Ilm, 1),
            "S": _group_err(g.source_sh(), ref_S, 1)}
    print(case, {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    g.close()
    for k, v in errs.items():
        assert v <= TARGET, f"{case} {k}: {v:.3e}"


def _solve_both(spec, tol_mixed=1e-6):
    o = oracle.Oracle(spec)
    ref = o.solve(tol=1e-10, max_iter=500, use_ng=True)
    g = B.Problem.from_spec(spec, precision=B.MIXED)
    g.solve(tol=tol_mixed, max_iter=300, use_ng=True)
    lab = moment_errors(g.moments(B.FRAME_LAB), o.moments_lab(ref["I_lab"]))
    co = moment_errors(g.moments(B.FRAME_COMOVING), o.moments_comoving(ref["I_lm"]))
    g.close()
    return lab, co


@pytest.mark.parametrize("name", ["uniform_slab", "small_jet", "small_compton_jet"])
def test_mixed_converged_moments(name):
    if name == "uniform_slab":
        spec = W.uniform_slab()
    elif name == "small_jet":
        spec = W.thomson_jet(n=8, ng=4, lmax=3, nmu=4, nphi=8, seed=2)
    else:
        # groups up to 200 keV: with L = 3 the truncated Klein-Nishina redistribution of
        # MeV photons is not a positive kernel and the Lambda iteration does not converge,
        # in the oracle either
        spec = W.compton_jet(n=8, ng=8, lmax=3, nmu=4, nphi=8, e_hi=200.0)
        spec["kte"] = None
    print(f"converged {name} mixed", flush=True)
    lab, co = _solve_both(spec)
    print(name, "lab", {k: f"{v:.2e}" for k, v in lab.items()}, "comoving", {k: f"{v:.2e}" for k, v in co.items()},
          flush=True)
    for frame, e in (("lab", lab), ("comoving", co)):
        for k in ("J", "H", "K", "f"):
            assert e[k] <= TARGET, f"{name} {frame} {k}: {e[k]:.3e}"


@pytest.mark.parametrize("emit", [True, False], ids=["faint_emission", "no_emission"])
def test_mixed_fold_of_rows_spanning_many_decades(emit):
    """The mixed ordinate -> SH product (L = 15, 16 x 32 ordinates) keeps one
    power-of-two scale per (point, group) row, set by the first block of 32
    ordinates with a nonzero value and lowered when a later block outgrows it.
    A beam exp(25 mu) entering through the bottom face of a nearly transparent
    medium at rest makes every row grow by more than nine decades from the
    downward to the upward rings (the ordinate order, one ring per block);
    without emission the downward rings are exactly zero, so the scale starts
    late.  The library's SH intensity is compared row by row with the FP64
    oracle's fold (Eq. 9 projection; the identity frame change at rest) of the
    library's own lab intensity, to 1e-4 of the row's largest coefficient."""
    n, ng, K = 6, 2, 512
    spec = W.random_medium(n=n, ng=ng, lmax=15, nmu=16, nphi=32, seed=5)
    P = n ** 3
    spec["beta"] = np.zeros((P, 3))
    spec["kappa"] = np.full((P, ng), 1e-3)
    spec["sigma"] = np.full(P, 1e-3)
    spec["bnu"] = np.full((P, ng), 1e-6 if emit else 0.0)
    o = oracle.Oracle(spec)
    mu = np.repeat(o.mu, spec["nphi"])
    beam = np.where(mu > 0, np.exp(25.0 * mu), 0.0)
    spec["bc_bot"] = np.broadcast_to(beam[:, None, None, None] * np.array([1.0, 1e-3]), (K, n, n, ng)).copy()
    spec["bc_top"] = np.zeros((K, n, n, ng))
    print(f"fold of rows spanning many decades, emission {emit}", flush=True)
    g = B.Problem.from_spec(spec, precision=B.MIXED)
    g.set_source_sh(oracle.Oracle(spec).initial_source())
    g.sweep()
    I_lab = g.sweep_intensity()
    got = g.intensity_sh()
    g.close()
    # the input has the structure the test is about
    blocks = np.abs(np.moveaxis(I_lab, 0, -1).reshape(-1, 16, 32)).max(axis=2)
    first = np.array([b[b > 0][0] for b in blocks])
    assert np.all(blocks.max(axis=1) > 1e9 * first)
    if not emit:
        assert np.all(blocks[:, :8] == 0.0)
    ref = oracle.Oracle(spec).fold(I_lab)
    r = ref.reshape(-1, ref.shape[-1])
    e = np.abs(got.reshape(r.shape) - r).max(axis=1) / np.abs(r).max(axis=1)
    print(f"worst row error {e.max():.2e} of the row's largest coefficient", flush=True)
    assert e.max() <= 1e-4
