"""Kernel variants and their autotuning, through the C ABI.

Every variant the autotuner may pick is checked against the FP64 oracle on one
sweep, to the tolerance of its precision; the autotuner's pick is one of the
candidates and is reused for a later problem of the same shape."""
import numpy as np
import pytest

import oracle
from paper_1507_05141_amd import binding as B
from test_gpu_parity import CASES, TOL, close_by_group, custom_spec

pytestmark = pytest.mark.gpu


def _sweep_against_oracle(case, prec, trace_groups, s6):
    spec = custom_spec(**CASES[case])
    o = oracle.Oracle(spec)
    g = B.Problem.from_spec(spec, precision=prec)
    g.set_variants(trace_groups=trace_groups, s6=s6)
    rs = np.random.default_rng(99)
    S = o.initial_source() + 0.3 * rs.normal(size=o.sh_shape()) * np.abs(o.initial_source()[..., :1]).mean()
    ref_I, ref_Ilm, ref_S, _ = o.sweep(S)
    g.set_source_sh(S)
    g.sweep()
    tol = 1e-3 if prec == B.MIXED else TOL[prec]
    close_by_group(g.sweep_intensity(), ref_I, tol, 2, "I_lab")
    close_by_group(g.intensity_sh(), ref_Ilm, tol, 1, "I_lm")
    close_by_group(g.source_sh(), ref_S, tol, 1, "S_new")
    assert g.variants() == {"trace_groups": trace_groups, "s6": s6, "tuned": False}
    g.close()


@pytest.mark.parametrize("s6", [0, 1, 2, 4], ids=["library", "rt1", "rt2", "rt4"])
@pytest.mark.parametrize("case", ["thomson_log", "high_gamma_L7"])
def test_s6_variants_fp32(case, s6):
    print(f"s6 variant {s6} {case} fp32", flush=True)
    _sweep_against_oracle(case, B.FP32, 1, s6)


@pytest.mark.parametrize("s6", [1, 2, 4], ids=["rt1", "rt2", "rt4"])
@pytest.mark.parametrize("case", ["thomson_log", "high_gamma_L7"])
def test_s6_variants_mixed(case, s6):
    print(f"s6 variant {s6} {case} mixed", flush=True)
    _sweep_against_oracle(case, B.MIXED, 1, s6)


@pytest.mark.parametrize("gc", [1, 2, 4, -1], ids=["gc1", "gc2", "gc4", "group_major"])
def test_trace_group_variants(gc):
    print(f"trace groups {gc}", flush=True)
    _sweep_against_oracle("grey_extinction_8g", B.FP32, gc, -1)


def test_unavailable_variants_are_rejected():
    spec = custom_spec(**CASES["thomson_log"])          # G = 3: only one group per workgroup divides it
    g = B.Problem.from_spec(spec, precision=B.FP32)
    with pytest.raises(B.RRTError):
        g.set_variants(trace_groups=2)
    with pytest.raises(B.RRTError):
        g.set_variants(s6=3)
    g.close()
    g = B.Problem.from_spec(spec, precision=B.FP64)
    with pytest.raises(B.RRTError):
        g.set_variants(s6=1)
    g.close()


def test_autotune_picks_a_candidate_and_reuses_it():
    spec = custom_spec(12, 12, 8, G=8, lmax=7, nmu=8, nphi=16, seed=31, grey_kappa=True)
    a = B.Problem.from_spec(spec, precision=B.FP32)
    assert a.variants()["tuned"] is False
    for _ in range(3):
        a.sweep()
    va = a.variants()
    print("tuned", va, flush=True)
    assert va["tuned"] and va["trace_groups"] in (1, 2, 4, -1) and va["s6"] in (0, 1, 2, 4)
    b = B.Problem.from_spec(spec, precision=B.FP32)
    for _ in range(2):
        b.sweep()
    assert b.variants() == va
    # the tuned problem still matches one with the same variants fixed
    c = B.Problem.from_spec(spec, precision=B.FP32)
    c.set_variants(trace_groups=va["trace_groups"], s6=va["s6"])
    for p in (b, c):
        p.set_intensity(None)
    rs = np.random.default_rng(5)
    S = np.abs(rs.normal(size=b.sh_shape()))
    for p in (b, c):
        p.set_source_sh(S)
        p.sweep()
    assert np.array_equal(b.source_sh(), c.source_sh())
    for p in (a, b, c):
        p.close()
