"""Sweeps replayed from captured HIP graphs against eager sweeps, through the C ABI.

A captured sweep runs the same kernels in the same order as an eager one, so
every replay must give bit-identical results.  Each test runs one problem with
graphs (the default) and an identical one without, with the library's own
eager work (residual reads, Ng extrapolation, chain copies, stage updates)
between the replays, and compares after every replay."""
import numpy as np
import pytest

from paper_1507_05141_amd import binding as B
from paper_1507_05141_amd import workloads as W

pytestmark = pytest.mark.gpu


def _specs():
    jet = W.thomson_jet(n=8, ng=4, lmax=3, nmu=4, nphi=8, seed=2)
    comp = W.compton_jet(n=6, ng=8, lmax=3, nmu=4, nphi=8, e_hi=200.0)
    comp["kte"] = None
    return {"thomson": jet, "compton": comp}


def _pair(spec, prec):
    a = B.Problem.from_spec(spec, precision=prec)
    b = B.Problem.from_spec(spec, precision=prec)
    b.set_graphs(False)
    return a, b


@pytest.mark.parametrize("prec", [B.FP32, B.MIXED, B.FP64], ids=["fp32", "mixed", "fp64"])
@pytest.mark.parametrize("case", ["thomson", "compton", "thomson_stage"])
def test_every_replayed_sweep_equals_eager(case, prec):
    spec = _specs()[case.split("_")[0]]
    dt_stage = 0.01 if case.endswith("stage") else 0.0
    print(f"graph sweeps {case} prec={prec}", flush=True)
    a, b = _pair(spec, prec)
    if dt_stage:
        rs = np.random.default_rng(3)
        I0 = rs.uniform(0.0, 1e-3, size=a.lab_shape())
        a.set_intensity(I0)
        b.set_intensity(I0)
    for i in range(8):
        ra = a.sweep(dt_stage)
        rb = b.sweep(dt_stage)
        assert ra["residual"] == rb["residual"], i
        assert np.array_equal(a.source_sh(), b.source_sh()), i
    n = a.graph_count()
    print("captured sweeps", n, flush=True)
    assert n >= 2                    # both source buffers' sweeps are replayed
    assert b.graph_count() == 0
    assert np.array_equal(a.sweep_intensity(), b.sweep_intensity())
    a.close()
    b.close()


@pytest.mark.parametrize("prec", [B.FP32, B.MIXED], ids=["fp32", "mixed"])
def test_solve_with_graphs_equals_eager(prec):
    spec = _specs()["compton"]
    print(f"graph solve prec={prec}", flush=True)
    a, b = _pair(spec, prec)
    ia = a.solve(tol=1e-6, max_iter=300, use_ng=True)
    ib = b.solve(tol=1e-6, max_iter=300, use_ng=True)
    assert ia["iters"] == ib["iters"] and ia["residual"] == ib["residual"]
    assert a.graph_count() >= 2
    for x, y in zip(a.moments(B.FRAME_LAB) + a.moments(B.FRAME_COMOVING),
                    b.moments(B.FRAME_LAB) + b.moments(B.FRAME_COMOVING)):
        assert np.array_equal(x, y)
    # a second solve replays the graphs captured by the first
    a.set_intensity(None)
    b.set_intensity(None)
    ia = a.solve(tol=1e-6, max_iter=300, use_ng=True)
    ib = b.solve(tol=1e-6, max_iter=300, use_ng=True)
    assert ia["iters"] == ib["iters"]
    assert np.array_equal(a.source_sh(), b.source_sh())
    a.close()
    b.close()


def test_time_steps_with_graphs_equal_eager():
    spec = _specs()["thomson"]
    print("graph time steps", flush=True)
    a, b = _pair(spec, B.FP32)
    dt = 0.5 / spec["nx"]
    for step in range(3):
        ia = a.advance(dt, nsteps=1, tol=1e-6, max_iter=100)
        ib = b.advance(dt, nsteps=1, tol=1e-6, max_iter=100)
        assert ia["iters"] == ib["iters"], step
        assert np.array_equal(a.intensity(), b.intensity()), step
    # four stages per step, each with its own stage input and 1/(c dt)
    assert a.graph_count() >= 4
    a.close()
    b.close()


def test_new_medium_drops_captured_sweeps():
    spec = _specs()["thomson"]
    a, b = _pair(spec, B.FP32)
    for _ in range(4):
        a.sweep()
        b.sweep()
    assert a.graph_count() >= 1
    other = W.thomson_jet(n=8, ng=4, lmax=3, nmu=4, nphi=8, seed=5)
    for p in (a, b):
        p.set_medium(other["kappa"], other["sigma"], other["bnu"], other.get("beta"))
        p.set_intensity(None)
    assert a.graph_count() == 0
    for i in range(6):
        a.sweep()
        b.sweep()
        assert np.array_equal(a.source_sh(), b.source_sh()), i
    a.close()
    b.close()
