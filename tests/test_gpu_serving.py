"""Batches and the continuous-batching request loop, through the C ABI.

A solve gives the same result alone and in a batch (the same kernels in the
same order on its own stream); admission respects the device-memory budget;
served requests match the FP64 oracle's converged moments."""
import numpy as np
import pytest

import oracle
from paper_1507_05141_amd import binding as B
from paper_1507_05141_amd import serving as SV
from paper_1507_05141_amd import workloads as W

pytestmark = pytest.mark.gpu


def _uneven_specs():
    a = W.thomson_jet(n=8, ng=4, lmax=3, nmu=4, nphi=8, seed=2)
    b = W.compton_jet(n=6, ng=8, lmax=3, nmu=4, nphi=8, e_hi=200.0)
    b["kte"] = None
    c = W.thomson_jet(n=10, ng=2, lmax=7, nmu=8, nphi=16, gamma_max=5.0, seed=7)
    return [a, b, c]


@pytest.mark.parametrize("prec", [B.FP32, B.MIXED], ids=["fp32", "mixed"])
def test_batch_results_equal_alone(prec):
    specs = _uneven_specs()
    alone = []
    for sp in specs:
        print(f"alone n={sp['nx']} lmax={sp['lmax']} {sp['scatter']}", flush=True)
        g = B.Problem.from_spec(sp, precision=prec)
        info = g.solve(tol=1e-6, max_iter=300, use_ng=True)
        alone.append((info["iters"], g.moments(B.FRAME_LAB), g.moments(B.FRAME_COMOVING)))
        g.close()
    print("batch of three", flush=True)
    batch = B.Batch(64 << 30)
    probs = [B.Problem.from_spec(sp, precision=prec) for sp in specs]
    for p in probs:
        assert batch.admit(p, tol=1e-6, max_iter=300, use_ng=True)
    rounds = 0
    while batch.step(1):
        rounds += 1
        assert rounds < 400
    for (it, lab, co), p in zip(alone, probs):
        done, info = batch.poll(p)
        assert done and info["converged"] and info["iters"] == it
        for a, b in zip(lab + co, p.moments(B.FRAME_LAB) + p.moments(B.FRAME_COMOVING)):
            assert np.array_equal(a, b)
        batch.remove(p)
        p.close()
    batch.close()


@pytest.mark.parametrize("prec", [B.FP32, B.MIXED], ids=["fp32", "mixed"])
def test_device_pool_reuses_freed_blocks(prec):
    """rrt_set_device_pool: a destroyed problem's blocks wait in the pool, the next
    problem of the same shape takes them, its solve equals a solve in fresh
    memory bit for bit, and a limit of 0 frees everything held."""
    sp = _uneven_specs()[2]
    assert B.set_device_pool(0) == 0
    g = B.Problem.from_spec(sp, precision=prec)
    ref = g.solve(tol=1e-6, max_iter=300, use_ng=True)
    ref_m = g.moments(B.FRAME_LAB)
    g.close()
    try:
        B.set_device_pool(1 << 30)
        g = B.Problem.from_spec(sp, precision=prec)
        g.solve(tol=1e-6, max_iter=300, use_ng=True)
        size = g.device_bytes()
        g.close()
        held = B.set_device_pool(1 << 30)
        print(f"pool holds {held} bytes after one problem of {size}", flush=True)
        assert held > 0
        g = B.Problem.from_spec(sp, precision=prec)
        assert B.set_device_pool(1 << 30) < held            # its blocks came from the pool
        info = g.solve(tol=1e-6, max_iter=300, use_ng=True)
        assert info["iters"] == ref["iters"]
        for a, b in zip(ref_m, g.moments(B.FRAME_LAB)):
            assert np.array_equal(a, b)
        g.close()
        assert B.set_device_pool(1000) <= 1000              # lowering the limit frees the excess
    finally:
        assert B.set_device_pool(0) == 0


def test_batch_admission_respects_budget():
    sp = W.thomson_jet(n=8, ng=4, lmax=3, nmu=4, nphi=8, seed=2)
    a = B.Problem.from_spec(sp)
    b = B.Problem.from_spec(sp)
    need = B.footprint_bytes(sp, B.FP32, use_ng=True)
    budget = max(a.device_bytes() + 4 * a.P * a.G * 16 * 4, need)
    batch = B.Batch(budget)
    assert batch.admit(a, tol=1e-6)
    assert not batch.admit(b, tol=1e-6)             # no room: the batch is unchanged
    batch.remove(a)
    assert batch.admit(b, tol=1e-6)
    while batch.step(4):
        pass
    done, info = batch.poll(b)
    assert done and info["converged"]
    batch.close()
    a.close()
    b.close()


@pytest.mark.parametrize("prec", [B.FP32, B.MIXED], ids=["fp32", "mixed"])
def test_served_requests_match_oracle(prec):
    """Eight requests arriving together (more than one round of admissions with a
    budget for about three problems): every result within 1e-3 of the oracle."""
    reqs = SV.poisson_requests(8, rate=0.0, seed=5, sizes=(6, 8), groups=(2, 4), lmaxes=(3,))
    budget = 3 * max(B.footprint_bytes(r["spec"], prec, use_ng=True) for r in reqs)
    out = {}

    def keep(i, pr):
        out[i] = pr.moments(B.FRAME_LAB)
        return {}

    recs, wall = SV.serve(reqs, precision=prec, budget_bytes=budget, tol=1e-7, max_iter=300, keep=keep)
    print(SV.summary(recs, wall), flush=True)
    assert all(r["converged"] for r in recs)
    for i, r in enumerate(reqs):
        o = oracle.Oracle(r["spec"])
        ref = o.solve(tol=1e-10, max_iter=500, use_ng=True)
        Jr, Hr, Kr = o.moments_lab(ref["I_lab"])
        J, H, K = out[i]
        assert np.max(np.abs(J - Jr) / np.abs(Jr)) <= 1e-3, f"request {i} J"
        for a, ar in ((H, Hr), (K, Kr)):
            for g in range(Jr.shape[1]):
                assert np.max(np.abs(a[:, g] - ar[:, g])) <= 1e-3 * np.max(np.abs(ar[:, g])), f"request {i}"
