"""Device-pointer boundary calls and the stand-alone S2 + S3 step.

The *_dev calls take and return device arrays (torch tensors here) and must
give exactly what the host calls give on the same problem; the lab source S~
of a sweep (SH -> ordinates, Eq. 9; comoving -> lab, Eqs. 7-8; time terms,
Eqs. 5-6) is compared with the FP64 oracle's sh2do + boost.
"""
import numpy as np
import pytest

import oracle
from paper_1507_05141_amd import binding as B
from paper_1507_05141_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {B.FP64: 1e-11, B.FP32: 1e-5}


def _spec():
    return W.random_medium(n=9, nz=7, ng=5, lmax=3, nmu=6, nphi=12, seed=41, gamma_max=4.0)


def _rel_by_group(got, ref, gaxis):
    g = np.moveaxis(got, gaxis, 0).reshape(got.shape[gaxis], -1)
    r = np.moveaxis(ref, gaxis, 0).reshape(ref.shape[gaxis], -1)
    return (np.abs(g - r).max(axis=1) / np.abs(r).max(axis=1)).max()


@pytest.mark.parametrize("prec", [B.FP64, B.FP32], ids=["fp64", "fp32"])
def test_lab_source_matches_the_oracle(prec):
    """S2 + S3 alone, steady and with the time terms of a stage."""
    spec = _spec()
    o = oracle.Oracle(spec)
    g = B.Problem.from_spec(spec, precision=prec)
    rs = np.random.default_rng(42)
    S = o.initial_source() * (1 + 0.3 * rs.uniform(size=o.sh_shape()))
    Ip = rs.uniform(0.0, 2.0, o.lab_shape())
    g.set_source_sh(S)
    g.set_intensity(Ip)
    for dt in (0.0, 0.05):
        inv = 1.0 / dt if dt else 0.0
        ref, _ = o.boost(o.sh2do(S), Ip if dt else None, inv)
        got = g.lab_source(dt)
        err = _rel_by_group(got, ref, 2)
        print(f"prec {prec} dt {dt}: S~ max error {err:.2e} of the group maximum", flush=True)
        assert err <= TOL[prec]
    g.close()


@pytest.mark.parametrize("prec", [B.FP64, B.FP32], ids=["fp64", "fp32"])
def test_device_calls_equal_the_host_calls(prec):
    spec = _spec()
    dt = torch.float64 if prec == B.FP64 else torch.float32
    h = B.Problem.from_spec(spec, precision=prec)
    d = B.Problem(spec, precision=prec, stream=torch.cuda.current_stream().cuda_stream)
    cu = lambda a, t=torch.float64: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda", t)
    d.set_medium_dev(cu(spec["kappa"]), cu(spec["sigma"]), cu(spec["bnu"]), cu(spec["beta"]))
    d.set_boundary(0, spec["bc_bot"])
    d.set_boundary(1, spec["bc_top"])
    rs = np.random.default_rng(43)
    S = rs.uniform(0.0, 1.0, h.sh_shape())
    Ip = rs.uniform(0.0, 1.0, h.lab_shape())
    h.set_source_sh(S)
    h.set_intensity(Ip)
    d.set_source_sh_dev(cu(S, dt))
    d.set_intensity_dev(cu(Ip, dt))
    torch.cuda.synchronize()
    assert np.array_equal(d.source_sh_dev().double().cpu().numpy(), h.source_sh())
    assert np.array_equal(d.intensity_dev().double().cpu().numpy(), h.intensity())
    assert np.array_equal(d.lab_source_dev(0.1).double().cpu().numpy(), h.lab_source(0.1))
    for p in (h, d):
        p.set_variants(trace_groups=1, s6=-1)
        p.sweep(0.1)
    assert np.array_equal(d.sweep_intensity_dev().double().cpu().numpy(), h.sweep_intensity())
    assert np.array_equal(d.intensity_sh_dev().double().cpu().numpy(), h.intensity_sh())
    assert np.array_equal(d.source_sh_dev().double().cpu().numpy(), h.source_sh())
    for fr in (B.FRAME_LAB, B.FRAME_COMOVING):
        for a, b in zip(d.moments_dev(fr), h.moments(fr)):
            assert np.array_equal(a.cpu().numpy(), b)
        a = d.moments_integrated_dev(fr).cpu().numpy()
        b = np.concatenate([x.reshape(h.P, -1) for x in h.moments_integrated(fr)], axis=1)
        assert np.array_equal(a, b)
    St = rs.uniform(0.0, 1.0, h.lab_shape())
    Xt = rs.uniform(0.5, 3.0, h.lab_shape())
    assert np.array_equal(d.ray_trace_dev(cu(St, dt), cu(Xt, dt)).double().cpu().numpy(), h.ray_trace(St, Xt))
    h.close()
    d.close()


def test_device_calls_refuse_bad_arguments():
    spec = _spec()
    d = B.Problem.from_spec(spec, precision=B.FP32)
    shape = d.lab_shape()
    St = torch.rand(shape, device="cuda")
    Xt = torch.rand(shape, device="cuda") + 0.5
    bad = Xt.clone()
    bad[3, 5, 1] = -1.0
    with pytest.raises(B.RRTError, match="chi~"):
        d.ray_trace_dev(St, bad)
    bad = St.clone()
    bad[0, 0, 0] = float("nan")
    with pytest.raises(B.RRTError, match="S~"):
        d.ray_trace_dev(bad, Xt)
    # host memory where device memory is required
    host = np.zeros(shape, dtype=np.float32)
    import ctypes
    st = B.lib().rrt_set_intensity_dev(d._h, ctypes.c_void_p(host.ctypes.data))
    assert st == B.RRT_E_INVALID
    assert "device memory" in B.lib().rrt_last_error().decode()
    d.close()
