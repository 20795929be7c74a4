"""The variable-Eddington-tensor hand-off on the GPU against the oracle
(oracle/vet.py): the Eddington tensor of the library's lab intensity state
closes the frequency-integrated moment equations, advanced on the device."""
import numpy as np
import pytest

import oracle
from oracle.vet import vet_step as oracle_vet_step
from paper_1507_05141_amd import binding as B
from test_gpu_parity import custom_spec

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _case(prec, seed=51):
    spec = custom_spec(11, 9, 7, G=4, lmax=3, nmu=6, nphi=12, seed=seed, gamma_max=3.0)
    P = 11 * 9 * 7
    o = oracle.Oracle(spec)
    g = B.Problem.from_spec(spec, precision=prec)
    rs = np.random.default_rng(seed + 1)
    # an anisotropic lab field: a beam-like ordinate dependence times a random spatial field
    I = rs.uniform(0.1, 1.0, o.lab_shape()) * (1.0 + 3.0 * (np.arange(o.K) % 7 == 0))[:, None, None]
    g.set_intensity(I)
    if prec != B.FP64:
        I = I.astype(np.float32).astype(np.float64)          # the state the library holds
    f = o.integrated(*o.moments_lab(I))[3]
    grid = (spec["nx"], spec["ny"], spec["nz"], spec["lx"], spec["ly"], spec["lz"])
    fields = dict(kappa_E=rs.uniform(0.0, 3.0, P), chi_F=rs.uniform(0.5, 4.0, P), B=rs.uniform(0.0, 2.0, P),
                  J=rs.uniform(0.2, 1.0, P), H=rs.uniform(-0.2, 0.2, (P, 3)))
    h = min(spec["lx"] / spec["nx"], spec["ly"] / spec["ny"], spec["lz"] / (spec["nz"] - 1))
    return spec, o, g, f, grid, fields, 0.5 * h


@pytest.mark.parametrize("prec", [B.FP64, B.FP32], ids=["fp64", "fp32"])
def test_vet_step_matches_the_oracle(prec):
    spec, o, g, f, grid, fl, dt = _case(prec)
    print(f"case vet {grid[:3]} prec {prec} dt {dt:.3g}", flush=True)
    J, H, G = g.vet_step(dt, 6, fl["kappa_E"], fl["chi_F"], fl["B"], fl["J"], fl["H"])
    rJ, rH, rG = oracle_vet_step(grid, f, fl["kappa_E"], fl["chi_F"], fl["B"], fl["J"], fl["H"], dt, 6)
    for got, ref, name in ((J, rJ, "J"), (H, rH, "H"), (G, rG, "G")):
        err = np.abs(got - ref).max() / np.abs(ref).max()
        print(f"  {name}: max error {err:.2e} of its maximum", flush=True)
        assert err < 1e-12, name
    g.close()


def test_vet_device_call_equals_the_host_call():
    spec, o, g, f, grid, fl, dt = _case(B.FP32, seed=61)
    J, H, G = g.vet_step(dt, 4, fl["kappa_E"], fl["chi_F"], fl["B"], fl["J"], fl["H"])
    cu = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    dJ, dH, dG = cu(fl["J"]), cu(fl["H"]), torch.empty((g.P, 4), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    g.vet_step_dev(dt, 4, cu(fl["kappa_E"]), cu(fl["chi_F"]), cu(fl["B"]), dJ, dH, dG)
    assert np.array_equal(dJ.cpu().numpy(), J) and np.array_equal(dH.cpu().numpy(), H)
    assert np.array_equal(dG.cpu().numpy(), G)
    bad = cu(fl["kappa_E"])
    bad[5] = -1.0
    with pytest.raises(B.RRTError, match="kappa_E"):
        g.vet_step_dev(dt, 1, bad, cu(fl["chi_F"]), cu(fl["B"]), dJ, dH)
    with pytest.raises(B.RRTError, match="dt"):
        g.vet_step(0.0, 1, fl["kappa_E"], fl["chi_F"], fl["B"], fl["J"], fl["H"])
    g.close()
