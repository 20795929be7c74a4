"""Sampled parity at the full size of the headline workload.

The 64^3 x 32-group x 512-ordinate, L = 15 thermal-Compton jet (electron
temperatures 10-100 keV) is swept on the GPU in FP32 exactly as the benchmark
times it (a stage of the four-stage scheme, autotuned kernel variants,
captured sweeps), and outputs the oracle can compute one at a time are
compared with it:

* S2 + S3 at sampled points: the oracle's sh2do and boost of that point's
  source and stage intensity (a one-point oracle problem with the point's
  medium) against the library's S~ of the sweep;
* S4 for sampled (ordinate, group) pairs: the oracle's march of that one
  ordinate and group over the whole grid, from the library's S~ and the
  oracle's own chi~, against the library's lab intensity;
* S5 + S6 and S1 at sampled points: the oracle's fold of the library's lab
  intensity at the point, and its source from the library's SH intensity.

The samples include the last point, ordinate and group, so every index range
of the arrays (more than 2^31 elements) is reached.  Tolerance 1e-5 of the
group maximum as in the reduced-size parity tests (groups much fainter than a
neighbour within 8 groups are held to 1e-5 of 1/100 of that neighbour) in
FP32; 1e-4 in mixed precision (the SH <-> ordinate products on FP16 matrix
cores with hi/lo operand pairs, about 22 significant bits).
"""
import numpy as np
import pytest

import oracle
from paper_1507_05141_amd import binding as B
from paper_1507_05141_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RTOL = {B.FP32: 1e-5, B.MIXED: 1e-4}


def close_by_group(got, ref, gaxis, what, rtol, reach=8):
    g = np.moveaxis(got, gaxis, 0).reshape(got.shape[gaxis], -1)
    r = np.moveaxis(ref, gaxis, 0).reshape(ref.shape[gaxis], -1)
    own = np.abs(r).max(axis=1)
    worst = 0.0
    for i in range(r.shape[0]):
        scale = max(own[i], 1e-2 * own[max(0, i - reach):i + reach + 1].max())
        err = np.max(np.abs(g[i] - r[i]))
        worst = max(worst, err / scale if scale > 0 else err)
        assert err <= rtol * scale + 1e-300, f"{what} group {i}: max err {err:.3e} vs scale {scale:.3e}"
    return worst


def point_oracle(spec, p):
    """Oracle problem of the single point p (its medium, the same groups,
    ordinates, SH order and temperature-node rule)."""
    sub = dict(spec)
    sub.update(nx=1, ny=1, nz=1, kappa=spec["kappa"][p:p + 1], sigma=spec["sigma"][p:p + 1],
               bnu=spec["bnu"][p:p + 1], beta=spec["beta"][p:p + 1], kte=spec["kte"][p:p + 1],
               bc_bot=None, bc_top=None)
    return oracle.Oracle(sub)


@pytest.mark.parametrize("prec", [B.FP32, B.MIXED], ids=["fp32", "mixed"])
def test_full_size_compton_jet_sampled_parity(prec):
    spec = W.compton_jet()
    rtol = RTOL[prec]
    n, G, K = spec["nx"], len(spec["edges"]) - 1, spec["nmu"] * spec["nphi"]
    P = n ** 3
    NL = (spec["lmax"] + 1) ** 2
    stream = torch.cuda.current_stream().cuda_stream
    print(f"case compton_jet {n}^3 G={G} K={K} L={spec['lmax']} precision {prec}", flush=True)
    g = B.Problem.from_spec(spec, precision=prec, stream=stream)
    dt_stage = 0.5 / n / 6.0
    inv_cdt = 1.0 / dt_stage
    bnu = torch.from_numpy(spec["bnu"]).to("cuda", torch.float32)
    Ip = bnu.unsqueeze(0).expand(K, P, G).contiguous()           # the stage-start intensity of the benchmark
    g.set_intensity_dev(Ip)
    del Ip
    S0 = torch.zeros((P, G, NL), dtype=torch.float32, device="cuda")
    S0[:, :, 0] = torch.from_numpy(np.sqrt(4 * np.pi) * spec["kappa"] * spec["bnu"]
                                   / (spec["kappa"] + spec["sigma"][:, None])).to("cuda", torch.float32)
    g.set_source_sh_dev(S0)
    del S0
    for _ in range(2):                                           # the second sweep autotunes
        g.sweep(dt_stage)
    print(f"variants: {g.variants()}", flush=True)

    mid = (n // 2 * n + n // 2) * n + n // 2
    bmag = np.linalg.norm(spec["beta"], axis=1)
    bmag[:n * n] = bmag[-n * n:] = 0.0          # the fastest point off the inflow planes (on them the
                                                # forward-beamed comoving field sees only the vacuum inflow)
    points = sorted({0, P - 1, mid, int(np.argmax(bmag)), int(np.argmax(spec["kte"])), 123457})
    cut = lambda a: np.ascontiguousarray(a, dtype=np.float64)
    pts = torch.tensor(points, device="cuda")
    S_old = g.source_sh_dev()
    S_old_p = S_old[pts].double().cpu().numpy()
    del S_old
    Ip_p = bnu[pts].double().cpu().numpy()                       # [npts][G], the same on every ordinate
    nmu, nphi = spec["nmu"], spec["nphi"]
    marches = [(K - 1, G - 1), (0, 0), (7 * nphi + 5, 20), (8 * nphi + 17, 12), (12 * nphi + 9, 28)]
    St = g.lab_source_dev(dt_stage)
    St_p = St[:, pts, :].double().cpu().numpy()                  # [K][npts][G]
    St_m = [St[k, :, gg].double().cpu().numpy() for k, gg in marches]
    del St
    g.sweep(dt_stage)
    print(f"graphs held: {g.graph_count()}", flush=True)
    I = g.sweep_intensity_dev()
    I_p = I[:, pts, :].double().cpu().numpy()
    I_m = [I[k, :, gg].double().cpu().numpy() for k, gg in marches]
    del I
    Ilm_p = g.intensity_sh_dev()[pts].double().cpu().numpy()
    S_new_p = g.source_sh_dev()[pts].double().cpu().numpy()
    g.close()
    torch.cuda.empty_cache()

    for i, p in enumerate(points):
        o1 = point_oracle(spec, p)
        ref_St, _ = o1.boost(o1.sh2do(S_old_p[i][None]), np.broadcast_to(Ip_p[i], (K, 1, G)), inv_cdt)
        w1 = close_by_group(St_p[:, i:i + 1, :], ref_St, 2, f"S~ at point {p}", rtol)
        ref_Ilm = o1.fold(cut(I_p[:, i:i + 1, :]))
        w2 = close_by_group(Ilm_p[i][None], ref_Ilm, 1, f"I_lm at point {p}", rtol)
        ref_S = o1.source(cut(Ilm_p[i][None]))
        w3 = close_by_group(S_new_p[i][None], ref_S, 1, f"S_new at point {p}", rtol)
        print(f"point {p}: S~ {w1:.1e}, fold {w2:.1e}, source {w3:.1e} (worst error / scale)", flush=True)

    o = oracle.Oracle(spec)
    for (k, gg), s_m, i_m in zip(marches, St_m, I_m):
        x_m = o.lab_extinction(k, gg, inv_cdt)
        ref = o.trace_one(k, gg, s_m, x_m)
        err = np.abs(i_m - ref).max() / np.abs(ref).max()
        print(f"march ordinate {k} group {gg}: max error {err:.2e} of its maximum {np.abs(ref).max():.2e}", flush=True)
        assert err <= rtol
