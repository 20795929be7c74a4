"""Benchmark: grid-point x ordinate x group updates per second of the
source-iteration sweep on one MI355X.

A step is one full sweep (SH -> comoving ordinates, Lorentz transform to the
lab frame with the implicit time terms, ray trace, inverse transform,
ordinates -> SH, new source function, residual) of the 64^3 relativistic
Compton jet (32 log groups over [1e-3, 1e3] keV, electron temperature
10-100 keV, L = 15, 16 x 32 ordinates, FP32) inside a time step of 0.5 cell
light-crossing times (the first stage of the four-stage scheme, dt/6), with
every input, including the stage's starting intensity, already resident in
HBM.  Prints one JSON line with the throughput, the roofline of the dominant
kernel (timed live with HIP events on the library's stream) and the FP64
oracle's rate on the host cores for a sample of the same physics.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "grid-pt·ordinate·group updates/s per sweep"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
KERNELS = ["trace", "sh2do", "boost", "unboost", "do2sh", "source", "reduce"]


def algorithmic(kernel, spec, esz, time_dependent, precision="fp32"):
    """Roofline quantity of one launch of each timed step of the sweep, from the
    method's own data movement and arithmetic: the reads and writes the step
    cannot avoid, once each, with no round trip of an intermediate array the
    method keeps on chip (the comoving ordinate values between the SH product
    and the frame transform, and between the inverse transform and the
    backward product), and the dense products counted in flops."""
    n = spec["nx"] * spec["ny"] * spec["nz"]
    G = len(spec["edges"]) - 1 if spec.get("edges") is not None else 1
    K = spec["nmu"] * spec["nphi"]
    NL = (spec["lmax"] + 1) ** 2
    compton = spec.get("scatter", "thomson") == "compton"
    # the residual's row sums are formed in the source pass: Thomson with NL dividing 64 or 256,
    # Compton on the matrix cores (FP32, G <= 32, L <= 15, NL / 4 dividing 64)
    if compton:
        fused = precision != "fp64" and G <= 32 and spec["lmax"] <= 15 and NL % 4 == 0 and 64 % (NL // 4) == 0
    else:
        fused = 64 % NL == 0 or (NL % 4 == 0 and 256 % NL == 0)
    grey_chi = not compton and spec.get("kappa") is not None and bool((spec["kappa"] == spec["kappa"][:, :1]).all())
    do, sh = n * G * K, n * G * NL
    mfma_peak = 2500.0 if precision == "mixed" else FP32_PEAK_TFLOPS
    table = {
        # S~ read, I written, and a per-group lab extinction read (a grey one is per point and ordinate)
        "trace": ("hbm", esz * (2 * do + (n * K if grey_chi else do))),
        # 2 NL flops per update (the product's output stays on chip in the method)
        "sh2do": ("mfma", 2.0 * NL * do, mfma_peak),
        # SH source read (the comoving values it transforms), the stage's starting intensity read, S~ written
        "boost": ("hbm", esz * ((2 if time_dependent else 1) * do + sh)),
        # lab intensity read, comoving SH intensity written (through the backward product)
        "unboost": ("hbm", esz * (do + sh)),
        "do2sh": ("mfma", 2.0 * NL * do, mfma_peak),
        # SH intensity read, new source written, and (where the residual's row sums are taken in
        # the same pass) the old source read
        "source": ("hbm", esz * (3 if fused else 2) * sh),
        # the residual: both sources read, or only the per-row sums where fused into the source
        "reduce": ("hbm", 16 * n * G if fused else esz * 2 * sh),
    }
    return table[kernel]


def traffic_from_profiles(kernel, workload, time_dependent, precision):
    """Measured HBM bytes per launch from the committed rocprofv3 counter
    summary, or None when absent or taken on a different kernel source, stage
    kind or precision."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("time_dependent") != time_dependent or rec.get("precision") != precision:
        return None
    src = os.path.join(ROOT, "paper_1507_05141_amd", "csrc", "rrt_kernels.hip")
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if rec.get("kernel_source_sha256") != h:
        return None
    return rec.get("bytes_per_launch")


def stage_start_intensity(spec, K):
    """Synthetic intensity at the start of the stage: the comoving thermal source
    on every lab ordinate, [K][P][G]."""
    import numpy as np
    return np.ascontiguousarray(np.broadcast_to(spec["bnu"][None, :, :], (K,) + spec["bnu"].shape))


def cpu_baseline(spec, inv_cdt, label):
    """The FP64 oracle, as it stands, timed on this host's cores over one full
    sweep of `spec` (the benchmark's physics, on a grid the host finishes in
    seconds) and stage."""
    import oracle
    o = oracle.Oracle(spec)
    I0 = stage_start_intensity(spec, o.K) if inv_cdt else None
    S = o.initial_source(I0)
    t0 = time.perf_counter()
    o.sweep(S, I0, inv_cdt)
    dt = time.perf_counter() - t0
    updates = o.P * o.G * o.K
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": updates / dt, "unit": "updates/s", "cores": cores, "kind": "oracle",
            "sample": f"one full FP64 sweep of {label} ({updates} updates, {dt:.1f} s; Compton tables not timed)"}


def serving_bench(args):
    """Solve requests drawn from the mix (grids 16^3-32^3, 4-16 groups, L = 3 or 7,
    Thomson or Compton), each to a residual below 1e-6 with Ng acceleration.
    Capacity: all requests at once, in FP32 with eager sweeps, in FP32 with
    captured sweeps and in mixed precision.  Latency: the same problems arriving
    as a Poisson stream at 0.8 x the FP32 capacity, in FP32 and in mixed precision."""
    from paper_1507_05141_amd import binding as B
    from paper_1507_05141_amd import serving as SV
    if args.mix == "full":
        # every grid, group count and SH order of the batched workload, up to 64^3 x 32 x L = 15
        mix = dict(sizes=(16, 24, 32, 48, 64), groups=(4, 8, 16, 32), lmaxes=(3, 7, 15))
        budget = 240 << 30
        workload = "request mix: n in {16,24,32,48,64}, G in {4,8,16,32}, L in {3,7,15}, Thomson/Compton"
        # Compton requests at n_e sigma_T near 10 do not converge (the FP64 oracle neither): a
        # request gives up after 150 Lambda iterations (converged ones need at most ~90)
        max_iter = 150
    else:
        mix = {}
        budget = 64 << 30
        workload = "request mix: n in {16,24,32}, G in {4,8,16}, L in {3,7}, Thomson/Compton"
        max_iter = 300
    burst = SV.poisson_requests(args.requests, rate=0.0, seed=5, **mix)
    # warm-up on the measured requests themselves, once per precision: the first use of a
    # shape autotunes its kernel variants and builds its Compton tables (both kept for the
    # process), which would otherwise land in whichever timed pass meets the shape first
    for prec in (B.FP32, B.MIXED):
        SV.serve(burst, precision=prec, budget_bytes=budget, max_iter=max_iter, release_pool=False)
    cap = {}
    runs = (("fp32_eager", B.FP32, False), ("fp32", B.FP32, True), ("mixed", B.MIXED, True))
    if args.mix == "full":
        runs = runs[1:]
    def progress(done, total):
        if args.mix == "full" or done % 8 == 0 or done == total:       # full mix: large requests finish minutes apart
            print(f"  {done}/{total} requests finished", file=sys.stderr, flush=True)

    for name, prec, graphs in runs:
        recs, wall = SV.serve(burst, precision=prec, budget_bytes=budget, graphs=graphs, progress=progress,
                              max_iter=max_iter, release_pool=False)
        cap[name] = SV.summary(recs, wall)
        print(f"capacity {name}: {cap[name]['solves_per_s']:.2f} solves/s", file=sys.stderr, flush=True)
    rate = 0.8 * cap["fp32"]["solves_per_s"]
    stream = SV.poisson_requests(args.requests, rate=rate, seed=5, **mix)
    res = {}
    for name, prec in (("fp32", B.FP32), ("mixed", B.MIXED)):
        recs, wall = SV.serve(stream, precision=prec, budget_bytes=budget, progress=progress, max_iter=max_iter,
                              release_pool=False)
        res[name] = SV.summary(recs, wall)
        print(f"stream {name}: p50 {res[name]['p50_ms']:.1f} ms p99 {res[name]['p99_ms']:.1f} ms", file=sys.stderr,
              flush=True)
    B.set_device_pool(0)
    return {"metric": "solves/s (continuous batching, all requests at once)", "value": cap["mixed"]["solves_per_s"],
            "unit": "solves/s", "n_gpus": 1, "higher_is_better": True, "vs_baseline": None,
            "dtype": "f32+f16mfma", "data": "synthetic",
            "p50_ms": res["mixed"]["p50_ms"], "p99_ms": res["mixed"]["p99_ms"],
            "config": {"workload": workload,
                       "requests": args.requests, "arrival_rate_per_s": rate, "tol": 1e-6, "max_iter": max_iter,
                       "hbm_budget_bytes": budget},
            "capacity": cap, "stream": res}


def vet_bytes(P):
    """Method bytes of one step of the VET hand-off, per kernel: the flux update
    reads J, f (6), H (3), chi_F and the momentum exchange (3) and writes H and
    the exchange; the energy update reads H (3), J, kappa_E, B and the energy
    exchange and writes J and the exchange (FP64)."""
    return {"vet_flux": 8 * P * (1 + 6 + 3 + 3 + 1 + 3 + 3), "vet_energy": 8 * P * (3 + 1 + 1 + 1 + 1 + 1 + 1)}


def vet_bench(args):
    """The variable-Eddington-tensor hand-off: nsteps FP64 steps of the
    frequency-integrated moment equations closed with the Eddington tensor of
    an anisotropic lab intensity state, on the 64^3 grid of the Compton jet
    (launch-bound: 262144 points) and on a 64 x 64 x 4096 grid (16.8 M
    points, streaming-bound; x-y planes of the size the ray trace holds); the
    roofline of the dominant kernel on the larger grid."""
    import numpy as np
    import torch

    from paper_1507_05141_amd import binding as B
    out = {"metric": "VET moment-update point-steps/s", "unit": "point-steps/s", "n_gpus": 1,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic"}
    runs = {}
    for n in (64, 4096):
        P = 64 * 64 * n
        spec = dict(nx=64, ny=64, nz=n, lx=1.0, ly=1.0, lz=n / 64.0, nmu=2, nphi=4, lmax=1, edges=None, log_centres=True,
                    scatter="thomson", kappa=np.full((P, 1), 0.5), sigma=np.full(P, 1.0), bnu=np.full((P, 1), 1.0),
                    beta=None, kte=None, bc_bot=None, bc_top=None)
        pr = B.Problem.from_spec(spec, precision=B.FP32, stream=torch.cuda.current_stream().cuda_stream)
        gen = torch.Generator(device="cuda").manual_seed(7)
        I = torch.rand((pr.K, P, 1), generator=gen, device="cuda") + 0.1
        I[0] *= 4.0                                                   # anisotropic: one bright ordinate
        pr.set_intensity_dev(I)
        del I
        cu = lambda lo, hi, shape: lo + (hi - lo) * torch.rand(shape, generator=gen, device="cuda", dtype=torch.float64)
        kap, chi, Bf = cu(0.0, 2.0, (P,)), cu(0.5, 3.0, (P,)), cu(0.0, 1.0, (P,))
        J, H, G = cu(0.2, 1.0, (P,)), cu(-0.1, 0.1, (P, 3)), torch.empty((P, 4), dtype=torch.float64, device="cuda")
        dt = 0.5 / 64
        steps = max(args.steps, 1) * (20 if n == 64 else 2)
        pr.vet_step_dev(dt, steps, kap, chi, Bf, J, H, G)            # warm-up
        torch.cuda.synchronize()
        pr.set_profiling(True)
        t0 = time.perf_counter()
        pr.vet_step_dev(dt, steps, kap, chi, Bf, J, H, G)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        kern = {}
        for k in ("vet_flux", "vet_energy"):
            c, ms = pr.kernel_time(k)
            kern[k] = {"launches": c, "avg_ms": ms / c}
        pr.set_profiling(False)
        pr.close()
        b = vet_bytes(P)
        runs[n] = {"grid": [64, 64, n], "steps": steps, "ms_per_step": el / steps * 1e3, "value": P * steps / el,
                   "kernels": kern,
                   "kernel_rooflines": {k: {"bound": "hbm", "achieved_GBps": b[k] / (v["avg_ms"] * 1e-3) / 1e9,
                                            "frac": b[k] / (v["avg_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS}
                                        for k, v in kern.items()}}
        print(f"  VET 64 x 64 x {n}: {el / steps * 1e3:.3f} ms per step", file=sys.stderr, flush=True)
    big = runs[4096]
    PB = 64 * 64 * 4096
    dom = max(big["kernels"], key=lambda k: big["kernels"][k]["avg_ms"])
    ach = vet_bytes(PB)[dom] / (big["kernels"][dom]["avg_ms"] * 1e-3) / 1e9
    out.update(value=big["value"], steps=big["steps"], warmup=big["steps"], ms_per_step=big["ms_per_step"],
               config={"workload": "vet_handoff_64x64x4096", "grid": big["grid"], "transport_grid_64c": runs[64]},
               roofline={"kernel": dom, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": ach / HBM_PEAK_GBS, "traffic": None,
                         "algorithmic_bytes_per_launch": vet_bytes(PB)[dom],
                         "avg_launch_ms": big["kernels"][dom]["avg_ms"]},
               kernels=big["kernels"], kernel_rooflines=big["kernel_rooflines"])
    if not args.no_cpu_baseline:
        from oracle.vet import vet_step as ovet
        n, steps = 64, 4
        P = n ** 3
        rs = np.random.default_rng(1)
        f = np.zeros((P, 6))
        f[:, :3] = rs.uniform(0.2, 0.5, (P, 3))
        t0 = time.perf_counter()
        ovet((n, n, n, 1.0, 1.0, 1.0), f, rs.uniform(0, 2, P), rs.uniform(0.5, 3, P), rs.uniform(0, 1, P),
             rs.uniform(0.2, 1, P), rs.uniform(-0.1, 0.1, (P, 3)), 0.5 / n, steps)
        el = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": P * steps / el, "unit": "point-steps/s", "cores": 1, "kind": "oracle",
                               "sample": f"{steps} steps of the NumPy oracle on 64^3 ({el:.1f} s)"}
    return out


def validation_runs(args):
    """The paper's validation problems (Sec. 3) at its own grid and ordinate
    sizes, in FP32 on the library, each checked against the closed form the
    paper compares with.  One JSON line per problem: wall time, sweeps,
    updates per second and the measured deviations."""
    import numpy as np
    from paper_1507_05141_amd import binding as B
    from paper_1507_05141_amd import workloads as W

    def beam_J(nmu, nphi):
        mu, wmu = np.polynomial.legendre.leggauss(nmu)
        return mu[-1], wmu[-1] * 2 * np.pi / nphi / (4 * np.pi)

    def run(spec, I0, how):
        g = B.Problem.from_spec(spec, precision=B.FP32)
        g.set_intensity(I0)
        t0 = time.perf_counter()
        info = how(g)
        sec = time.perf_counter() - t0
        J, H, _ = g.moments(B.FRAME_LAB)
        I = g.intensity() if spec["nmu"] * spec["nphi"] * spec["nx"] * spec["nz"] <= (1 << 26) else None
        g.close()
        ups = spec["nx"] * spec["nz"] * spec["nmu"] * spec["nphi"]
        return dict(seconds=round(sec, 3), sweeps=info["sweeps"], updates_per_s=info["sweeps"] * ups / sec), J, H, I

    def advance(dt, nsteps, scheme, tol, max_iter, use_ng):
        def how(g):
            i = g.advance(dt, nsteps=nsteps, scheme=scheme, tol=tol, max_iter=max_iter, use_ng=use_ng)
            return dict(sweeps=i["iters"])
        return how

    def steady(g):
        i = g.solve(tol=1e-10, max_iter=5, use_ng=False)
        return dict(sweeps=i["iters"])

    def emit(rec):
        print(json.dumps(rec), flush=True)

    # searchlight beam, 512^2, (4, 8), one cell per step, t = 0.25 s
    n = 512
    mu, Jb = beam_J(4, 8)
    dt = 1.0 / (n - 1)
    nsteps = int(round(0.25 * W.SECOND / dt))
    ct = nsteps * dt
    prof = {}
    for alpha_cm in (0.0, 1e-10):
        spec, I0 = W.searchlight(n, alpha_cm=alpha_cm)
        rec, J, _, _ = run(spec, I0, advance(dt, nsteps, B.SCHEME_RK4, 1e-10, 5, False))
        J = J[:, 0].reshape(spec["nz"], n)
        z = np.arange(spec["nz"]) / (spec["nz"] - 1)
        xi = ((0.3 + z * np.sqrt(1 - mu * mu) / mu) % 1.0) * n
        i0 = np.floor(xi).astype(int)
        f = xi - i0
        rows = np.arange(spec["nz"])
        Jr = (1 - f) * J[rows, i0 % n] + f * J[rows, (i0 + 1) % n]
        s = z / mu
        att = np.exp(-alpha_cm * W.DOMAIN_CM * s)
        rel = Jr / Jb / att
        behind = s < ct - 0.25
        prof[alpha_cm] = rel
        emit(dict(problem="searchlight", alpha_per_cm=alpha_cm, grid=[n, n], ordinates=[4, 8], t_s=0.25, **rec,
                  max_dev_behind_front=float(np.max(np.abs(rel[behind] - 1))),
                  front_half_point_minus_ct=float(s[np.argmin(np.abs(rel - 0.5))] - ct), cell_path=1.0 / (n - 1) / mu))
    emit(dict(problem="searchlight", check="front shape with / without absorption",
              max_diff=float(np.max(np.abs(prof[1e-10] - prof[0.0])))))

    # two beams and a shadow, 512^2, (4, 8), steady state
    Js = {}
    for beams in ((0,), (1,), (0, 1)):
        spec, I0 = W.two_beam_shadow(n, beams=beams)
        rec, J, _, _ = run(spec, I0, steady)
        Js[beams] = J[:, 0].reshape(spec["nz"], n) / Jb
    both, nz = Js[(0, 1)], spec["nz"]

    def at(x, z):
        return float(both[int(round(z * (nz - 1))), int(round(x * n)) % n])
    emit(dict(problem="two_beam_shadow", grid=[n, n], ordinates=[4, 8], **rec,
              superposition_dev=float(np.max(np.abs(both - Js[(0,)] - Js[(1,)]))),
              J_over_beam={"lit_both(0.1,0.05)": at(0.1, 0.05), "above_shadows(0.5,0.9)": at(0.5, 0.9),
                           "one_shadow(0.75,0.7)": at(0.75, 0.7), "one_shadow(0.25,0.7)": at(0.25, 0.7),
                           "both_shadows(0.5,0.52)": at(0.5, 0.52)}))

    # optically thin pulse, 128^2, (64, 128), t = 0.1 s: peak of J r against free streaming
    spec, I0 = W.radiative_pulse(128, nmu=64, nphi=128)
    n, nz = spec["nx"], spec["nz"]
    dt = 1.0 / (nz - 1)
    nsteps = int(round(0.1 * W.SECOND / dt))
    rec, J, _, _ = run(spec, I0, advance(dt, nsteps, B.SCHEME_RK4, 1e-10, 5, False))
    J = J[:, 0].reshape(nz, n)
    t = nsteps * dt
    mid = (nz - 1) // 2
    r = np.arange(n // 2) / n
    mq, wq = np.polynomial.legendre.leggauss(256)
    ph = (np.arange(512) + 0.5) * np.pi / 256
    M, PH = np.meshgrid(mq, ph, indexing="ij")
    nxv, nzv = np.sqrt(1 - M ** 2) * np.cos(PH), M
    exact = np.array([(wq[:, None] * 100 * np.exp(-((rr - t * nxv) ** 2 + (t * nzv) ** 2) / 0.09 ** 2)).sum()
                      * (np.pi / 256) / (4 * np.pi) for rr in r])
    emit(dict(problem="thin_pulse", grid=[n, nz], ordinates=[64, 128], t_s=0.1, **rec,
              exact_peak_r=float(r[np.argmax(exact)]), exact_peak_J=float(exact.max()),
              x_axis_peak_r=float(r[np.argmax(J[mid, n // 2:])]), x_axis_peak_J=float(J[mid, n // 2:].max()),
              z_axis_peak_r=float(r[np.argmax(J[mid:mid + n // 2, n // 2])]),
              z_axis_peak_J=float(J[mid:mid + n // 2, n // 2].max()), centre_J=float(J[mid, n // 2]),
              exact_centre_J=float(exact[0])))

    # optically thick pulse, 128^2, (32, 64), backward Euler, dt = 1/20 to t = 1 (c = 1)
    spec, I0 = W.radiative_pulse(128, nmu=32, nphi=64, thick=True)
    n, nz = spec["nx"], spec["nz"]
    rec, J, _, _ = run(spec, I0, advance(0.05, 20, B.SCHEME_EULER, 1e-6, 400, True))
    J = J[:, 0].reshape(nz, n)
    x = np.arange(n) / n - 0.5
    Dc, t, w = 1.0 / (3 * 300.0), 1.0, 0.09
    Jd = 100 * w / np.sqrt(w ** 2 + 4 * Dc * t) * np.exp(-x ** 2 / (w ** 2 + 4 * Dc * t))
    emit(dict(problem="thick_pulse", grid=[n, nz], ordinates=[32, 64], t_units=t, **rec,
              max_dev_over_peak=float(np.max(np.abs(J[(nz - 1) // 2] - Jd)) / Jd.max())))

    # relativistic beaming, 128^2, (32, 64), steady state, beta along x
    nmu, nphi = 32, 64
    mq = np.polynomial.legendre.leggauss(nmu)[0]
    for bx in (0.0, 0.1, 0.5, 0.9, 0.99, 0.995):
        spec, I0 = W.beaming_cylinder(128, nmu=nmu, nphi=nphi, beta=(bx, 0.0))
        rec, J, H, I = run(spec, I0, steady)
        n, nz = spec["nx"], spec["nz"]
        I = I[:, :, 0].reshape(nmu * nphi, nz, n)
        worst = 0.0
        for a in range(nmu):
            st = np.sqrt(1 - mq[a] ** 2)
            for b in range(nphi):
                cph = np.cos(2 * np.pi * b / nphi)
                if cph <= 0:
                    continue
                ratio = ((1 + bx * st * cph) / (1 - bx * st * cph)) ** 3
                A, Mr = I[a * nphi + b], I[a * nphi + (nphi // 2 - b) % nphi][:, (-np.arange(n)) % n]
                lit = A > 1e-6 * A.max()
                if lit.any():
                    worst = max(worst, float(np.max(np.abs(A[lit] / (Mr[lit] * ratio) - 1))))
        emit(dict(problem="beaming_cylinder", beta_x=bx, gamma=1 / np.sqrt(1 - bx * bx), grid=[n, nz],
                  ordinates=[nmu, nphi], **rec, mirror_D3_ratio_max_dev=worst,
                  flux_x_over_J=float(H[:, 0, 0].sum() / J[:, 0].sum())))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["fp32", "fp64", "mixed"], default=None,
                    help="mixed: FP32 with the SH <-> ordinate products on FP16 matrix cores (the default for "
                         "the Compton jet, which is specified with 16-bit matrix-core transforms and FP32 "
                         "accumulation); fp32 the default for the Thomson jet")
    ap.add_argument("--workload", choices=["thomson_jet", "compton_jet"], default="compton_jet",
                    help="compton_jet (default): 64^3, 32 groups, L=15, electron temperature 10-100 keV; "
                         "thomson_jet: 32^3, 16 groups, L=7")
    ap.add_argument("--steady", action="store_true", help="time steady-state sweeps instead of a time-step stage")
    ap.add_argument("--serving", action="store_true",
                    help="continuous batching of a stream of solve requests instead of sweeps: solves/s, p50/p99 latency")
    ap.add_argument("--requests", type=int, default=48, help="requests in the --serving stream")
    ap.add_argument("--mix", choices=["small", "full"], default="small",
                    help="--serving request mix: small (n <= 32, G <= 16, L <= 7) or full (n <= 64, G <= 32, L <= 15)")
    ap.add_argument("--vet", action="store_true",
                    help="time the variable-Eddington-tensor hand-off (moment update closed with the transport's f)")
    ap.add_argument("--validation", action="store_true",
                    help="run the paper's validation problems (Sec. 3) at its sizes instead of the sweep benchmark")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device-to-device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the sweep is measured on one MI355X "
              "(multi-GPU sharding is a design note only).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1507_05141_amd import binding as B
    from paper_1507_05141_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    torch.cuda.set_device(0)
    if args.serving:
        print(json.dumps(serving_bench(args)), flush=True)
        return
    if args.vet:
        print(json.dumps(vet_bench(args)), flush=True)
        return
    if args.validation:
        validation_runs(args)
        return
    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload == "thomson_jet":
        spec = W.thomson_jet()
        workload = "thomson_jet_32c_g16_l7_16x32"
    else:
        spec = W.compton_jet()
        workload = "compton_jet_64c_g32_l15_16x32_kte10-100"
    if args.precision is None:
        args.precision = "mixed" if args.workload == "compton_jet" else "fp32"
    prec = {"fp32": B.FP32, "fp64": B.FP64, "mixed": B.MIXED}[args.precision]
    esz = 8 if prec == B.FP64 else 4
    stream = torch.cuda.current_stream().cuda_stream
    pr = B.Problem.from_spec(spec, precision=prec, stream=stream)
    # time step of half a cell light-crossing time, first stage (dt/6) of the
    # four-stage scheme; c = 1 and the cell is 1/nx
    dt = 0.5 / spec["nx"]
    dt_stage = 0.0 if args.steady else dt / 6.0
    if dt_stage:
        pr.set_intensity(stage_start_intensity(spec, pr.K))
    # the initial source of the solve (thermal emission only), resident on the device
    nl = (spec["lmax"] + 1) ** 2
    S0 = np.zeros((pr.P, pr.G, nl))
    S0[:, :, 0] = np.sqrt(4 * np.pi) * spec["kappa"] * spec["bnu"] / (spec["kappa"] + spec["sigma"][:, None])
    pr.set_source_sh(S0)
    for _ in range(args.warmup):
        pr.sweep(dt_stage)
    pr.synchronize()
    torch.cuda.synchronize()
    pr.set_profiling(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        pr.sweep(dt_stage)
    pr.synchronize()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kern = {}
    for k in KERNELS:
        n, ms = pr.kernel_time(k)
        if n:
            kern[k] = {"launches": n, "avg_ms": ms / n}
    pr.set_profiling(False)
    updates = pr.P * pr.G * pr.K
    value = updates * args.steps / elapsed
    dom = max(kern, key=lambda k: kern[k]["avg_ms"] * kern[k]["launches"])
    rl = algorithmic(dom, spec, esz, bool(dt_stage), args.precision)
    if rl[0] == "hbm":
        achieved = rl[1] / (kern[dom]["avg_ms"] * 1e-3) / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS,
                "traffic": traffic_from_profiles(dom, workload, bool(dt_stage), args.precision),
                "algorithmic_bytes_per_launch": rl[1], "avg_launch_ms": kern[dom]["avg_ms"]}
    else:
        achieved = rl[1] / (kern[dom]["avg_ms"] * 1e-3) / 1e12
        roof = {"kernel": dom, "bound": "mfma", "achieved": achieved, "peak": rl[2], "unit": "TFLOP/s",
                "frac": achieved / rl[2], "traffic": None,
                "algorithmic_flops_per_launch": rl[1], "avg_launch_ms": kern[dom]["avg_ms"]}
    # every timed step against its own roofline
    per_kernel = {}
    for k, v in kern.items():
        r = algorithmic(k, spec, esz, bool(dt_stage), args.precision)
        if r[0] == "hbm":
            a = r[1] / (v["avg_ms"] * 1e-3) / 1e9
            per_kernel[k] = {"bound": "hbm", "achieved_GBps": a, "frac": a / HBM_PEAK_GBS}
        else:
            a = r[1] / (v["avg_ms"] * 1e-3) / 1e12
            per_kernel[k] = {"bound": "mfma", "achieved_TFLOPs": a, "frac": a / r[2]}
    out = {
        "metric": METRIC, "value": value, "unit": "updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": {"fp32": "f32", "fp64": "f64", "mixed": "f32+f16mfma"}[args.precision],
        "data": "synthetic",
        "config": {"workload": workload, "grid": [spec["nx"], spec["ny"], spec["nz"]], "groups": pr.G,
                   "lmax": spec["lmax"], "ordinates": [spec["nmu"], spec["nphi"]], "scatter": spec["scatter"],
                   "gamma_max": 10.0, "updates_per_sweep": updates,
                   "electron_temperature_keV": [10.0, 100.0] if spec.get("kte") is not None else None,
                   "sh_products": {"mixed": "FP16 matrix cores (hi/lo operand pairs), FP32 accumulation",
                                   "fp32": "FP32 matrix cores", "fp64": "FP64 matrix cores"}[args.precision],
                   "stage": "steady" if not dt_stage else f"time step dt = {dt:.6g}, stage dt/6 (four-stage scheme)"},
        "roofline": roof,
        "kernels": kern,
        "kernel_rooflines": per_kernel,
    }
    pr.close()
    if not args.no_cpu_baseline:
        if args.workload == "thomson_jet":
            out["cpu_baseline"] = cpu_baseline(W.thomson_jet(), 1.0 / dt_stage if dt_stage else 0.0,
                                               "the same workload")
        else:
            # the same physics (groups, temperature field, L, ordinates, jet) on 16^3: a full
            # 64^3 oracle sweep would take hours on the host
            small = W.compton_jet(n=16)
            out["cpu_baseline"] = cpu_baseline(small, 6.0 / (0.5 / small["nx"]) if dt_stage else 0.0,
                                               "the 64^3 Compton jet's physics on a 16^3 grid")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
