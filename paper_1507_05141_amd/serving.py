"""Continuous batching of steady-state radiative-transfer solves.

Requests (a problem description each) arrive over time; the loop admits them
in arrival order while the device-memory budget has room, advances every
running solve by one Lambda iteration per round through the library's batch
(`rrt_batch_*`: each problem on its own stream, so uneven solves overlap on
the GPU), and retires each request when its solve finishes, freeing its slot
and memory for the next arrival.  Problems keep their fields and source
function on the device from admission to retirement.  Latency is measured
from arrival to the round in which the result is seen.

The request mix follows the batched and served workloads: grids n^3 with n in
`sizes`, G groups, SH order L (8 x 16 ordinates for L = 3, 16 x 32 above), a
jet with Gamma_max log-uniform in [1.1, 20], a spatially uniform n_e sigma_T
log-uniform in [0.1, 10], Thomson or Compton scattering with equal odds.
Thomson problems take the Thomson jet's frequency set-up; Compton problems
take log groups from 1e-3 keV to 200 keV with a 1 keV blackbody seed (with
L = 3, groups reaching MeV energies give a non-positive truncated
Klein-Nishina kernel whose Lambda iteration does not converge).
"""
import time

import numpy as np

from . import binding as B
from . import workloads as W


def request_spec(gen, sizes=(16, 24, 32), groups=(4, 8, 16), lmaxes=(3, 7)):
    """One problem of the mix, drawn from the generator `gen`."""
    n = int(gen.choice(sizes))
    G = int(gen.choice(groups))
    L = int(gen.choice(lmaxes))
    nmu, nphi = (8, 16) if L <= 3 else (16, 32)
    gmax = float(np.exp(gen.uniform(np.log(1.1), np.log(20.0))))
    sig = float(10.0 ** gen.uniform(-1.0, 1.0))
    seed = int(gen.integers(1 << 30))
    if gen.uniform() < 0.5:
        spec = W.thomson_jet(n=n, ng=G, lmax=L, nmu=nmu, nphi=nphi, gamma_max=gmax, seed=seed)
        kind = "thomson"
    else:
        spec = W.compton_jet(n=n, ng=G, lmax=L, nmu=nmu, nphi=nphi, gamma_max=gmax, seed=seed, e_hi=200.0)
        kind = "compton"
    spec["sigma"] = np.full(n ** 3, sig)
    meta = {"n": n, "G": G, "lmax": L, "gamma_max": gmax, "sigma": sig, "scatter": kind}
    return spec, meta


def poisson_requests(count, rate, seed, **mix):
    """`count` requests with exponential inter-arrival times of mean 1/rate
    (seconds; rate 0: all at once).  The problems come from one stream of the
    seed and the arrival times from another, so the same seed gives the same
    problems at any rate."""
    gen = np.random.Generator(np.random.PCG64([seed, 0]))
    arr = np.random.Generator(np.random.PCG64([seed, 1]))
    t = 0.0
    out = []
    for _ in range(count):
        t += float(arr.exponential(1.0 / rate)) if rate > 0 else 0.0
        spec, meta = request_spec(gen, **mix)
        out.append({"arrival": t, "spec": spec, "meta": meta})
    return out


def serve(requests, precision=B.FP32, budget_bytes=64 << 30, tol=1e-6, max_iter=300, use_ng=True, keep=None,
          graphs=True, progress=None, autotune=False, pool_bytes=None, release_pool=True):
    """Run the request stream; returns per-request records and the run's wall time.

    keep(i, problem) -> dict, if given, is called on each finished problem
    before it is destroyed (e.g. to read its moments).  graphs=False runs every
    sweep eagerly instead of replaying captured sweeps.  progress(done, total),
    if given, is called whenever a request finishes or is rejected.  Requests
    run the library's default kernel variants unless autotune is set (timing
    candidates inside a request would add to its latency and, with other
    requests sharing the GPU, measure contention as much as the kernels).

    Device memory that retired requests free is kept for the next requests of
    the same sizes (rrt_set_device_pool, up to pool_bytes, default a quarter of the budget):
    freeing device memory would synchronise the device and stall the running
    requests at every retirement; release_pool empties the pool on return."""
    # a quarter of the budget by default: the pool's blocks are not in the budget, so a pool as
    # large as a near-full budget would leave allocations to fail and empty it
    B.set_device_pool(budget_bytes // 4 if pool_bytes is None else pool_bytes)
    batch = B.Batch(budget_bytes)
    pending = list(range(len(requests)))           # not yet admitted, in arrival order
    running = {}                                    # request -> Problem
    reserved = {}                                   # request -> bytes counted at admission
    used = 0
    blocked = False                                 # the head request did not fit: wait for a retirement
    recs = [None] * len(requests)
    t0 = time.perf_counter()
    now = lambda: time.perf_counter() - t0
    try:
        while pending or running:
            # admit arrived requests in order while the budget allows
            while pending and not blocked and requests[pending[0]]["arrival"] <= now():
                i = pending[0]
                spec = requests[i]["spec"]
                need = B.footprint_bytes(spec, precision, time_dependent=False, use_ng=use_ng)
                if used + need > budget_bytes and running:
                    break
                t_adm = now()
                pr = B.Problem.from_spec(spec, precision=precision)
                if not graphs:
                    pr.set_graphs(False)
                if not autotune:
                    pr.set_autotune(False)
                if not batch.admit(pr, tol=tol, max_iter=max_iter, use_ng=use_ng):
                    pr.close()
                    if running:
                        blocked = True
                        break
                    # larger than the whole budget: rejected
                    pending.pop(0)
                    recs[i] = {"arrival": requests[i]["arrival"], "rejected": True, "latency": now() - requests[i]["arrival"],
                               "iters": 0, "converged": False, **requests[i]["meta"]}
                    if progress is not None:
                        progress(sum(r is not None and "latency" in r for r in recs), len(requests))
                    continue
                pending.pop(0)
                running[i] = pr
                reserved[i] = need
                used += need
                recs[i] = {"arrival": requests[i]["arrival"], "admitted": t_adm, **requests[i]["meta"]}
            if not running:
                if pending:
                    time.sleep(max(0.0, min(0.01, requests[pending[0]]["arrival"] - now())))
                continue
            batch.step(1)
            for i in list(running):
                done, info = batch.poll(running[i])
                if not done:
                    continue
                pr = running.pop(i)
                t_done = now()
                recs[i].update(finished=t_done, latency=t_done - recs[i]["arrival"], iters=info["iters"],
                               residual=info["residual"], converged=info["converged"])
                batch.remove(pr)
                if keep is not None:
                    recs[i].update(keep(i, pr))
                pr.close()
                used -= reserved.pop(i)
                blocked = False
                if progress is not None:
                    progress(sum(r is not None and "latency" in r for r in recs), len(requests))
    finally:
        for pr in running.values():
            pr.close()
        batch.close()
        if release_pool:
            B.set_device_pool(0)
    return recs, now()


def summary(recs, wall):
    """Solves per second, latency percentiles and iteration counts of the served
    (not rejected) requests."""
    done = [r for r in recs if not r.get("rejected")]
    lat = np.array([r["latency"] for r in done]) if done else np.zeros(1)
    return {"requests": len(recs), "rejected": len(recs) - len(done), "solves_per_s": len(done) / wall, "wall_s": wall,
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_iters": float(np.mean([r["iters"] for r in done])) if done else 0.0,
            "not_converged": sum(not r["converged"] for r in done),
            "all_converged": bool(all(r["converged"] for r in done))}
