"""Serving sample for bench.py: continuous batching of whole solves.

Requests are shaped like the serving workload (N = 2^round(U[10,16]), D in
{2,3,4}, ballistic-like kernel with a ~ U[0,0.9], float-float spectra) with a
step inside explicit Heun's stability interval and 20..200 steps per request,
so the sample finishes in seconds.  First all requests are
submitted at once (closed loop) to measure the saturated rate mu_sat; then the
same requests arrive as a Poisson process at 0.8 * mu_sat and the latency
(finish - submit) percentiles are reported.
"""
from __future__ import annotations

import time

import numpy as np


def _drain(eng, tickets, Ns, deadline_s=600.0):
    done = {}
    t0 = time.perf_counter()
    while len(done) < len(tickets):
        for t, N in zip(tickets, Ns):
            if t in done:
                continue
            rc, out, st = eng.poll(t, N)
            if rc != 1:
                done[t] = (rc, out, st)
        if time.perf_counter() - t0 > deadline_s:
            raise RuntimeError("serving sample did not finish")
        time.sleep(0.0005)
    return done


def run_serving(count: int, steps_range=(20, 200), log=print, seed: int = 4, nsample: int = 6):
    """Returns (summary, sample): the sample is ``nsample`` served results with
    their requests (the cheapest ones to re-solve on the host: smallest N times
    steps), which bench.py checks against the oracle after all GPU work."""
    import paper_1905_09071_amd as agg
    import synth

    reqs = synth.serving_requests(count, seed=seed, steps_range=steps_range)
    eng = agg.Engine(0)
    try:
        # closed loop: everything submitted at t = 0
        t0 = time.perf_counter()
        tickets = [eng.submit(r["D"], r["N"], r["kernel"], r["n0"], r["dt"], r["t_end"], "fp32c") for r in reqs]
        done = _drain(eng, tickets, [r["N"] for r in reqs])
        makespan = time.perf_counter() - t0
        mu_sat = count / makespan
        bad = sum(1 for v in done.values() if v[0] != 0)
        log(f"[serving] closed loop: {count} solves in {makespan:.3f} s -> {mu_sat:.1f} solves/s, {bad} failed")

        # open loop: Poisson arrivals at 0.8 mu_sat
        lam = 0.8 * mu_sat
        gaps = np.random.default_rng(seed + 1).exponential(1.0 / lam, size=count)
        arrivals = np.cumsum(gaps)
        tickets = []
        t0 = time.perf_counter()
        for r, ta in zip(reqs, arrivals):
            while time.perf_counter() - t0 < ta:
                time.sleep(0.0002)
            tickets.append(eng.submit(r["D"], r["N"], r["kernel"], r["n0"], r["dt"], r["t_end"], "fp32c"))
        done = _drain(eng, tickets, [r["N"] for r in reqs])
        span = time.perf_counter() - t0
        lat = np.array([(v[2].t_finish - v[2].t_submit) for v in done.values()])
        cost = [r["N"] * round(r["t_end"] / r["dt"]) * (1 << (2 * r["D"])) for r in reqs]
        pick = sorted(range(count), key=lambda i: cost[i])[:nsample]
        sample = [(done[tickets[i]][1], reqs[i]) for i in pick if done[tickets[i]][0] == 0]
        queue = np.array([(v[2].t_admit - v[2].t_submit) for v in done.values()])
        steps = int(sum(v[2].steps for v in done.values()))
        bad = sum(1 for v in done.values() if v[0] != 0)
        res = {
            "requests": count,
            "precision": "fp32c",
            "steps_per_request": list(steps_range),
            "dt": "min(1e-3, 1/(D^2 N^a)) per request",
            "mu_sat_solves_per_s": round(mu_sat, 2),
            "arrival_rate_per_s": round(lam, 2),
            "solves_per_s": round(count / span, 2),
            "p50_latency_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
            "p99_latency_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
            "p50_queue_ms": round(float(np.percentile(queue, 50)) * 1e3, 3),
            "heun_steps": steps,
            "failed": bad,
        }
        log(f"[serving] poisson at {lam:.1f}/s: p50 {res['p50_latency_ms']} ms, p99 {res['p99_latency_ms']} ms")
        return res, sample
    finally:
        eng.close()
