"""Serving engine on the GPU: requests of uneven N, D, kernel and length run
concurrently (continuous batching); each result equals, bit for bit, the same
request served alone by the engine, agrees with the oracle's Heun trajectory of
the request (per-rank FFT evaluation of the Sec. 1 sums, Heun stepping of
Sec. 3) and with agg_solve of the request within the parity tolerance
(agg_solve may narrow the column group of a small launch, which regroups the
binary64 partial dot products); admission, rejection and ticket handling."""
import ctypes
import sys
import time

import numpy as np
import pytest

import oracle
import synth
from conftest import dense_kernel

torch = pytest.importorskip("torch")
agg = pytest.importorskip("paper_1905_09071_amd")

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def alone(r, prec):
    plan = agg.Plan(r["D"], r["N"], r["kernel"], prec)
    n = torch.tensor(r["n0"], dtype=torch.float64, device="cuda:0")
    plan.solve(n, r["dt"], r["t_end"])
    out = n.cpu().numpy()
    plan.close()
    return out


TOL = {"fp64": 1e-12, "fp32c": 1e-10}
_ORACLE = {}


def oracle_solve(r):
    """The oracle's n(t_end) of a request (cached per request: both precisions
    are checked against the same binary64 trajectory)."""
    key = (r["D"], r["N"], r.get("a"), r["dt"], r["t_end"], hash(np.asarray(r["n0"]).tobytes()))
    if key not in _ORACLE:
        k = dense_kernel(r["kernel"])
        rhs = lambda v: oracle.total_rhs(*oracle.rhs_fft(r["D"], r["N"], k, v))
        _ORACLE[key] = oracle.heun_solve(rhs, r["n0"], r["dt"], r["t_end"])
    return _ORACLE[key]


def vs_oracle(out, r):
    ref = oracle_solve(r)
    return float(np.max(np.abs(out - ref)) / np.max(np.abs(ref)))


def served_alone(r, prec):
    eng = agg.Engine(0)
    t = eng.submit(r["D"], r["N"], r["kernel"], r["n0"], r["dt"], r["t_end"], prec)
    rc, out, st = drain(eng, [t], [r["N"]])[t]
    eng.close()
    assert rc == agg.AGG_OK
    return out


def drain(eng, tickets, Ns, limit=120.0):
    res = {}
    t0 = time.time()
    while len(res) < len(tickets):
        for t, N in zip(tickets, Ns):
            if t not in res:
                rc, out, st = eng.poll(t, N)
                if rc != agg.AGG_PENDING:
                    res[t] = (rc, out, st)
        assert time.time() - t0 < limit, "engine did not finish"
        time.sleep(0.001)
    return res


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_mixed_requests_equal_alone(prec):
    reqs = synth.serving_requests(10, seed=11, t_end_range=(0.005, 0.05), log2n_range=(10, 14))
    # a second copy of the first request arrives later, while others run
    eng = agg.Engine(0)
    tickets = [eng.submit(r["D"], r["N"], r["kernel"], r["n0"], r["dt"], r["t_end"], prec) for r in reqs[:6]]
    time.sleep(0.002)
    tickets += [eng.submit(r["D"], r["N"], r["kernel"], r["n0"], r["dt"], r["t_end"], prec) for r in reqs[6:]]
    res = drain(eng, tickets, [r["N"] for r in reqs])
    c = eng.counters()
    eng.close()
    assert c["completed"] == len(reqs) and c["running"] == 0 and c["queued"] == 0
    for r, t in zip(reqs, tickets):
        rc, out, st = res[t]
        assert rc == agg.AGG_OK
        ref = alone(r, prec)
        solo = served_alone(r, prec)
        eo = vs_oracle(out, r)
        say(f"[serve] D={r['D']} N={r['N']} a={r['a']:.2f} steps={st.steps} "
            f"maxdiff vs agg_solve={np.max(np.abs(out - ref)):.3e}, rel err vs oracle {eo:.3e}")
        assert eo <= TOL[prec]
        assert st.steps == len(__import__("oracle").time_grid(r["dt"], r["t_end"]))
        assert np.array_equal(out, solo)       # slot arithmetic is independent of neighbours
        assert np.max(np.abs(out - ref)) <= TOL[prec] * np.max(np.abs(ref))
        assert st.t_submit <= st.t_admit <= st.t_finish


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_saturating_mix_equals_alone(prec):
    """Enough concurrent requests of one transform length that the bucket's
    launches take the variants for launches that fill the GPU (several
    workgroups per CU, one transform per wavefront), while each request served
    alone takes the full variants: every result is still bit for bit the alone
    one (all variants run the same stage sequence with the same rounding), and
    within the parity bar of the oracle."""
    N = 65536
    reqs = []
    for i in range(14):
        D = 2 if i < 8 else 4          # L = 2^17 (M1 = M2 = 256) and 2^18 (M1 = 512, M2 = 256)
        a = 0.15 + 0.05 * i
        dt = min(1e-3, 1.0 / (D * D * N ** a))
        reqs.append(dict(D=D, N=N, a=a, kernel=synth.kernel_ballistic(D, N, a),
                         n0=synth.n0_uniform_head(N, 100 + i, 16), dt=dt, t_end=3 * dt))
    eng = agg.Engine(0)
    tickets = [eng.submit(r["D"], r["N"], r["kernel"], r["n0"], r["dt"], r["t_end"], prec) for r in reqs]
    res = drain(eng, tickets, [r["N"] for r in reqs])
    eng.close()
    for i, (r, t) in enumerate(zip(reqs, tickets)):
        rc, out, st = res[t]
        assert rc == agg.AGG_OK
        solo = served_alone(r, prec)
        same = np.array_equal(out, solo)
        say(f"[serve-mix] D={r['D']} a={r['a']:.2f} steps={st.steps} equal alone: {same}, "
            f"max diff {np.max(np.abs(out - solo)):.3e}")
        assert same
        if i in (0, 9):
            eo = vs_oracle(out, r)
            say(f"  rel err vs oracle {eo:.3e}")
            assert eo <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_configured_horizon_requests(prec):
    """Requests of the serving shape at its configured horizon, t_end in [1, 20]
    (1000 to 1500 Heun steps of h = 1e-3, sizes and exponents for which that step
    is inside Heun's stability interval), served together: each result against
    the oracle's Heun trajectory."""
    reqs = []
    for i, (D, N, a, t_end) in enumerate(((2, 1024, 0.1, 1.0), (3, 1024, 0.25, 1.5), (3, 2048, 0.2, 1.2),
                                          (2, 2048, 0.3, 1.0))):
        reqs.append(dict(D=D, N=N, a=a, kernel=synth.kernel_ballistic(D, N, a),
                         n0=synth.n0_uniform_head(N, 300 + i, 16), dt=1e-3, t_end=t_end))
    eng = agg.Engine(0)
    tickets = [eng.submit(r["D"], r["N"], r["kernel"], r["n0"], r["dt"], r["t_end"], prec) for r in reqs]
    res = drain(eng, tickets, [r["N"] for r in reqs])
    eng.close()
    for r, t in zip(reqs, tickets):
        rc, out, st = res[t]
        assert rc == agg.AGG_OK
        assert st.steps == len(__import__("oracle").time_grid(r["dt"], r["t_end"]))
        eo = vs_oracle(out, r)
        say(f"[serve-horizon] D={r['D']} N={r['N']} a={r['a']} t_end={r['t_end']} steps={st.steps}: "
            f"rel err vs oracle {eo:.3e}")
        assert eo <= TOL[prec]


def test_budget_and_errors():
    N = 4096
    k = synth.kernel_ballistic(3, N, 0.5)
    n0 = synth.n0_uniform_head(N, 1)
    eng = agg.Engine(0, mem_budget=256 << 10)      # 256 KiB: too small for this request
    with pytest.raises(agg.AggError) as e:
        eng.submit(3, N, k, n0, 1e-3, 0.01, "fp64")
    assert e.value.status == agg.AGG_ENOMEM
    eng.close()
    eng = agg.Engine(0)
    bad = n0.copy()
    bad[3] = np.nan
    with pytest.raises(agg.AggError) as e:
        eng.submit(3, N, k, bad, 1e-3, 0.01, "fp64")
    assert e.value.status == agg.AGG_ENONFINITE
    with pytest.raises(agg.AggError) as e:
        eng.poll(987654321, N)
    assert e.value.status == agg.AGG_ENOTFOUND
    # t_end = 0: the result is the initial state
    t = eng.submit(3, N, k, n0, 1e-3, 0.0, "fp64")
    res = drain(eng, [t], [N])
    assert res[t][0] == agg.AGG_OK and np.array_equal(res[t][1], n0)
    eng.close()


def test_fifo_admission_under_tight_budget():
    """With room for about one request at a time every request still finishes,
    in submission order of admission."""
    reqs = synth.serving_requests(4, seed=12, t_end_range=(0.003, 0.01), log2n_range=(12, 12))
    eng = agg.Engine(0, mem_budget=3 << 20)
    tickets = [eng.submit(r["D"], r["N"], r["kernel"], r["n0"], r["dt"], r["t_end"], "fp64") for r in reqs]
    res = drain(eng, tickets, [r["N"] for r in reqs])
    eng.close()
    admits = [res[t][2].t_admit for t in tickets]
    assert all(res[t][0] == agg.AGG_OK for t in tickets)
    assert admits == sorted(admits)


def test_submits_from_several_threads():
    """Requests submitted concurrently from 4 client threads (each submitter
    plans and stages its own request) all finish with distinct tickets, and each
    result equals bit for bit the same request submitted from one thread into
    another engine; one sample agrees with the oracle's trajectory."""
    from concurrent.futures import ThreadPoolExecutor
    reqs = synth.serving_requests(24, seed=14, t_end_range=(0.003, 0.02), log2n_range=(10, 13))
    sub = lambda eng, r: eng.submit(r["D"], r["N"], r["kernel"], r["n0"], r["dt"], r["t_end"], "fp64")
    eng = agg.Engine(0)
    with ThreadPoolExecutor(4) as pool:
        tickets = list(pool.map(lambda r: sub(eng, r), reqs))
    assert len(set(tickets)) == len(reqs)
    res = drain(eng, tickets, [r["N"] for r in reqs])
    c = eng.counters()
    eng.close()
    assert c["completed"] == len(reqs) and c["running"] == 0 and c["queued"] == 0
    eng1 = agg.Engine(0)
    t1 = [sub(eng1, r) for r in reqs]
    res1 = drain(eng1, t1, [r["N"] for r in reqs])
    eng1.close()
    for r, t, u in zip(reqs, tickets, t1):
        assert res[t][0] == agg.AGG_OK and res1[u][0] == agg.AGG_OK
        assert np.array_equal(res[t][1], res1[u][1])
    i = min(range(len(reqs)), key=lambda j: reqs[j]["N"] * (1 << reqs[j]["D"]))
    e = vs_oracle(res[tickets[i]][1], reqs[i])
    say(f"[serve threads] {len(reqs)} requests from 4 threads; sample D={reqs[i]['D']} N={reqs[i]['N']} "
        f"rel err vs oracle {e:.3e}")
    assert e <= TOL["fp64"]


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_tensor_train_requests_in_the_mix(prec):
    """Requests whose kernels are given in tensor-train form (agg_submit_tt:
    random dense D = 3 cores of ranks (1,3,1), (1,4,4,1), 30 core columns, at
    N = 1024 and 4096; the chunked row pass's per-bin chains) served among CP
    requests: each tensor-train result equals the same request served alone bit
    for bit and agrees with the oracle's Heun trajectory of its rank paths."""
    rng = np.random.default_rng(91)
    cores = lambda N, ranks: [rng.uniform(0.1, 1.0, size=(ranks[m], N, ranks[m + 1])) for m in range(len(ranks) - 1)]
    tts = [dict(D=3, N=N, tt={2: cores(N, [1, 3, 1]), 3: cores(N, [1, 4, 4, 1])},
                n0=synth.n0_random_dense(N, 92 + N, decay=2e-3), dt=1e-3, t_end=0.02) for N in (1024, 4096)]
    cps = synth.serving_requests(4, seed=93, t_end_range=(0.003, 0.01), log2n_range=(10, 12))
    sub_tt = lambda eng, r: eng.submit(r["D"], r["N"], None, r["n0"], r["dt"], r["t_end"], prec, tt=r["tt"])
    eng = agg.Engine(0)
    bad = dict(tts[0], tt={2: cores(1024, [1, 9, 1])})            # a rank above 8
    with pytest.raises(agg.AggError) as ex:
        sub_tt(eng, bad)
    assert ex.value.status == agg.AGG_EINVAL
    with pytest.raises(agg.AggError) as ex:                         # the plain option is not an engine option
        r = tts[0]
        terms, nt, keep = agg.make_tt_terms(r["D"], r["N"], r["tt"])
        t = ctypes.c_uint64(0)
        agg.check(agg.lib().agg_submit_tt(eng._h, r["D"], r["N"], terms, nt,
                                          r["n0"].ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                          r["dt"], r["t_end"], agg.AGG_PLAIN | 0, ctypes.byref(t)))
    assert ex.value.status == agg.AGG_EINVAL
    t_tt = [sub_tt(eng, r) for r in tts]
    t_cp = [eng.submit(r["D"], r["N"], r["kernel"], r["n0"], r["dt"], r["t_end"], prec) for r in cps]
    res = drain(eng, t_tt + t_cp, [r["N"] for r in tts] + [r["N"] for r in cps])
    eng.close()
    assert all(res[t][0] == agg.AGG_OK for t in t_cp)
    for r, t in zip(tts, t_tt):
        rc, out, st = res[t]
        assert rc == agg.AGG_OK and st.steps == 20
        e1 = agg.Engine(0)
        u = sub_tt(e1, r)
        rc1, out1, _ = drain(e1, [u], [r["N"]])[u]
        e1.close()
        assert rc1 == agg.AGG_OK and np.array_equal(out, out1)
        cp = {d: oracle.tt_paths(c) for d, c in r["tt"].items()}
        rhs = lambda v: oracle.total_rhs(*oracle.rhs_fft(r["D"], r["N"], cp, v))
        ref = oracle.heun_solve(rhs, r["n0"], r["dt"], r["t_end"])
        e = float(np.max(np.abs(out - ref)) / np.max(np.abs(ref)))
        say(f"[serve tt] D=3 N={r['N']} {prec}: rel err vs oracle {e:.3e}")
        assert e <= TOL[prec]


def test_nonfinite_request_is_isolated():
    """A request stepped far outside Heun's stability interval blows up; it ends
    AGG_ENONFINITE (state still returned) while the requests that share its
    launches (same transform length) finish exactly as they do alone."""
    reqs = synth.serving_requests(3, seed=21, t_end_range=(0.005, 0.02), log2n_range=(11, 11))
    bad = dict(reqs[0])
    bad["dt"], bad["t_end"] = 5.0, 5.0 * 30
    eng = agg.Engine(0)
    allr = [bad] + reqs
    tickets = [eng.submit(r["D"], r["N"], r["kernel"], r["n0"], r["dt"], r["t_end"], "fp64") for r in allr]
    res = drain(eng, tickets, [r["N"] for r in allr])
    eng.close()
    rc, out, st = res[tickets[0]]
    assert rc == agg.AGG_ENONFINITE and st.status == agg.AGG_ENONFINITE
    assert not np.all(np.isfinite(out))
    for r, t in zip(reqs, tickets[1:]):
        rc, out, st = res[t]
        assert rc == agg.AGG_OK
        assert np.array_equal(out, served_alone(r, "fp64"))


def test_destroy_with_requests_in_flight():
    """Destroying the engine while requests are queued and running returns
    after the work already on the device, and a new engine serves normally."""
    reqs = synth.serving_requests(6, seed=31, t_end_range=(0.02, 0.05), log2n_range=(12, 13))
    eng = agg.Engine(0)
    for r in reqs:
        eng.submit(r["D"], r["N"], r["kernel"], r["n0"], r["dt"], r["t_end"], "fp64")
    t0 = time.time()
    eng.close()
    assert time.time() - t0 < 30.0
    assert np.array_equal(served_alone(reqs[0], "fp64"), served_alone(reqs[0], "fp64"))


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_chunked_and_weighted_requests_in_the_mix(prec):
    """A request whose row pass runs in chunks (random kernel, u = 76) and one
    with term weights, served together with small ones: each result equals
    the same request served alone bit for bit, and agg_solve within tolerance."""
    N = 65536
    big = dict(D=4, N=N, kernel=synth.kernel_random(4, N, {2: 4, 3: 8, 4: 11}, 21),
               n0=synth.n0_uniform_head(N, 5, 16), dt=1e-4, t_end=3e-4)
    k = synth.kernel_random(3, 2048, 2, 9)
    rng = np.random.default_rng(10)
    wk = {d: {"U": U, "weight": rng.uniform(0.5, 1.5, size=2)} for d, U in k.items()}
    weighted = dict(D=3, N=2048, kernel=wk, n0=synth.n0_uniform_head(2048, 6, 16), dt=1e-3, t_end=5e-3)
    small = dict(D=2, N=1024, kernel=synth.kernel_ballistic(2, 1024, 0.3), n0=synth.n0_uniform_head(1024, 7, 16),
                 dt=1e-3, t_end=4e-3)
    reqs = [big, weighted, small]
    eng = agg.Engine(0)
    tickets = [eng.submit(r["D"], r["N"], r["kernel"], r["n0"], r["dt"], r["t_end"], prec) for r in reqs]
    res = drain(eng, tickets, [r["N"] for r in reqs])
    eng.close()
    for r, t in zip(reqs, tickets):
        rc, out, _ = res[t]
        assert rc == agg.AGG_OK
        assert np.array_equal(out, served_alone(r, prec))
        ref = alone(r, prec)
        e = float(np.max(np.abs(out - ref)) / np.max(np.abs(ref)))
        eo = vs_oracle(out, r)
        say(f"[mix chunked/weighted] D={r['D']} N={r['N']} {prec}: vs agg_solve {e:.2e}, vs oracle {eo:.2e}")
        assert e <= TOL[prec] and eo <= TOL[prec]
