"""GPU parity at mixed-radix transform lengths (3 2^a and 5 2^a: a radix-3 or
radix-5 first stage in the column transforms, AGG_MIXED_RADIX): the HIP path
against the oracle, element by element, at every supported column length, in
launches of one state and saturating batches, through Heun steps and the
serving engine, and at the two largest workloads: D = 5, N = 2^20 (L = 5 2^20
instead of 2^23) and the pure ternary D = 3, N = 2^19 (L = 3 2^19 instead of
2^21).  Tolerances as in the power-of-two parity tests."""
import sys
import time

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
agg = pytest.importorskip("paper_1905_09071_amd")

pytestmark = pytest.mark.gpu

RHS_TOL = {"fp64": 1e-12, "fp32": 1e-5, "fp32c": 1e-10}
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def gpu_rhs(D, N, kernel, n, prec, batch=1, mixed=True):
    plan = agg.Plan(D, N, kernel, prec=prec, batch=batch, mixed=mixed)
    out = plan.rhs(torch.tensor(np.asarray(n).reshape(-1), dtype=torch.float64, device=DEV))
    torch.cuda.synchronize()
    r = out.cpu().numpy()
    plan.close()
    return r.reshape(batch, N) if batch > 1 else r


# (label, D, N, kernel, state): each case's mixed length and column length M1
# (from the planner's rules) in the label
CASES = [
    ("M1-96-L6144", 5, 1025, lambda: synth.kernel_random(5, 1025, 1, 21), lambda: synth.n0_random_dense(1025, 1)),
    ("C2-M1-96-L12288", 3, 4096, lambda: synth.kernel_brownian_sum(3, 4096), lambda: synth.n0_exponential(4096)),
    ("M1-160-L20480-d2", 2, 10240, lambda: synth.kernel_random(2, 10240, 1, 22),
     lambda: synth.n0_random_dense(10240, 2)),
    ("M1-160-L20480", 5, 3282, lambda: synth.kernel_random(5, 3282, 1, 23), lambda: synth.n0_random_dense(3282, 3)),
    ("M1-192-L24576", 5, 4133, lambda: synth.kernel_random(5, 4133, 1, 24), lambda: synth.n0_random_dense(4133, 4)),
    ("M1-320-L81920", 5, 13124, lambda: synth.kernel_random(5, 13124, 1, 25),
     lambda: synth.n0_random_dense(13124, 5, decay=1e-4)),
    ("M1-384-L98304", 5, 16417, lambda: synth.kernel_random(5, 16417, 1, 26),
     lambda: synth.n0_random_dense(16417, 6, decay=1e-4)),
    ("M1-640-L163840", 5, 26222, lambda: synth.kernel_random(5, 26222, 1, 27),
     lambda: synth.n0_random_dense(26222, 7, decay=1e-4)),
    ("M1-768-L196608", 5, 32771, lambda: synth.kernel_random(5, 32771, 1, 28),
     lambda: synth.n0_random_dense(32771, 8, decay=1e-4)),
    ("M1-1280-L327680", 5, 52455, lambda: synth.kernel_random(5, 52455, 1, 29),
     lambda: synth.n0_random_dense(52455, 9, decay=1e-4)),
    ("M1-1536-L393216", 5, 65553, lambda: synth.kernel_random(5, 65553, 1, 30),
     lambda: synth.n0_random_dense(65553, 10, decay=1e-4)),
]
_REF = {}


def _case(label):
    c = next(c for c in CASES if c[0] == label)
    if label not in _REF:
        _, D, N, kf, nf = c
        k, n = kf(), nf()
        _REF[label] = (D, N, k, n, oracle.total_rhs(*oracle.rhs_fft(D, N, k, n)))
    return _REF[label]


@pytest.mark.parametrize("prec", ["fp64", "fp32c", "fp32"])
@pytest.mark.parametrize("label", [c[0] for c in CASES])
def test_mixed_rhs_vs_oracle(label, prec):
    D, N, k, n, ref = _case(label)
    tab = agg.plan_tables(D, N, k, prec, mixed=True)
    L, M1 = int(tab[0]), int(tab[1])
    assert L & (L - 1) != 0, "the case must take a mixed length"
    if prec != "fp32":   # binary32 rows are half as wide: the split may differ
        assert f"M1-{M1}-" in label and f"L{L}" in label
    say(f"[mixed rhs] {label} D={D} N={N} L={L} M1={M1} M2={int(tab[2])} {prec}")
    e = rel(gpu_rhs(D, N, k, n, prec), ref)
    say(f"  err {e:.3e}")
    assert e <= RHS_TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
@pytest.mark.parametrize("label,batch", [("M1-96-L6144", 128), ("M1-160-L20480", 64), ("M1-320-L81920", 16),
                                         ("M1-768-L196608", 8)])
def test_mixed_saturating_batch_members_equal_single(label, batch, prec):
    """A batch large enough for the saturating (lean) variants: members of equal
    state bitwise equal, and within the parity tolerance of the oracle and of the
    one-state launch (which narrows its column group, so its binary64 partial dot
    products are grouped differently)."""
    D, N, k, n, ref = _case(label)
    nb = np.tile(n, batch)
    say(f"[mixed batch] {label} B={batch} {prec}")
    fb = gpu_rhs(D, N, k, nb, prec, batch=batch)
    f1 = gpu_rhs(D, N, k, n, prec)
    for b in (batch // 2, batch - 1):
        assert np.array_equal(fb[b], fb[0]), f"member {b} differs from member 0"
    e, e1 = rel(fb[batch - 1], ref), rel(fb[0], f1)
    say(f"  err {e:.3e}, vs one state {e1:.3e}")
    assert e <= RHS_TOL[prec] and e1 <= RHS_TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_mixed_and_power_of_two_agree(prec):
    """The same right-hand side through both lengths (different transforms,
    equal sums up to rounding)."""
    D, N, k, n, ref = _case("M1-384-L98304")
    a = gpu_rhs(D, N, k, n, prec, mixed=True)
    b = gpu_rhs(D, N, k, n, prec, mixed=False)
    assert rel(a, b) <= 2 * RHS_TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_mixed_c2_solve_vs_oracle_heun(prec):
    """20 Heun steps of the C2 kernel at L = 12288 against the oracle's trajectory."""
    D, N = 3, 4096
    k = synth.kernel_brownian_sum(D, N)
    n0 = synth.n0_exponential(N)
    h, steps = 1e-3, 20
    plan = agg.Plan(D, N, k, prec, mixed=True)
    n = torch.tensor(n0, dtype=torch.float64, device=DEV)
    st = plan.solve(n, h, steps * h)
    assert st.steps == steps
    torch.cuda.synchronize()
    got = n.cpu().numpy()
    plan.close()
    rhs = lambda v: oracle.total_rhs(*oracle.rhs_fft(D, N, k, v))
    ref = oracle.heun_solve(rhs, n0, h, steps * h)
    e = rel(got, ref)
    say(f"[mixed C2 solve] {prec}: err {e:.3e}")
    assert e <= 1e-10


def test_mixed_served_equals_alone_and_oracle():
    """Requests submitted with the mixed option (one 3 2^a and one 5 2^a length,
    one power-of-two request beside them) run concurrently; each result equals
    the request served alone and the oracle's Heun trajectory."""
    reqs = [
        dict(D=3, N=4096, kernel=synth.kernel_brownian_sum(3, 4096), n0=synth.n0_exponential(4096),
             dt=1e-3, t_end=8e-3),
        dict(D=2, N=10240, kernel=synth.kernel_ballistic(2, 10240, 0.3), n0=synth.n0_uniform_head(10240, 7, 16),
             dt=1e-3, t_end=6e-3),
        dict(D=2, N=2048, kernel=synth.kernel_ballistic(2, 2048, 0.5), n0=synth.n0_uniform_head(2048, 8, 16),
             dt=1e-3, t_end=5e-3),
    ]

    def run(rs):
        eng = agg.Engine(0)
        ts = [eng.submit(r["D"], r["N"], r["kernel"], r["n0"], r["dt"], r["t_end"], "fp32c", mixed=True)
              for r in rs]
        out = {}
        t0 = time.time()
        while len(out) < len(ts):
            for t, r in zip(ts, rs):
                if t not in out:
                    rc, o, st = eng.poll(t, r["N"])
                    if rc != agg.AGG_PENDING:
                        assert rc == agg.AGG_OK
                        out[t] = o
            assert time.time() - t0 < 120.0, "engine did not finish"
            time.sleep(0.001)
        eng.close()
        return [out[t] for t in ts]

    assert [int(agg.plan_tables(r["D"], r["N"], r["kernel"], "fp32c", mixed=True)[0]) for r in reqs] == \
        [12288, 20480, 4096]
    say("[mixed serving] 3 requests together, then each alone")
    together = run(reqs)
    for r, got in zip(reqs, together):
        alone = run([r])[0]
        assert np.array_equal(got, alone)
        rhs = lambda v, r=r: oracle.total_rhs(*oracle.rhs_fft(r["D"], r["N"], r["kernel"], v))
        ref = oracle.heun_solve(rhs, r["n0"], r["dt"], r["t_end"])
        e = rel(got, ref)
        say(f"  D={r['D']} N={r['N']}: err {e:.3e}")
        assert e <= 1e-10


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_mixed_d5_n2e20_batch(prec):
    """D = 5, N = 2^20, additive kernel, 64 states (initial data uniform on
    [1,16], seeds 0..63) at L = 5 2^20 (M1 = 1280, M2 = 2048): sampled members'
    right-hand sides and one Heun step against the oracle at full N."""
    c = synth.config("C5a")
    D, N, B, k = c["D"], c["N"], c["n0"].shape[0], c["kernel"]
    tab = agg.plan_tables(D, N, k, prec, mixed=True)
    assert (int(tab[0]), int(tab[1]), int(tab[2])) == (5 << 20, 1280, 2048)
    say(f"[mixed D5] N={N} B={B} L=5*2^20 {prec}")
    plan = agg.Plan(D, N, k, prec, batch=B, mixed=True)
    n = torch.tensor(c["n0"].reshape(-1), device=DEV)
    f = plan.rhs(n)
    torch.cuda.synchronize()
    f = f.cpu().numpy().reshape(B, N)
    for b in (0, 29, 63):
        ref = oracle.total_rhs(*oracle.rhs_conv(D, N, k, c["n0"][b]))
        e = rel(f[b], ref)
        say(f"  rhs member {b}: err {e:.3e}")
        assert e <= RHS_TOL[prec]
    h = c["dt"]
    plan.rk2_step(n, h)
    torch.cuda.synchronize()
    nb = n.cpu().numpy().reshape(B, N)
    plan.close()
    for b in (0, 63):
        rhs = lambda v: oracle.total_rhs(*oracle.rhs_conv(D, N, k, v))
        ref = oracle.heun_solve(rhs, c["n0"][b], h, h)
        e = rel(nb[b], ref)
        say(f"  heun member {b}: err {e:.3e}")
        assert e <= RHS_TOL[prec]


def test_mixed_ternary_n2e19():
    """The pure ternary D = 3, N = 2^19 generalized Brownian kernel (exponents
    1/3, -1/3, 0; one rank-one term per permutation, six in all) at
    L = 3 2^19 (M1 = 1536, M2 = 512): the right-hand side against the oracle and
    against the power-of-two plan, binary64."""
    D, N = 3, 1 << 19
    k = {3: synth.kernel_generalized_brownian(N, [1.0 / 3.0, -1.0 / 3.0, 0.0])}
    tab = agg.plan_tables(D, N, k, "fp64", mixed=True)
    assert (int(tab[0]), int(tab[1]), int(tab[2])) == (3 << 19, 1536, 512)
    n = synth.n0_uniform_head(N, 3, 16)
    say("[mixed ternary] D=3 N=2^19 L=3*2^19 fp64")
    f = gpu_rhs(D, N, k, n, "fp64")
    ref = oracle.total_rhs(*oracle.rhs_conv(D, N, k, n))
    e = rel(f, ref)
    say(f"  err {e:.3e}")
    assert e <= RHS_TOL["fp64"]
    f2 = gpu_rhs(D, N, k, n, "fp64", mixed=False)
    assert rel(f, f2) <= 2 * RHS_TOL["fp64"]
