"""GPU parity for kernels given in tensor-train form (Sec. 2): the generalized
Brownian kernels built from the TT cores of the proof of Sec. 2's rank theorem,
expanded by the library into rank-one paths (which the planner merges), against
the oracle evaluating the same kernel from its independently built CP form
(one rank-one term per permutation).  Cases: D = 4 with orders 2..4 at
N = 4096 (dense state), and the pure ternary D = 3 kernel [1/3, -1/3, 0] at
N = 2^19 (the shape of the paper's Table 1) on a state with short support,
RHS and one Heun step."""
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
agg = pytest.importorskip("paper_1905_09071_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = {"fp64": 1e-12, "fp32c": 1e-10, "fp32": 1e-5}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("prec", ["fp64", "fp32c", "fp32"])
def test_tt_brownian_orders_2_to_4(prec):
    D, N = 4, 4096
    mus = [0.3, -0.3, 0.1, 0.0]
    k_tt = {d: agg.tt_expand(N, synth.brownian_tt_cores(N, mus[:d])) for d in range(2, D + 1)}
    k_cp = {d: synth.kernel_generalized_brownian(N, mus[:d]) for d in range(2, D + 1)}
    n = synth.n0_random_dense(N, 61, decay=1e-3)
    plan = agg.Plan(D, N, k_tt, prec)
    f = plan.rhs(torch.tensor(n, device=DEV))
    torch.cuda.synchronize()
    f = f.cpu().numpy()
    plan.close()
    ref = oracle.total_rhs(*oracle.rhs_fft(D, N, k_cp, n))
    e = rel(f, ref)
    say(f"[tt brownian] D={D} N={N} {prec}: rhs err {e:.3e}")
    assert e <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_tt_pure_ternary_table1_shape(prec):
    D, N = 3, 1 << 19
    mus = [1 / 3, -1 / 3, 0.0]
    k_tt = {3: agg.tt_expand(N, synth.brownian_tt_cores(N, mus))}
    k_cp = {3: synth.kernel_generalized_brownian(N, mus)}
    n0 = synth.n0_uniform_head(N, 3, 16)
    say(f"[tt ternary] D={D} N={N} {prec}: paths {k_tt[3].shape[1]}")
    plan = agg.Plan(D, N, k_tt, prec)
    n = torch.tensor(n0, device=DEV)
    f = plan.rhs(n)
    torch.cuda.synchronize()
    f = f.cpu().numpy()

    def rhs_short(v, kmax):
        nz = np.nonzero(v)[0]
        assert (nz[-1] + 1) * D <= kmax
        p, q = oracle.rhs_conv(D, N, k_cp, v, kmax=kmax)
        p[:, kmax:] = 0.0
        return oracle.total_rhs(p, q)

    e = rel(f, rhs_short(n0, 64))
    say(f"  rhs err {e:.3e}")
    assert e <= TOL[prec]
    h = 1e-3
    plan.rk2_step(n, h)
    torch.cuda.synchronize()
    ref = oracle.heun_solve(lambda v: rhs_short(v, 200), n0, h, h)
    e = rel(n.cpu().numpy(), ref)
    say(f"  heun err {e:.3e}")
    assert e <= TOL[prec]
    plan.close()


# ---- the tensor-train chain (agg_plan_create_tt): one transform per core
# column, a product of the cores' matrices of spectra per frequency bin -------

def _cores(rng, N, ranks):
    return [rng.uniform(0.1, 1.0, size=(ranks[m], N, ranks[m + 1])) for m in range(len(ranks) - 1)]


def _tt_rhs(D, N, tt, n, prec, batch=1, step=None):
    plan = agg.Plan(D, N, prec=prec, tt=tt, batch=batch)
    nt = torch.tensor(np.tile(n, batch), device=DEV)
    f = plan.rhs(nt)
    out = [f.cpu().numpy().reshape(batch, N)]
    if step is not None:
        plan.rk2_step(nt, step)
        out.append(nt.cpu().numpy().reshape(batch, N))
    torch.cuda.synchronize()
    plan.close()
    return out


@pytest.mark.parametrize("prec", ["fp64", "fp32c", "fp32"])
@pytest.mark.parametrize("N", [9, 13])
def test_tt_chain_tiny_vs_literal_sums(prec, N):
    """Random dense cores of orders 2..4 (ranks (1,2,1), (1,3,2,1), (1,2,3,2,1)),
    one core column all zero and one shared between orders, against the
    literal sums over the kernel tensors rebuilt from the cores."""
    rng = np.random.default_rng(70 + N)
    D = 4
    tt = {2: _cores(rng, N, [1, 2, 1]), 3: _cores(rng, N, [1, 3, 2, 1]), 4: _cores(rng, N, [1, 2, 3, 2, 1])}
    tt[3][1][2, :, 0] = 0.0
    tt[4][3][1, :, 0] = tt[2][1][0, :, 0]
    n = rng.uniform(0.0, 1.0, size=N)
    f, = _tt_rhs(D, N, tt, n, prec)
    ref = oracle.total_rhs(*[np.atleast_2d(x) for x in oracle.rhs_dense(D, N, {d: oracle.tt_full(c) for d, c in tt.items()}, n)])
    e = rel(f[0], ref)
    say(f"[tt chain tiny] N={N} {prec}: rhs err {e:.3e}")
    assert e <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32c", "fp32"])
def test_tt_chain_random_dense_ranks_6(prec):
    """D = 4, random dense cores with ranks (1,3,1), (1,4,4,1), (1,6,6,6,1) at
    N = 4096 (84 + 16 + 3 distinct core columns), dense state, two states in a
    batch: RHS and one Heun step against the oracle's CP-FFT evaluation of the
    kernel written as its rank paths (216 + 16 + 3 rank-one terms)."""
    rng = np.random.default_rng(80)
    D, N = 4, 4096
    tt = {2: _cores(rng, N, [1, 3, 1]), 3: _cores(rng, N, [1, 4, 4, 1]), 4: _cores(rng, N, [1, 6, 6, 6, 1])}
    cp = {d: oracle.tt_paths(c) for d, c in tt.items()}
    n = synth.n0_random_dense(N, 81, decay=2e-3)
    h = 1e-5
    f, after = _tt_rhs(D, N, tt, n, prec, batch=2, step=h)
    rhs = lambda v: oracle.total_rhs(*oracle.rhs_fft(D, N, cp, v))
    e = rel(f[1], rhs(n))
    say(f"[tt chain ranks 6] {prec}: rhs err {e:.3e}")
    assert e <= TOL[prec]
    assert np.array_equal(f[0], f[1])
    e = rel(after[0], oracle.heun_solve(rhs, n, h, h))
    say(f"  heun err {e:.3e}")
    assert e <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_tt_chain_brownian_equals_the_path_expansion(prec):
    """The generalized Brownian cores of Sec. 2 (zero columns and ranks C(D, m))
    through the chain agree with the same cores through the rank-path
    expansion (both library paths), and with the oracle, at N = 65536."""
    D, N = 4, 65536
    mus = [0.3, -0.3, 0.1, 0.0]
    tt = {d: synth.brownian_tt_cores(N, mus[:d]) for d in range(2, D + 1)}
    n = synth.n0_random_dense(N, 62, decay=1e-4)
    f, = _tt_rhs(D, N, tt, n, prec)
    plan = agg.Plan(D, N, {d: agg.tt_expand(N, c) for d, c in tt.items()}, prec)
    g = plan.rhs(torch.tensor(n, device=DEV)).cpu().numpy()
    plan.close()
    ref = oracle.total_rhs(*oracle.rhs_fft(D, N, {d: synth.kernel_generalized_brownian(N, mus[:d])
                                                  for d in range(2, D + 1)}, n))
    e1, e2 = rel(f[0], ref), rel(f[0], g)
    say(f"[tt chain brownian] {prec}: vs oracle {e1:.3e}, vs path expansion {e2:.3e}")
    assert e1 <= TOL[prec] and e2 <= TOL[prec]


_REF = {}


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_tt_chain_across_chunks(prec):
    """The ranks-6 kernel set at N = 65536: the row pass holds 69 columns at a
    time, so the 114 core columns come in three chunks and the order-4 chain
    carries its per-bin vector across them.  Against the oracle's CP-FFT
    evaluation of the rank paths (computed once for both precisions)."""
    rng = np.random.default_rng(82)
    D, N = 4, 65536
    tt = {2: _cores(rng, N, [1, 3, 1]), 3: _cores(rng, N, [1, 4, 4, 1]), 4: _cores(rng, N, [1, 6, 6, 6, 1])}
    ref_tables = oracle.plan_tables_tt(D, N, tt, prec)
    assert len(ref_tables["chunks"]) == 3 and ref_tables["M2"] == 64
    n = synth.n0_random_dense(N, 83, decay=1e-4)
    f, = _tt_rhs(D, N, tt, n, prec)
    if "ref" not in _REF:
        cp = {d: oracle.tt_paths(c) for d, c in tt.items()}
        _REF["ref"] = oracle.total_rhs(*oracle.rhs_fft(D, N, cp, n))
    e = rel(f[0], _REF["ref"])
    say(f"[tt chain chunks] {prec}: rhs err {e:.3e}")
    assert e <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32c", "fp32"])
def test_split_column_pass_is_exact(prec):
    """A launch with fewer column groups than CUs splits each group's 114
    distinct core columns over several workgroups (N = 4096: 16 groups of one
    column at one state, 16 shares; binary32 spectra, half the bytes per row,
    give rows of 32 values: 32 groups, 8 shares); a batch of 16 states (8 in
    binary32) fills the CUs with unsplit groups of the same width (a larger
    batch would widen the groups, which regroups the binary64 partial dot
    products).  Each batch member's RHS, and its state after a 5-step solve
    (stage 2 reading stage 1's kept state), equals the single-state plan's
    result bit for bit; member 0 also against the oracle."""
    rng = np.random.default_rng(84)
    D, N = 4, 4096
    B = 8 if prec == "fp32" else 16
    tt = {2: _cores(rng, N, [1, 3, 1]), 3: _cores(rng, N, [1, 4, 4, 1]), 4: _cores(rng, N, [1, 6, 6, 6, 1])}
    ref_tables = oracle.plan_tables_tt(D, N, tt, prec)
    assert ref_tables["M2"] == (32 if prec == "fp32" else 16) and ref_tables["u"] == 114
    states = np.stack([synth.n0_random_dense(N, 85 + b, decay=2e-3) for b in range(B)])
    h = 1e-5
    batch = agg.Plan(D, N, prec=prec, tt=tt, batch=B)
    nb = torch.tensor(states.ravel(), device=DEV)
    fb = batch.rhs(nb).cpu().numpy().reshape(B, N)
    batch.solve(nb, h, 5 * h, stats=False)
    sb = nb.cpu().numpy().reshape(B, N)
    batch.close()
    one = agg.Plan(D, N, prec=prec, tt=tt)
    for b in (0, B // 2 - 1, B - 1):
        n1 = torch.tensor(states[b], device=DEV)
        f1 = one.rhs(n1).cpu().numpy()
        one.solve(n1, h, 5 * h, stats=False)
        s1 = n1.cpu().numpy()
        say(f"[split column pass] {prec} member {b}: rhs equal {np.array_equal(f1, fb[b])}, "
            f"solve equal {np.array_equal(s1, sb[b])}")
        assert np.array_equal(f1, fb[b]) and np.array_equal(s1, sb[b])
        if b == 0:
            cp = {d: oracle.tt_paths(c) for d, c in tt.items()}
            e = rel(f1, oracle.total_rhs(*oracle.rhs_fft(D, N, cp, states[0])))
            say(f"  rhs err vs oracle {e:.3e}")
            assert e <= TOL[prec]
    one.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_many_term_combine_shared_by_lanes(prec):
    """The ranks-6 kernel written as its 235 rank paths (114 distinct columns)
    at N = 4096, rows of 16 values: each bin pair's gain terms are shared by 8
    lanes of a wavefront.  One state (the full row-pass variant) and two states
    (the lean variant) give bit for bit the same RHS and Heun step, which agree
    with the oracle."""
    rng = np.random.default_rng(80)
    D, N = 4, 4096
    tt = {2: _cores(rng, N, [1, 3, 1]), 3: _cores(rng, N, [1, 4, 4, 1]), 4: _cores(rng, N, [1, 6, 6, 6, 1])}
    paths = {d: agg.tt_expand(N, c) for d, c in tt.items()}
    assert agg.plan_tables(D, N, paths, prec)[2] == 16
    n = synth.n0_random_dense(N, 86, decay=2e-3)
    h = 1e-5
    out = {}
    for B in (1, 2):
        plan = agg.Plan(D, N, paths, prec, batch=B)
        nt = torch.tensor(np.tile(n, B), device=DEV)
        f = plan.rhs(nt).cpu().numpy().reshape(B, N)
        plan.rk2_step(nt, h)
        out[B] = (f, nt.cpu().numpy().reshape(B, N))
        plan.close()
    assert np.array_equal(out[1][0][0], out[2][0][1]) and np.array_equal(out[1][1][0], out[2][1][1])
    cp = {d: oracle.tt_paths(c) for d, c in tt.items()}
    rhs = lambda v: oracle.total_rhs(*oracle.rhs_fft(D, N, cp, v))
    e1 = rel(out[1][0][0], rhs(n))
    e2 = rel(out[1][1][0], oracle.heun_solve(rhs, n, h, h))
    say(f"[many-term combine] {prec}: rhs err {e1:.3e}, heun err {e2:.3e}")
    assert e1 <= TOL[prec] and e2 <= TOL[prec]


@pytest.mark.parametrize("N,prec", [(4096, "fp64"), (4096, "fp32c"), (4096, "fp32"),
                                    (65536, "fp64"), (65536, "fp32c")])
def test_tt_chain_mixed_radix(N, prec):
    """Random dense D = 3 cores (ranks (1,3,1), (1,4,4,1); 30 distinct columns)
    with the mixed-radix option: L = 3 2^12 (columns of 96 values) at N = 4096
    and L = 3 2^16 (columns of 1536 values, rows of 64) at N = 65536, instead of
    2^14 and 2^18.  RHS and one Heun step against the oracle's CP-FFT
    evaluation of the rank paths."""
    rng = np.random.default_rng(87)
    D = 3
    tt = {2: _cores(rng, N, [1, 3, 1]), 3: _cores(rng, N, [1, 4, 4, 1])}
    t = oracle.plan_tables_tt(D, N, tt, prec, mixed=True)
    assert t["L"] == 3 * N and t["M1"] == {4096: 96, 65536: 1536}[N]
    assert agg.plan_tables_tt(D, N, tt, prec, mixed=True).tolist() == t["flat"].tolist()
    n = synth.n0_random_dense(N, 88, decay=2e-3 if N == 4096 else 1e-4)
    h = 1e-5
    plan = agg.Plan(D, N, prec=prec, tt=tt, mixed=True)
    nt = torch.tensor(n, device=DEV)
    f = plan.rhs(nt).cpu().numpy()
    plan.rk2_step(nt, h)
    after = nt.cpu().numpy()
    plan.close()
    cp = {d: oracle.tt_paths(c) for d, c in tt.items()}
    rhs = lambda v: oracle.total_rhs(*oracle.rhs_fft(D, N, cp, v))
    e1 = rel(f, rhs(n))
    e2 = rel(after, oracle.heun_solve(rhs, n, h, h))
    say(f"[tt chain mixed] N={N} L={t['L']} M1={t['M1']} M2={t['M2']} {prec}: rhs err {e1:.3e}, heun err {e2:.3e}")
    assert e1 <= TOL[prec] and e2 <= TOL[prec]


def test_tt_chain_refusals():
    rng = np.random.default_rng(5)
    N = 64
    with pytest.raises(agg.AggError) as e:   # rank above 8
        agg.Plan(3, N, prec="fp64", tt={3: _cores(rng, N, [1, 9, 2, 1])})
    assert e.value.status == agg.AGG_EINVAL
    with pytest.raises(agg.AggError) as e:   # rows longer than 512 values
        agg.Plan(2, 1 << 22, prec="fp64", tt={2: [np.ones((1, 1 << 22, 1)), np.ones((1, 1 << 22, 1))]})
    assert e.value.status == agg.AGG_EUNSUPPORTED


def _ballistic(a):
    s = a.astype(np.float64)
    return np.sum(s ** (1 / 3), axis=1) ** 2 * np.sqrt(np.sum(1.0 / s, axis=1))


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_tt_cross_kernel_through_the_chain(prec):
    """A non-separable kernel with no CP or TT construction (the ballistic
    kernel, cube roots squared times the root of the summed inverse sizes, at
    orders 2 and 3) compressed by agg_tt_cross to ranks <= 8, then evaluated
    through the chain: parity with the oracle's evaluation of the same cores
    at N = 4096, and at N = 20 agreement with the literal sums over the exact
    kernel to the compression's error."""
    D = 3
    for N in (20, 4096):
        tt = {d: agg.tt_cross(d, N, _ballistic, tol=1e-12, rmax=8, seed=d)[0] for d in (2, 3)}
        n = synth.n0_random_dense(N, 90, decay=1e-3 if N > 100 else 0.1)
        f, = _tt_rhs(D, N, tt, n, prec)
        if N == 4096:
            ref = oracle.total_rhs(*oracle.rhs_fft(D, N, {d: oracle.tt_paths(c) for d, c in tt.items()}, n))
            e = rel(f[0], ref)
            say(f"[tt cross chain] N={N} {prec}: rhs err vs the cores' oracle evaluation {e:.3e}")
            assert e <= TOL[prec]
        else:
            grid = lambda d: np.array(list(__import__("itertools").product(range(1, N + 1), repeat=d)))
            exact = {d: _ballistic(grid(d)).reshape((N,) * d) for d in (2, 3)}
            ref = oracle.total_rhs(*[np.atleast_2d(x) for x in oracle.rhs_dense(D, N, exact, n)])
            e = rel(f[0], ref)
            say(f"[tt cross chain] N={N} {prec}: rhs err vs the exact kernel {e:.3e}")
            assert e <= 1e-5
