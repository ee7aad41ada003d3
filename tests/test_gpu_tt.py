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
