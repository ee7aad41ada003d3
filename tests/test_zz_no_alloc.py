"""agg_rhs_noalloc through the C ABI: the allocation-free right-hand side gives
what agg_rhs gives on the same plan and states (bit for bit: the same launches
over a static workspace instead of the plan's), on two calls in a row, the
second with a smaller input, and refuses a batch beyond its static array."""
import ctypes
import sys

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
agg = pytest.importorskip("paper_1905_09071_amd")
from paper_1905_09071_amd import _lib  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def both(plan, n, batch):
    """(agg_rhs of the plan on the batch, agg_rhs_noalloc on its first `batch` states)"""
    L = _lib.lib()
    ref = torch.empty_like(n)
    assert L.agg_rhs(plan._h, ptr(n), ptr(ref)) == 0, L.agg_last_error()
    out = torch.full((batch * plan.N,), float("nan"), dtype=torch.float64, device="cuda:0")
    rc = L.agg_rhs_noalloc(plan._h, ptr(n), ptr(out), batch)
    assert rc == 0, L.agg_last_error()
    torch.cuda.synchronize()
    return ref.cpu().numpy()[:batch * plan.N], out.cpu().numpy()


def test_noalloc_equals_agg_rhs_twice_then_smaller():
    c = synth.config("C3")
    D, N = c["D"], c["N"]
    # first call: the D=4, N=65536 workload, two states (8.4 MB of workspace each)
    plan = agg.Plan(D, N, c["kernel"], "fp64", batch=2)
    n = torch.tensor(np.concatenate([c["n0"], synth.n0_random_dense(N, 5, decay=1e-3)]),
                     dtype=torch.float64, device="cuda:0")
    say(f"[noalloc] call 1: D={D} N={N} fp64 batch 2")
    ref, out = both(plan, n, 2)
    assert np.array_equal(ref, out), float(np.max(np.abs(ref - out)))
    plan.close()
    # second call: a smaller input (D=3, N=4096, float-float spectra, one state),
    # over the workspace the first call left behind
    c2 = synth.config("C2")
    plan = agg.Plan(c2["D"], c2["N"], c2["kernel"], "fp32c", batch=1)
    n = torch.tensor(synth.n0_random_dense(c2["N"], 9, decay=1e-2), dtype=torch.float64, device="cuda:0")
    say(f"[noalloc] call 2: D={c2['D']} N={c2['N']} fp32c batch 1")
    ref, out = both(plan, n, 1)
    assert np.array_equal(ref, out), float(np.max(np.abs(ref - out)))
    assert np.max(np.abs(ref)) > 0
    plan.close()


def test_noalloc_smaller_batch_of_a_plan():
    # first `batch` states of a plan of four: equal to agg_rhs of a plan of that
    # batch (the launch geometry depends on the batch, so that is the same launch)
    c = synth.config("C2")
    D, N = c["D"], c["N"]
    states = np.concatenate([synth.n0_random_dense(N, s, decay=1e-2) for s in range(4)])
    n = torch.tensor(states, dtype=torch.float64, device="cuda:0")
    big = agg.Plan(D, N, c["kernel"], "fp64", batch=4)
    for b in (4, 2):
        small = agg.Plan(D, N, c["kernel"], "fp64", batch=b)
        nb = n[:b * N].clone()
        ref, _ = both(small, nb, b)
        out = torch.empty(b * N, dtype=torch.float64, device="cuda:0")
        assert _lib.lib().agg_rhs_noalloc(big._h, ptr(n), ptr(out), b) == 0
        torch.cuda.synchronize()
        say(f"[noalloc] D={D} N={N} fp64: plan batch 4, call batch {b}")
        assert np.array_equal(ref, out.cpu().numpy())
        small.close()
    big.close()


def test_noalloc_refuses_beyond_its_array():
    c = synth.config("C3")
    L = _lib.lib()
    plan = agg.Plan(c["D"], c["N"], c["kernel"], "fp64", batch=8)
    n = torch.zeros(8 * c["N"], dtype=torch.float64, device="cuda:0")
    out = torch.zeros_like(n)
    assert L.agg_rhs_noalloc(plan._h, ptr(n), ptr(out), 8) == agg.AGG_EUNSUPPORTED
    assert b"static scratch" in L.agg_last_error()
    assert L.agg_rhs_noalloc(plan._h, ptr(n), ptr(out), 9) == agg.AGG_EINVAL
    assert L.agg_rhs_noalloc(plan._h, ptr(n), ptr(out), 0) == agg.AGG_EINVAL
    assert L.agg_rhs_noalloc(None, ptr(n), ptr(out), 1) == agg.AGG_EINVAL
    plan.close()


def test_noalloc_tensor_train_plan():
    """A kernel in tensor-train form (random dense cores of ranks (1,3,1),
    (1,4,4,1), (1,6,6,6,1) at N = 4096: 114 core columns, so the column passes
    split each group's columns over several workgroups, and the chunked row
    pass's per-bin chains) through agg_rhs_noalloc: two states, then one, each
    bit for bit agg_rhs."""
    rng = np.random.default_rng(95)
    N = 4096
    cores = lambda ranks: [rng.uniform(0.1, 1.0, size=(ranks[m], N, ranks[m + 1])) for m in range(len(ranks) - 1)]
    tt = {2: cores([1, 3, 1]), 3: cores([1, 4, 4, 1]), 4: cores([1, 6, 6, 6, 1])}
    plan = agg.Plan(4, N, prec="fp64", tt=tt, batch=2)
    n = torch.tensor(np.concatenate([synth.n0_random_dense(N, 96, decay=2e-3), synth.n0_random_dense(N, 97)]),
                     dtype=torch.float64, device="cuda:0")
    for batch in (2, 1):
        say(f"[noalloc] tensor-train D=4 N={N} fp64 batch {batch}")
        ref, out = both(plan, n, batch)
        assert np.array_equal(ref, out), float(np.max(np.abs(ref - out)))
        assert np.max(np.abs(ref)) > 0
    plan.close()
