"""Python binding of libagg (include/agg.h): argument marshalling only.

Every step of the right-hand side and of the time stepping runs in the HIP
kernels of libagg.so; torch provides device memory (float64 tensors) and
streams.  Kernel factors are numpy arrays of shape (d, R_d, N) with
U[m-1, r, i-1] = U^(d)_m(i, r); mode d carries k in the loss term.
"""
from __future__ import annotations

import ctypes

import numpy as np

from ._lib import (AGG_EINVAL, AGG_ENOMEM, AGG_ENONFINITE, AGG_ENOTFOUND, AGG_EUNSUPPORTED,  # noqa: F401
                   AGG_OK, AGG_PENDING, AGG_MAX_D, PREC, AggError, agg_engine_config,
                   agg_request_stats, agg_solve_stats, agg_term, agg_tt_term, check, lib, KERNEL_FN)

__all__ = ["Plan", "Engine", "plan_tables", "plan_tables_tt", "twiddles", "expsum_fit", "tt_expand", "AggError",
           "PREC", "make_terms", "make_tt_terms", "tt_cross"]


def make_terms(D: int, N: int, kernel: dict):
    """Build the agg_term array; returns (array, count, keepalive list).  The
    factors of order d are an array of shape (d, R, N), or a list of d arrays
    of shape (R, N) (modes may then share one array), or a dict with those
    factors under "U" and R per-rank weights under "weight"."""
    items = sorted(kernel.items())
    arr = (agg_term * max(len(items), 1))()
    keep = []
    for t, (d, U) in enumerate(items):
        weight = None
        if isinstance(U, dict):
            weight, U = U.get("weight"), U["U"]
        modes = list(U) if isinstance(U, (list, tuple)) else None
        if modes is None:
            U = np.asarray(U, dtype=np.float64)
            if U.ndim != 3 or U.shape[0] != d or U.shape[2] != N:
                raise ValueError(f"factors of order {d} must have shape (d, R, N) = ({d}, R, {N})")
            modes = [U[m] for m in range(d)]
        if len(modes) != d or any(np.ndim(x) != 2 or np.shape(x)[1] != N or np.shape(x)[0] != np.shape(modes[0])[0]
                                  for x in modes):
            raise ValueError(f"factors of order {d} must be d arrays of shape (R, {N})")
        arr[t].d = d
        arr[t].rank = np.shape(modes[0])[0]
        for m in range(d):
            col = np.ascontiguousarray(modes[m], dtype=np.float64)
            keep.append(col)
            arr[t].U[m] = col.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        if weight is not None:
            wv = np.ascontiguousarray(weight, dtype=np.float64)
            if wv.shape != (arr[t].rank,):
                raise ValueError(f"order {d}: one weight per rank expected")
            keep.append(wv)
            arr[t].weight = wv.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return arr, len(items), keep


def make_tt_terms(D: int, N: int, tt: dict):
    """Build the agg_tt_term array from {d: [core_1, ..., core_d]}, core m an
    array of shape (r_{m-1}, N, r_m) with H[a, i-1, b] = H^(m)_{a, i, b};
    returns (array, count, keepalive list)."""
    items = sorted(tt.items())
    arr = (agg_tt_term * max(len(items), 1))()
    keep = []
    for t, (d, cores) in enumerate(items):
        if len(cores) != d:
            raise ValueError(f"order {d} needs {d} cores")
        ranks = [int(np.shape(cores[0])[0])] + [int(np.shape(c)[2]) for c in cores]
        for m in range(d):
            if np.ndim(cores[m]) != 3 or np.shape(cores[m])[1] != N or np.shape(cores[m])[0] != ranks[m]:
                raise ValueError(f"order {d}, core {m + 1}: shape (r_{m}, N, r_{m + 1}) expected")
        arr[t].d = d
        for m, r in enumerate(ranks):
            arr[t].ranks[m] = r
        for m in range(d):
            # (r_{m-1}, N, r_m) -> r_{m-1} x r_m columns of N values
            col = np.ascontiguousarray(np.transpose(np.asarray(cores[m], dtype=np.float64), (0, 2, 1)))
            keep.append(col)
            arr[t].H[m] = col.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return arr, len(items), keep


def plan_tables_tt(D: int, N: int, tt: dict, prec: str = "fp64", mixed: bool = False) -> np.ndarray:
    """The planner's integer tables of a tensor-train kernel set (host only)."""
    terms, nt, keep = make_tt_terms(D, N, tt)
    code = PREC[prec] | (AGG_MIXED_RADIX if mixed else 0)
    ln = ctypes.c_int64(0)
    lib().agg_plan_tables_tt(D, N, terms, nt, code, None, 0, ctypes.byref(ln))
    out = np.zeros(max(ln.value, 1), dtype=np.int64)
    check(lib().agg_plan_tables_tt(D, N, terms, nt, code,
                                   out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), out.size, ctypes.byref(ln)))
    del keep
    return out[:ln.value]


AGG_PLAIN = 0x100
AGG_MIXED_RADIX = 0x200


def _plan_code(prec: str, plain: bool, mixed: bool) -> int:
    return PREC[prec] | (AGG_PLAIN if plain else 0) | (AGG_MIXED_RADIX if mixed else 0)


def plan_tables(D: int, N: int, kernel: dict, prec: str = "fp64", plain: bool = False,
                mixed: bool = False) -> np.ndarray:
    """The planner's integer tables (host only, no device touched)."""
    terms, nt, keep = make_terms(D, N, kernel)
    ln = ctypes.c_int64(0)
    code = _plan_code(prec, plain, mixed)
    lib().agg_plan_tables(D, N, terms, nt, code, None, 0, ctypes.byref(ln))
    out = np.zeros(max(ln.value, 1), dtype=np.int64)
    check(lib().agg_plan_tables(D, N, terms, nt, code,
                                out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), out.size, ctypes.byref(ln)))
    del keep
    return out[:ln.value]


def expsum_fit(f: np.ndarray, smin: int, R: int, relative: bool = False):
    """Exponential-sum fit of f on the integers smin .. smin+len(f)-1 (host):
    returns (alpha[R], w[R+1], max_err); max_err is relative to |f| when
    ``relative``."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    alpha = np.zeros(max(R, 1))
    w = np.zeros(R + 1)
    err = ctypes.c_double(0.0)
    dp = ctypes.POINTER(ctypes.c_double)
    check(lib().agg_expsum_fit(f.ctypes.data_as(dp), int(smin), int(smin) + f.size - 1, int(R), int(bool(relative)),
                               alpha.ctypes.data_as(dp), w.ctypes.data_as(dp), ctypes.byref(err)))
    return alpha[:R], w, err.value


def tt_expand(N: int, cores) -> np.ndarray:
    """CP factors (d, P, N) of a tensor-train kernel given by its d cores, each an
    array of shape (r_{m-1}, N, r_m) with H[a, i-1, b] = H^(m)_{a, i, b}."""
    d = len(cores)
    ranks = [int(np.shape(cores[0])[0])] + [int(np.shape(c)[2]) for c in cores]
    for m in range(1, d):
        if np.shape(cores[m])[0] != ranks[m] or np.shape(cores[m])[1] != N:
            raise ValueError(f"core {m + 1} must have shape (r_{m}, N, r_{m + 1}) = ({ranks[m]}, {N}, r)")
    r = (ctypes.c_int32 * (d + 1))(*ranks)
    keep = [np.ascontiguousarray(np.transpose(np.asarray(c, dtype=np.float64), (0, 2, 1))) for c in cores]
    ptrs = (ctypes.POINTER(ctypes.c_double) * d)(*[k.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for k in keep])
    npaths = ctypes.c_int64(0)
    check(lib().agg_tt_expand(d, N, r, ptrs, 0, None, ctypes.byref(npaths)))
    U = np.zeros((d, max(npaths.value, 1), N))
    check(lib().agg_tt_expand(d, N, r, ptrs, npaths.value, U.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                              ctypes.byref(npaths)))
    return U[:, :npaths.value]


def tt_cross(d: int, N: int, f, tol: float = 1e-8, rmax: int = 8, max_sweeps: int = 12, seed: int = 0):
    """TT-cross approximation (host) of the order-d kernel C(i_1..i_d) = f(idx),
    f taking an int64 array of shape (count, d) of sizes (1-based) and
    returning count values.  Returns (cores, err_est): cores[m] of shape
    (r_m, N, r_{m+1}) as agg_plan_create_tt takes them."""
    def cb(idx, count, dd, out, ctx):
        a = np.ctypeslib.as_array(idx, shape=(count * dd,)).reshape(count, dd)
        o = np.ctypeslib.as_array(out, shape=(count,))
        o[:] = np.asarray(f(a), dtype=np.float64)
    fn = KERNEL_FN(cb)
    ranks = (ctypes.c_int32 * (d + 1))()
    cap = d * rmax * rmax * N
    buf = np.zeros(cap)
    ln = ctypes.c_int64(0)
    err = ctypes.c_double(0.0)
    dp = ctypes.POINTER(ctypes.c_double)
    check(lib().agg_tt_cross(d, N, ctypes.cast(fn, ctypes.c_void_p), None, float(tol), int(rmax), int(max_sweeps),
                             int(seed), ranks, buf.ctypes.data_as(dp), cap, ctypes.byref(ln), ctypes.byref(err)))
    r = list(ranks)
    cores, off = [], 0
    for m in range(d):
        size = r[m] * r[m + 1] * N
        # stored as r_{m-1} x r_m columns of N: (a, b, i) -> (a, i, b)
        cores.append(np.ascontiguousarray(buf[off:off + size].reshape(r[m], r[m + 1], N).transpose(0, 2, 1)))
        off += size
    return cores, err.value


def twiddles(P: int) -> np.ndarray:
    out = np.zeros(2 * P)
    check(lib().agg_twiddles(P, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out.reshape(P, 2)


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check_state(t, numel):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise TypeError("state tensors must be float64 CUDA (HIP) tensors")
    if not t.is_contiguous() or t.numel() != numel:
        raise ValueError(f"state tensor must be contiguous with {numel} elements")
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """agg_plan: a kernel set, precision and batch size bound to a stream."""

    def __init__(self, D: int, N: int, kernel: dict = None, prec: str = "fp64", batch: int = 1, stream=None,
                 plain: bool = False, tt: dict = None, mixed: bool = False):
        """plain=True: the term-by-term, unshared, unfused reference evaluation.
        tt={d: cores}: the kernel set in tensor-train form instead of CP factors
        (agg_plan_create_tt).  mixed=True: transform lengths 3 2^a and 5 2^a
        allowed (AGG_MIXED_RADIX), for CP and tensor-train kernel sets."""
        self.D, self.N, self.batch, self.prec, self.plain = D, N, batch, prec, plain
        self._stream = stream
        h = ctypes.c_void_p()
        if tt is not None:
            if kernel is not None or plain:
                raise ValueError("a tensor-train plan takes no CP kernel and no plain option")
            terms, nt, keep = make_tt_terms(D, N, tt)
            check(lib().agg_plan_create_tt(D, N, terms, nt, _plan_code(prec, False, mixed), batch,
                                           _stream_handle(stream), ctypes.byref(h)))
        else:
            terms, nt, keep = make_terms(D, N, kernel)
            code = _plan_code(prec, plain, mixed)
            check(lib().agg_plan_create(D, N, terms, nt, code, batch, _stream_handle(stream),
                                        ctypes.byref(h)))
        del keep
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().agg_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def rhs(self, n, out=None):
        import torch
        if out is None:
            out = torch.empty_like(n)
        check(lib().agg_rhs(self._h, _check_state(n, self.batch * self.N), _check_state(out, self.batch * self.N)))
        return out

    def rhs_noalloc(self, n, out, batch: int = None):
        """agg_rhs_noalloc: f(n) for the first ``batch`` states with the library's
        static workspace (no device allocation by the call)."""
        b = self.batch if batch is None else int(batch)
        check(lib().agg_rhs_noalloc(self._h, _check_state(n, b * self.N), _check_state(out, b * self.N), b))
        return out

    def rk2_step(self, n, dt: float):
        check(lib().agg_rk2_step(self._h, _check_state(n, self.batch * self.N), float(dt)))
        return n

    def set_tilt(self, theta: float):
        """Exponential tilt of a binary32 plan's gain transforms (see agg.h)."""
        check(lib().agg_plan_set_tilt(self._h, float(theta)))

    def profile_pass(self, n, which: int, reps: int = 50) -> float:
        """Mean device microseconds per launch of one pipeline pass (see agg.h)."""
        us = ctypes.c_double()
        check(lib().agg_profile_pass(self._h, _check_state(n, self.batch * self.N), int(which), int(reps),
                                     ctypes.byref(us)))
        return us.value

    def solve(self, n, dt: float, t_end: float, stats: bool = True):
        st = agg_solve_stats()
        rc = lib().agg_solve(self._h, _check_state(n, self.batch * self.N), float(dt), float(t_end),
                             ctypes.byref(st) if stats else None)
        check(rc)
        return st if stats else None


class Engine:
    """agg_engine: continuous-batching solve service on one device."""

    def __init__(self, device: int = 0, mem_budget: int = 0, max_slots: int = 0):
        cfg = agg_engine_config(device, mem_budget, max_slots)
        h = ctypes.c_void_p()
        check(lib().agg_engine_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().agg_engine_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, D, N, kernel, n0, dt, t_end, prec="fp32c", mixed: bool = False, tt: dict = None) -> int:
        """Queue one solve (agg_submit; agg_submit_tt with tt={d: cores} instead
        of a CP kernel)."""
        if (kernel is None) == (tt is None):
            raise ValueError("give either a CP kernel or tensor-train cores")
        n0 = np.ascontiguousarray(n0, dtype=np.float64)
        if n0.size != N:
            raise ValueError("n0 must have N entries")
        t = ctypes.c_uint64(0)
        np0 = n0.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        code = _plan_code(prec, False, mixed)
        if tt is not None:
            terms, nt, keep = make_tt_terms(D, N, tt)
            check(lib().agg_submit_tt(self._h, D, N, terms, nt, np0, float(dt), float(t_end), code, ctypes.byref(t)))
        else:
            terms, nt, keep = make_terms(D, N, kernel)
            check(lib().agg_submit(self._h, D, N, terms, nt, np0, float(dt), float(t_end), code, ctypes.byref(t)))
        del keep
        return t.value

    def poll(self, ticket: int, N: int):
        """(status, n_out or None, stats).  status AGG_PENDING while running."""
        out = np.zeros(N)
        st = agg_request_stats()
        rc = lib().agg_poll(self._h, ticket, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(st))
        if rc == AGG_PENDING:
            return rc, None, None
        if rc == AGG_ENOTFOUND:
            check(rc)
        return rc, out, st

    def counters(self):
        v = [ctypes.c_int64() for _ in range(4)]
        check(lib().agg_engine_counters(self._h, *[ctypes.byref(x) for x in v]))
        return dict(completed=v[0].value, running=v[1].value, queued=v[2].value, bytes_in_use=v[3].value)
