#!/usr/bin/env python3
"""Benchmark of the multi-particle aggregation right-hand side on one MI355X.

Workload (a "step" = one Heun step = two right-hand-side evaluations over the
whole pipeline): D = 4, N = 65536, ballistic-like kernel
C^(d) = sum_{m != l} (i_m/i_l)^0.4 in CP form, n_k(0) uniform random on
k in [1, 16] (PCG64 seed 3), Heun step dt = 5e-4; 1000 steps are the whole
t = 0.5 solve.  The state is resident in HBM before the timed region starts.

Prints ONE JSON line.  `value` is right-hand-side evaluations per second in
the primary precision (float-float compensated by default); the binary64 and
binary32 rates of the same workload are reported beside it, with the serving
sample's latency percentiles, the oracle's CPU rate and the factored CPU
version's rate on every host thread.

Every GPU line also states its error against the binary64 oracle.  The GPU legs
keep the outputs they check (computed outside the timed regions); the one leg
that runs the oracle (`cpu_legs`, after all GPU work) times it, times the
factored CPU version, and computes the reference values of those outputs.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PREC_BYTES = {"fp64": 16, "fp32": 8, "fp32c": 16}
PASS_NAMES = {0: "forward column pass", 1: "row pass", 2: "inverse column pass + f",
              3: "fused column pass (inverse + Heun + forward)"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pass_bytes(which: int, N: int, u: int, M: int, cs: int) -> float:
    """Algorithmic HBM bytes of one launch of a pass for one state.

    Spectra: each of the u forward half-length spectra (M stored complex values
    of cs bytes) is written once and read once, and the combined spectrum is
    written once and read once; state-sized vectors are binary64.
      0 forward column pass: read n and u columns, write u spectra
      1 row pass:            read u spectra, write the combined spectrum
      2 inverse column + f:  read combined spectrum, n, u columns; write f
      3 fused column pass:   read combined spectrum, n, u columns;
                             write k1, n~ and u spectra
    """
    if which == 0:
        return 8.0 * N * (1 + u) + u * M * cs
    if which == 1:
        return u * M * cs + M * cs
    if which == 2:
        return M * cs + 8.0 * N * (1 + u) + 8.0 * N
    return M * cs + 8.0 * N * (1 + u) + 2 * 8.0 * N + u * M * cs


def rhs_flops(N: int, u: int, L: int, tsum: int, T: int) -> float:
    """Algorithmic flops of one right-hand-side evaluation of one state: u + 1
    real transforms of length L at 2.5 L log2 L each, the spectral combine over
    H = L/2 + 1 bins (6 flops per complex product, sum_t (|t| - 1) products,
    2 flops per term for its coefficient and sum), the weighting and dot
    products (4 N u) and the loss term with the update (10 N)."""
    H = L // 2 + 1
    return (u + 1) * 2.5 * L * math.log2(L) + H * (6 * tsum + 2 * T) + 4.0 * N * u + 10.0 * N


def gain_terms(tables, kernel) -> tuple:
    """(sum over gain terms of (length - 1), number of gain terms) from the flat plan tables."""
    Tp = int(tables[5])
    pos = 8 + sum(d * (U.shape[1] if hasattr(U, "shape") else len(U[0])) for d, U in kernel.items())
    tsum = 0
    for _ in range(Tp):
        ln = int(tables[pos])
        tsum += ln - 1
        pos += 2 + ln
    return tsum, Tp


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("kernels.hip", "fft_lds.h", "arith.h", "kernels.h"):
        with open(os.path.join(ROOT, "paper_1905_09071_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(which: int, prec: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None
    when it is missing or was taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic_c3.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch", {}).get(f"{prec}:{which}")


def write_traffic(fetch_csv: str, write_csv: str, copy_mib: int, prec: str, out_path: str = None) -> dict:
    """Turn two rocprofv3 counter runs (FETCH_SIZE, then WRITE_SIZE, KiB per
    dispatch) of `bench.py --quick --copy-probe MIB` into bytes per launch of the
    column and row passes, calibrated by the counters of the plain device copy
    of known size; writes profiles/traffic_c3.json and returns its content."""
    import csv
    import statistics

    def per_kernel(path, counter):
        out = {}
        with open(path, newline="") as f:
            for row in csv.DictReader(f):
                if row["Counter_Name"] == counter:
                    out.setdefault(row["Kernel_Name"], []).append(float(row["Counter_Value"]))
        return out

    F, W = per_kernel(fetch_csv, "FETCH_SIZE"), per_kernel(write_csv, "WRITE_SIZE")
    copy_f = max(max(v) for k, v in F.items() if "copyBuffer" in k)
    copy_w = max(max(v) for k, v in W.items() if "copyBuffer" in k)
    fs, ws = copy_mib * 1024.0 / copy_f, copy_mib * 1024.0 / copy_w
    med, per_launch = {}, {}
    for k in F:
        for tag, which in (("agg::col_kernel", 3), ("agg::row_kernel", 1)):
            if tag in k and k in W:
                short = k.split("(")[0].replace("void agg::", "")
                mf, mw = statistics.median(F[k]), statistics.median(W[k])
                med[short] = {"FETCH_SIZE": mf, "WRITE_SIZE": mw}
                per_launch[f"{prec}:{which}"] = round(mf * 1024 * fs + mw * 1024 * ws)
    t = {"workload": f"D=4 N=65536 ballistic a=0.4, one state, {prec}",
         "kernel_source_hash": kernel_source_hash(), "copy_probe_MiB": copy_mib,
         "copy_fetch_KiB": copy_f, "copy_write_KiB": copy_w,
         "fetch_scale": round(fs, 4), "write_scale": round(ws, 4),
         "bytes_per_launch": per_launch, "median_KiB_per_dispatch": med}
    with open(out_path or os.path.join(ROOT, "profiles", "traffic_c3.json"), "w") as f:
        json.dump(t, f, indent=1)
    return t


def time_steps(plan, n, dt, steps, warmup, torch):
    # at least 18 warm-up steps, so that the solve's captured graph of 16 steps
    # is built outside the timed region whatever --warmup asks for; then, for a
    # short solve, the timed call itself twice untimed, so that the timed call
    # replays the captured whole solve (built at the second identical call)
    plan.solve(n, dt, max(warmup, 18) * dt, stats=False)
    if steps <= 64:
        plan.solve(n, dt, steps * dt, stats=False)
        plan.solve(n, dt, steps * dt, stats=False)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    plan.solve(n, dt, steps * dt, stats=False)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / 1000.0, wall


def copy_bandwidth(torch, mib: int = 2048, reps: int = 5) -> float:
    """Device-to-device copy rate (read + write bytes per second, GB/s) of a
    plain torch copy of `mib` MiB, median of `reps`: the measured ceiling that
    the roofline is also quoted against."""
    src = torch.ones(mib * 131072, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    rates = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        rates.append(2 * src.numel() * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    del src, dst
    torch.cuda.empty_cache()
    rates.sort()
    return rates[len(rates) // 2]


def cpu_baseline(c, budget_s: float):
    """The oracle (per-rank numpy FFT evaluation) on the host, bounded sample."""
    import oracle
    import synth
    n = synth.n0_random_dense(c["N"], 5, decay=1e-4)
    evals = 0
    t0 = time.perf_counter()
    while True:
        oracle.rhs_fft(c["D"], c["N"], c["kernel"], n)
        evals += 1
        el = time.perf_counter() - t0
        if el >= budget_s or evals >= 400:
            break
    return evals / el, evals, el


def cpu_factored(c, budget_s: float):
    """The factored CPU version (oracle/factored.c: distinct columns, own binary64
    FFT, OpenMP over every host thread) on the same workload, bounded sample."""
    import oracle
    import synth
    n = synth.n0_random_dense(c["N"], 5, decay=1e-4)
    oracle.rhs_factored(c["D"], c["N"], c["kernel"], n)      # first call: threads, pages
    evals, threads = 0, 0
    t0 = time.perf_counter()
    while True:
        _, threads = oracle.rhs_factored(c["D"], c["N"], c["kernel"], n)
        evals += 1
        el = time.perf_counter() - t0
        if el >= budget_s or evals >= 5000:
            break
    return evals / el, evals, el, threads


def rel_err(got, ref) -> float:
    import numpy as np
    return float(np.max(np.abs(np.asarray(got) - ref)) / max(float(np.max(np.abs(ref))), 1e-300))


def dense_factors(kernel) -> dict:
    """A kernel dict as the oracle takes it: (d, R, N) factor arrays without
    weights (a rank's weight multiplies its mode-1 column)."""
    import numpy as np
    out = {}
    for d, v in kernel.items():
        w = None
        if isinstance(v, dict):
            w, v = v.get("weight"), v["U"]
        U = np.array([np.asarray(x, dtype=np.float64) for x in v])
        if w is not None:
            U[0] = U[0] * np.asarray(w, dtype=np.float64)[:, None]
        out[d] = U
    return out


def oracle_reference(chk: dict):
    """Reference value of one recorded GPU output.  kind "rhs": the oracle's
    right-hand side of chk["n"] (per-rank FFT evaluation; with "kmax", per-rank
    direct convolutions up to kmax, exact for a state whose support lies in
    [1, kmax/D]); kind "solve": the oracle's Heun trajectory from chk["n"] to
    chk["t_end"] with step chk["dt"]."""
    import numpy as np
    import oracle
    D, N = chk["D"], chk["N"]
    # a tensor-train kernel set enters as its rank-path CP factors
    k = ({d: oracle.tt_paths(c) for d, c in chk["tt"].items()} if "tt" in chk else dense_factors(chk["kernel"]))

    def rhs(v):
        if chk.get("kmax"):
            p, q = oracle.rhs_conv(D, N, k, v, kmax=chk["kmax"])
            p[:, chk["kmax"]:] = 0.0
            return oracle.total_rhs(p, q)
        return oracle.total_rhs(*oracle.rhs_fft(D, N, k, v))

    if chk["kind"] == "rhs":
        return rhs(chk["n"])
    _ = np
    return oracle.heun_solve(rhs, chk["n"], chk["dt"], chk["t_end"])


def cpu_legs(c, budget_s: float, checks: dict, log=print):
    """Everything that runs the oracle, after all GPU work: the oracle's CPU rate,
    the factored CPU version's rate, and the error of every recorded GPU output
    (``checks``: name -> (GPU output, reference spec)) against the oracle."""
    import os as _os
    out = {"cpu_baseline": None, "cpu_factored": None, "errors": {}}
    if budget_s > 0:
        rate, evals, el = cpu_baseline(c, budget_s)
        out["cpu_baseline"] = {"value": round(rate, 4), "unit": "RHS evals/s", "cores": 1, "kind": "oracle",
                               "sample": f"{evals} oracle RHS evaluations (per-rank numpy FFT, D=4 N=65536, "
                                         f"dense state) in {el:.1f} s on one host thread"}
        log(f"[bench] cpu oracle: {rate:.2f} RHS/s")
        rate, evals, el, th = cpu_factored(c, budget_s)
        out["cpu_factored"] = {"value": round(rate, 3), "unit": "RHS evals/s", "cores": th, "kind": "factored",
                               "host_cpus": _os.cpu_count(),
                               "sample": f"{evals} RHS evaluations of the factored CPU version (oracle/factored.c: "
                                         f"3 distinct columns, own radix-2 binary64 FFT of length 2^18, "
                                         f"OpenMP) in {el:.1f} s on {th} threads, D=4 N=65536 dense state"}
        log(f"[bench] cpu factored: {rate:.2f} RHS/s on {th} threads")
    for name, (got, chk) in checks.items():
        t0 = time.perf_counter()
        out["errors"][name] = float(f"{rel_err(got, oracle_reference(chk)):.3e}")
        log(f"[bench] accuracy {name}: {out['errors'][name]:.3e} ({time.perf_counter() - t0:.1f} s)")
    return out


def tensor_train_lines(agg, synth, torch, np, checks, log):
    """Kernels in tensor-train form (Sec. 2) through the per-bin matrix chain
    (agg_plan_create_tt), D=4, N=65536, 20 Heun steps of one state:
    random dense cores of ranks (1,3,1), (1,4,4,1), (1,6,6,6,1) against the
    same kernel as rank paths (agg_tt_expand: 3 + 16 + 216 rank-one terms);
    and the ballistic kernel at orders 2 and 3 (no CP or TT form known)
    compressed by agg_tt_cross to ranks <= 8."""
    h, steps = 1e-6, 20
    out = {}
    for N in (4096, 65536):
        rng = np.random.default_rng(80)
        cores = lambda ranks: [rng.uniform(0.1, 1.0, size=(ranks[m], N, ranks[m + 1]))
                               for m in range(len(ranks) - 1)]
        tt = {2: cores([1, 3, 1]), 3: cores([1, 4, 4, 1]), 4: cores([1, 6, 6, 6, 1])}
        n0 = synth.n0_uniform_head(N, 3, 16)
        rates, refused = {}, None
        for prec in ("fp64", "fp32c"):
            for how in ("chain", "paths"):
                try:
                    if how == "chain":
                        plan = agg.Plan(4, N, prec=prec, tt=tt)
                    else:
                        plan = agg.Plan(4, N, {d: agg.tt_expand(N, c) for d, c in tt.items()}, prec)
                except agg.AggError as e:
                    refused = str(e)
                    log(f"[bench] TT ranks 6 D=4 N={N} {how} {prec}: refused ({e})")
                    continue
                n = torch.tensor(n0, dtype=torch.float64, device="cuda:0")
                t, _ = time_steps(plan, n, h, steps, 2, torch)
                rates[f"{how}_{prec}"] = round(2 * steps / t, 1)
                if how == "chain":
                    f = plan.rhs(torch.tensor(n0, dtype=torch.float64, device="cuda:0"))
                    checks[f"tt_chain_ranks6_n{N}_rhs_{prec}"] = (
                        f.cpu().numpy(), dict(kind="rhs", D=4, N=N, tt=tt, n=n0, kmax=64))
                plan.close()
                del n
                log(f"[bench] TT ranks 6 D=4 N={N} {how} {prec}: {rates[f'{how}_{prec}']} RHS/s")
        out[f"ranks6_n{N}"] = {
            "workload": f"D=4 N={N}, random dense TT cores ranks (1,3,1),(1,4,4,1),(1,6,6,6,1) (114 core "
                        "columns), n0 uniform on [1,16], 20 Heun steps h=1e-6; chain = agg_plan_create_tt, "
                        "paths = the same kernel as 3+16+216 rank-one terms (agg_tt_expand)",
            "rhs_per_s": rates,
            "chain_vs_paths": {p: round(rates[f"chain_{p}"] / rates[f"paths_{p}"], 3)
                               for p in ("fp64", "fp32c") if f"paths_{p}" in rates and f"chain_{p}" in rates},
            "paths_refused": refused}
    N = 65536
    n0 = synth.n0_uniform_head(N, 3, 16)

    def ballistic(a):
        s = a.astype(np.float64)
        return np.sum(s ** (1 / 3), axis=1) ** 2 * np.sqrt(np.sum(1.0 / s, axis=1))
    t0 = time.perf_counter()
    cross = {d: agg.tt_cross(d, N, ballistic, tol=1e-12, rmax=8, seed=d) for d in (2, 3)}
    tcross = time.perf_counter() - t0
    ttb = {d: c for d, (c, _) in cross.items()}
    rates, rates_mixed = {}, {}
    Lm = int(agg.plan_tables_tt(3, N, ttb, "fp64", mixed=True)[0])
    for mixed in (False, True):
        for prec in ("fp64", "fp32c"):
            plan = agg.Plan(3, N, prec=prec, tt=ttb, mixed=mixed)
            n = torch.tensor(n0, dtype=torch.float64, device="cuda:0")
            t, _ = time_steps(plan, n, h, steps, 2, torch)
            (rates_mixed if mixed else rates)[prec] = round(2 * steps / t, 1)
            f = plan.rhs(torch.tensor(n0, dtype=torch.float64, device="cuda:0"))
            key = f"tt_cross_ballistic{'_L3x2e16' if mixed else ''}_rhs_{prec}"
            checks[key] = (f.cpu().numpy(), dict(kind="rhs", D=3, N=N, tt=ttb, n=n0, kmax=48))
            plan.close()
            del n
            log(f"[bench] TT-cross ballistic D=3 N={N} {prec}{f' L={Lm}' if mixed else ''}: "
                f"{(rates_mixed if mixed else rates)[prec]} RHS/s")
    out["tt_cross_ballistic"] = {
        "workload": "D=3 N=65536, kernel (sum_m i_m^(1/3))^2 (sum_m 1/i_m)^(1/2) at orders 2 and 3, "
                    "compressed on the host by agg_tt_cross (rmax 8), n0 uniform on [1,16], 20 Heun steps h=1e-6",
        "ranks": {d: [1] + [int(x.shape[2]) for x in c] for d, (c, _) in cross.items()},
        "cross_err_est": {d: float(f"{e:.3e}") for d, (_, e) in cross.items()},
        "cross_seconds": round(tcross, 2),
        "rhs_per_s": rates,
        "mixed_radix": {"L": Lm, "rhs_per_s": rates_mixed}}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--prec", default="fp32c", choices=["fp32c", "fp64", "fp32"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="oracle CPU sample budget (0 = skip)")
    ap.add_argument("--serving", type=int, default=512, help="requests in the serving sample (0 = skip)")
    ap.add_argument("--batch", type=int, default=64, help="states of the batched C3 line (0 = skip)")
    ap.add_argument("--c5", type=int, default=1, help="run the D=5 N=2^20 batch-64 line (0 = skip)")
    ap.add_argument("--table1", type=int, default=1,
                    help="run the D=3 pure ternary N=2^19 tensor-train kernel line (0 = skip)")
    ap.add_argument("--c5b", type=int, default=64,
                    help="states of the D=5 N=2^20 compressed (sum i)^(1/2) line (0 = skip)")
    ap.add_argument("--tt", type=int, default=1,
                    help="run the tensor-train lines (matrix chain vs rank paths; TT-cross kernel) (0 = skip)")
    ap.add_argument("--quick", action="store_true",
                    help="profiling aid: time only the primary precision (on --batch states if > 0), "
                         "no pass timing, no other lines")
    ap.add_argument("--quick-d5", type=int, default=0, choices=[0, 1, 2],
                    help="profiling aid: time the passes of the D=5 N=2^20 batch (additive kernel, --batch states, "
                         "default 64) at L = 2^23 (1) or 5 2^20 (2) and exit")
    ap.add_argument("--quick-tt", action="store_true",
                    help="profiling aid: run only the tensor-train lines and print their JSON")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="profiling aid: also copy a float64 tensor of this many MiB (counter calibration)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="no GPU: turn the two counter runs of --quick --copy-probe into profiles/traffic_c3.json")
    args = ap.parse_args()
    if args.traffic_from:
        t = write_traffic(args.traffic_from[0], args.traffic_from[1], args.copy_probe or 256, args.prec)
        print(json.dumps(t))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1905_09071_amd as agg
    import synth

    if args.quick_d5:
        # the D=5, N=2^20 batch's row and fused column passes, a few launches each
        cc = synth.config("C5a")
        B5 = args.batch if args.batch > 0 else cc["n0"].shape[0]
        mixed = args.quick_d5 == 2
        t5 = agg.plan_tables(cc["D"], cc["N"], cc["kernel"], args.prec, mixed=mixed)
        plan = agg.Plan(cc["D"], cc["N"], cc["kernel"], args.prec, batch=B5, mixed=mixed)
        n = torch.tensor(cc["n0"][:B5].reshape(-1), dtype=torch.float64, device="cuda:0")
        us = {w: plan.profile_pass(n, w, reps=2) for w in (1, 3)}
        print(json.dumps({"quick_d5": True, "prec": args.prec, "batch": B5, "L": int(t5[0]), "M1": int(t5[1]),
                          "M2": int(t5[2]), "row_us": round(us[1], 1), "fused_col_us": round(us[3], 1)}))
        return

    if args.quick_tt:
        tt_out = tensor_train_lines(agg, synth, torch, np, {}, log)
        print(json.dumps({"quick_tt": True, "tensor_train": tt_out}))
        return

    c = synth.config("C3")
    D, N, dt = c["D"], c["N"], c["dt"]
    tables = agg.plan_tables(D, N, c["kernel"], args.prec)
    L, M1, M2, g, u = (int(x) for x in tables[:5])
    M = L // 2
    log(f"[bench] C3 D={D} N={N} L={L} M1={M1} M2={M2} g={g} u={u} steps={args.steps} warmup={args.warmup}")

    if args.copy_probe > 0:
        src = torch.ones(args.copy_probe * 131072, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy probe: {args.copy_probe} MiB copied")
        del src, dst

    results = {}
    checks = {}    # name -> (GPU output, oracle reference spec); checked in cpu_legs
    nd = synth.n0_random_dense(N, 5, decay=1e-4)   # dense state of the accuracy checks
    order = [args.prec] + [p for p in ("fp64", "fp32", "fp32c") if p != args.prec]
    if args.quick:
        order = [args.prec]
    # --quick with --batch B > 0 times the primary precision on B states instead
    qb = args.batch if (args.quick and args.batch > 0) else 1
    for prec in order:
        plan = agg.Plan(D, N, c["kernel"], prec, batch=qb)
        n = torch.tensor(np.tile(c["n0"], qb), dtype=torch.float64, device="cuda:0")
        t_gpu, t_wall = time_steps(plan, n, dt, args.steps, args.warmup, torch)
        rate = 2 * args.steps * qb / t_gpu
        if args.quick:
            results[prec] = dict(seconds=t_gpu, wall=t_wall, rhs_per_s=rate, passes_us={w: 1.0 for w in range(4)})
            log(f"[bench] {prec}: {args.steps} steps of {qb} state(s) in {t_gpu*1e3:.2f} ms -> {rate:.1f} RHS/s (quick)")
            plan.close()
            del n
            continue
        passes = {w: plan.profile_pass(n, w, reps=200) for w in (0, 1, 2, 3)}
        results[prec] = dict(seconds=t_gpu, wall=t_wall, rhs_per_s=rate, passes_us=passes)
        f = plan.rhs(torch.tensor(nd, dtype=torch.float64, device="cuda:0"))
        checks[f"c3_rhs_{prec}"] = (f.cpu().numpy(), dict(kind="rhs", D=D, N=N, kernel=c["kernel"], n=nd))
        log(f"[bench] {prec}: {args.steps} steps in {t_gpu*1e3:.2f} ms (wall {t_wall*1e3:.2f}) -> "
            f"{rate:.1f} RHS/s; pass us: " + ", ".join(f"{w}:{v:.2f}" for w, v in passes.items()))
        plan.close()
        del n

    if args.quick:
        print(json.dumps({"quick": True, "prec": args.prec, "batch": qb,
                          "rhs_per_s": round(results[args.prec]["rhs_per_s"], 2)}))
        return

    # the plain fp64 reference evaluation (term by term, unshared, unfused)
    plan = agg.Plan(D, N, c["kernel"], "fp64", plain=True)
    n = torch.tensor(c["n0"], dtype=torch.float64, device="cuda:0")
    psteps = max(5, args.steps // 20)
    t_plain, _ = time_steps(plan, n, dt, psteps, 2, torch)
    plain_rate = 2 * psteps / t_plain
    log(f"[bench] plain fp64: {psteps} steps in {t_plain*1e3:.2f} ms -> {plain_rate:.1f} RHS/s")
    plan.close()
    del n

    # batched throughput: B states sharing the kernel (C3 shape) and the D=5,
    # N=2^20 batch of 64 states (transform length 2^23)
    batched = {}
    roof_b = None
    if args.batch > 0:
        for prec in ("fp64", "fp32c", "fp32"):
            plan = agg.Plan(D, N, c["kernel"], prec, batch=args.batch)
            n = torch.tensor(np.tile(c["n0"], args.batch), dtype=torch.float64, device="cuda:0")
            bsteps = 20
            t_b, _ = time_steps(plan, n, dt, bsteps, 2, torch)
            batched[prec] = round(2 * bsteps * args.batch / t_b, 1)
            f = plan.rhs(torch.tensor(np.tile(nd, args.batch), dtype=torch.float64, device="cuda:0"))
            checks[f"c3_batch_rhs_{prec}_last_member"] = (
                f.cpu().numpy()[(args.batch - 1) * N:], dict(kind="rhs", D=D, N=N, kernel=c["kernel"], n=nd))
            log(f"[bench] C3 batch {args.batch} {prec}: {2 * bsteps * args.batch / t_b:.1f} RHS/s")
            if prec == args.prec:
                # the same byte model at saturation: B states per launch
                bp = {w: plan.profile_pass(n, w, reps=20) for w in (1, 3)}
                wd = max(bp, key=bp.get)
                byts = pass_bytes(wd, N, u, M, PREC_BYTES[prec]) * args.batch
                ach = byts / (bp[wd] * 1e-6) / 1e9
                roof_b = {"batch": args.batch, "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                          "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "kernel": PASS_NAMES[wd],
                          "bytes_per_launch": byts, "us_per_launch": round(bp[wd], 3)}
            plan.close()
            del n
            torch.cuda.empty_cache()
    c5 = {}
    c5_mixed = {}
    if args.c5:
        cc = synth.config("C5a")
        B5 = cc["n0"].shape[0]
        # transform length 2^23, then (mixed-radix option) 5 2^20
        for mixed, dst in ((False, c5), (True, c5_mixed)):
            for prec in ("fp64", "fp32c"):
                plan = agg.Plan(cc["D"], cc["N"], cc["kernel"], prec, batch=B5, mixed=mixed)
                n = torch.tensor(cc["n0"].reshape(-1), dtype=torch.float64, device="cuda:0")
                s5 = 10
                t5, _ = time_steps(plan, n, cc["dt"], s5, 1, torch)
                dst[prec] = round(2 * s5 * B5 / t5, 2)
                f = plan.rhs(torch.tensor(cc["n0"].reshape(-1), dtype=torch.float64, device="cuda:0"))
                f = f.cpu().numpy().reshape(B5, cc["N"])
                tag = "_L5x2e20" if mixed else ""
                for b in ((0, B5 - 1) if not mixed else (B5 - 1,)):
                    checks[f"d5_n2e20{tag}_rhs_{prec}_member{b}"] = (
                        f[b], dict(kind="rhs", D=cc["D"], N=cc["N"], kernel=cc["kernel"], n=cc["n0"][b], kmax=80))
                L5 = int(agg.plan_tables(cc["D"], cc["N"], cc["kernel"], prec, mixed=mixed)[0])
                log(f"[bench] D=5 N=2^20 batch {B5} {prec} L={L5}: {s5} steps in {t5*1e3:.1f} ms -> "
                    f"{dst[prec]} RHS/s")
                plan.close()
                del n
                torch.cuda.empty_cache()

    c5b = None
    if args.c5b:
        # (i_1+..+i_d)^(1/2), compressed on the host to rank 32 per order (not timed)
        D5, N5, B = 5, 1 << 20, args.c5b
        fv = synth.sum_kernel_values(2, D5 * N5)
        t0 = time.perf_counter()
        alpha, w, ferr = agg.expsum_fit(fv, 2, 31)
        tfit = time.perf_counter() - t0
        k5 = synth.kernel_expsum(D5, N5, alpha, w, weighted=True)   # 32 columns shared by all orders
        n0 = np.stack([synth.n0_uniform_head(N5, s, 16) for s in range(B)])
        c5b = {"batch": B, "rank_per_order": 32, "distinct_columns": 32,
               "fit_max_err_over_max_C": float(f"{ferr / fv.max():.3e}"), "fit_seconds": round(tfit, 2)}
        for mixed, prec in ((False, "fp64"), (False, "fp32c"), (True, "fp64"), (True, "fp32c")):
            plan = agg.Plan(D5, N5, k5, prec, batch=B, mixed=mixed)
            L5 = int(agg.plan_tables(D5, N5, k5, prec, mixed=mixed)[0])
            n = torch.tensor(n0.reshape(-1), dtype=torch.float64, device="cuda:0")
            h, s5 = 1e-4, 3
            plan.solve(n, h, h, stats=False)      # one untimed step
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            plan.solve(n, h, s5 * h, stats=False)
            e1.record()
            torch.cuda.synchronize()
            t5 = e0.elapsed_time(e1) / 1000.0
            key = prec + ("_L5x2e20" if mixed else "")
            c5b[key] = round(2 * s5 * B / t5, 2)
            f = plan.rhs(torch.tensor(n0.reshape(-1), dtype=torch.float64, device="cuda:0"))
            checks[f"d5_n2e20_sqrt_sum_rhs_{key}_member0"] = (
                f.cpu().numpy()[:N5], dict(kind="rhs", D=D5, N=N5, kernel=k5, n=n0[0], kmax=80))
            log(f"[bench] D=5 N=2^20 sqrt-sum kernel (rank 32, u=32) batch {B} {prec} L={L5}: {s5} steps in "
                f"{t5*1e3:.1f} ms -> {c5b[key]} RHS/s")
            plan.close()
            del n
            torch.cuda.empty_cache()

    table1 = None
    if args.table1:
        # the shape of the paper's Table 1: pure ternary aggregation, 3-dimensional
        # generalized Brownian kernel given by its TT cores, N = 2^19, 100 Heun steps
        D1, N1, h1, s1 = 3, 1 << 19, 1e-3, 100
        mus = [1.0 / 3.0, -1.0 / 3.0, 0.0]
        k1 = {3: agg.tt_expand(N1, synth.brownian_tt_cores(N1, mus))}
        plan = agg.Plan(D1, N1, k1, "fp64")
        n = torch.tensor(synth.n0_uniform_head(N1, 3, 16), dtype=torch.float64, device="cuda:0")
        t1, _ = time_steps(plan, n, h1, s1, 1, torch)
        tab1 = agg.plan_tables(D1, N1, k1, "fp64")
        # the same with the mixed-radix length 3 2^19
        plan_m = agg.Plan(D1, N1, k1, "fp64", mixed=True)
        n_m = torch.tensor(synth.n0_uniform_head(N1, 3, 16), dtype=torch.float64, device="cuda:0")
        t1m, _ = time_steps(plan_m, n_m, h1, s1, 1, torch)
        L1m = int(agg.plan_tables(D1, N1, k1, "fp64", mixed=True)[0])
        nt1m = synth.n0_uniform_head(N1, 3, 16)
        fm = plan_m.rhs(torch.tensor(nt1m, dtype=torch.float64, device="cuda:0"))
        checks["table1_shape_L3x2e19_rhs_fp64"] = (fm.cpu().numpy(),
                                                   dict(kind="rhs", D=D1, N=N1, kernel=k1, n=nt1m, kmax=48))
        plan_m.close()
        del n_m
        log(f"[bench] Table-1 shape, L={L1m}: 100 steps in {t1m*1e3:.1f} ms")
        nt1 = synth.n0_uniform_head(N1, 3, 16)
        f = plan.rhs(torch.tensor(nt1, dtype=torch.float64, device="cuda:0"))
        checks["table1_shape_rhs_fp64"] = (f.cpu().numpy(), dict(kind="rhs", D=D1, N=N1, kernel=k1, n=nt1, kmax=48))
        table1 = {"workload": "D=3 pure ternary (d=3 only), generalized Brownian kernel [1/3, -1/3, 0] from "
                              "its TT cores (ranks 1,3,3,1; 6 paths merged into 1 gain term), N=2^19, "
                              "n0 uniform on [1,16] seed 3, 100 Heun steps h=1e-3, fp64",
                  "L": int(tab1[0]), "seconds_100_steps": round(t1, 5), "rhs_per_s": round(2 * s1 / t1, 1),
                  "mixed_radix": {"L": L1m, "seconds_100_steps": round(t1m, 5),
                                  "rhs_per_s": round(2 * s1 / t1m, 1)},
                  "paper_seconds_100_steps": {"1 core": 257.80, "128 cores": 12.22},
                  "paper_context": "Table 1: TT path with MKL ClusterFFT on CPU cores (kernel exponents and "
                                   "initial data not stated in the paper)"}
        log(f"[bench] Table-1 shape (D=3 ternary N=2^19 TT Brownian): 100 steps in {t1*1e3:.1f} ms")
        plan.close()
        del n
        torch.cuda.empty_cache()

    tt_lines = None
    if args.tt:
        tt_lines = tensor_train_lines(agg, synth, torch, np, checks, log)

    prim = results[args.prec]
    cs = PREC_BYTES[args.prec]
    # dominant kernel of a time step: the pass with the largest device time
    dom = max((1, 3), key=lambda w: prim["passes_us"][w])
    bytes_dom = pass_bytes(dom, N, u, M, cs)
    achieved = bytes_dom / (prim["passes_us"][dom] * 1e-6) / 1e9
    copy_gbs = copy_bandwidth(torch)
    log(f"[bench] device copy: {copy_gbs:.0f} GB/s")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(dom, args.prec),
                "kernel": PASS_NAMES[dom], "bytes_per_launch": bytes_dom,
                "us_per_launch": round(prim["passes_us"][dom], 3),
                "measured_copy_gbs": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4)}

    tsum, Tp = gain_terms(tables, c["kernel"])
    F = rhs_flops(N, u, L, tsum, Tp)
    fpeak = 78.6 if args.prec == "fp64" else 157.3
    flop_roof = {"flops_per_rhs": round(F), "achieved_tflops": round(F * prim["rhs_per_s"] / 1e12, 3),
                 "peak_tflops": fpeak, "frac": round(F * prim["rhs_per_s"] / 1e12 / fpeak, 5),
                 "note": "algorithmic flops; fp32c executes several binary32 operations per flop"
                         if args.prec == "fp32c" else "algorithmic flops"}

    serving = None
    if args.serving > 0:
        from serving_bench import run_serving
        serving, served = run_serving(args.serving, log=log)
        for i, (out, r) in enumerate(served):
            checks[f"serving_sample_{i}"] = (out, dict(kind="solve", D=r["D"], N=r["N"], kernel=r["kernel"],
                                                      n=r["n0"], dt=r["dt"], t_end=r["t_end"]))

    # the one leg that runs the oracle: CPU rates and the reference values
    legs = cpu_legs(c, args.cpu_seconds, checks, log=log)
    cpu = legs["cpu_baseline"]
    errors = legs["errors"]
    if serving is not None:
        se = [v for k, v in errors.items() if k.startswith("serving_sample_")]
        serving["max_err_vs_oracle_sampled"] = max(se) if se else None
        serving["accuracy_sample"] = (f"{len(se)} served results (fp32c) against the oracle's Heun trajectory, "
                                      "max_k |n - n_ref| / max_k n_ref")

    ms_per_step = prim["seconds"] / args.steps * 1e3
    line = {
        "metric": "RHS evals/s at D=4 N=65536 (FP32-comp vs FP64) + serving p50/p99 latency",
        "value": round(prim["rhs_per_s"], 2),
        "unit": "RHS evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32c": "f32x2 (float-float)", "fp64": "f64", "fp32": "f32"}[args.prec],
        "data": "synthetic",
        "config": {"workload": "C3: D=4 N=65536 ballistic a=0.4 CP (u=3 distinct columns), "
                               "n0 uniform on [1,16] seed 3, Heun dt=5e-4, one state",
                   "L": L, "M1": M1, "M2": M2, "parallelism": "single GPU"},
        "rhs_per_s": {p: round(r["rhs_per_s"], 2) for p, r in results.items()},
        "ratio_fp32c_vs_fp64": round(results["fp32c"]["rhs_per_s"] / results["fp64"]["rhs_per_s"], 4),
        "plain_fp64_rhs_per_s": round(plain_rate, 2),
        "batched_rhs_per_s": {"batch": args.batch, **batched} if batched else None,
        "d5_n2e20_batch64_rhs_per_s": c5 or None,
        "d5_n2e20_batch64_L5x2e20_rhs_per_s": c5_mixed or None,
        "d5_n2e20_sqrt_sum_kernel_rhs_per_s": c5b,
        "paper_table1_shape": table1,
        "tensor_train": tt_lines,
        "ratio_fp32c_vs_plain_fp64": round(results["fp32c"]["rhs_per_s"] / plain_rate, 3),
        "pass_us": {p: {PASS_NAMES[w]: round(v, 3) for w, v in r["passes_us"].items()} for p, r in results.items()},
        "roofline": roofline,
        "roofline_batched": dict(roof_b, measured_copy_gbs=round(copy_gbs, 1),
                                 frac_of_copy=round(roof_b["achieved"] / copy_gbs, 4)) if roof_b else None,
        "flop_roofline": flop_roof,
        "cpu_baseline": cpu,
        "cpu_factored": legs["cpu_factored"],
        "gpu_vs_cpu_factored": (round(prim["rhs_per_s"] / legs["cpu_factored"]["value"], 1)
                                if legs["cpu_factored"] else None),
        "rhs_err_vs_oracle": errors,
        "err_norm": "max_k |f - f_ref| / max_k |f_ref| per RHS (the oracle's binary64 evaluation)",
        "serving": serving,
    }
    _ = np
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
