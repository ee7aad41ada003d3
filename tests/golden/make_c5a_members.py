"""Writes c5a_members_t5e-6.txt: the oracle's n(t = 5e-6) for two members of the
D=5, N=2^20 additive-kernel batch (C^(d) = sum_m i_m in CP form, rank d; the
members' initial states are uniform on [1,16] with PCG64 seeds 0 and 37),
10 Heun steps of h = 5e-7 (Sec. 3; inside Heun's stability interval for the
loss rate of the largest size), sampled.  Calls only the oracle (per-rank
numpy FFT evaluation of the Sec. 1 sums, Heun stepping) and the seeded input
generators.  The run time it took is written into the header.

    python tests/golden/make_c5a_members.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402

MEMBERS = (0, 37)


def main():
    c = synth.config("C5a")
    D, N, k, dt, t_end = c["D"], c["N"], c["kernel"], c["dt"], c["t_end"]
    sizes = np.arange(1, N + 1, dtype=np.float64)
    idx = sorted(set(range(1, 257)) | set(range(300, 4097, 16)) | set(range(5000, N + 1, 8191)) | {N})
    t0 = time.time()
    out = []
    for s in MEMBERS:
        n = oracle.heun_solve(lambda v: oracle.total_rhs(*oracle.rhs_fft(D, N, k, v)), c["n0"][s], dt, t_end,
                              callback=lambda j, v: print(f"member {s} step {j + 1}", flush=True))
        assert np.all(np.isfinite(n))
        out.append(n)
    el = time.time() - t0
    with open(os.path.join(HERE, "c5a_members_t5e-6.txt"), "w") as f:
        f.write("# n(t=5e-6) of batch members 0 and 37, D=5 N=2^20 additive kernel sum_m i_m (CP rank d),\n")
        f.write("# n0 uniform on [1,16] with seed = member index, 10 Heun steps h=5e-7 (Sec. 3), RHS by\n")
        f.write("# the oracle's per-rank FFT evaluation of the Sec. 1 sums (binary64).  Written by\n")
        f.write(f"# tests/golden/make_c5a_members.py in {el:.0f} s on one host thread.\n")
        for s, n in zip(MEMBERS, out):
            f.write(f"# MEMBER {s} M0 {np.sum(n):.17e} M1 {np.sum(sizes * n):.17e} MAX {np.max(n):.17e}\n")
        f.write("# k n_k(member 0) n_k(member 37)\n")
        for i in idx:
            f.write(f"{i} {out[0][i - 1]:.17e} {out[1][i - 1]:.17e}\n")


if __name__ == "__main__":
    main()
