"""Writes c2_trajectory_t10.txt: the oracle's n(t = 10) for the D=3, N=4096
generalized Brownian workload, C^(d) = (sum_m i_m^(1/3)) (sum_l i_l^(-1/3)),
n_k(0) = exp(-k/8)/Z, 10000 Heun steps of h = 1e-3 (Sec. 3), sampled, with the
zeroth and first moments at every 1000th step.  Calls only the oracle
(per-rank numpy FFT evaluation of the Sec. 1 sums, Heun stepping) and the
seeded input generators.  The run time it took is written into the header.

    python tests/golden/make_c2_trajectory.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402


def main():
    c = synth.config("C2")
    D, N, k, dt, t_end = c["D"], c["N"], c["kernel"], c["dt"], c["t_end"]
    sizes = np.arange(1, N + 1, dtype=np.float64)
    moments = []

    def cb(j, n):
        if (j + 1) % 1000 == 0:
            moments.append((j + 1, float(np.sum(n)), float(np.sum(sizes * n))))
            print(f"step {j + 1}: M0 {moments[-1][1]:.6e}", flush=True)

    t0 = time.time()
    n = oracle.heun_solve(lambda v: oracle.total_rhs(*oracle.rhs_fft(D, N, k, v)), c["n0"], dt, t_end,
                          callback=cb)
    el = time.time() - t0
    assert np.all(np.isfinite(n))
    idx = sorted(set(range(1, 129)) | set(range(160, N + 1, 32)) | {N})
    with open(os.path.join(HERE, "c2_trajectory_t10.txt"), "w") as f:
        f.write("# n(t=10), D=3 N=4096 generalized Brownian kernel (sum i^(1/3))(sum i^(-1/3)) in CP form\n")
        f.write("# (ranks 4 and 9), n0 = exp(-k/8)/Z, 10000 Heun steps h=1e-3 (Sec. 3), RHS by the oracle's\n")
        f.write("# per-rank FFT evaluation of the Sec. 1 sums (binary64).  Written by\n")
        f.write(f"# tests/golden/make_c2_trajectory.py in {el:.0f} s on one host thread.\n")
        f.write(f"# M0 {np.sum(n):.17e}\n# M1 {np.sum(sizes * n):.17e}\n# MAX {np.max(n):.17e}\n")
        for step, m0, m1 in moments:
            f.write(f"# STEP {step} M0 {m0:.17e} M1 {m1:.17e}\n")
        f.write("# k n_k\n")
        for i in idx:
            f.write(f"{i} {n[i - 1]:.17e}\n")


if __name__ == "__main__":
    main()
