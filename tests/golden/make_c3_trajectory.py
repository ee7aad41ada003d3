"""Writes c3_trajectory_t0.5.txt: the oracle's n(t = 0.5) for the D=4, N=65536
ballistic workload (1000 Heun steps of h = 5e-4 from the seeded initial state),
sampled.  Calls only the oracle (per-rank numpy FFT evaluation of the Sec. 1
sums, Heun stepping of Sec. 3) and the seeded input generators.  About 25
minutes on one host thread (the written file's header records the time taken).

    python tests/golden/make_c3_trajectory.py
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
    c = synth.config("C3")
    D, N, k, dt, t_end = c["D"], c["N"], c["kernel"], c["dt"], c["t_end"]
    t0 = time.time()
    n = oracle.heun_solve(lambda v: oracle.total_rhs(*oracle.rhs_fft(D, N, k, v)), c["n0"], dt, t_end)
    el = time.time() - t0
    idx = sorted(set(range(1, 65)) | set(range(128, N + 1, 512)) | {N})
    sizes = np.arange(1, N + 1, dtype=np.float64)
    with open(os.path.join(HERE, "c3_trajectory_t0.5.txt"), "w") as f:
        f.write("# n(t=0.5), D=4 N=65536 ballistic a=0.4 CP kernel (u=3), n0 uniform on [1,16] seed 3,\n")
        f.write("# 1000 Heun steps h=5e-4 (Sec. 3), RHS by the oracle's per-rank FFT evaluation of the\n")
        f.write("# Sec. 1 sums (binary64).  Written by tests/golden/make_c3_trajectory.py "
                f"in {el:.0f} s.\n")
        f.write(f"# M0 {np.sum(n):.17e}\n# M1 {np.sum(sizes * n):.17e}\n# MAX {np.max(n):.17e}\n")
        f.write("# k n_k\n")
        for i in idx:
            f.write(f"{i} {n[i - 1]:.17e}\n")


if __name__ == "__main__":
    main()
