"""Write the oracle's trajectories of three SBM instances of the 256-instance batch workload into
tests/golden/batch_sbm_instances_rk4_2000.txt.

The batch is gen.batch_instances_iter() (256 instances, N log-uniform in [1024, 65536], all-to-all
or equal-community SBM with communities of about 1024 nodes, rho 0.97, p_out 2e-4, K swept over
[0, 6], omega ~ N(0, 1), seed 1004). The instances stored are the two smallest SBM instances and
the smallest SBM instance above 16000 nodes. Each is integrated by the oracle (straightforward
summation of Sec. 3 eq. KuramotoGraph, classical RK4 of Sec. 2, FP64, unwrapped phases) for 2000
steps of dt 0.01 from the inputs an FP32 batch sees: theta0, omega, K and dt rounded to FP32.

Per instance the file holds its batch index, size and K, the order parameter r every 10 steps
(Sec. 2, eq. OrderParameter), and theta(T) of every row (instances below 4096 nodes) or of a
seeded 1/8 of the rows (instance-local user numbering). Beside each phase it stores the row's
sensitivity: the largest change of the oracle's own theta(T) over two runs whose theta0 and
omega carry seeded relative perturbations of FP32 rounding size (2^-24). A partially
synchronised instance has drifting oscillators whose phase at T moves far more than the inputs
do; an FP32 trajectory can only be compared with the oracle within that sensitivity.

Only gen and oracle are used. Runs on the CPU (about half an hour on 8 cores):

    python tests/golden/make_batch_sbm_instances.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import gen  # noqa: E402
import oracle  # noqa: E402

STEPS = 2000
R_EVERY = 10
DT = 0.01
OUT = os.path.join(HERE, "batch_sbm_instances_rk4_2000.txt")


def f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def sample_rows(i: int, n: int) -> np.ndarray:
    if n < 4096:
        return np.arange(n)
    return np.sort(np.random.default_rng(1000 + i).choice(n, n // 8, replace=False))


def main():
    small, large = [], None
    for i, w in enumerate(gen.batch_instances_iter()):
        if w.meta["kind"] != "sbm":
            continue
        n = w.graph.n
        if n <= 2048:
            small.append((n, i, w))
            small = sorted(small, key=lambda x: x[:2])[:2]
        elif n > 16000 and (large is None or (n, i) < large[:2]):
            large = (n, i, w)
    pick = [s for s in small] + [large]
    with open(OUT, "w") as f:
        f.write("# Oracle (FP64, straightforward summation of Sec. 3 eq. KuramotoGraph, classical RK4 of Sec. 2,\n")
        f.write("# unwrapped phases) on SBM instances of gen.batch_instances_iter() (256 instances, seed 1004):\n")
        f.write("# the two smallest SBM instances and the smallest above 16000 nodes; inputs theta0, omega, K\n")
        f.write("# and dt rounded to FP32; %d steps; written by tests/golden/make_batch_sbm_instances.py\n" % STEPS)
        f.write("# 'instance <index> <n> <K as run>' starts a block; 'r <step> <r>' every %d steps;\n" % R_EVERY)
        f.write("# 'theta <row> <theta(T)> <sensitivity>' (instance-local user row; the sensitivity is the\n")
        f.write("# largest |change of theta(T)| over two runs with inputs perturbed by relative 2^-24)\n")
        for n, i, w in pick:
            t0 = time.time()
            K = float(np.float32(w.K))
            om, th0, dt = f32(w.omega), f32(w.theta0), float(np.float32(DT))
            th, r, _ = oracle.rk4(w.graph, om, K, th0, dt, STEPS, r_every=R_EVERY)
            spread = np.zeros(n)
            rng = np.random.default_rng(4242 + i)
            for _ in range(2):
                u = 2.0 ** -24
                thp, _, _ = oracle.rk4(w.graph, om * (1 + u * rng.standard_normal(n)), K,
                                       th0 * (1 + u * rng.standard_normal(n)), dt, STEPS)
                d = np.abs(np.remainder(thp - th + np.pi, 2 * np.pi) - np.pi)
                spread = np.maximum(spread, d)
            f.write("instance %d %d %.17g\n" % (i, n, K))
            for s in range(len(r)):
                f.write("r %d %.17g\n" % (s * R_EVERY, r[s]))
            for m in sample_rows(i, n):
                f.write("theta %d %.17g %.6g\n" % (m, th[m], spread[m]))
            print("instance %d (n = %d, K = %.4f): %.0f s, r(T) %.4f" % (i, n, K, time.time() - t0, r[-1]),
                  flush=True)


if __name__ == "__main__":
    main()
