"""Write the oracle's discrete adjoint of a down-scaled adjoint workload into tests/golden/.

The workload is the adjoint workload on a smaller graph: gen.sbm_equal(n_comm=4) (N = 4096 in 4
planted communities of 1024 nodes, intra pair probability 0.97, cross pair probability 2e-4,
nodes permuted, omega ~ N(0, 1), theta0 ~ U[0, 2 pi), K = 4, dt = 0.01, seed 1002), 200 RK4
steps, and the loss L = (1 - r(T))^2 + (1/N) sum_m 2 (1 - cos(theta_m(T) - target_m)) with the
workload's seeded target phases (oracle.loss_and_seed). The oracle integrates (Sec. 3 eq.
KuramotoGraph, classical RK4 of Sec. 2, FP64) and runs the discrete adjoint of its own RK4 with
the whole trajectory stored.

Two fixtures, one per input precision:
  sbm4x1024_adjoint_200_f64in.txt   FP64 theta0, omega, K, dt
  sbm4x1024_adjoint_200_f32in.txt   theta0, omega, K and dt rounded to FP32 (the oracle still
                                    runs in FP64)
Each holds L, dL/dK, and for a seeded 1/4 of the rows (user order) theta(T), dL/dtheta0 and
dL/domega.

Only gen and oracle are used. Runs on the CPU (about two minutes on 8 cores):

    python tests/golden/make_sbm4x1024_adjoint.py
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

STEPS = 200
ROW_SEED = 4


def workload():
    return gen.sbm_equal(n_comm=4, steps=STEPS)


def sample_rows(n: int) -> np.ndarray:
    return np.sort(np.random.default_rng(ROW_SEED).choice(n, n // 4, replace=False))


def f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def write(path, w, omega, theta0, K, dt, label):
    t0 = time.time()
    thT, _, _ = oracle.rk4(w.graph, omega, K, theta0, dt, STEPS)
    L, seed = oracle.loss_and_seed(thT, w.target)
    gt, gw, gk = oracle.adjoint_rk4(w.graph, omega, K, theta0, dt, STEPS, seed)
    rows = sample_rows(w.graph.n)
    with open(path, "w") as f:
        f.write("# Oracle discrete adjoint of its RK4 (FP64) on gen.sbm_equal(n_comm=4): N = %d, %d steps,\n"
                % (w.graph.n, STEPS))
        f.write("# loss (1 - r(T))^2 + mean chordal distance 2 (1 - cos(theta(T) - target)) to the seeded target.\n")
        f.write("# inputs: %s; K = %.17g, dt = %.17g\n" % (label, K, dt))
        f.write("# written by tests/golden/make_sbm4x1024_adjoint.py (gen + oracle only)\n")
        f.write("# 'L <loss>', 'gK <dL/dK>', then 'row <m> <theta(T)> <dL/dtheta0> <dL/domega>' for a\n")
        f.write("# seeded 1/4 of the rows\n")
        f.write("L %.17g\n" % L)
        f.write("gK %.17g\n" % gk)
        for m in rows:
            f.write("row %d %.17g %.17g %.17g\n" % (m, thT[m], gt[m], gw[m]))
    print("%s: %.0f s, L %.6f, dL/dK %.3e" % (os.path.basename(path), time.time() - t0, L, gk), flush=True)


def main():
    w = workload()
    assert w.graph.n == 4096
    write(os.path.join(HERE, "sbm4x1024_adjoint_200_f64in.txt"), w, w.omega, w.theta0, w.K, w.dt, "FP64")
    write(os.path.join(HERE, "sbm4x1024_adjoint_200_f32in.txt"), w, f32(w.omega), f32(w.theta0),
          float(np.float32(w.K)), float(np.float32(w.dt)), "theta0, omega, K, dt rounded to FP32")


if __name__ == "__main__":
    main()
