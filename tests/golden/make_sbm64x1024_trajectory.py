"""Write the oracle's phases after 1000 RK4 steps of the 64 x 1024 SBM workload into tests/golden/.

The workload is the equal-community stochastic block model of gen.sbm_equal() (N = 65536 in 64
planted communities of 1024 nodes, intra pair probability 0.97, cross pair probability 2e-4,
nodes randomly permuted, omega ~ N(0, 1), theta0 ~ U[0, 2 pi), K = 4, dt = 0.01, seed 1002).
The right-hand side is Sec. 3, eq. KuramotoGraph with uniform scaling K/N; the integrator is the
classical RK4 of Sec. 2 on unwrapped phases.

Two fixtures are written, one per input precision:
  sbm64x1024_rk4_1000_f64in.txt   FP64 theta0, omega, K, dt
  sbm64x1024_rk4_1000_f32in.txt   theta0, omega, K and dt first rounded to FP32 (the inputs an FP32
                                  run sees); the oracle still integrates in FP64
Each holds the order parameter r, psi (Sec. 2, eq. OrderParameter) every 10 steps over all rows,
and the unwrapped theta(T) of a seeded 1/16 of the rows (user order).

Only gen and oracle are used: nothing here comes from the GPU library. Runs on the CPU, about
17 minutes per fixture on 8 cores:

    python tests/golden/make_sbm64x1024_trajectory.py
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

STEPS = 1000
R_EVERY = 10
ROW_SEED = 16


def sample_rows(n: int) -> np.ndarray:
    return np.sort(np.random.default_rng(ROW_SEED).choice(n, n // 16, replace=False))


def f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def write(path, w, omega, theta0, K, dt, label):
    t0 = time.time()
    th, r, psi = oracle.rk4(w.graph, omega, K, theta0, dt, STEPS, r_every=R_EVERY)
    rows = sample_rows(w.graph.n)
    with open(path, "w") as f:
        f.write("# Oracle (FP64, straightforward summation of Sec. 3 eq. KuramotoGraph, classical RK4 of Sec. 2,\n")
        f.write("# unwrapped phases) on gen.sbm_equal(): N = %d, 64 x 1024, rho_in 0.97, p_out 2e-4, seed 1002.\n"
                % w.graph.n)
        f.write("# inputs: %s; K = %.17g, dt = %.17g, %d steps\n" % (label, K, dt, STEPS))
        f.write("# written by tests/golden/make_sbm64x1024_trajectory.py (gen + oracle only)\n")
        f.write("# 'r <step> <r> <psi>': order parameter over all rows every %d steps (Sec. 2 eq. OrderParameter)\n"
                % R_EVERY)
        f.write("# 'theta <row> <theta(T)>': unwrapped phase of user row <row>, seeded 1/16 of the rows\n")
        for i in range(len(r)):
            f.write("r %d %.17g %.17g\n" % (i * R_EVERY, r[i], psi[i]))
        for m in rows:
            f.write("theta %d %.17g\n" % (m, th[m]))
    print("%s: %.0f s, max|theta| %.3f, r(T) %.6f" % (os.path.basename(path), time.time() - t0,
                                                     np.abs(th).max(), r[-1]), flush=True)


def main():
    w = gen.sbm_equal()
    assert w.steps == STEPS and w.graph.n == 65536
    write(os.path.join(HERE, "sbm64x1024_rk4_1000_f64in.txt"), w, w.omega, w.theta0, w.K, w.dt, "FP64")
    write(os.path.join(HERE, "sbm64x1024_rk4_1000_f32in.txt"), w, f32(w.omega), f32(w.theta0),
          float(np.float32(w.K)), float(np.float32(w.dt)), "theta0, omega, K, dt rounded to FP32")


if __name__ == "__main__":
    main()
