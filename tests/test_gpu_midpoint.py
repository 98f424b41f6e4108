"""GPU tests of kur_step_midpoint (implicit midpoint rule by fixed-point iteration) against the
oracle's midpoint integrator on the same inputs: FP64 unwrapped phases within 1e-12 relative,
FP32 wrapped phases and r within 1e-5 after 200 steps; time symmetry of the converged rule;
a run that continues an RK4 run; batches."""
import numpy as np
import pytest

import oracle
from paper_2102_07167_amd import Kuramoto

from test_gpu_adjoint import ragged_sbm
from test_gpu_batch import small_instances

pytestmark = pytest.mark.gpu
TWO_PI = 2 * np.pi


def wrap(x):
    return np.remainder(x + np.pi, TWO_PI) - np.pi


def ctx(w, dtype, opts=None):
    k = Kuramoto(dtype, device=0)
    for key, v in (opts or {}).items():
        k.set_option(key, v)
    k.set_graph(w.graph)
    k.set_params(w.omega, w.K)
    k.set_phases(w.theta0)
    return k


@pytest.mark.parametrize("iters", [1, 2, 6])
@pytest.mark.parametrize("opts", [dict(), dict(chunk=64, tile_rows=64, flat_min_vec=0.5), dict(scaling=1)])
def test_midpoint_fp64_matches_oracle(need_gpu, iters, opts):
    w = ragged_sbm(41)
    steps, r_every = 100, 10
    with ctx(w, "f64", opts) as k:
        r, _ = k.step_midpoint(w.dt, steps, iters, r_every)
        th = k.get_phases(wrapped=False)
    tho, ro, _ = oracle.midpoint(w.graph, w.omega, w.K, w.theta0, w.dt, steps, iters, r_every=r_every,
                                 scaling=opts.get("scaling", 0))
    assert np.abs(th - tho).max() <= 1e-12 * max(1.0, np.abs(tho).max())
    assert np.abs(r - ro).max() < 1e-12


def test_midpoint_fp32_matches_oracle(need_gpu):
    w = ragged_sbm(42)
    w.omega = w.omega.astype(np.float32).astype(np.float64)
    w.theta0 = w.theta0.astype(np.float32).astype(np.float64)
    steps = 200
    with ctx(w, "f32") as k:
        r, _ = k.step_midpoint(w.dt, steps, 6, 20)
        th = k.get_phases()
    dt32 = float(np.float32(w.dt))
    tho, ro, _ = oracle.midpoint(w.graph, w.omega, float(np.float32(w.K)), w.theta0, dt32, steps, 6, r_every=20)
    assert np.abs(wrap(th - tho)).max() < 1e-5
    assert np.abs(r - ro).max() < 1e-5


def test_midpoint_is_time_symmetric(need_gpu):
    w = ragged_sbm(43)
    with ctx(w, "f64") as k:
        k.step_midpoint(0.05, 20, 40)
        k.step_midpoint(-0.05, 20, 40)
        th = k.get_phases(wrapped=False)
    assert np.abs(th - w.theta0).max() < 1e-11


def test_midpoint_continues_an_rk4_run(need_gpu):
    w = ragged_sbm(44)
    with ctx(w, "f64") as k:
        k.step_rk4(w.dt, 10)
        k.step_midpoint(w.dt, 10, 5)
        k.step_rk4(w.dt, 7, r_every=7)
        th = k.get_phases(wrapped=False)
    t1, _, _ = oracle.rk4(w.graph, w.omega, w.K, w.theta0, w.dt, 10)
    t2, _, _ = oracle.midpoint(w.graph, w.omega, w.K, t1, w.dt, 10, 5)
    t3, _, _ = oracle.rk4(w.graph, w.omega, w.K, t2, w.dt, 7)
    assert np.abs(th - t3).max() <= 1e-12 * max(1.0, np.abs(t3).max())


def test_midpoint_on_a_batch(need_gpu):
    inst = small_instances(seed=12, count=5)
    dt, steps = 0.01, 80
    with Kuramoto("f64", device=0) as k:
        k.set_batch(inst)
        rf = k.batch_info()
        k.step_midpoint(dt, steps, 4)
        th = k.get_phases()
    for i, (g, K, om, th0) in enumerate(inst):
        tho, _, _ = oracle.midpoint(g, om, K, th0, dt, steps, 4)
        assert np.abs(wrap(th[rf[i]:rf[i + 1]] - tho)).max() < 1e-12 * max(1.0, np.abs(tho).max()), i
