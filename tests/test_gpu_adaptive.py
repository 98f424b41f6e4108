"""GPU tests of kur_step_adaptive (variable-step embedded Runge-Kutta pair of orders 4(5))
against the oracle's integrator with the same tableau and step-size controller: in FP64 the
same accepted and rejected steps and time reached, the next step size within 1e-9 relative
(the error estimate cancels), phases within 1e-10; in FP32 (atol 1e-4) phases within 1e-4 of the FP64 oracle; exact for K = 0."""
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


@pytest.mark.parametrize("atol", [1e-5, 1e-9])
@pytest.mark.parametrize("opts", [dict(), dict(chunk=64, tile_rows=64, flat_min_vec=0.5), dict(scaling=1),
                                  dict(mask_min=0.0, chunk=512)])
def test_adaptive_fp64_matches_oracle(need_gpu, atol, opts):
    w = ragged_sbm(51)
    with ctx(w, "f64", opts) as k:
        st = k.step_adaptive(1.0, 0.3, atol)
        th = k.get_phases(wrapped=False)
    tho, sto = oracle.rkf45(w.graph, w.omega, w.K, w.theta0, 1.0, 0.3, atol, scaling=opts.get("scaling", 0))
    assert (st["accepted"], st["rejected"]) == (int(sto[2]), int(sto[3]))
    # the error estimate is a difference of nearly equal weighted sums (e ~ atol from terms of
    # size |F| h), so its rounding relative to itself is about eps |F| h / e, and the proposed
    # step carries a fifth of that
    assert abs(st["t"] - sto[0]) < 1e-12 and abs(st["dt"] - sto[1]) <= 1e-9 * sto[1]
    assert np.abs(th - tho).max() < 1e-10


def test_adaptive_fp32_close_to_oracle(need_gpu):
    w = ragged_sbm(52)
    w.omega = w.omega.astype(np.float32).astype(np.float64)
    w.theta0 = w.theta0.astype(np.float32).astype(np.float64)
    with ctx(w, "f32") as k:
        st = k.step_adaptive(2.0, 0.1, 1e-4)
        th = k.get_phases()
    tho, sto = oracle.rkf45(w.graph, w.omega, float(np.float32(w.K)), w.theta0, 2.0, 0.1, 1e-4)
    assert abs(st["t"] - 2.0) < 1e-6 and abs(st["accepted"] - sto[2]) <= 2
    assert np.abs(wrap(th - tho)).max() < 1e-4


def test_adaptive_exact_without_coupling_and_continues(need_gpu):
    w = ragged_sbm(53)
    with ctx(w, "f64") as k:
        k.set_params(w.omega, 0.0)
        st = k.step_adaptive(3.0, 0.01, 1e-8)
        th = k.get_phases(wrapped=False)
        assert st["rejected"] == 0 and st["t"] == 3.0
        assert np.abs(th - (w.theta0 + 3.0 * w.omega)).max() < 1e-12
        # continue with RK4 from the adaptive state
        k.set_params(w.omega, w.K)
        k.step_rk4(w.dt, 10)
        th2 = k.get_phases(wrapped=False)
    t2, _, _ = oracle.rk4(w.graph, w.omega, w.K, w.theta0 + 3.0 * w.omega, w.dt, 10)
    assert np.abs(th2 - t2).max() <= 1e-12 * max(1.0, np.abs(t2).max())


def test_adaptive_on_a_batch(need_gpu):
    """One common step size for the union of instances; checked against the oracle integrating
    the union (the same step decisions) instance by instance on the final phases."""
    inst = small_instances(seed=13, count=4)
    with Kuramoto("f64", device=0) as k:
        k.set_batch(inst)
        rf = k.batch_info()
        st = k.step_adaptive(0.5, 0.05, 1e-8)
        th = k.get_phases(wrapped=False)
    assert st["t"] == 0.5
    for i, (g, K, om, th0) in enumerate(inst):
        ref, _, _ = oracle.rk4(g, om, K, th0, 0.5 / 500, 500)
        assert np.abs(th[rf[i]:rf[i + 1]] - ref).max() < 1e-6, i
