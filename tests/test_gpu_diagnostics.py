"""GPU tests of kur_diagnostics: the potential V (eq. ExtendedPotentialConservation; eq.
Potential for the complete graph) against the oracle's plain double sum at the GPU's own
unwrapped phases, its decrease along RK4 trajectories of the gradient system (symmetric A,
uniform scaling), and the mean deviation of eq. Means: zero for symmetric A (eq.
KuramotoGraphConservation), the oracle's nonzero value for an asymmetric A.

Tolerances relative to S = sum_m |omega_m theta_m| + K/2 sum_m scale_m deg_m, the size of the
terms V sums: FP64 1e-12, FP32 1e-5 (FP32 coupling sums)."""
import numpy as np
import pytest

import gen
import oracle
from paper_2102_07167_amd import Kuramoto
from paper_2102_07167_amd.kur import KurError, KUR_ESTATE

from test_gpu_adjoint import ragged_sbm

pytestmark = pytest.mark.gpu


def scale_of(g, omega, K, theta, scaling):
    deg = np.diff(g.row_ptr) if not g.complete else np.full(g.n, g.n - 1)
    sc = np.where(deg > 0, 1.0 / np.maximum(deg, 1), 0.0) if scaling else np.full(g.n, 1.0 / g.n)
    return np.abs(omega * theta).sum() + 0.5 * K * (sc * deg).sum()


def ctx(g, dtype, omega, K, theta, scaling=0):
    k = Kuramoto(dtype, device=0)
    k.set_option("scaling", scaling)
    k.set_graph(g)
    k.set_params(omega, K)
    k.set_phases(theta)
    return k


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("scaling", [0, 1])
@pytest.mark.parametrize("symmetric", [True, False])
def test_potential_matches_oracle(need_gpu, dtype, scaling, symmetric):
    w = ragged_sbm(21)
    g = w.graph
    if not symmetric:
        rng = np.random.default_rng(4)
        A = g.dense()
        drop = rng.random(A.shape) < 0.2
        A[drop] = 0
        g = gen.from_dense(A, g.labels)
    om, th0 = w.omega, w.theta0
    if dtype == "f32":
        om, th0 = om.astype(np.float32).astype(np.float64), th0.astype(np.float32).astype(np.float64)
    with ctx(g, dtype, om, w.K, th0, scaling) as k:
        k.step_rk4(w.dt, 25)
        th = k.get_phases(wrapped=False)
        d = k.diagnostics()
    Vo = oracle.potential(g, om, w.K, th, scaling=scaling)
    S = scale_of(g, om, w.K, th, scaling)
    tol = 1e-12 if dtype == "f64" else 1e-5
    assert abs(d["V"] - Vo) <= tol * S, (d["V"], Vo, S)
    assert abs(d["mean_theta"] - th.mean()) <= tol * max(1.0, np.abs(th).max())
    assert abs(d["mean_omega"] - om.mean()) <= tol * max(1.0, np.abs(om).max())


def test_potential_complete_graph(need_gpu):
    rng = np.random.default_rng(8)
    n = 700
    g = gen.complete_graph(n)
    om, th = rng.standard_normal(n), rng.uniform(0, 2 * np.pi, n)
    with ctx(g, "f64", om, 2.0, th) as k:
        d = k.diagnostics()
    Vo = oracle.potential(g, om, 2.0, th)
    assert abs(d["V"] - Vo) <= 1e-12 * scale_of(g, om, 2.0, th, 0)


def test_potential_decreases_and_mean_is_conserved(need_gpu):
    """Gradient system: V(theta(t)) does not increase; (1/N) sum (theta - theta0 - t omega) = 0."""
    w = ragged_sbm(23)
    with ctx(w.graph, "f64", w.omega, 3.0, w.theta0) as k:
        d0 = k.diagnostics()
        Vs = [d0["V"]]
        for i in range(20):
            k.step_rk4(0.02, 10)
            d = k.diagnostics()
            Vs.append(d["V"])
            t = 0.02 * 10 * (i + 1)
            assert abs(d["mean_theta"] - d0["mean_theta"] - t * d0["mean_omega"]) < 1e-12
    S = scale_of(w.graph, w.omega, 3.0, w.theta0, 0)
    assert np.all(np.diff(Vs) <= 1e-12 * S), np.diff(Vs)
    assert Vs[-1] < Vs[0]


def test_mean_deviation_nonzero_for_asymmetric(need_gpu):
    rng = np.random.default_rng(5)
    n = 300
    A = (rng.random((n, n)) < 0.2).astype(np.uint8)
    np.fill_diagonal(A, 0)
    g = gen.from_dense(A, rng.integers(0, 3, n).astype(np.int32))
    om, th0 = rng.standard_normal(n), rng.uniform(0, 2 * np.pi, n)
    with ctx(g, "f64", om, 4.0, th0) as k:
        d0 = k.diagnostics()
        k.step_rk4(0.01, 100)
        d1 = k.diagnostics()
    dev = d1["mean_theta"] - d0["mean_theta"] - 1.0 * d0["mean_omega"]
    tho, _, _ = oracle.rk4(g, om, 4.0, th0, 0.01, 100)
    dev_o = np.mean(tho - th0 - 1.0 * om)
    assert abs(dev_o) > 1e-4
    assert abs(dev - dev_o) < 1e-11


def test_diagnostics_reject_batch(need_gpu):
    g = gen.complete_graph(100)
    rng = np.random.default_rng(1)
    with Kuramoto("f64", device=0) as k:
        k.set_batch([(g, 1.0, rng.standard_normal(100), rng.uniform(0, 6, 100))])
        with pytest.raises(KurError) as ei:
            k.diagnostics()
        assert ei.value.status == KUR_ESTATE
