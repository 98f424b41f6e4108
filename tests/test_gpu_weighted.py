"""GPU tests of integer-weighted graphs (0/1 layers per block, prevalent value as the number of
layers evaluated with localised order parameters, weighted inter-block edges): right-hand side,
RK4 trajectory, implicit midpoint rule, adjoint and potential against the oracle on the same
weighted adjacency. Tolerances as for 0/1 graphs (FP64 1e-12, FP32 1e-5, adjoint 1e-10)."""
import numpy as np
import pytest

import gen
import oracle
from paper_2102_07167_amd import Kuramoto

pytestmark = pytest.mark.gpu
TWO_PI = 2 * np.pi


def wrap(x):
    return np.remainder(x + np.pi, TWO_PI) - np.pi


def weighted_graph(seed=71):
    rng = np.random.default_rng(seed)
    sizes = [150, 1, 97, 260, 33]
    n = sum(sizes)
    g = gen.weighted_sbm(sizes, [3, 0, 0, 2, 5], 0.2, 5, 0.02, rng, uperm=rng.permutation(n).astype(np.int32))
    return g, rng.standard_normal(n), rng.uniform(0, TWO_PI, n)


def ctx(g, dtype, om, K, th, opts=None):
    k = Kuramoto(dtype, device=0)
    for key, v in (opts or {}).items():
        k.set_option(key, v)
    k.set_graph(g)
    k.set_params(om, K)
    k.set_phases(th)
    return k


@pytest.mark.parametrize("opts", [dict(), dict(chunk=64, tile_rows=64, flat_min_vec=0.5), dict(scaling=1)])
def test_weighted_fp64_rhs_and_rk4(need_gpu, opts):
    g, om, th = weighted_graph()
    K, dt, steps = 0.8, 0.01, 100
    sc = opts.get("scaling", 0)
    with ctx(g, "f64", om, K, th, opts) as k:
        info = k.graph_info()
        assert info["symmetric"] == 1 and info["dense_blocks"] == 3
        F = k.eval_rhs()
        k.step_rk4(dt, steps)
        thT = k.get_phases(wrapped=False)
    Fo = oracle.rhs(g, om, K, th, scaling=sc)
    assert np.abs(F - Fo).max() <= 1e-12 * np.abs(Fo).max()
    tho, _, _ = oracle.rk4(g, om, K, th, dt, steps, scaling=sc)
    assert np.abs(thT - tho).max() <= 1e-12 * max(1.0, np.abs(tho).max())


def test_weighted_fp32_rk4(need_gpu):
    g, om, th = weighted_graph(72)
    om, th = om.astype(np.float32).astype(np.float64), th.astype(np.float32).astype(np.float64)
    with ctx(g, "f32", om, 0.8, th) as k:
        r, _ = k.step_rk4(0.01, 200, r_every=20)
        thT = k.get_phases()
    tho, ro, _ = oracle.rk4(g, om, float(np.float32(0.8)), th, float(np.float32(0.01)), 200, r_every=20)
    assert np.abs(wrap(thT - tho)).max() < 1e-5
    assert np.abs(r - ro).max() < 1e-5


def test_weighted_midpoint_adjoint_and_potential(need_gpu):
    g, om, th = weighted_graph(73)
    K, dt = 0.8, 0.02
    with ctx(g, "f64", om, K, th) as k:
        d = k.diagnostics()
        k.step_midpoint(dt, 20, 5)
        thm = k.get_phases(wrapped=False)
        seed = np.random.default_rng(1).standard_normal(g.n)
        gt, gw, gk = k.adjoint_rk4(dt, 25, seed, theta0=th, ckpt_every=6)
    Vo = oracle.potential(g, om, K, th)
    assert abs(d["V"] - Vo) <= 1e-12 * (np.abs(om * th).sum() + K * g.dense().sum() / g.n)
    tmo, _, _ = oracle.midpoint(g, om, K, th, dt, 20, 5)
    assert np.abs(thm - tmo).max() <= 1e-12 * max(1.0, np.abs(tmo).max())
    go = oracle.adjoint_rk4(g, om, K, th, dt, 25, seed)
    assert np.abs(gt - go[0]).max() <= 1e-10 * np.abs(go[0]).max()
    assert np.abs(gw - go[1]).max() <= 1e-10 * np.abs(go[1]).max()
    assert abs(gk - go[2]) <= 1e-10 * max(abs(go[2]), np.abs(go[1]).max())
