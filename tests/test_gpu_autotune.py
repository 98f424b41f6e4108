"""GPU tests of the layout autotuner: re-tiling keeps the phase state bit for bit and every
result within the parity tolerances of the oracle (RHS, RK4 trajectory, order parameter of
every batch instance, adjoint); the full tuner stores its choice in the cache and a second
context configured from the cache builds the same layout. Tolerances as in test_gpu_parity
(FP64 1e-12 relative, FP32 1e-5 on wrapped phases) and test_gpu_adjoint (FP64 1e-10)."""
import numpy as np
import pytest

import gen
import oracle
from paper_2102_07167_amd import Kuramoto
from paper_2102_07167_amd.kur import KurError, KUR_ESTATE

from test_gpu_adjoint import ragged_sbm
from test_gpu_batch import small_instances

pytestmark = pytest.mark.gpu
TWO_PI = 2 * np.pi


def wrap(x):
    return np.remainder(x + np.pi, TWO_PI) - np.pi


@pytest.mark.parametrize("opts", [dict(), dict(mask_min=0.0, chunk=512, mask_sub=128, mask_item=20000)])
def test_tune_tiles_keeps_state_and_parity(need_gpu, opts):
    """Re-tiling (which also re-cuts the bitmask items of a layout with bitmask segments) keeps
    the state bit for bit, and the RHS, the trajectory and the adjoint stay within parity."""
    w = ragged_sbm(13)
    with Kuramoto("f64", device=0) as k:
        for key, v in opts.items():
            k.set_option(key, v)
        k.set_graph(w.graph)
        if opts:
            assert k.graph_masks()["mask_segments"] > 0
        k.set_params(w.omega, w.K)
        k.set_phases(w.theta0)
        k.step_rk4(w.dt, 5)
        s0 = k.get_state()
        rep = k.tune_tiles(1)
        assert k.get_state() == s0
        assert rep["timed"] >= 10 and 0 < rep["ms_per_step"] <= rep["ms_per_step_start"]
        th5 = k.get_phases(wrapped=False)
        F = k.eval_rhs()
        Fo = oracle.rhs(w.graph, w.omega, w.K, th5)
        assert np.abs(F - Fo).max() <= 1e-12 * np.abs(Fo).max()
        k.step_rk4(w.dt, 25)
        thT = k.get_phases(wrapped=False)
        tho, _, _ = oracle.rk4(w.graph, w.omega, w.K, w.theta0, w.dt, 30)
        assert np.abs(thT - tho).max() <= 1e-12 * max(1.0, np.abs(tho).max())
        seed = np.random.default_rng(2).standard_normal(w.graph.n)
        gt, gw, gk = k.adjoint_rk4(w.dt, 20, seed, theta0=w.theta0, ckpt_every=6)
    gt_o, gw_o, gk_o = oracle.adjoint_rk4(w.graph, w.omega, w.K, w.theta0, w.dt, 20, seed)
    assert np.abs(gt - gt_o).max() <= 1e-10 * np.abs(gt_o).max()
    assert np.abs(gw - gw_o).max() <= 1e-10 * np.abs(gw_o).max()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_tune_tiles_on_a_batch(need_gpu, dtype):
    inst = small_instances(seed=8, count=6)
    if dtype == "f32":
        inst = [(g, float(np.float32(K)), om.astype(np.float32).astype(np.float64),
                 th.astype(np.float32).astype(np.float64)) for g, K, om, th in inst]
    dt, steps, r_every = 0.01, 100, 10
    with Kuramoto(dtype, device=0) as k:
        k.set_batch(inst)
        rf = k.batch_info()
        k.tune_tiles(1)
        r, _ = k.batch_step(dt, steps, r_every)
        th = k.get_phases()
    tol = 1e-12 if dtype == "f64" else 1e-5
    for i, (g, K, om, th0) in enumerate(inst):
        thT, ro, _ = oracle.rk4(g, om, K, th0, dt, steps, r_every=r_every)
        scale = max(1.0, np.abs(thT).max()) if dtype == "f64" else 1.0
        assert np.abs(wrap(th[rf[i]:rf[i + 1]] - thT)).max() < tol * scale, i
        assert np.abs(r[:, i] - ro).max() < tol, i


def test_autotune_stores_and_reloads(need_gpu, tmp_path):
    rng = np.random.default_rng(21)
    sizes = np.array([900, 300, 1500, 64, 700, 1200])
    rho = np.array([0.35, 0.45, 0.55, 0.9, 0.65, 0.97])
    n = int(sizes.sum())
    g = gen.sbm(sizes, rho, 0.003, key=4242, uperm=rng.permutation(n).astype(np.int32))
    om, th0 = rng.standard_normal(n), rng.uniform(0, TWO_PI, n)
    om32, th32 = om.astype(np.float32).astype(np.float64), th0.astype(np.float32).astype(np.float64)
    path = str(tmp_path / "tuned.tsv")
    with Kuramoto("f32", device=0) as k:
        rep = k.autotune(g, effort=1, cache=path)
        key = k.tune_key(g)
        assert rep["cache"] == 0 and rep["builds"] >= 1 and rep["timed"] >= 10
        assert 0 < rep["ms_per_step"] <= rep["ms_per_step_start"]
        with pytest.raises(KurError) as ei:
            k.eval_rhs()
        assert ei.value.status == KUR_ESTATE
        info = k.graph_info()
        assert info["chunk"] == rep["chunk"]
        k.set_params(om32, 3.0)
        k.set_phases(th32)
        k.step_rk4(0.01, 100)
        thA = k.get_phases()
    lines = open(path).read().splitlines()
    assert len(lines) == 1 and lines[0].startswith(key + "\t") and "gfx950" in key
    tho, _, _ = oracle.rk4(g, om32, float(np.float32(3.0)), th32, float(np.float32(0.01)), 100)
    assert np.abs(wrap(thA - tho)).max() < 1e-5
    with Kuramoto("f32", device=0) as k2:
        rep2 = k2.autotune(g, effort=1, cache=path)
        assert rep2["cache"] == 1 and rep2["timed"] == 0
        for key in ("tau", "chunk", "threads", "tile_rows", "tile_min_cost", "flat_min_vec", "xcds"):
            assert rep2[key] == rep[key], key
        assert k2.graph_info() == info
        k2.set_params(om32, 3.0)
        k2.set_phases(th32)
        k2.step_rk4(0.01, 100)
        assert np.array_equal(k2.get_phases(), thA)


def test_autotune_with_dense_offdiagonal_blocks(need_gpu, tmp_path):
    """The tuner on a graph with dense off-diagonal blocks (its density thresholds also decide
    those blocks) keeps the result within the oracle's tolerance."""
    rng = np.random.default_rng(41)
    sizes = [300, 200, 257, 130]
    V = np.array([[1, 1, 0, 0], [1, 1, 0, 1], [0, 0, 1, 0], [0, 1, 0, 1]], dtype=np.int32)
    n = sum(sizes)
    g = gen.block_model(sizes, V, 0.4, 1, rng, uperm=rng.permutation(n).astype(np.int32))
    om, th = rng.standard_normal(n), rng.uniform(0, TWO_PI, n)
    with Kuramoto("f64", device=0) as k:
        rep = k.autotune(g, effort=1, cache=str(tmp_path / "cache.tsv"))
        assert rep["timed"] >= 2
        k.set_params(om, 1.5)
        F = k.eval_rhs(th)
    Fo = oracle.rhs(g, om, 1.5, th)
    assert np.abs(F - Fo).max() <= 1e-12 * np.abs(Fo).max()
