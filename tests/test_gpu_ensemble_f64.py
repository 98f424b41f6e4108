"""GPU tests of the shared-graph ensemble path in FP64: the dense products on the FP64 matrix
cores (exact 0/1 entries, FP64 accumulation) plus CSR rows for the rest. Every checked replica
is compared with the oracle integrating it alone on the same inputs.

Tolerances (FP64 path, FP64 oracle; the two differ only in the order of the sums): right-hand
side |F - F_o| <= 1e-12 max|F_o|; wrapped phases and r within 1e-12 after 200 RK4 steps; the
two ways of forming the dense-block sums (matrix cores or CSR rows) agree to the same 1e-12."""
import numpy as np
import pytest

import gen
import oracle
from paper_2102_07167_amd import Kuramoto

pytestmark = pytest.mark.gpu
TWO_PI = 2 * np.pi


def wrap(x):
    return np.remainder(x + np.pi, TWO_PI) - np.pi


def ragged_graph(seed=12):
    rng = np.random.default_rng(seed)
    sizes = np.array([300, 1, 97, 1000, 33, 257, 130])
    rho = np.array([0.9, 0.5, 0.35, 0.7, 1.0, 0.55, 0.3])
    n = int(sizes.sum())
    return gen.sbm(sizes, rho, 0.01, key=9090 + seed, uperm=rng.permutation(n).astype(np.int32))


def paired_graph(seed=21):
    """Dense off-diagonal blocks 0-2, 1-3 and 4-5 next to the diagonal ones, and a partner
    below 32 nodes (block 6)."""
    rng = np.random.default_rng(seed)
    sizes = [300, 97, 257, 130, 64, 96, 20]
    V = np.zeros((7, 7), dtype=np.int32)
    for a, c in [(0, 0), (1, 1), (2, 2), (3, 3), (5, 5), (6, 6), (0, 2), (1, 3), (4, 5), (2, 6)]:
        V[a, c] = V[c, a] = 1
    n = sum(sizes)
    return gen.block_model(sizes, V, 0.1, 1, rng, uperm=rng.permutation(n).astype(np.int32))


def replicas(n, B, seed=3):
    rng = np.random.default_rng(seed)
    K = np.linspace(0.5, 6.0, B)
    om = rng.standard_normal((B, n))
    th = rng.uniform(0, TWO_PI, (B, n))
    return K, om, th


def ens_ctx(g, tau, K, om, th):
    k = Kuramoto("f64", device=0)
    k.set_option("ens_tau", tau)
    k.ens_set_graph(g)
    k.ens_set_params(K, om)
    k.ens_set_phases(th)
    return k


def checked(B):
    return sorted(set([0, B - 1, B // 2, min(B - 1, 63), min(B - 1, 64)]))


@pytest.mark.parametrize("tau", [0.0, 0.5, 2.0])
@pytest.mark.parametrize("B", [1, 70, 200])
def test_ens_f64_rhs_matches_oracle(need_gpu, tau, B):
    g = ragged_graph()
    K, om, th = replicas(g.n, B)
    with ens_ctx(g, tau, K, om, th) as k:
        info = k.ens_info()
        if tau == 0.0:
            assert info["gemm_blocks"] == 6 and info["gemm_rows"] == g.n - 1
        F = k.ens_eval_rhs()
        th_back = k.ens_get_phases(wrapped=False)
    assert np.abs(th_back - th).max() <= 1e-15 * TWO_PI
    for e in checked(B):
        Fo = oracle.rhs(g, om[e], float(K[e]), th[e])
        assert np.abs(F[e] - Fo).max() <= 1e-12 * np.abs(Fo).max(), (e, np.abs(F[e] - Fo).max())


@pytest.mark.parametrize("tau", [0.0, 0.5])
def test_ens_f64_rk4_matches_oracle(need_gpu, tau):
    g = ragged_graph(13)
    B, dt, steps, r_every = 70, 0.01, 200, 10
    K, om, th = replicas(g.n, B, seed=5)
    with ens_ctx(g, tau, K, om, th) as k:
        r, psi = k.ens_step(dt, steps, r_every)
        thT = k.ens_get_phases(wrapped=False)
    assert r.shape == (steps // r_every + 1, B) and np.isfinite(r).all()
    for e in checked(B):
        tho, ro, _ = oracle.rk4(g, om[e], float(K[e]), th[e], dt, steps, r_every=r_every)
        assert np.abs(wrap(thT[e] - tho)).max() < 1e-12, (e, np.abs(wrap(thT[e] - tho)).max())
        assert np.abs(r[:, e] - ro).max() < 1e-12, e


def test_ens_f64_matrix_cores_agree_with_csr(need_gpu):
    g = ragged_graph(14)
    B, dt, steps = 130, 0.01, 200
    K, om, th = replicas(g.n, B, seed=6)
    out = {}
    for tau in (0.0, 2.0):
        with ens_ctx(g, tau, K, om, th) as k:
            r, _ = k.ens_step(dt, steps, 50)
            out[tau] = (k.ens_get_phases(), r)
    assert np.abs(wrap(out[0.0][0] - out[2.0][0])).max() < 1e-12
    assert np.abs(out[0.0][1] - out[2.0][1]).max() < 1e-12


@pytest.mark.parametrize("tau", [0.0, 0.5])
def test_ens_f64_dense_offdiagonal_blocks(need_gpu, tau):
    g = paired_graph()
    B = 130
    K, om, th = replicas(g.n, B, seed=8)
    with ens_ctx(g, tau, K, om, th) as k:
        if tau == 0.5:
            assert k.ens_info()["offdiag_blocks"] == 6
        F = k.ens_eval_rhs()
        r, _ = k.ens_step(0.01, 100, 50)
        thT = k.ens_get_phases()
    for e in checked(B):
        Fo = oracle.rhs(g, om[e], float(K[e]), th[e])
        assert np.abs(F[e] - Fo).max() <= 1e-12 * np.abs(Fo).max(), e
        tho, ro, _ = oracle.rk4(g, om[e], float(K[e]), th[e], 0.01, 100, r_every=50)
        assert np.abs(wrap(thT[e] - tho)).max() < 1e-12, e
        assert np.abs(r[:, e] - ro).max() < 1e-12, e


def test_ens_f64_equals_single_system_path(need_gpu):
    """Replica e of the FP64 ensemble against the single-system FP64 path on the same graph."""
    g = ragged_graph(15)
    B, dt, steps = 64, 0.01, 100
    K, om, th = replicas(g.n, B, seed=7)
    with ens_ctx(g, 0.5, K, om, th) as k:
        k.ens_step(dt, steps)
        thE = k.ens_get_phases()
    for e in (0, 31, 63):
        with Kuramoto("f64", device=0) as s:
            s.set_graph(g)
            s.set_params(om[e], float(K[e]))
            s.set_phases(th[e])
            s.step_rk4(dt, steps)
            assert np.abs(wrap(s.get_phases() - thE[e])).max() < 1e-12, e


def test_ens_f64_sbm_64x1024_sampled(need_gpu):
    """The equal-community SBM (64 x 1024, rho 0.97) with 128 replicas in FP64: sampled rows
    of the right-hand side against the oracle, and mean(theta - theta0 - t omega) conserved
    over 20 steps for every replica (symmetric A)."""
    w = gen.sbm_equal(steps=20, seed=1002)
    g = w.graph
    B = 128
    K, om, th = replicas(g.n, B, seed=11)
    rows = np.sort(np.random.default_rng(1).choice(g.n, 64, replace=False))
    with ens_ctx(g, 0.5, K, om, th) as k:
        assert k.ens_info()["gemm_blocks"] == 64
        F = k.ens_eval_rhs()
        k.ens_step(0.01, 20)
        thT = k.ens_get_phases(wrapped=False)
    for e in (0, 50, 100, 127):
        Fo = oracle.rhs_rows(g, om[e], float(K[e]), th[e], rows)
        assert np.abs(F[e, rows] - Fo).max() <= 1e-12 * np.abs(Fo).max(), e
    drift = np.abs(np.mean(thT - th - 0.2 * om, axis=1))
    assert drift.max() < 1e-11, drift.max()
