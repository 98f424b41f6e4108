"""GPU tests of the shared-graph ensemble path: matrix-core products of the dense blocks
(bitmask A, X split exactly into three bf16 terms, FP32 accumulation) plus CSR rows for the
rest. Every checked replica is compared with the oracle integrating it alone on the same
FP32-rounded inputs.

Tolerances (FP32 path, FP64 oracle): right-hand side |F - F_o| <= 1e-5 max|F_o|; wrapped
phases <= 1e-5 and r <= 1e-5 after 200 RK4 steps (the bound stated for 1000 steps); the two
ways of forming the dense-block sums (matrix cores or CSR rows) agree to the same 1e-5."""
import numpy as np
import pytest

import gen
import oracle
from paper_2102_07167_amd import Kuramoto

pytestmark = pytest.mark.gpu
TWO_PI = 2 * np.pi


def wrap(x):
    return np.remainder(x + np.pi, TWO_PI) - np.pi


def f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def ragged_graph(seed=12):
    rng = np.random.default_rng(seed)
    sizes = np.array([300, 1, 97, 1000, 33, 257, 130])
    rho = np.array([0.9, 0.5, 0.35, 0.7, 1.0, 0.55, 0.3])
    n = int(sizes.sum())
    return gen.sbm(sizes, rho, 0.01, key=9090 + seed, uperm=rng.permutation(n).astype(np.int32))


def replicas(n, B, seed=3):
    rng = np.random.default_rng(seed)
    K = f32(np.linspace(0.5, 6.0, B))
    om = f32(rng.standard_normal((B, n)))
    th = f32(rng.uniform(0, TWO_PI, (B, n)))
    return K, om, th


def ens_ctx(g, tau, K, om, th):
    k = Kuramoto("f32", device=0)
    k.set_option("ens_tau", tau)
    k.ens_set_graph(g)
    k.ens_set_params(K, om)
    k.ens_set_phases(th)
    return k


def checked(B):
    return sorted(set([0, B - 1, B // 2, min(B - 1, 63), min(B - 1, 64)]))


@pytest.mark.parametrize("tau", [0.0, 0.5, 2.0])
@pytest.mark.parametrize("B", [1, 70, 200])
def test_ens_rhs_matches_oracle(need_gpu, tau, B):
    g = ragged_graph()
    K, om, th = replicas(g.n, B)
    with ens_ctx(g, tau, K, om, th) as k:
        info = k.ens_info()
        assert info["B"] == B and info["Bp"] == (B + 63) // 64 * 64
        if tau == 0.0:
            assert info["gemm_blocks"] == 6 and info["gemm_rows"] == g.n - 1
        if tau == 2.0:
            assert info["gemm_blocks"] == 0
        F = k.ens_eval_rhs()
    for e in checked(B):
        Fo = oracle.rhs(g, om[e], float(K[e]), th[e])
        assert np.abs(F[e] - Fo).max() <= 1e-5 * np.abs(Fo).max(), (e, np.abs(F[e] - Fo).max())


@pytest.mark.parametrize("tau", [0.0, 0.5])
def test_ens_rk4_matches_oracle(need_gpu, tau):
    g = ragged_graph(13)
    B, dt, steps, r_every = 70, 0.01, 200, 10
    K, om, th = replicas(g.n, B, seed=5)
    with ens_ctx(g, tau, K, om, th) as k:
        r, psi = k.ens_step(dt, steps, r_every)
        thT = k.ens_get_phases(wrapped=False)
    assert r.shape == (steps // r_every + 1, B) and np.isfinite(r).all()
    dt32 = float(np.float32(dt))
    for e in checked(B):
        tho, ro, po = oracle.rk4(g, om[e], float(K[e]), th[e], dt32, steps, r_every=r_every)
        assert np.abs(wrap(thT[e] - tho)).max() < 1e-5, e
        assert np.abs(r[:, e] - ro).max() < 1e-5, e


def test_ens_matrix_cores_agree_with_csr(need_gpu):
    g = ragged_graph(14)
    B, dt, steps = 130, 0.01, 200
    K, om, th = replicas(g.n, B, seed=6)
    out = {}
    for tau in (0.0, 2.0):
        with ens_ctx(g, tau, K, om, th) as k:
            r, _ = k.ens_step(dt, steps, 50)
            out[tau] = (k.ens_get_phases(), r)
    assert np.abs(wrap(out[0.0][0] - out[2.0][0])).max() < 1e-5
    assert np.abs(out[0.0][1] - out[2.0][1]).max() < 1e-5


def test_ens_equals_single_system_path(need_gpu):
    """Replica e of the ensemble against the single-system FP32 path on the same graph."""
    g = ragged_graph(15)
    B, dt, steps = 64, 0.01, 100
    K, om, th = replicas(g.n, B, seed=7)
    with ens_ctx(g, 0.5, K, om, th) as k:
        k.ens_step(dt, steps)
        thE = k.ens_get_phases()
    for e in (0, 31, 63):
        with Kuramoto("f32", device=0) as s:
            s.set_graph(g)
            s.set_params(om[e], float(K[e]))
            s.set_phases(th[e])
            s.step_rk4(dt, steps)
            assert np.abs(wrap(s.get_phases() - thE[e])).max() < 1e-5, e


def test_ens_one_full_block_and_small_blocks(need_gpu):
    """A single all-to-all community of 700 (rho = 1), and blocks of 2 and 3 nodes."""
    rng = np.random.default_rng(9)
    for sizes, rho in (([700], [1.0]), ([2, 3, 2, 40], [1.0, 1.0, 0.0, 0.6])):
        sizes = np.array(sizes)
        n = int(sizes.sum())
        g = gen.sbm(sizes, np.array(rho), 0.2 if len(sizes) > 1 else 0.0, key=31,
                    uperm=rng.permutation(n).astype(np.int32))
        B = 5
        K, om, th = replicas(n, B, seed=8)
        with ens_ctx(g, 0.0, K, om, th) as k:
            F = k.ens_eval_rhs()
            k.ens_step(0.01, 100)
            thT = k.ens_get_phases()
        for e in range(B):
            Fo = oracle.rhs(g, om[e], float(K[e]), th[e])
            assert np.abs(F[e] - Fo).max() <= 1e-5 * np.abs(Fo).max(), e
            tho, _, _ = oracle.rk4(g, om[e], float(K[e]), th[e], float(np.float32(0.01)), 100)
            assert np.abs(wrap(thT[e] - tho)).max() < 1e-5, e


def test_ens_sbm_64x1024_sampled(need_gpu):
    """The equal-community SBM (64 x 1024, rho 0.97, p_out 2e-4) with 128 replicas: sampled rows
    of the right-hand side of four replicas against the oracle, and conservation of
    mean(theta - theta0 - t omega) over 50 steps for every replica (symmetric A)."""
    w = gen.sbm_equal(steps=50, seed=1002)
    g = w.graph
    B = 128
    K, om, th = replicas(g.n, B, seed=11)
    rows = np.sort(np.random.default_rng(1).choice(g.n, 64, replace=False))
    with ens_ctx(g, 0.5, K, om, th) as k:
        assert k.ens_info()["gemm_blocks"] == 64
        F = k.ens_eval_rhs()
        k.ens_step(0.01, 50)
        thT = k.ens_get_phases(wrapped=False)
    for e in (0, 50, 100, 127):
        Fo = oracle.rhs_rows(g, om[e], float(K[e]), th[e], rows)
        assert np.abs(F[e, rows] - Fo).max() <= 1e-5 * np.abs(Fo).max(), e
    T = 50 * float(np.float32(0.01))
    drift = np.abs(np.mean(thT - th - T * om, axis=1))
    assert drift.max() < 2e-5, drift.max()


def paired_graph(seed=21):
    """Dense off-diagonal blocks 0-2 (0.9), 1-3 (0.9), a sparse community 4 with a dense
    partner 5, and a partner below 32 nodes (block 6)."""
    rng = np.random.default_rng(seed)
    sizes = [300, 97, 257, 130, 64, 96, 20]
    V = np.zeros((7, 7), dtype=np.int32)
    for a, c in [(0, 0), (1, 1), (2, 2), (3, 3), (5, 5), (6, 6), (0, 2), (1, 3), (4, 5), (2, 6)]:
        V[a, c] = V[c, a] = 1
    n = sum(sizes)
    return gen.block_model(sizes, V, 0.1, 1, rng, uperm=rng.permutation(n).astype(np.int32))


@pytest.mark.parametrize("tau", [0.0, 0.5, 2.0])
@pytest.mark.parametrize("B", [1, 130])
def test_ens_dense_offdiagonal_blocks(need_gpu, tau, B):
    """Off-diagonal dense blocks on the matrix cores (accumulated with the row block's own
    product in one pass along k) against the oracle: RHS, then 100 RK4 steps."""
    g = paired_graph()
    K, om, th = replicas(g.n, B, seed=8)
    with ens_ctx(g, tau, K, om, th) as k:
        info = k.ens_info()
        if tau == 0.5:
            assert info["offdiag_blocks"] == 6  # 0-2, 1-3, 4-5 both ways
        F = k.ens_eval_rhs()
        r, _ = k.ens_step(0.01, 100, 50)
        thT = k.ens_get_phases()
    for e in checked(B):
        Fo = oracle.rhs(g, om[e], float(K[e]), th[e])
        assert np.abs(F[e] - Fo).max() <= 1e-5 * np.abs(Fo).max(), (e, np.abs(F[e] - Fo).max())
        tho, ro, _ = oracle.rk4(g, om[e], float(K[e]), th[e], float(np.float32(0.01)), 100, r_every=50)
        assert np.abs(wrap(thT[e] - tho)).max() < 1e-5
        assert np.abs(r[:, e] - ro).max() < 1e-5


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_ens_autotune_then_matches_oracle(need_gpu, dtype):
    """kur_ens_autotune_csr times whole RK4 steps for candidate thresholds (effort 0: 0, 0.5 and
    2, the last putting no block on the matrix cores), installs the graph with the fastest and
    leaves the replicas unset; the installed layout then matches the oracle at the dtype's bound."""
    g = paired_graph(23)
    B = 70
    K, om, th = replicas(g.n, B, seed=10)
    tol = 1e-5 if dtype == "f32" else 1e-12
    with Kuramoto(dtype, device=0) as k:
        rep = k.ens_autotune(g, B, 0)
        assert rep["ens_tau"] in (0.0, 0.5, 2.0) and 2 <= rep["timed"] <= 3
        assert rep["ms_per_step"] > 0
        assert rep["ms_per_step"] <= np.nanmin([rep["ms_all_gemm"], rep["ms_no_gemm"]]) + 1e-9
        info = k.ens_info()
        assert info["B"] == 0
        if rep["ens_tau"] == 2.0:
            assert info["gemm_blocks"] == 0
        else:
            assert info["gemm_blocks"] > 0
        k.ens_set_params(K, om)
        k.ens_set_phases(th)
        F = k.ens_eval_rhs()
        k.ens_step(0.01, 50)
        thT = k.ens_get_phases()
    dt = float(np.float32(0.01)) if dtype == "f32" else 0.01
    for e in (0, 35, 69):
        Fo = oracle.rhs(g, om[e], float(K[e]), th[e])
        assert np.abs(F[e] - Fo).max() <= tol * np.abs(Fo).max(), e
        tho, _, _ = oracle.rk4(g, om[e], float(K[e]), th[e], dt, 50)
        assert np.abs(wrap(thT[e] - tho)).max() < tol, e
