"""GPU parity: the HIP path through the C ABI against the CPU oracle on the same seeded inputs.

Tolerances (from the arithmetic and the stated targets):
  FP64 right-hand side   max |dF| <= 1e-12 * max |F_oracle|
  FP64 phases            max |wrap(dtheta)| <= 1e-12 * max(1, max |theta_oracle|)  (unwrapped scale)
  FP32 phases            max |wrap(dtheta)| <= 1e-5 after 1000 RK4 steps; the oracle integrates in FP64
                         from the FP32-rounded theta0, omega, K and dt
  FP32 right-hand side   |dG_m| <= 1e-5 * scale_m * (deg_m + 2 s_b [block of row m stores zeros])
                         where G = F - omega (rounding scale of the complement form:
                         u * (|S_b| + |C_b| + sum |terms|); summed for every column group of the row)
"""
import math

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
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def make(w, dtype, **opts):
    k = Kuramoto(dtype, device=0)
    for key, v in opts.items():
        k.set_option(key, v)
    k.set_graph(w.graph)
    k.set_params(w.omega, w.K)
    k.set_phases(w.theta0)
    return k


def rel_err(a, b):
    return np.abs(a - b).max() / max(1.0, np.abs(b).max())


def dense_term(k, g):
    """Per user row, sum over the column groups whose localised order parameters enter the row
    (its own community when that block stores its zeros, and dense off-diagonal blocks) of
    2 x group size x factor: the rounding scale |S_b| + |C_b| <= 2 s_b of the complement form,
    which rows summed straightforwardly do not carry. Blocks follow the label order."""
    if g.complete:
        return np.full(g.n, 2.0 * g.n)
    _, inv, cnt = np.unique(g.labels, return_inverse=True, return_counts=True)
    assert k.graph_info()["blocks"] == len(cnt)
    per_block = np.zeros(len(cnt))
    for b in range(len(cnt)):
        blk, md = k.block_groups(b)
        per_block[b] = 2.0 * float((cnt[blk] * md).sum())
    return per_block[inv]


def fp32_rhs_bound(k, w, theta=None):
    """Per-row rounding scale for an FP32 evaluation (see module docstring)."""
    g = w.graph
    deg = np.diff(g.row_ptr) if not g.complete else np.full(g.n, g.n - 1)
    return 1e-5 * (w.K / g.n) * (deg + dense_term(k, g)) + 1e-6 * np.abs(w.omega) + 1e-7


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_all_to_all_n512(need_gpu, dtype):
    """Classical model as one dense block with an empty list (Sec. 2, eq. KuramotoReformulation)."""
    w = gen.all_to_all()
    if dtype == "f32":
        w.omega, w.theta0, w.K, w.dt = f32(w.omega), f32(w.theta0), float(np.float32(w.K)), float(np.float32(w.dt))
    with make(w, dtype) as k:
        F = k.eval_rhs()
        Fo = oracle.rhs(w.graph, w.omega, w.K, w.theta0)
        tol = 1e-12 if dtype == "f64" else 1e-5
        assert rel_err(F, Fo) < tol
        r, psi = k.step_rk4(w.dt, w.steps, r_every=1)
        th = k.get_phases()
        tho, ro, psio = oracle.rk4(w.graph, w.omega, w.K, w.theta0, w.dt, w.steps, r_every=1)
        ptol = 1e-12 * max(1.0, np.abs(tho).max()) if dtype == "f64" else 1e-5
        assert np.abs(wrap(th - tho)).max() < ptol
        assert np.abs(r - ro).max() < (1e-12 if dtype == "f64" else 1e-5)
        assert len(r) == w.steps + 1


def small_sbm(seed=21, n_comm=8, comm_size=512, steps=1000, **kw):
    return gen.sbm_equal(n_comm=n_comm, comm_size=comm_size, rho_in=0.97, p_out=2e-3, K=4.0, dt=0.01,
                         steps=steps, seed=seed, **kw)


@pytest.mark.parametrize("flat", [0.1, 8.0])
def test_sbm_fp64_rhs_and_trajectory(need_gpu, flat):
    w = small_sbm()
    with make(w, "f64", flat_min_vec=flat) as k:
        F = k.eval_rhs()
        Fo = oracle.rhs(w.graph, w.omega, w.K, w.theta0)
        assert rel_err(F, Fo) < 1e-12
        k.step_rk4(w.dt, w.steps)
        th = k.get_phases()
    tho, _, _ = oracle.rk4(w.graph, w.omega, w.K, w.theta0, w.dt, w.steps)
    assert np.abs(wrap(th - tho)).max() < 1e-12 * max(1.0, np.abs(tho).max())


@pytest.mark.parametrize("flat", [0.1, 8.0])
def test_sbm_fp32_trajectory_1000_steps(need_gpu, flat):
    w = small_sbm()
    om, th0, Kf, dtf = f32(w.omega), f32(w.theta0), float(np.float32(w.K)), float(np.float32(w.dt))
    w.omega, w.theta0, w.K = om, th0, Kf
    with make(w, "f32", flat_min_vec=flat) as k:
        k.step_rk4(dtf, w.steps)
        th = k.get_phases()
        thw = k.get_phases(wrapped=True)
    tho, _, _ = oracle.rk4(w.graph, om, Kf, th0, dtf, w.steps)
    err = np.abs(wrap(th - tho)).max()
    assert err < 1e-5, err
    assert np.abs(wrap(thw - tho)).max() < 1e-5
    assert np.all(thw >= -np.pi) and np.all(thw < np.pi)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("opts", [dict(chunk=64, tile_rows=64), dict(tau=0.0, chunk=128), dict(tau=1.0),
                                  dict(threads=256, tile_rows=128), dict(threads=1024), dict(threads=128, tile_rows=64, chunk=128),
                                  dict(threads=128, xcds=8),
                                  dict(flat_min_vec=0.1, chunk=128, tile_rows=64), dict(flat_min_vec=0.1, tau=0.0),
                                  dict(flat_min_vec=0), dict(tile_min_cost=1), dict(tile_min_cost=1, tiles=100000),
                                  dict(xcds=8, tile_min_cost=1), dict(xcds=8, tile_rows=64, chunk=128),
                                  dict(xcds=3, tile_min_cost=64),
                                  dict(mask_min=0.0, chunk=512), dict(mask_min=0.0, chunk=512, threads=256, tile_rows=64, xcds=8),
                                  dict(mask_min=0.0, chunk=1024, threads=128), dict(mask_min=0.1, chunk=2048, flat_min_vec=0.1),
                                  dict(mask_min=0.0, chunk=1024, mask_sub=128, mask_item=1),
                                  dict(mask_min=0.0, chunk=512, tile_rows=64, mask_sub=128, mask_item=20000),
                                  dict(mask_min=0.0, chunk=2048, tile_rows=512, mask_sub=1024, mask_item=10**9)])
def test_ragged_layouts(need_gpu, dtype, opts):
    """Odd block sizes, several chunks per block, several tiles per block, all-dense and
    all-sparse evaluation, a size-1 block and a complete block; launch orders for 8 and 3 XCDs
    (tiles of a block on one XCD, empty slots in the launch order); bitmask segments, with
    bitmask items of one sub-chunk, of a few sub-chunks starting and ending inside segments, and
    of a whole tile."""
    rng = np.random.default_rng(77)
    sizes = np.array([333, 1, 129, 700, 64, 2, 515])
    rho = np.array([0.95, 0.5, 0.3, 0.75, 1.0, 1.0, 0.55])
    n = int(sizes.sum())
    g = gen.sbm(sizes, rho, 0.01, key=2024, uperm=rng.permutation(n).astype(np.int32))
    w = gen.Workload("ragged", g, rng.standard_normal(n), rng.uniform(0, TWO_PI, n), 3.0, 0.01, 50)
    if dtype == "f32":
        w.omega, w.theta0 = f32(w.omega), f32(w.theta0)
    with make(w, dtype, **opts) as k:
        F = k.eval_rhs()
        Fo = oracle.rhs(g, w.omega, w.K, w.theta0)
        if dtype == "f64":
            assert rel_err(F, Fo) < 1e-12
        else:
            assert np.all(np.abs(F - Fo) <= fp32_rhs_bound(k, w, w.theta0))
        k.step_rk4(w.dt, w.steps)
        th = k.get_phases()
    tho, _, _ = oracle.rk4(g, w.omega, w.K, w.theta0, w.dt, w.steps)
    tol = 1e-12 * max(1.0, np.abs(tho).max()) if dtype == "f64" else 1e-5
    assert np.abs(wrap(th - tho)).max() < tol


def test_asymmetric_and_degree_scaling(need_gpu):
    rng = np.random.default_rng(8)
    n = 600
    labels = rng.integers(0, 5, n).astype(np.int32)
    A = (rng.random((n, n)) < 0.02).astype(np.uint8)
    same = labels[:, None] == labels[None, :]
    A |= (same & (rng.random((n, n)) < 0.8)).astype(np.uint8)
    A[:7, :] = 0  # zero rows: theta' = omega under degree scaling
    np.fill_diagonal(A, 0)
    g = gen.from_dense(A, labels)
    omega, th0 = rng.standard_normal(n), rng.uniform(0, TWO_PI, n)
    for scaling in (0, 1):
        with Kuramoto("f64", device=0) as k:
            k.set_option("scaling", scaling)
            k.set_graph(g)
            k.set_params(omega, 2.5)
            k.set_phases(th0)
            F = k.eval_rhs()
            assert rel_err(F, oracle.rhs(g, omega, 2.5, th0, scaling=scaling)) < 1e-12
            k.step_rk4(0.02, 100)
            th = k.get_phases()
        tho, _, _ = oracle.rk4(g, omega, 2.5, th0, 0.02, 100, scaling=scaling)
        assert np.abs(wrap(th - tho)).max() < 1e-12 * max(1, np.abs(tho).max())


def test_empty_graph_and_single_node(need_gpu):
    rng = np.random.default_rng(1)
    n = 50
    g = gen.Graph(n=n, labels=rng.integers(0, 3, n).astype(np.int32), row_ptr=np.zeros(n + 1, np.int64),
                  col=np.zeros(0, np.int32))
    om, th0 = rng.standard_normal(n), rng.uniform(0, TWO_PI, n)
    with Kuramoto("f64", device=0) as k:
        k.set_graph(g)
        k.set_params(om, 5.0)
        k.set_phases(th0)
        assert np.array_equal(k.eval_rhs(), om)
        k.step_rk4(0.1, 10)
        assert np.abs(k.get_phases() - (th0 + om)).max() < 1e-13
    with Kuramoto("f32", device=0) as k:
        k.set_graph(gen.Graph(n=1, labels=np.zeros(1, np.int32), row_ptr=np.zeros(2, np.int64),
                              col=np.zeros(0, np.int32)))
        k.set_params(np.array([0.5]), 1.0)
        k.set_phases(np.array([3.0]))
        k.step_rk4(0.5, 4)
        assert abs(k.get_phases()[0] - 4.0) < 1e-6
        r, _ = k.order_parameter()
        assert abs(r - 1.0) < 1e-6


@pytest.mark.parametrize("opts", [dict(), dict(mask_min=0.0, chunk=512, mask_sub=128, mask_item=20000)])
def test_state_roundtrip_bitwise_and_determinism(need_gpu, opts):
    """A run resumed from a saved state repeats an uninterrupted run bit for bit (lists only,
    and with bitmask segments summed in items of a few sub-chunks)."""
    w = small_sbm(n_comm=4, comm_size=300, steps=40)
    for dtype in ("f32", "f64"):
        with make(w, dtype, **opts) as k1:
            k1.step_rk4(w.dt, 40)
            a = k1.get_state()
        with make(w, dtype, **opts) as k2:
            k2.step_rk4(w.dt, 20)
            blob = k2.get_state()
        with make(w, dtype, **opts) as k3:
            k3.set_state(blob)
            k3.step_rk4(w.dt, 20)
            b = k3.get_state()
        assert a == b  # bitwise: resume and rerun agree exactly


def test_conservation_and_fixed_point(need_gpu):
    """Symmetric A, uniform scaling: the mean of theta - theta0 - t omega stays 0 (Sec. 3, eq.
    KuramotoGraphConservation); omega = 0 with equal phases is a fixed point."""
    w = small_sbm(n_comm=8, comm_size=256, steps=200)
    with make(w, "f64") as k:
        k.step_rk4(w.dt, 200)
        th = k.get_phases()
        dev = math.fsum(th - w.theta0 - 200 * w.dt * w.omega) / w.graph.n
        assert abs(dev) < 1e-11
        k.set_params(np.zeros(w.graph.n), w.K)
        k.set_phases(np.full(w.graph.n, 0.3))
        F = k.eval_rhs()
        assert np.abs(F).max() < 1e-12
        k.step_rk4(w.dt, 50)
        assert np.abs(k.get_phases() - 0.3).max() < 1e-12


def test_order_parameter_samples(need_gpu):
    w = small_sbm(n_comm=4, comm_size=256, steps=100)
    with make(w, "f64") as k:
        r, psi = k.step_rk4(w.dt, 100, r_every=10)
        r1, psi1 = k.order_parameter()
    tho, ro, psio = oracle.rk4(w.graph, w.omega, w.K, w.theta0, w.dt, 100, r_every=10)
    assert len(r) == 11
    assert np.abs(r - ro).max() < 1e-12
    assert np.abs(wrap(psi - psio)).max() < 1e-10
    assert abs(r1 - ro[-1]) < 1e-12


def test_eval_at_given_theta(need_gpu):
    w = small_sbm(n_comm=4, comm_size=256, steps=1)
    rng = np.random.default_rng(4)
    th = rng.uniform(-50, 50, w.graph.n)
    with make(w, "f64") as k:
        F = k.eval_rhs(th)
    assert rel_err(F, oracle.rhs(w.graph, w.omega, w.K, th)) < 1e-12


def test_sbm_64x1024_sampled_rows(need_gpu):
    """N = 65536 = 64 x 1024, rho 0.97, p_out 2e-4: FP64 and FP32 right-hand side on a seeded
    1/64 subsample of rows at theta0 and at a partially synchronised state; conservation over
    100 steps."""
    w = gen.sbm_equal()
    g = w.graph
    rows = np.sort(np.random.default_rng(0).choice(g.n, g.n // 64, replace=False))
    rng = np.random.default_rng(5)
    th_sync = (g.labels * 0.7 + 0.1 * rng.standard_normal(g.n))
    for dtype in ("f64", "f32"):
        with make(w, dtype) as k:
            for th in (w.theta0, th_sync):
                thx = th if dtype == "f64" else f32(th)
                F = k.eval_rhs(thx)
                Fo = oracle.rhs_rows(g, w.omega, w.K, thx, rows)
                if dtype == "f64":
                    assert np.abs(F[rows] - Fo).max() < 1e-12 * np.abs(Fo).max()
                else:
                    bound = fp32_rhs_bound(k, w, thx)[rows]
                    assert np.all(np.abs(F[rows] - Fo) <= bound)
            if dtype == "f64":
                k.step_rk4(w.dt, 100)
                th = k.get_phases()
                dev = math.fsum(th - w.theta0 - 100 * w.dt * w.omega) / g.n
                assert abs(dev) < 1e-10


def load_trajectory_fixture(name):
    """(steps of the r samples, r, psi, rows, theta(T) of those rows) of a fixture written by
    tests/golden/make_sbm64x1024_trajectory.py (oracle only)."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)
    rs, rows, th = [], [], []
    with open(path) as f:
        for line in f:
            p = line.split()
            if not p or p[0].startswith("#"):
                continue
            if p[0] == "r":
                rs.append((int(p[1]), float(p[2]), float(p[3])))
            elif p[0] == "theta":
                rows.append(int(p[1]))
                th.append(float(p[2]))
    rs = np.array(rs)
    return rs[:, 0].astype(int), rs[:, 1], rs[:, 2], np.array(rows, dtype=np.int64), np.array(th)


# The committed cached layout of the 64 x 1024 SBM (tile options chosen by the tuner on MI355X,
# launch order for 8 XCDs); FP64 contexts take the same tile options with their own chunk width.
SBM64_CACHED = dict(tile_rows=128, tile_min_cost=16384, flat_min_vec=8, xcds=8, inter_gather=0)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("layout", ["default", "cached"])
def test_sbm_64x1024_trajectory_1000_steps(need_gpu, dtype, layout):
    """The 64 x 1024 SBM workload at full size (N = 65536, rho 0.97, p_out 2e-4, permuted), 1000
    RK4 steps: phases of a seeded 1/16 of the rows and r every 10 steps (all rows) against the
    oracle's trajectory stored in tests/golden/ (Sec. 3, eq. KuramotoGraph; classical RK4).
    FP64 from the FP64 inputs: |wrap(dtheta)| and |dr| <= 1e-12 max(1, max |theta_oracle|).
    FP32 from the FP32-rounded inputs (the oracle integrated those in FP64): <= 1e-5. Run in the
    default layout and in the committed tuned layout (8-XCD launch order), the one bench.py uses."""
    import os
    w = gen.sbm_equal()
    g = w.graph
    steps_r, ro, psio, rows, tho = load_trajectory_fixture(
        "sbm64x1024_rk4_1000_%sin.txt" % ("f64" if dtype == "f64" else "f32"))
    om, th0, K, dt = w.omega, w.theta0, w.K, w.dt
    if dtype == "f32":
        om, th0, K, dt = f32(om), f32(th0), float(np.float32(K)), float(np.float32(dt))
    with Kuramoto(dtype, device=0) as k:
        if layout == "cached" and dtype == "f32":
            cache = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                                 "paper_2102_07167_amd", "tuned_layouts.tsv")
            rep = k.autotune(g, effort=1, cache=cache)
            assert rep["cache"] == 1 and rep["xcds"] == 8 and rep["inter_gather"] == 0
        else:
            if layout == "cached":
                for key, v in SBM64_CACHED.items():
                    k.set_option(key, v)
            k.set_graph(g)
        k.set_params(om, K)
        k.set_phases(th0)
        r, psi = k.step_rk4(dt, 1000, r_every=10)
        th = k.get_phases(wrapped=False)
    assert np.array_equal(np.arange(0, 1001, 10), steps_r)
    tol = 1e-12 * max(1.0, np.abs(tho).max()) if dtype == "f64" else 1e-5
    err = np.abs(wrap(th[rows] - tho)).max()
    assert err <= tol, (err, tol)
    assert np.abs(r - ro).max() <= tol
    live = ro > 1e-3
    assert np.abs(wrap(psi - psio)[live]).max() <= tol / 1e-3


@pytest.fixture(scope="module")
def het_workload():
    """The heterogeneous N = 2^20 SBM workload, generated once for the tests of this module."""
    return gen.sbm_heterogeneous()


def test_het_sbm_n2p20_sampled_rows(need_gpu, het_workload):
    """Heterogeneous SBM, N = 2^20 (power-law communities in [256, 16384], densities U[0.3, 1],
    inter mean degree 8), FP32, in the layout bench.py times (installed through the committed
    tuning cache). The coupling sums of a seeded 1/64 subsample of rows (omega = 0 so that the
    FP32 rounding of the Cauchy frequencies does not hide them) against the FP64 oracle within
    K/N (1e-7 (deg + 2 block size) + 1e-5), a bound far above FP32 summation error and far
    below the ~0.6 K/N of one missing or extra edge; then, with the real omega, the conserved
    mean over 20 RK4 steps and r against the GPU's own phases."""
    import os
    w = het_workload
    g = w.graph
    cache = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2102_07167_amd",
                         "tuned_layouts.tsv")
    rows = np.sort(np.random.default_rng(0).choice(g.n, g.n // 64, replace=False))
    th0 = f32(w.theta0)
    K = float(np.float32(w.K))
    scale = K / g.n
    _, inv, cnt = np.unique(g.labels, return_inverse=True, return_counts=True)
    sb = cnt[inv][rows]
    deg = np.diff(g.row_ptr)[rows]
    with Kuramoto("f32", device=0) as k:
        k.autotune(g, effort=1, cache=cache)
        k.set_params(np.zeros(g.n), K)
        F = k.eval_rhs(th0)
        Fo = oracle.rhs_rows(g, np.zeros(g.n), K, th0, rows)
        err = np.abs(F[rows] - Fo) / scale
        assert np.all(err <= 1e-7 * (deg + 2 * sb) + 1e-5), err.max()
        om = f32(w.omega)
        k.set_params(om, K)
        k.set_phases(th0)
        k.step_rk4(w.dt, 20)
        th = k.get_phases(wrapped=False)
        r, _ = k.order_parameter()
    T = 20 * float(np.float32(w.dt))
    assert abs(math.fsum(th - th0 - T * om) / g.n) < 1e-5
    ro, _ = oracle.order_parameter(th)
    assert abs(r - ro) < 1e-5


def test_het_sbm_n2p20_evolved_states(need_gpu, het_workload):
    """Heterogeneous SBM, N = 2^20, FP32 with the real Cauchy(0, 0.5) frequencies, in the layout
    bench.py times: at the GPU's own states after 0, 100, ..., 500 RK4 steps (dt 0.005), the
    coupling sums G = F - omega of a seeded 1/64 of the rows against the FP64 oracle at the same
    (FP32) phases, within 1e-5 (K/N)(deg_m + 2 s_b [dense]) (Sec. 3, eq. KuramotoGraphApproach);
    G is evaluated with omega = 0 so that the FP32 rounding of F = omega + G at the Cauchy tails
    does not hide it, and F with the real omega within that bound plus half an FP32 ulp of |F|.
    r at every state against the oracle's r of the same phases."""
    import os
    w = het_workload
    g = w.graph
    cache = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2102_07167_amd",
                         "tuned_layouts.tsv")
    rows = np.sort(np.random.default_rng(0).choice(g.n, g.n // 64, replace=False))
    th0 = f32(w.theta0)
    om = f32(w.omega)
    K = float(np.float32(w.K))
    dt = float(np.float32(w.dt))
    scale = K / g.n
    deg = np.diff(g.row_ptr)[rows]
    zero = np.zeros(g.n)
    with Kuramoto("f32", device=0) as k:
        k.autotune(g, effort=1, cache=cache)
        dense = dense_term(k, g)[rows]
        k.set_params(om, K)
        k.set_phases(th0)
        for n_done in range(0, 501, 100):
            if n_done:
                k.step_rk4(dt, 100)
            th = f32(k.get_phases(wrapped=True))
            r, _ = k.order_parameter()
            F = k.eval_rhs(th)[rows]
            k.set_params(zero, K)
            G = k.eval_rhs(th)[rows]
            k.set_params(om, K)
            # set_params keeps the phase state; the next steps continue from it
            Go = oracle.rhs_rows(g, zero, K, th, rows)
            bound = 1e-5 * scale * (deg + dense)
            assert np.all(np.abs(G - Go) <= bound), (n_done, np.max(np.abs(G - Go) / bound))
            Fo = Go + om[rows]
            assert np.all(np.abs(F - Fo) <= bound + 2.0 ** -24 * np.abs(Fo) + 1e-30), n_done
            ro, _ = oracle.order_parameter(th)
            assert abs(r - ro) < 1e-5, n_done


def test_paper_four_communities(need_gpu):
    """The paper-shaped workload of the bench (M = 4096 in four equal communities, the special
    omega with omega0 = 2, splay theta0, K = 3): RHS and 200 FP64 RK4 steps against the oracle
    at 1e-12; then the whole T = 200 integration (20000 steps) keeps the mean of
    theta - theta0 - t omega at 0 (symmetric A) and stays finite."""
    w = gen.paper_four_communities()
    g = w.graph
    assert g.n == 4096 and w.steps == 20000
    with Kuramoto("f64", device=0) as k:
        k.set_graph(g)
        k.set_params(w.omega, w.K)
        k.set_phases(w.theta0)
        F = k.eval_rhs()
        Fo = oracle.rhs(g, w.omega, w.K, w.theta0)
        assert np.abs(F - Fo).max() <= 1e-12 * np.abs(Fo).max()
        k.step_rk4(w.dt, 200)
        th = k.get_phases(wrapped=False)
        tho, _, _ = oracle.rk4(g, w.omega, w.K, w.theta0, w.dt, 200)
        assert np.abs(th - tho).max() <= 1e-12 * max(1.0, np.abs(tho).max())
        k.set_phases(w.theta0)
        r, _ = k.step_rk4(w.dt, w.steps, 1000)
        thT = k.get_phases(wrapped=False)
    assert np.isfinite(r).all() and np.isfinite(thT).all()
    T = w.steps * w.dt
    assert abs(np.mean(thT - w.theta0 - T * w.omega)) < 1e-9


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n", [1, 2, 97, 512, 1000, 1024, 1025])
def test_complete_graph_one_workgroup_run(need_gpu, dtype, n):
    """Complete graphs of at most 1024 nodes run kur_step_rk4 in one workgroup (option
    persistent, default 1); 1025 nodes take the row kernel. Against the row kernel (persistent = 0)
    and the oracle: phases and r samples (including step 0 and a last step that is not a multiple
    of r_every) at 1e-12 (FP64) or 1e-5 (FP32), both scalings; the order parameter and the
    right-hand side afterwards come from the updated state."""
    rng = np.random.default_rng(n)
    om = rng.standard_normal(n)
    th0 = rng.uniform(0, 2 * np.pi, n)
    K, dt, steps, r_every = 2.5, 0.01, 203, 10
    if dtype == "f32":
        om, th0, K, dt = f32(om), f32(th0), float(np.float32(K)), float(np.float32(dt))
    tol = 1e-12 if dtype == "f64" else 1e-5
    g = gen.complete_graph(n)
    for scaling in (0, 1):
        out = {}
        for pers in (1, 0):
            with Kuramoto(dtype, device=0) as k:
                k.set_option("persistent", pers)
                k.set_option("scaling", scaling)
                k.set_graph(g)
                k.set_params(om, K)
                k.set_phases(th0)
                r, psi = k.step_rk4(dt, steps, r_every)
                r2, _ = k.step_rk4(dt, 7, 7)  # a second call continues from the updated state
                th = k.get_phases(wrapped=False)
                rn, _ = k.order_parameter()
                F = k.eval_rhs()
                out[pers] = (r, psi, r2, th, rn, F)
        a, b = out[1], out[0]
        assert a[0].shape == (steps // r_every + 1,)
        assert np.abs(a[0] - b[0]).max() < tol and np.abs(a[2] - b[2]).max() < tol
        live = a[0] > 1e-3  # psi is defined where r is not 0
        if live.any():
            assert np.abs(wrap(a[1] - b[1])[live]).max() < (1e-9 if dtype == "f64" else 1e-3)
        assert np.abs(a[3] - b[3]).max() <= tol * max(1.0, np.abs(b[3]).max())
        assert abs(a[4] - a[2][-1]) < tol
        assert np.abs(a[5] - b[5]).max() <= tol * max(1.0, np.abs(b[5]).max())
        if n <= 512:  # the oracle's complete graph costs n^2 per evaluation
            tho, ro, _ = oracle.rk4(g, om, K, th0, dt, steps + 7, r_every=1, scaling=scaling)
            assert np.abs(wrap(a[3] - tho)).max() < (tol * max(1.0, np.abs(tho).max()) if dtype == "f64" else 1e-5)
            assert np.abs(a[0] - ro[:steps + 1:r_every]).max() < tol


def test_complete_graph_one_workgroup_zero_steps(need_gpu):
    """nsteps = 0 with sampling: one sample, of the initial phases; nothing else changes."""
    rng = np.random.default_rng(3)
    n = 300
    th0 = rng.uniform(0, 2 * np.pi, n)
    with Kuramoto("f64", device=0) as k:
        k.set_graph(gen.complete_graph(n))
        k.set_params(rng.standard_normal(n), 1.0)
        k.set_phases(th0)
        r, psi = k.step_rk4(0.01, 0, 5)
        th = k.get_phases(wrapped=False)
    ro, po = oracle.order_parameter(th0)
    assert r.shape == (1,) and abs(r[0] - ro) < 1e-14 and abs(psi[0] - po) < 1e-12
    assert np.abs(th - th0).max() < 1e-15 * 2 * np.pi


@pytest.mark.parametrize("r_every", [0, 1000, 7])
def test_complete_graph_one_workgroup_long_run(need_gpu, r_every):
    """A call longer than one launch of the one-workgroup run (launches of whole sampling
    periods, at most about 65536 steps): 70001 steps give the same phases and r samples as the
    row kernel, with every sample present exactly once."""
    rng = np.random.default_rng(5)
    n, K, dt, steps = 64, 5.0, 0.002, 70001  # synchronised regime: differences in rounding contract
    om = rng.standard_normal(n)
    th0 = rng.uniform(0, 2 * np.pi, n)
    out = {}
    for pers in (1, 0):
        with Kuramoto("f64", device=0) as k:
            k.set_option("persistent", pers)
            k.set_graph(gen.complete_graph(n))
            k.set_params(om, K)
            k.set_phases(th0)
            r, psi = k.step_rk4(dt, steps, r_every)
            out[pers] = (r, k.get_phases(wrapped=False))
    if r_every:
        assert out[1][0].shape == (steps // r_every + 1,)
        assert np.abs(out[1][0] - out[0][0]).max() < 1e-10
    assert np.abs(out[1][1] - out[0][1]).max() < 1e-9 * max(1.0, np.abs(out[0][1]).max())
