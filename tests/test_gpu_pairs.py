"""GPU tests of dense off-diagonal blocks (a submatrix of two communities evaluated with the
localised order parameters of its column community minus its list of zeros, Sec. 3, extension
to submatrices [M1..M2] x [M3..M4]): right-hand side, RK4, midpoint, adaptive pair, adjoint and
potential against the oracle, which sums the adjacency directly. Tolerances as for the diagonal
blocks: FP64 1e-12 relative, FP32 1e-5 on phases and r, adjoint 1e-10; the FP32 right-hand side
within 1e-5 (K/N)(deg_m + 2 sum_q mode_q s_q) + 1e-6 |omega_m|, the rounding scale of the
complement form summed over the row's column groups q (sizes s_q, factors mode_q)."""
import numpy as np
import pytest

import gen
import oracle
from paper_2102_07167_amd import Kuramoto

pytestmark = pytest.mark.gpu
TWO_PI = 2 * np.pi


def wrap(x):
    return np.remainder(x + np.pi, TWO_PI) - np.pi


def pair_graph(seed, sizes, V, exception=0.1, J=1):
    rng = np.random.default_rng(seed)
    n = int(np.sum(sizes))
    g = gen.block_model(sizes, V, exception, J, rng, uperm=rng.permutation(n).astype(np.int32))
    return g, rng.standard_normal(n), rng.uniform(0, TWO_PI, n)


# blocks 0-2 and 1-3 dense off-diagonal, 2-4 dense but block 4 below pair_min, 5 ragged (257)
SIZES = [150, 70, 100, 40, 20, 257]
V6 = np.zeros((6, 6), dtype=np.int32)
for a, c in [(0, 0), (1, 1), (2, 2), (5, 5), (0, 2), (1, 3), (2, 4), (0, 5), (3, 5)]:
    V6[a, c] = V6[c, a] = 1


def ctx(g, dtype, om, K, th, opts=None):
    k = Kuramoto(dtype, device=0)
    for key, v in (opts or {}).items():
        k.set_option(key, v)
    k.set_graph(g)
    k.set_params(om, K)
    k.set_phases(th)
    return k


def group_scale(g, opts=None):
    """Per user node: sum over its row block's column groups of mode_q * s_q (host layout)."""
    k = Kuramoto("f64", device=-1)
    for key, v in (opts or {}).items():
        if key in ("tau", "chunk", "pairs", "pair_min"):
            k.set_option(key, v)
    k.set_graph(g)
    bp, _ = k.blocks()
    perm = k.perm()
    per_block = np.zeros(len(bp) - 1)
    for b in range(len(bp) - 1):
        gb, gm = k.block_groups(b)
        per_block[b] = float(np.sum(gm * np.diff(bp)[gb]))
    k.close()
    blk_of = np.repeat(np.arange(len(bp) - 1), np.diff(bp))
    return per_block[blk_of[perm]]


def deg_of(g):
    if g.weight is None:
        return np.diff(g.row_ptr).astype(np.float64)
    return np.add.reduceat(g.weight.astype(np.float64), g.row_ptr[:-1]) * (np.diff(g.row_ptr) > 0)


@pytest.mark.parametrize("opts", [dict(), dict(chunk=64, tile_rows=64, flat_min_vec=0.5),
                                  dict(chunk=64, threads=256, flat_min_vec=1000), dict(scaling=1),
                                  dict(mask_min=0.0, chunk=512)])
def test_pairs_fp64_rhs_and_rk4(need_gpu, opts):
    g, om, th = pair_graph(81, SIZES, V6)
    K, dt, steps = 0.8, 0.01, 100
    sc = opts.get("scaling", 0)
    with ctx(g, "f64", om, K, th, opts) as k:
        assert k.graph_pairs() == 8
        F = k.eval_rhs()
        k.step_rk4(dt, steps)
        thT = k.get_phases(wrapped=False)
    Fo = oracle.rhs(g, om, K, th, scaling=sc)
    assert np.abs(F - Fo).max() <= 1e-12 * np.abs(Fo).max()
    tho, _, _ = oracle.rk4(g, om, K, th, dt, steps, scaling=sc)
    assert np.abs(thT - tho).max() <= 1e-12 * max(1.0, np.abs(tho).max())


def test_pairs_on_and_off_agree(need_gpu):
    g, om, th = pair_graph(82, SIZES, V6)
    out = []
    for pairs in (1, 0):
        with ctx(g, "f64", om, 1.3, th, dict(pairs=pairs, chunk=128)) as k:
            assert (k.graph_pairs() > 0) == bool(pairs)
            out.append(k.eval_rhs())
    assert np.abs(out[0] - out[1]).max() <= 1e-12 * np.abs(out[1]).max()


@pytest.mark.parametrize("threads", [128, 256, 512, 1024])
def test_pairs_more_groups_than_waves(need_gpu, threads):
    """Twelve mutually dense blocks: every row block has twelve column groups, more than the
    waves of a 128-, 256- or 512-thread workgroup."""
    sizes = [33, 40, 47, 54, 61, 68, 75, 82, 89, 96, 103, 110]
    g, om, th = pair_graph(83, sizes, np.ones((12, 12), dtype=np.int32), exception=0.15)
    K = 1.1
    with ctx(g, "f64", om, K, th, dict(threads=threads, chunk=64, tile_rows=64)) as k:
        assert k.graph_pairs() == 132
        F = k.eval_rhs()
    Fo = oracle.rhs(g, om, K, th)
    assert np.abs(F - Fo).max() <= 1e-12 * np.abs(Fo).max()
    om32, th32 = om.astype(np.float32).astype(np.float64), th.astype(np.float32).astype(np.float64)
    K32 = float(np.float32(K))
    with ctx(g, "f32", om32, K, th32, dict(threads=threads)) as k:
        F32 = k.eval_rhs()
    Fo = oracle.rhs(g, om32, K32, th32)
    bound = 1e-5 * K32 / g.n * (deg_of(g) + 2 * group_scale(g)) + 1e-6 * np.abs(om32)
    assert np.all(np.abs(F32 - Fo) <= bound)


def test_pairs_fp32_rk4(need_gpu):
    g, om, th = pair_graph(84, SIZES, V6)
    om, th = om.astype(np.float32).astype(np.float64), th.astype(np.float32).astype(np.float64)
    K32, dt32 = float(np.float32(0.8)), float(np.float32(0.01))
    with ctx(g, "f32", om, 0.8, th) as k:
        F = k.eval_rhs()
        r, _ = k.step_rk4(0.01, 200, r_every=20)
        thT = k.get_phases()
    Fo = oracle.rhs(g, om, K32, th)
    bound = 1e-5 * K32 / g.n * (deg_of(g) + 2 * group_scale(g)) + 1e-6 * np.abs(om)
    assert np.all(np.abs(F - Fo) <= bound)
    tho, ro, _ = oracle.rk4(g, om, K32, th, dt32, 200, r_every=20)
    assert np.abs(wrap(thT - tho)).max() < 1e-5
    assert np.abs(r - ro).max() < 1e-5


def test_pairs_weighted_midpoint_adjoint_potential(need_gpu):
    """Integer-weighted off-diagonal blocks with prevalent values 1 and 2 (J = 3)."""
    sizes = [90, 70, 60, 33, 129]
    V = np.array([[2, 1, 0, 0, 0],
                  [1, 0, 2, 0, 1],
                  [0, 2, 3, 0, 0],
                  [0, 0, 0, 1, 2],
                  [0, 1, 0, 2, 1]], dtype=np.int32)
    g, om, th = pair_graph(85, sizes, V, exception=0.2, J=3)
    assert g.weight is not None
    K, dt = 0.8, 0.02
    with ctx(g, "f64", om, K, th, dict(chunk=64)) as k:
        assert k.graph_pairs() == 8  # 0-1, 1-2, 1-4, 3-4, both ways
        F = k.eval_rhs()
        d = k.diagnostics()
        k.step_midpoint(dt, 20, 5)
        thm = k.get_phases(wrapped=False)
        seed = np.random.default_rng(1).standard_normal(g.n)
        gt, gw, gk = k.adjoint_rk4(dt, 25, seed, theta0=th, ckpt_every=6)
    Fo = oracle.rhs(g, om, K, th)
    assert np.abs(F - Fo).max() <= 1e-12 * np.abs(Fo).max()
    Vo = oracle.potential(g, om, K, th)
    assert abs(d["V"] - Vo) <= 1e-12 * (np.abs(om * th).sum() + K * g.dense().sum() / g.n)
    tmo, _, _ = oracle.midpoint(g, om, K, th, dt, 20, 5)
    assert np.abs(thm - tmo).max() <= 1e-12 * max(1.0, np.abs(tmo).max())
    go = oracle.adjoint_rk4(g, om, K, th, dt, 25, seed)
    assert np.abs(gt - go[0]).max() <= 1e-10 * np.abs(go[0]).max()
    assert np.abs(gw - go[1]).max() <= 1e-10 * np.abs(go[1]).max()
    assert abs(gk - go[2]) <= 1e-10 * max(abs(go[2]), np.abs(go[1]).max())


def test_pairs_adaptive(need_gpu):
    g, om, th = pair_graph(86, SIZES, V6)
    K, atol = 1.5, 1e-8
    with ctx(g, "f64", om, K, th) as k:
        st = k.step_adaptive(1.0, 0.3, atol)
        thT = k.get_phases(wrapped=False)
    tho, sto = oracle.rkf45(g, om, K, th, 1.0, 0.3, atol)
    assert (st["accepted"], st["rejected"]) == (int(sto[2]), int(sto[3]))
    assert abs(st["t"] - sto[0]) < 1e-12
    assert np.abs(thT - tho).max() < 1e-10


def test_pairs_full_size_sampled_rows(need_gpu):
    """64 communities of 1024 coupled in pairs (density 0.9): the RHS on a seeded 1/64 row
    sample against the oracle, and the mean phase and r after 20 RK4 steps."""
    g = gen.paired_sbm()
    rng = np.random.default_rng(87)
    om = rng.standard_normal(g.n)
    th = rng.uniform(0, TWO_PI, g.n)
    om, th = om.astype(np.float32).astype(np.float64), th.astype(np.float32).astype(np.float64)
    K = float(np.float32(2.0))
    rows = np.sort(rng.choice(g.n, g.n // 64, replace=False))
    with Kuramoto("f32", device=0) as k:
        k.set_graph(g)
        assert k.graph_pairs() == 64
        k.set_params(np.zeros(g.n), K)
        F = k.eval_rhs(th)
        k.set_params(om, K)
        k.set_phases(th)
        r, _ = k.step_rk4(0.01, 20, r_every=20)
        thT = k.get_phases(wrapped=False)
    Fo = oracle.rhs_rows(g, np.zeros(g.n), K, th, rows)
    deg = np.diff(g.row_ptr)[rows].astype(np.float64)
    bound = 1e-5 * K / g.n * (deg + 2 * 2 * 1024)
    assert np.all(np.abs(F[rows] - Fo) <= bound)
    # symmetric coupling: the mean phase moves with the mean frequency
    assert abs(thT.mean() - th.mean() - 0.2 * om.mean()) < 1e-5
    ro, _ = oracle.order_parameter(thT)
    assert abs(r[-1] - ro) < 1e-5
