"""CPU pins of the seeded synthetic workloads the bench and the full-size tests use: the recipes
stated for them (community sizes, densities, inter-community degree, symmetry, planted labels)
hold for the generated graphs. The generator holds none of the method's arithmetic; these tests
check that the inputs are the ones described."""
import math

import numpy as np

import gen


def _intra_inter(g):
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    same = g.labels[rows] == g.labels[g.col]
    return rows, same


def _symmetric(g):
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    a = rows.astype(np.int64) * g.n + g.col
    b = g.col.astype(np.int64) * g.n + rows
    return np.array_equal(np.sort(a), np.sort(b))


def test_heterogeneous_n2p20_community_sizes():
    """The N = 2^20 bench workload's communities (seed 1003): power-law sizes with density
    ~ s^-2 above 256, clipped at 16384, summing to 2^20, and densities ~ U[0.3, 1]: 794
    communities, 579 of them at density >= 1/2 (the blocks stored as zeros at tau = 1/2)."""
    g_rng, *_ = gen.streams(1003)
    s = gen.powerlaw_sizes(g_rng, 1 << 20)
    rho = g_rng.uniform(0.3, 1.0, size=len(s))
    assert s.sum() == 1 << 20 and s.min() >= 256 and s.max() <= 16384
    assert len(s) == 794 and int((rho >= 0.5).sum()) == 579
    # P(s < 2 smin) = 1/2 for density s^-2 above smin (before the clip)
    assert 0.45 < np.mean(s < 512) < 0.55
    assert 0.3 <= rho.min() and rho.max() <= 1.0


def test_heterogeneous_recipe_on_a_small_instance():
    """The same generator at N = 2^15 (sizes clipped to [256, 2048]): symmetric, no self loops,
    planted labels of the drawn sizes, realised intra densities close to their draws, and a
    mean inter-community degree close to 8."""
    w = gen.sbm_heterogeneous(n=1 << 15, smax=2048, seed=77)
    g = w.graph
    assert g.n == 1 << 15 and _symmetric(g)
    rows, same = _intra_inter(g)
    assert not np.any(rows == g.col)
    inter_deg = np.count_nonzero(~same) / g.n
    assert abs(inter_deg - 8.0) < 0.5, inter_deg
    g_rng, *_ = gen.streams(77)
    sizes = gen.powerlaw_sizes(g_rng, 1 << 15, 256, 2048)
    rho = g_rng.uniform(0.3, 1.0, size=len(sizes))
    _, counts = np.unique(g.labels, return_counts=True)
    assert sorted(counts.tolist()) == sorted(sizes.tolist())
    intra_per_label = np.bincount(g.labels[rows[same]], minlength=len(sizes))
    for c in range(len(sizes)):
        s = int(np.count_nonzero(g.labels == c))
        if s >= 512:
            dens = intra_per_label[c] / (s * (s - 1))
            assert abs(dens - rho[c]) < 0.02, (c, dens, rho[c])
    assert np.all(np.isfinite(w.omega)) and w.K == 3.0 and w.dt == 0.005


def test_paired_sbm_recipe():
    """Paired SBM (small instance): communities 2i and 2i + 1 joined by a block of density
    ~0.9, the diagonal blocks at ~0.97, everything else at ~p_out."""
    g = gen.paired_sbm(n_comm=8, comm_size=256, rho_in=0.97, rho_pair=0.9, p_out=2e-3, seed=5)
    assert g.n == 2048 and _symmetric(g)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    la, lc = g.labels[rows], g.labels[g.col]
    s = 256
    diag = np.count_nonzero(la == lc) / (8 * s * (s - 1))
    pair = np.count_nonzero((la != lc) & (la // 2 == lc // 2)) / (8 * s * s)
    rest = np.count_nonzero(la // 2 != lc // 2) / (8 * s * (8 * s - 2 * s))
    assert abs(diag - 0.97) < 0.01 and abs(pair - 0.9) < 0.01 and abs(rest - 2e-3) < 5e-4


def test_batch_instance_list():
    """The 256-instance batch: N log-uniform in [1024, 65536], all-to-all or SBM by a coin,
    K = linspace(0, 6, 256); generated lazily, the plan is fixed by the seed."""
    ns, kinds, Ks = [], [], []
    for w in gen.batch_instances_iter():
        ns.append(w.graph.n)
        kinds.append(w.meta["kind"])
        Ks.append(w.K)
        if w.meta["kind"] == "a2a":
            assert w.graph.complete
        else:
            _, counts = np.unique(w.graph.labels, return_counts=True)
            assert counts.max() - counts.min() <= 1 and abs(counts.mean() - 1024) < 512
    assert len(ns) == 256 and min(ns) >= 1024 and max(ns) <= 65536
    assert np.allclose(Ks, np.linspace(0.0, 6.0, 256))
    assert 100 < kinds.count("a2a") < 156
    logs = np.log(ns)
    # log-uniform: the mean of log N is near the midpoint of [log 1024, log 65536]
    assert abs(logs.mean() - 0.5 * (math.log(1024) + math.log(65536))) < 0.3
    assert sum(ns) == 3656930
