"""CPU tests of the shared-graph ensemble layout on host-only contexts: the regroup, the choice
of matrix-core blocks at "ens_tau", the bitmask rows of those blocks and the CSR of every other
edge, checked against the dense adjacency; argument validation."""
import numpy as np
import pytest

import gen
from paper_2102_07167_amd import kur as K

from test_abi_host import host_ctx


def mixed_sbm(seed=5, symmetric=True):
    rng = np.random.default_rng(seed)
    sizes = np.array([70, 1, 33, 130, 2, 64])
    rho = np.array([0.8, 0.5, 0.3, 0.6, 1.0, 0.95])
    n = int(sizes.sum())
    if symmetric:
        return gen.sbm(sizes, rho, 0.03, key=77, uperm=rng.permutation(n).astype(np.int32))
    A = (rng.random((n, n)) < 0.2).astype(np.uint8)
    np.fill_diagonal(A, 0)
    labels = rng.integers(0, 5, n).astype(np.int32)
    return gen.from_dense(A, labels)


def check_ens_layout(k, g, tau, pair_min=32, pair_floor=0.01):
    """The matrix-core ranges of every row block (its own block when at least tau dense, then its
    off-diagonal blocks of two communities of >= pair_min nodes at least max(tau, pair_floor)
    dense), their bit patterns and the CSR rows rebuild the dense adjacency exactly."""
    A = g.dense()
    n = g.n
    perm = k.ens_perm()
    order = np.lexsort((np.arange(n), g.labels))
    assert np.array_equal(perm[order], np.arange(n))
    B = A[np.ix_(order, order)]
    np.fill_diagonal(B, 0)
    labs = g.labels[order]
    bp = np.r_[np.flatnonzero(np.r_[True, labs[1:] != labs[:-1]]), n]
    nb = len(bp) - 1
    modes, dens = k.ens_block_modes()
    info = k.ens_info()
    assert info["blocks"] == nb == len(modes)
    gemm_blocks = gemm_rows = gemm_cells = csr = offdiag = 0
    for b in range(nb):
        s0, s1 = bp[b], bp[b + 1]
        s = s1 - s0
        sub = B[s0:s1, s0:s1]
        rho = sub.sum() / (s * (s - 1)) if s > 1 else 0.0
        assert abs(dens[b] - rho) < 1e-12
        assert modes[b] == (1 if (s >= 2 and rho >= tau) else 0), (b, rho, tau)
        cols_on = np.zeros(n, dtype=bool)  # columns of the row block's matrix-core ranges
        if modes[b]:
            cols_on[s0:s1] = True
            gemm_cells += s * s
        for c in range(nb):
            c0, c1 = bp[c], bp[c + 1]
            sc = c1 - c0
            if c == b or s < pair_min or sc < pair_min:
                continue
            r = B[s0:s1, c0:c1].sum() / (s * sc)
            if r >= max(tau, pair_floor):
                cols_on[c0:c1] = True
                gemm_cells += s * sc
                offdiag += 1
        if cols_on.any():
            gemm_blocks += 1
            gemm_rows += s
        for m in range(s0, s1):
            cols, dense = k.ens_row_pattern(m)
            assert np.all(np.diff(cols) > 0)
            assert not np.any(cols_on[cols])
            assert not np.any(dense[~cols_on])
            csr += len(cols)
            got = dense.astype(np.uint8).copy()
            got[cols] += 1
            assert np.array_equal(got, B[m]), (b, m)
    assert (info["gemm_blocks"], info["gemm_rows"], info["gemm_pairs"], info["csr_entries"], info["offdiag_blocks"]) == \
        (gemm_blocks, gemm_rows, gemm_cells, csr, offdiag)


@pytest.mark.parametrize("tau", [0.0, 0.5, 0.9, 2.0])
def test_ensemble_layout_matches_dense_adjacency(tau):
    g = mixed_sbm()
    with host_ctx("f32", ens_tau=tau) as k:
        k.ens_set_graph(g)
        assert k.ens_info()["symmetric"] == 1
        check_ens_layout(k, g, tau)


def test_ensemble_layout_asymmetric_with_self_loops():
    g = mixed_sbm(7, symmetric=False)
    A = g.dense()
    A[np.arange(0, g.n, 7), np.arange(0, g.n, 7)] = 1  # diagonal entries are ignored
    g2 = gen.from_dense(A, g.labels)
    with host_ctx("f32", ens_tau=0.1) as k:
        k.ens_set_graph(g2)
        assert k.ens_info()["symmetric"] == 0
        A0 = A.copy()
        np.fill_diagonal(A0, 0)
        check_ens_layout(k, gen.from_dense(A0, g.labels), 0.1)


def test_ensemble_validation():
    g = mixed_sbm()
    # FP64 contexts build the same layout; their product tiles are 128 rows high (256 in FP32)
    issued = {}
    for dt in ("f32", "f64"):
        with host_ctx(dt) as k:
            k.ens_set_graph(g)
            info = k.ens_info()
            issued[dt] = info["gemm_cells_issued"]
            if dt == "f64":
                check_ens_layout(k, g, 0.5)
    assert issued["f64"] <= issued["f32"]
    with host_ctx("f32") as k:
        with pytest.raises(K.KurError) as ei:
            k.ens_info()
        assert ei.value.status == K.KUR_ESTATE
        bad = gen.Graph(n=g.n, labels=g.labels, row_ptr=g.row_ptr.copy(), col=g.col.copy())
        r = next(u for u in range(g.n) if g.row_ptr[u + 1] - g.row_ptr[u] >= 2)
        bad.col[g.row_ptr[r] + 1] = bad.col[g.row_ptr[r]]
        with pytest.raises(K.KurError) as ei:
            k.ens_set_graph(bad)
        assert ei.value.status == K.KUR_EINVAL and "duplicate" in str(ei.value)
        k.ens_set_graph(g)
        with pytest.raises(K.KurError) as ei:
            k.ens_set_params([1.0], np.zeros((1, g.n)))
        assert ei.value.status == K.KUR_EDEVICE
        cols, _ = k.ens_row_pattern(0)
        if len(cols):
            cap = K.I64(len(cols) - 1)
            buf = np.empty(len(cols), dtype=np.int32)
            assert k._L.kur_ens_row_pattern(k._h, 0, K._ptr(buf), K.ctypes.byref(cap), None) == K.KUR_EINVAL
        with pytest.raises(K.KurError):
            k.set_option("ens_tau", -0.1)


@pytest.mark.parametrize("tau", [0.0, 0.3, 0.8])
def test_ensemble_layout_dense_offdiagonal_blocks(tau):
    """Communities 0-2 and 1-3 joined by dense off-diagonal blocks (density 0.9), 0-1 at 0.1, a
    partner below 32 nodes; 0 is sparse itself, so its row block holds only its partner range."""
    rng = np.random.default_rng(17)
    sizes = [90, 70, 100, 40, 20, 50]
    V = np.zeros((6, 6), dtype=np.int32)
    for a, c in [(1, 1), (2, 2), (3, 3), (4, 4), (0, 2), (1, 3), (2, 4), (5, 5), (0, 1)]:
        V[a, c] = V[c, a] = 1
    V[0, 1] = V[1, 0] = 0
    n = sum(sizes)
    g = gen.block_model(sizes, V, 0.1, 1, rng, uperm=rng.permutation(n).astype(np.int32))
    with host_ctx("f32", ens_tau=tau) as k:
        k.ens_set_graph(g)
        check_ens_layout(k, g, tau)
        if tau == 0.3:
            assert k.ens_info()["offdiag_blocks"] == 4  # 0-2 and 1-3, both ways
