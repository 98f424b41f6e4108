"""CPU tests of the C ABI: the library loads and exports every declared symbol, and the host
preprocessing (regroup by label, dense/sparse choice, chunked lists, inter CSR) is checked on
host-only contexts against the dense adjacency. No GPU call is made."""
import ctypes
import os
import re

import numpy as np
import pytest

import gen
from paper_2102_07167_amd import kur as K

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "kur.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(kur_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = K.lib()
    names = declared_symbols()
    assert len(names) >= 20
    for nm in names:
        assert hasattr(L, nm), nm
    assert set(names) == set(K.SIGNATURES), set(names) ^ set(K.SIGNATURES)
    assert L.kur_version() >= 100


def host_ctx(dtype="f32", **opts):
    k = K.Kuramoto(dtype, device=-1)
    for key, v in opts.items():
        k.set_option(key, v)
    return k


def rebuild_row(k, m, b, bp, groups):
    """Row m of the block-order adjacency from the stored layout: every group's factor on its
    columns (not m itself), minus one per zero entry, plus one per one entry and per inter entry."""
    n = int(bp[-1])
    blk_of = np.repeat(np.arange(len(bp) - 1), np.diff(bp))
    R = np.zeros(n, dtype=np.int64)
    for c, v in groups.items():
        R[bp[c]:bp[c + 1]] += v
    if b in groups:
        R[m] -= groups[b]
    cols, lay = k.row_layers(m)
    for col, t in zip(cols, lay):
        R[col] += -1 if t <= groups.get(int(blk_of[col]), 0) else 1
    _, itr = k.row_lists(m)
    np.add.at(R, itr, 1)
    return R


def check_layout(k, g, tau, pair_min=32, pairs=True):
    """Compare the stored layout with the dense adjacency of g (user order)."""
    A = g.dense()
    perm = k.perm()
    n = g.n
    # stable counting sort by label: block order sorted by (label, user index)
    order = np.lexsort((np.arange(n), g.labels))
    assert np.array_equal(perm[order], np.arange(n))
    bp, mode = k.blocks()
    labs = g.labels[order]
    starts = np.flatnonzero(np.r_[True, labs[1:] != labs[:-1]])
    assert np.array_equal(bp[:-1], starts) and bp[-1] == n
    B = A[np.ix_(order, order)]  # block-order adjacency P A P^T
    nb = len(mode)
    blk_of = np.repeat(np.arange(nb), np.diff(bp))
    npairs = 0
    for b in range(nb):
        s0, s1 = bp[b], bp[b + 1]
        sub = B[s0:s1, s0:s1]
        s = s1 - s0
        rho = sub.sum() / (s * (s - 1)) if s > 1 else 0.0
        assert mode[b] == (1 if (s >= 2 and rho >= tau) else 0)
        # dense off-diagonal blocks: both sides >= pair_min, nonzero, density >= tau
        want = {b: 1} if mode[b] else {}
        for c in range(nb):
            sc = bp[c + 1] - bp[c]
            nnz = int(B[s0:s1, bp[c]:bp[c + 1]].sum())
            if pairs and c != b and s >= pair_min and sc >= pair_min and nnz > 0 and nnz / (s * sc) >= tau:
                want[c] = 1
                npairs += 1
        gb, gm = k.block_groups(b)
        groups = {int(c): int(v) for c, v in zip(gb, gm)}
        assert groups == want, b
        assert list(gb) == sorted(gb, key=lambda c: (c != b, c))  # own block first, then block order
        for m in range(s0, s1):
            lst, itr = k.row_lists(m)
            r = m - s0
            if mode[b]:
                want_l = [c for c in range(s) if c != r and sub[r, c] == 0]
            else:
                want_l = list(np.flatnonzero(sub[r]))
            assert list(lst) == want_l, (b, m)
            cross = [c for c in np.flatnonzero(B[m]) if blk_of[c] != b and int(blk_of[c]) not in groups]
            assert list(itr) == cross
            assert np.array_equal(rebuild_row(k, m, b, bp, groups), B[m].astype(np.int64)), (b, m)
    assert k.graph_pairs() == npairs


@pytest.mark.parametrize("chunk", [64, 8128])
@pytest.mark.parametrize("tau", [0.0, 0.5, 1.0])
def test_preprocessing_matches_dense_adjacency(chunk, tau):
    rng = np.random.default_rng(3)
    sizes = np.array([130, 1, 64, 200, 7])
    rho = np.array([0.9, 0.5, 0.3, 0.7, 1.0])
    g = gen.sbm(sizes, rho, 0.02, key=12345, uperm=rng.permutation(sizes.sum()).astype(np.int32))
    with host_ctx(chunk=chunk, tau=tau, tile_rows=64) as k:
        k.set_graph(g)
        info = k.graph_info()
        assert info["n"] == g.n and info["blocks"] == 5 and info["chunk"] == chunk
        # tau = 0 also makes every nonzero off-diagonal block of two large enough blocks dense
        assert tau == 0.0 or info["inter_entries"] == sum(
            int(np.sum(g.labels[g.col[g.row_ptr[u]:g.row_ptr[u + 1]]] != g.labels[u])) for u in range(g.n))
        check_layout(k, g, tau)


def test_preprocessing_asymmetric_and_labels_unordered():
    rng = np.random.default_rng(9)
    n = 150
    A = (rng.random((n, n)) < 0.3).astype(np.uint8)
    np.fill_diagonal(A, 0)
    labels = rng.choice([7, 3, 100, 42], size=n).astype(np.int32)
    # make the blocks denser than the rest
    for i in range(n):
        for j in range(n):
            if i != j and labels[i] == labels[j] and rng.random() < 0.7:
                A[i, j] = 1
    g = gen.from_dense(A, labels)
    with host_ctx(chunk=64) as k:
        k.set_graph(g)
        check_layout(k, g, 0.5)


def test_block_form_roundtrip():
    """kur_set_graph with the lists exported from a CSR-built layout rebuilds the same layout."""
    rng = np.random.default_rng(5)
    sizes = np.array([100, 60, 90])
    g = gen.sbm(sizes, np.array([0.95, 0.2, 0.6]), 0.05, key=99, uperm=rng.permutation(250).astype(np.int32))
    with host_ctx(chunk=64) as k1:
        k1.set_graph(g)
        bp, mode = k1.blocks()
        perm = k1.perm()
        lp, lc, ip, ic = [0], [], [0], []
        for m in range(g.n):
            lst, itr = k1.row_lists(m)
            lc += list(lst)
            ic += list(itr)
            lp.append(len(lc))
            ip.append(len(ic))
        with host_ctx(chunk=128) as k2:
            k2.set_graph_blocks(g.n, bp, mode, np.array(lp), np.array(lc), np.array(ip), np.array(ic), perm)
            assert np.array_equal(k2.perm(), perm)
            bp2, mode2 = k2.blocks()
            assert np.array_equal(bp2, bp) and np.array_equal(mode2, mode)
            for m in range(g.n):
                a1, b1 = k1.row_lists(m)
                a2, b2 = k2.row_lists(m)
                assert np.array_equal(a1, a2) and np.array_equal(b1, b2)
            assert k2.graph_info()["list_entries"] == k1.graph_info()["list_entries"]


def test_complete_graph_has_empty_lists():
    with host_ctx() as k:
        k.set_graph_complete(1000)
        info = k.graph_info()
        assert info["blocks"] == 1 and info["dense_blocks"] == 1 and info["list_entries"] == 0


def _expect(status, fn, *a):
    with pytest.raises(K.KurError) as ei:
        fn(*a)
    assert ei.value.status == status, str(ei.value)


def test_validation_errors_before_device_work():
    with host_ctx() as k:
        rp = np.array([0, 1, 2], dtype=np.int64)
        _expect(K.KUR_EINVAL, k.set_graph_csr, 2, np.array([0, 2, 1]), np.array([1, 0]), np.zeros(2))
        _expect(K.KUR_EINVAL, k.set_graph_csr, 2, rp, np.array([1, 2]), np.zeros(2))       # col out of range
        _expect(K.KUR_EINVAL, k.set_graph_csr, 2, rp, np.array([1, 0]), np.array([0, -1]))  # negative label
        _expect(K.KUR_EINVAL, k.set_graph_csr, 2, np.array([0, 2, 2]), np.array([1, 1]), np.zeros(2))  # dup
        _expect(K.KUR_EINVAL, k.set_graph_csr, 0, np.array([0]), np.zeros(0), np.zeros(0))
        for key, v in [("tau", -0.1), ("chunk", 100), ("chunk", 8192), ("tile_rows", 10), ("threads", 64),
                       ("scaling", 2), ("nonsense", 1.0), ("tau", float("nan")), ("flat_min_vec", -1),
                       ("mask_sub", 192), ("mask_sub", 2048), ("mask_sub", 0), ("mask_item", 0), ("mask_item", 1.5)]:
            _expect(K.KUR_EINVAL, k.set_option, key, v)
        with host_ctx("f64") as k64:
            _expect(K.KUR_EINVAL, k64.set_option, "chunk", 4096)
            k64.set_option("chunk", 4032)
        # calls out of order
        _expect(K.KUR_ESTATE, k.graph_info)
        k.set_graph_complete(4)
        # no device on a host-only context
        _expect(K.KUR_EDEVICE, k.set_params, np.zeros(4), 1.0)
        _expect(K.KUR_EINVAL, k.set_params, np.array([0, np.nan, 0, 0]), 1.0)
        _expect(K.KUR_EINVAL, k.set_params, np.zeros(4), float("inf"))
        _expect(K.KUR_EINVAL, k.set_phases, np.array([0, 0, np.inf, 0]))
        _expect(K.KUR_EDEVICE, k.step_rk4, 0.01, 1)
        _expect(K.KUR_EINVAL, k.step_rk4, 0.0, 1)
        _expect(K.KUR_EINVAL, k.step_rk4, 0.01, -1)


def test_block_form_validation():
    with host_ctx() as k:
        z = np.zeros(5, dtype=np.int64)
        ok = dict(n=4, block_ptr=np.array([0, 2, 4]), mode=np.array([1, 0]), list_ptr=z, list_col=np.zeros(1),
                  inter_ptr=z, inter_col=np.zeros(1))
        k.set_graph_blocks(**ok)
        bad = [dict(block_ptr=np.array([0, 2, 5])), dict(block_ptr=np.array([0, 2, 2, 4]), mode=np.array([1, 0, 1])),
               dict(list_ptr=np.array([0, 1, 1, 1, 1]), list_col=np.array([0])),        # diagonal
               dict(list_ptr=np.array([0, 1, 1, 1, 1]), list_col=np.array([2])),        # out of block
               dict(inter_ptr=np.array([0, 1, 1, 1, 1]), inter_col=np.array([1])),      # own block
               dict(inter_ptr=np.array([0, 2, 2, 2, 2]), inter_col=np.array([2, 2])),   # duplicate
               dict(perm=np.array([0, 1, 1, 3]))]
        for b in bad:
            args = dict(ok)
            args.update(b)
            _expect(K.KUR_EINVAL, k.set_graph_blocks, *[args[x] for x in
                                                        ["n", "block_ptr", "mode", "list_ptr", "list_col",
                                                         "inter_ptr", "inter_col"]], args.get("perm"))


def test_batch_layout_is_block_diagonal():
    """A batch is the block-diagonal union of its instances: every instance keeps its own lists
    and inter-block columns, shifted to its rows; complete instances store no list."""
    rng = np.random.default_rng(12)
    parts = []
    g1 = gen.sbm(np.array([40, 25]), np.array([0.9, 0.3]), 0.05, key=1, uperm=rng.permutation(65).astype(np.int32))
    parts.append((g1, 1.0, np.zeros(65), np.zeros(65)))
    parts.append((gen.complete_graph(30), 2.0, np.zeros(30), np.zeros(30)))
    g3 = gen.sbm(np.array([50]), np.array([0.6]), 0.0, key=3)
    parts.append((g3, 3.0, np.zeros(50), np.zeros(50)))
    with host_ctx(chunk=64) as k:
        k.set_batch(parts)
        rf = k.batch_info()
        assert list(rf) == [0, 65, 95, 145]
        perm = k.perm()
        for i, (g, *_rest) in enumerate(parts):
            lo, hi = rf[i], rf[i + 1]
            assert set(perm[lo:hi]) == set(range(lo, hi))
            with host_ctx(chunk=64) as k1:
                if g.complete:
                    k1.set_graph_complete(g.n)
                else:
                    k1.set_graph(g)
                assert np.array_equal(k1.perm() + lo, perm[lo:hi])
                for m in range(g.n):
                    a1, b1 = k1.row_lists(m)
                    a2, b2 = k.row_lists(m + lo)
                    assert np.array_equal(a1, a2) and np.array_equal(b1 + lo, b2)
        info = k.graph_info()
        assert info["blocks"] == 4 and info["symmetric"] == 1


def test_complete_graph_beyond_u16_block():
    with host_ctx() as k:
        k.set_graph_complete(70000)
        info = k.graph_info()
        assert info["blocks"] == 1 and info["list_entries"] == 0 and info["max_block"] == 70000


def check_weighted_layout(k, g, pair_min=32):
    """Rebuild every row of the weighted adjacency from its 0/1 layers, groups and inter list."""
    A = g.dense()
    n = g.n
    perm = k.perm()
    order = np.lexsort((np.arange(n), g.labels))
    assert np.array_equal(perm[order], np.arange(n))
    B = A[np.ix_(order, order)]
    bp, mode = k.blocks()
    nb = len(mode)
    for b in range(nb):
        s0, s1 = bp[b], bp[b + 1]
        s = s1 - s0
        sub = B[s0:s1, s0:s1]
        if s >= 2:
            full = np.bincount(sub[~np.eye(s, dtype=bool)], minlength=256)
            assert mode[b] == int(np.argmax(full)), b
        # groups: the block itself when its prevalent value is positive, then every off-diagonal
        # block (both sides >= pair_min) whose prevalent value, zeros included, is positive
        want = {b: int(mode[b])} if mode[b] else {}
        for c in range(nb):
            sc = bp[c + 1] - bp[c]
            if c == b or s < pair_min or sc < pair_min:
                continue
            v = int(np.argmax(np.bincount(B[s0:s1, bp[c]:bp[c + 1]].ravel(), minlength=256)))
            if v > 0:
                want[c] = v
        gb, gm = k.block_groups(b)
        groups = {int(c): int(v) for c, v in zip(gb, gm)}
        assert groups == want, b
        for m in range(s0, s1):
            _, lay = k.row_layers(m)
            assert lay.min(initial=1) >= 1 and lay.max(initial=1) <= max(1, int(B[m].max()))
            assert np.array_equal(rebuild_row(k, m, b, bp, groups), B[m].astype(np.int64)), (b, m)


@pytest.mark.parametrize("chunk", [64, 4096])
def test_weighted_layout_matches_dense(chunk):
    rng = np.random.default_rng(62)
    g = gen.weighted_sbm([90, 1, 70, 130], [2, 0, 0, 3], 0.25, 4, 0.03, rng,
                         uperm=rng.permutation(291).astype(np.int32))
    with host_ctx(chunk=chunk, tile_rows=64) as k:
        k.set_graph(g)
        info = k.graph_info()
        assert info["symmetric"] == 1
        check_weighted_layout(k, g)
    with host_ctx() as k:
        bad = gen.Graph(n=g.n, labels=g.labels, row_ptr=g.row_ptr, col=g.col, weight=g.weight.copy())
        bad.weight[0] = 300
        with pytest.raises(K.KurError):
            k.set_graph(bad)


# ------------------------------------------------------------------------------------------------
# Dense off-diagonal blocks (Sec. 3, extension to submatrices [M1..M2] x [M3..M4])
# ------------------------------------------------------------------------------------------------

def _pair_graph(rng, sizes, V, exception=0.1, J=1):
    n = int(np.sum(sizes))
    return gen.block_model(sizes, V, exception, J, rng, uperm=rng.permutation(n).astype(np.int32))


@pytest.mark.parametrize("chunk", [64, 4096])
@pytest.mark.parametrize("tau", [0.3, 0.5, 0.95])
def test_dense_pairs_layout(chunk, tau):
    """Blocks 0-2 and 1-3 are dense off-diagonal blocks (density 0.9), 0-1 about 0.1; block 4 is
    below pair_min. Every row rebuilds exactly from groups, layers and inter entries."""
    rng = np.random.default_rng(71)
    sizes = [150, 70, 100, 40, 20]
    V = np.zeros((5, 5), dtype=np.int32)
    V[0, 0] = V[1, 1] = V[2, 2] = 1
    V[0, 2] = V[2, 0] = V[1, 3] = V[3, 1] = 1
    V[2, 4] = V[4, 2] = 1  # dense, but block 4 is smaller than pair_min
    g = _pair_graph(rng, sizes, V)
    with host_ctx(chunk=chunk, tau=tau, tile_rows=64) as k:
        k.set_graph(g)
        check_layout(k, g, tau)
        if tau <= 0.5:
            assert k.graph_pairs() == 4
        assert k.graph_info()["symmetric"] == 1


def test_dense_pairs_options():
    rng = np.random.default_rng(72)
    sizes = [64, 48, 80]
    V = np.ones((3, 3), dtype=np.int32)
    g = _pair_graph(rng, sizes, V, exception=0.2)
    with host_ctx(chunk=64, pairs=0) as k:
        k.set_graph(g)
        check_layout(k, g, 0.5, pairs=False)
        assert k.graph_pairs() == 0
        inter_off = k.graph_info()["inter_entries"]
    with host_ctx(chunk=64, pair_min=50) as k:
        k.set_graph(g)
        check_layout(k, g, 0.5, pair_min=50)
        assert k.graph_pairs() == 2  # 0-2 and 2-0 (block 1 has 48 nodes)
    with host_ctx(chunk=64) as k:
        k.set_graph(g)
        check_layout(k, g, 0.5)
        assert k.graph_pairs() == 6
        assert k.graph_info()["inter_entries"] == 0 < inter_off
    with host_ctx() as k:
        with pytest.raises(K.KurError):
            k.set_option("pairs", 2)
        with pytest.raises(K.KurError):
            k.set_option("pair_min", 0)


@pytest.mark.parametrize("chunk", [64, 4096])
def test_dense_pairs_weighted_layout(chunk):
    """Integer-weighted off-diagonal blocks with prevalent values 1 and 2 (two zero layers) and
    a sparse weighted block; J = 3 gives one or two layers of ones above the prevalent value."""
    rng = np.random.default_rng(73)
    sizes = [90, 70, 60, 33]
    V = np.array([[2, 1, 0, 0],
                  [1, 0, 2, 0],
                  [0, 2, 3, 0],
                  [0, 0, 0, 1]], dtype=np.int32)
    g = _pair_graph(rng, sizes, V, exception=0.2, J=3)
    assert g.weight is not None
    with host_ctx(chunk=chunk, tile_rows=64) as k:
        k.set_graph(g)
        check_weighted_layout(k, g)
        assert k.graph_pairs() == 4


def test_dense_pairs_in_batch():
    """A batch of instances with dense off-diagonal blocks keeps every instance's groups."""
    rng = np.random.default_rng(74)
    V = np.array([[1, 1], [1, 0]], dtype=np.int32)
    gs = [_pair_graph(rng, [40 + 10 * i, 50], V) for i in range(3)]
    with host_ctx(chunk=64) as k:
        k.set_batch([(g, 1.0, np.zeros(g.n), np.zeros(g.n)) for g in gs])
        assert k.graph_pairs() == 6
        off = 0
        nb_off = 0
        bp, _ = k.blocks()
        for g in gs:
            with host_ctx(chunk=64) as k1:
                k1.set_graph(g)
                bp1, _ = k1.blocks()
                for b in range(len(bp1) - 1):
                    g1, m1 = k1.block_groups(b)
                    g2, m2 = k.block_groups(b + nb_off)
                    assert np.array_equal(g1 + nb_off, g2) and np.array_equal(m1, m2)
                for m in range(g.n):
                    c1, l1 = k1.row_layers(m)
                    c2, l2 = k.row_layers(m + off)
                    assert np.array_equal(c1 + off, c2) and np.array_equal(l1, l2)
                off += g.n
                nb_off += len(bp1) - 1


def test_transpose_option_values():
    with host_ctx() as k:
        k.set_option("transpose", 1)
        k.set_option("transpose", 0)
        with pytest.raises(K.KurError):
            k.set_option("transpose", 2)
        # host-only contexts build no device layouts; an asymmetric graph still installs
        k.set_option("transpose", 1)
        rng = np.random.default_rng(8)
        g = gen.random_dense(50, 0.3, rng, symmetric=False)
        k.set_graph(g)
        assert k.graph_info()["symmetric"] == 0


# ------------------------------------------------------------------------------------------------
# Bitmask segments (option "mask_min")
# ------------------------------------------------------------------------------------------------

def _same_rows(k1, k2, n, off=0):
    """Row lists and layers of k2 (rows shifted by off) equal those of k1."""
    for m in range(n):
        a1, b1 = k1.row_lists(m)
        a2, b2 = k2.row_lists(m + off)
        assert np.array_equal(a1, a2) and np.array_equal(b1 + off, b2), m
        c1, l1 = k1.row_layers(m)
        c2, l2 = k2.row_layers(m + off)
        assert np.array_equal(c1 + off, c2) and np.array_equal(l1, l2), m


@pytest.mark.parametrize("mask_min", [0.0, 0.1])
def test_mask_segments_match_lists(mask_min):
    """With bitmask segments the layout holds the same entries as with lists: every row's listed
    columns, layers and inter entries are unchanged, the adjacency rebuilds exactly, and the
    lists keep only the segments below the threshold."""
    rng = np.random.default_rng(81)
    sizes = np.array([700, 1, 64, 1300, 7, 530])
    rho = np.array([0.9, 0.5, 0.3, 0.6, 1.0, 0.97])
    g = gen.sbm(sizes, rho, 0.004, key=777, uperm=rng.permutation(sizes.sum()).astype(np.int32))
    with host_ctx(chunk=512, tile_rows=64) as k0, host_ctx(chunk=512, tile_rows=64, mask_min=mask_min) as k1:
        k0.set_graph(g)
        k1.set_graph(g)
        assert k0.graph_masks() == {"mask_segments": 0, "mask_bytes": 0}
        ms = k1.graph_masks()
        assert ms["mask_segments"] > 0
        i0, i1 = k0.graph_info(), k1.graph_info()
        assert i1["list_padded"] < i0["list_padded"] and i1["list_entries"] < i0["list_entries"]
        assert i1["inter_entries"] == i0["inter_entries"]
        # 16 bytes per 128-column unit and row of every bitmask segment
        assert ms["mask_bytes"] % 16 == 0
        _same_rows(k0, k1, g.n)
        check_layout(k1, g, 0.5)
    # below the least chunk width nothing is converted
    with host_ctx(chunk=448, mask_min=0.0) as k:
        k.set_graph(g)
        assert k.graph_masks()["mask_segments"] == 0


def test_mask_segments_weighted_and_pairs():
    """Weighted layers and dense off-diagonal blocks convert segment by segment as well."""
    rng = np.random.default_rng(82)
    gw = gen.weighted_sbm([600, 1, 70, 650], [2, 0, 0, 3], 0.25, 4, 0.03, rng,
                          uperm=rng.permutation(1321).astype(np.int32))
    V = np.zeros((3, 3), dtype=np.int32)
    V[0, 0] = V[1, 1] = V[0, 1] = V[1, 0] = 1
    gp = _pair_graph(rng, [600, 540, 40], V)
    for g in (gw, gp):
        with host_ctx(chunk=512, tile_rows=64) as k0, host_ctx(chunk=512, tile_rows=64, mask_min=0.0) as k1:
            k0.set_graph(g)
            k1.set_graph(g)
            assert k1.graph_masks()["mask_segments"] > 0
            assert k1.graph_pairs() == k0.graph_pairs()
            _same_rows(k0, k1, g.n)
        if g is gw:
            with host_ctx(chunk=512, tile_rows=64, mask_min=0.0) as k:
                k.set_graph(g)
                check_weighted_layout(k, g)
        else:
            with host_ctx(chunk=512, tile_rows=64, mask_min=0.0) as k:
                k.set_graph(g)
                check_layout(k, g, 0.5)


def test_mask_segments_in_batch():
    """A batch keeps every instance's bitmask segments, with their offsets shifted."""
    rng = np.random.default_rng(83)
    gs = [gen.sbm(np.array([520 + 40 * i, 600]), np.array([0.8, 0.4]), 0.01, key=90 + i,
                  uperm=rng.permutation(1120 + 40 * i).astype(np.int32)) for i in range(3)]
    with host_ctx(chunk=512, mask_min=0.0) as k:
        k.set_batch([(g, 1.0, np.zeros(g.n), np.zeros(g.n)) for g in gs])
        total = k.graph_masks()
        off = 0
        segs = 0
        for g in gs:
            with host_ctx(chunk=512, mask_min=0.0) as k1:
                k1.set_graph(g)
                segs += k1.graph_masks()["mask_segments"]
                _same_rows(k1, k, g.n, off)
            off += g.n
        assert total["mask_segments"] == segs > 0


@pytest.mark.parametrize("opts", [dict(), dict(mask_sub=128, mask_item=1), dict(mask_sub=256, mask_item=20000),
                                  dict(mask_sub=1024, mask_item=10**9, tile_rows=512, chunk=1024)])
def test_mask_items_cover_every_bitmask_unit(opts):
    """The bitmask work items (one workgroup each) hold every 128-column unit of every row of
    every bitmask segment exactly once: rows x units x 16 bytes summed over the items equals the
    layout's bitmask bytes. An item of more than one sub-chunk stays within mask_item cells;
    items launch largest first; their partial-sum rows are disjoint runs of their tile's rows
    covering the item buffer; a tile's items follow its segments in order."""
    rng = np.random.default_rng(81)
    sizes = np.array([700, 1, 64, 1300, 7, 530])
    rho = np.array([0.9, 0.5, 0.3, 0.6, 1.0, 0.97])
    g = gen.sbm(sizes, rho, 0.004, key=777, uperm=rng.permutation(sizes.sum()).astype(np.int32))
    base = dict(chunk=512, tile_rows=64, mask_min=0.0)
    base.update(opts)
    with host_ctx(**base) as k:
        k.set_graph(g)
        ms = k.graph_masks()
        it = k.graph_mask_items()
    assert ms["mask_segments"] > 0 and len(it) > 0
    tile, block, seg, sub, nsub, rows, units, cells, out = it.T
    assert np.all(nsub >= 1) and np.all(rows >= 1)
    assert int(np.sum(rows * units)) * 16 == ms["mask_bytes"]
    budget = opts.get("mask_item", 32768)
    assert np.all((nsub == 1) | (cells <= budget))
    assert np.all(np.diff(cells) <= 0)
    o = np.argsort(out, kind="stable")
    assert out[o][0] == 0 and np.array_equal(out[o][1:], (out + rows)[o][:-1])
    for t in np.unique(tile):
        m = np.flatnonzero(tile == t)
        m = m[np.argsort(out[m])]
        assert len(set(block[m])) == 1 and len(set(rows[m])) == 1
        assert list(zip(seg[m], sub[m])) == sorted(zip(seg[m], sub[m]))
    with host_ctx() as k:
        _expect(K.KUR_ESTATE, k.graph_mask_items)
