"""CPU tests of the layout autotuner's host side: the tuning-cache signature, cache lookup
(last matching line wins, malformed lines skipped, out-of-range values rejected) and the
layout a cached choice installs, which is checked against the dense adjacency. Timing needs a
device: without a cached entry a host-only context must refuse."""
import numpy as np
import pytest

import gen
from paper_2102_07167_amd import kur as K

from test_abi_host import check_layout, host_ctx


def small_sbm(seed=3):
    rng = np.random.default_rng(seed)
    sizes = np.array([130, 1, 64, 200, 7])
    rho = np.array([0.9, 0.5, 0.3, 0.7, 1.0])
    return gen.sbm(sizes, rho, 0.02, key=12345, uperm=rng.permutation(sizes.sum()).astype(np.int32))


def test_tune_key_identifies_graph_and_dtype():
    g1, g2 = small_sbm(3), small_sbm(4)
    g3 = gen.sbm(np.array([130, 1, 64, 200, 7]), np.array([0.9, 0.5, 0.3, 0.7, 0.95]), 0.02, key=999,
                 uperm=np.arange(402, dtype=np.int32))
    with host_ctx("f32") as a, host_ctx("f64") as b:
        k1 = a.tune_key(g1)
        assert k1 == a.tune_key(g1) and " host " in k1 and k1.startswith("kur2 f32")
        assert b.tune_key(g1).startswith("kur2 f64") and b.tune_key(g1) != k1
        assert a.tune_key(g2) != k1  # same sizes, other labels order
        assert a.tune_key(g3) != k1  # other edges


def test_autotune_without_cache_needs_device(tmp_path):
    g = small_sbm()
    with host_ctx() as k:
        with pytest.raises(K.KurError) as ei:
            k.autotune(g, effort=0, cache=str(tmp_path / "none.tsv"))
        assert ei.value.status == K.KUR_EDEVICE
        with pytest.raises(K.KurError) as ei:
            k.autotune(g, effort=0)
        assert ei.value.status == K.KUR_EDEVICE


def test_tune_tiles_needs_device():
    g = small_sbm()
    with host_ctx() as k:
        k.set_graph(g)
        with pytest.raises(K.KurError) as ei:
            k.tune_tiles(0)
        assert ei.value.status == K.KUR_EDEVICE
        with pytest.raises(K.KurError) as ei:
            k.tune_tiles(3)
        assert ei.value.status == K.KUR_EINVAL


def test_cached_choice_installs_its_layout(tmp_path):
    g = small_sbm()
    path = tmp_path / "tune.tsv"
    with host_ctx() as k:
        key = k.tune_key(g)
        path.write_text(
            "kur2 f32 host n=1 nnz=0 h=0000000000000000\t0.9 64 256 64 1 1 8 1\n"
            + key + "\t0.6 128 256 64 4096 2 8 1.5\n"
            + key + "\tgarbage\n"
            + key + "\t0.4 192 512 128 8192 4 1 1.25\n"
            + "no tab here\n")
        rep = k.autotune(g, effort=1, cache=str(path))
        assert rep["cache"] == 1 and rep["builds"] == 1 and rep["timed"] == 0
        assert (rep["tau"], rep["chunk"], rep["threads"], rep["tile_rows"], rep["tile_min_cost"],
                rep["flat_min_vec"], rep["xcds"], rep["ms_per_step"]) == (0.4, 192, 512, 128, 8192, 4.0, 1, 1.25)
        assert np.isnan(rep["ms_per_step_start"])
        info = k.graph_info()
        assert info["chunk"] == 192
        check_layout(k, g, 0.4)
        # the cached options stay in force for the next build
        k.set_graph(g)
        assert k.graph_info()["chunk"] == 192
        check_layout(k, g, 0.4)


def test_cached_gather_choice(tmp_path):
    """A cache line's optional ninth field selects the inter-block gathers (0 pairs, 1 phases);
    lines without it report -1 (the dtype's default); a ninth field other than 0 or 1 makes the
    line malformed, so an earlier matching line wins."""
    g = small_sbm()
    path = tmp_path / "tune.tsv"
    with host_ctx() as k:
        key = k.tune_key(g)
        path.write_text(key + "\t0.5 128 512 256 16384 8 1 1.0\n")
        assert k.autotune(g, cache=str(path))["inter_gather"] == -1
        path.write_text(key + "\t0.5 128 512 256 16384 8 1 1.0 0\n")
        assert k.autotune(g, cache=str(path))["inter_gather"] == 0
        path.write_text(key + "\t0.5 128 512 256 16384 8 1 1.0 1\n" + key + "\t0.5 128 512 256 16384 8 1 2.0 5\n")
        rep = k.autotune(g, cache=str(path))
        assert rep["inter_gather"] == 1 and rep["ms_per_step"] == 1.0


def test_cached_choice_out_of_range_is_rejected(tmp_path):
    g = small_sbm()
    path = tmp_path / "tune.tsv"
    with host_ctx() as k:
        path.write_text(k.tune_key(g) + "\t0.5 100 512 256 16384 8 8 1\n")
        with pytest.raises(K.KurError) as ei:
            k.autotune(g, cache=str(path))
        assert ei.value.status == K.KUR_EINVAL


def test_cached_mask_choice(tmp_path):
    """A cache line's optional tenth field is the bitmask threshold: the graph is built with
    bitmask segments from it; lines without it build lists only; a negative tenth field makes the
    line malformed, so an earlier matching line wins."""
    g = small_sbm()
    path = tmp_path / "tune.tsv"
    with host_ctx() as k:
        key = k.tune_key(g)
        path.write_text(key + "\t0.5 512 512 256 16384 8 1 1.0 1\n")
        k.autotune(g, cache=str(path))
        assert k.graph_masks()["mask_segments"] == 0
        path.write_text(key + "\t0.5 512 512 256 16384 8 1 1.0 1 0\n")
        k.autotune(g, cache=str(path))
        with_masks = k.graph_masks()
        assert with_masks["mask_segments"] > 0 and with_masks["mask_bytes"] > 0
        path.write_text(key + "\t0.5 512 512 256 16384 8 1 1.0 1 0\n" + key + "\t0.5 512 512 256 16384 8 1 2.0 1 -1\n")
        rep = k.autotune(g, cache=str(path))
        assert rep["ms_per_step"] == 1.0 and k.graph_masks() == with_masks
