"""GPU: kur_diagnostics_noalloc (fixed scratch, no device allocation) against kur_diagnostics.

Both run the same kernels in the same order, so the three diagnostics agree bit for bit: on two
calls in a row, the second on a smaller graph (the scratch keeps the first call's larger
contents, which the second must not read), on a second context of the same device, and after
RK4 steps. A graph above the scratch's 2^24 nodes is refused with KUR_EINVAL.
"""
import numpy as np
import pytest

import gen
from paper_2102_07167_amd import Kuramoto
from paper_2102_07167_amd.kur import KUR_EINVAL, KurError

pytestmark = pytest.mark.gpu


def setup(k, w):
    k.set_graph(w.graph)
    k.set_params(w.omega, w.K)
    k.set_phases(w.theta0)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_matches_diagnostics(need_gpu, dtype):
    big = gen.sbm_equal(n_comm=16, comm_size=700, rho_in=0.9, p_out=1e-3, K=3.0, seed=71)
    small = gen.sbm_equal(n_comm=3, comm_size=257, rho_in=0.6, p_out=5e-3, K=1.5, seed=72)
    with Kuramoto(dtype, device=0) as k:
        setup(k, big)
        a = k.diagnostics_noalloc()
        b = k.diagnostics()
        assert a == b
        setup(k, small)  # a smaller input on the same context: fewer partials than the scratch holds
        a = k.diagnostics_noalloc()
        b = k.diagnostics()
        assert a == b
        k.step_rk4(small.dt, 25)
        assert k.diagnostics_noalloc() == k.diagnostics()
        with Kuramoto(dtype, device=0) as k2:  # a second context on the same device
            setup(k2, big)
            k2.set_option("timing", 1)
            assert k2.diagnostics_noalloc() == k2.diagnostics()
        assert k.diagnostics_noalloc() == k.diagnostics()


def test_noalloc_rejects_graphs_above_its_scratch(need_gpu):
    n = (1 << 24) + 1
    with Kuramoto("f32", device=0) as k:
        k.set_graph_csr(n, np.zeros(n + 1, np.int64), np.zeros(1, np.int32), (np.arange(n) % 1024).astype(np.int32))
        k.set_params(np.zeros(n), 1.0)
        k.set_phases(np.zeros(n))
        with pytest.raises(KurError) as ei:
            k.diagnostics_noalloc()
        assert ei.value.status == KUR_EINVAL and "16777216" in str(ei.value)
