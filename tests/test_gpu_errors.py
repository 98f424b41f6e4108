"""GPU: the runtime error paths of the C ABI, forced from the host with valid arguments.

KUR_ENONFINITE: finite inputs whose RK4 stages overflow (omega = 1e300 with a step that makes
dt omega infinite in FP64; in FP32 omega itself rounds to infinity on upload) give a non-finite
order-parameter sample, which kur_step_rk4 reports. KUR_ENOMEM: a recording run whose stage
record (16 n reals per step) exceeds the device's memory is refused before any launch, with the
size in kur_last_error. After either failure the same context takes new inputs and matches the
oracle again. Every kernel runs to its normal end: non-finite values only flow through
arithmetic, and the refused allocation launches nothing.
"""
import numpy as np
import pytest

import gen
import oracle
from paper_2102_07167_amd import Kuramoto
from paper_2102_07167_amd.kur import KUR_ENOMEM, KUR_ENONFINITE, KurError

pytestmark = pytest.mark.gpu


def wrap(x):
    return np.remainder(x + np.pi, 2 * np.pi) - np.pi


def small():
    return gen.sbm_equal(n_comm=4, comm_size=256, rho_in=0.9, p_out=2e-3, K=3.0, steps=50, seed=17)


def check_recovers(k, w, dtype):
    k.set_params(w.omega, w.K)
    k.set_phases(w.theta0)
    k.step_rk4(w.dt, w.steps)
    th = k.get_phases()
    tho, _, _ = oracle.rk4(w.graph, w.omega, w.K, w.theta0, w.dt, w.steps)
    tol = 1e-12 * max(1.0, np.abs(tho).max()) if dtype == "f64" else 1e-5
    assert np.abs(wrap(th - tho)).max() <= tol


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_nonfinite_phases_are_reported(need_gpu, dtype):
    w = small()
    if dtype == "f32":
        w.omega = w.omega.astype(np.float32).astype(np.float64)
        w.theta0 = w.theta0.astype(np.float32).astype(np.float64)
    with Kuramoto(dtype, device=0) as k:
        k.set_graph(w.graph)
        k.set_params(np.full(w.graph.n, 1e300), w.K)
        k.set_phases(w.theta0)
        dt = 1e9 if dtype == "f64" else 0.01
        with pytest.raises(KurError) as ei:
            k.step_rk4(dt, 3, r_every=1)
        assert ei.value.status == KUR_ENONFINITE
        assert "non-finite" in str(ei.value)
        check_recovers(k, w, dtype)


def test_stage_record_beyond_device_memory(need_gpu):
    w = gen.sbm_equal(n_comm=64, comm_size=1024, steps=20)
    n = w.graph.n
    nsteps = 100000  # 16 n reals per step of FP64: 8.4 MB per step, 839 GB in all
    with Kuramoto("f64", device=0) as k:
        k.set_graph(w.graph)
        k.set_params(w.omega, w.K)
        k.set_phases(w.theta0)
        k.set_option("checkpoint_every", 1000)
        k.set_option("record_stages", 1)
        with pytest.raises(KurError) as ei:
            k.step_rk4(w.dt, nsteps)
        assert ei.value.status == KUR_ENOMEM
        msg = str(ei.value)
        assert "stage record" in msg and "GB" in msg
        gb = float(msg.split("(")[1].split(" GB")[0])
        assert abs(gb - 16 * 8 * n * nsteps / 1e9) <= 1e-3 * gb
        assert k.recorded_run()[0] == 0
        # nothing ran: the phases are those set before the call
        assert np.abs(k.get_phases() - w.theta0).max() < 1e-14
        k.set_option("checkpoint_every", 0)
        k.set_option("record_stages", 0)
        w.steps = 20
        check_recovers(k, w, "f64")
