"""GPU adjoint: the discrete adjoint of the RK4 trajectory against the oracle's discrete adjoint,
exact cases, central differences of the GPU FP64 forward, and the autograd wrapper.

Tolerances: FP64 vs oracle adjoint max |dg| <= 1e-10 max |g| (both are the same discrete
adjoint; the difference is rounding); FP32 vs oracle <= 1e-3 max |g|. Central differences with
step h on the FP64 forward carry an error of about eps |L| / h + h^2 |L3| / 6 (L3 the third
derivative), so they are compared to 1e-6 of max(|g_fd|, 1e-3 max |g|) plus that error (see the
full-size test).
"""
import math

import numpy as np
import pytest

import gen
import oracle
from paper_2102_07167_amd import Kuramoto

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


def ctx(w, dtype, **opts):
    k = Kuramoto(dtype, device=0)
    for key, v in opts.items():
        k.set_option(key, v)
    k.set_graph(w.graph)
    k.set_params(w.omega, w.K)
    k.set_phases(w.theta0)
    return k


def ragged_sbm(seed=3):
    rng = np.random.default_rng(seed)
    sizes = np.array([150, 1, 97, 260, 33])
    rho = np.array([0.9, 0.5, 0.35, 0.7, 1.0])
    n = int(sizes.sum())
    g = gen.sbm(sizes, rho, 0.02, key=777, uperm=rng.permutation(n).astype(np.int32))
    return gen.Workload("ragged", g, rng.standard_normal(n), rng.uniform(0, 2 * np.pi, n), 2.5, 0.02, 30,
                        target=rng.uniform(0, 2 * np.pi, n))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("ckpt", [1, 7, 100])
@pytest.mark.parametrize("opts", [dict(), dict(chunk=64, tile_rows=64, flat_min_vec=0.5), dict(scaling=1),
                                  dict(mask_min=0.0, chunk=512)])
def test_adjoint_matches_oracle(need_gpu, dtype, ckpt, opts):
    w = ragged_sbm()
    scaling = opts.get("scaling", 0)
    if dtype == "f32":
        w.omega = w.omega.astype(np.float32).astype(np.float64)
        w.theta0 = w.theta0.astype(np.float32).astype(np.float64)
    thT, _, _ = oracle.rk4(w.graph, w.omega, w.K, w.theta0, w.dt, w.steps, scaling=scaling)
    _, seed = oracle.loss_and_seed(thT, w.target)
    gt_o, gw_o, gk_o = oracle.adjoint_rk4(w.graph, w.omega, w.K, w.theta0, w.dt, w.steps, seed, scaling=scaling)
    with ctx(w, dtype, **opts) as k:
        assert k.graph_info()["symmetric"] == 1
        gt, gw, gk = k.adjoint_rk4(w.dt, w.steps, seed, theta0=w.theta0, ckpt_every=ckpt)
    tol = 1e-10 if dtype == "f64" else 1e-3
    for a, b in ((gt, gt_o), (gw, gw_o)):
        assert np.abs(a - b).max() <= tol * np.abs(b).max(), (np.abs(a - b).max(), np.abs(b).max())
    assert abs(gk - gk_o) <= tol * max(abs(gk_o), np.abs(gw_o).max())


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n", [1, 2, 97, 512, 1024, 1025])
def test_adjoint_complete_graph_one_workgroup(need_gpu, dtype, n):
    """Complete graphs of at most 1024 nodes run the whole adjoint in one workgroup (forward in
    the one-workgroup RK4 run, each checkpoint segment recomputed and swept back inside one
    launch); 1025 nodes take the row kernel. 30 steps, checkpoints every 7 (a ragged last
    segment), both scalings: against the oracle's discrete adjoint (1e-10 FP64, 1e-3 FP32, of
    the largest gradient) and against the row-kernel adjoint (option persistent = 0); the
    recorded variant (checkpoints kept by kur_step_rk4) gives the same gradients."""
    rng = np.random.default_rng(100 + n)
    om, th0, tgt = rng.standard_normal(n), rng.uniform(0, 2 * np.pi, n), rng.uniform(0, 2 * np.pi, n)
    K, dt, steps = 2.5, 0.01, 30
    if dtype == "f32":
        r32 = lambda x: np.asarray(x, dtype=np.float32).astype(np.float64)
        om, th0, K, dt = r32(om), r32(th0), float(np.float32(K)), float(np.float32(dt))
    tol = 1e-10 if dtype == "f64" else 1e-3
    g = gen.complete_graph(n)
    for scaling in (0, 1):
        thT, _, _ = oracle.rk4(g, om, K, th0, dt, steps, scaling=scaling)
        _, seed = oracle.loss_and_seed(thT, tgt)
        go = oracle.adjoint_rk4(g, om, K, th0, dt, steps, seed, scaling=scaling)
        got = {}
        for pers in (1, 0):
            with Kuramoto(dtype, device=0) as k:
                k.set_option("persistent", pers)
                k.set_option("scaling", scaling)
                k.set_graph(g)
                k.set_params(om, K)
                k.set_phases(th0)
                got[pers] = k.adjoint_rk4(dt, steps, seed, theta0=th0, ckpt_every=7)
                if pers:
                    k.set_option("checkpoint_every", 7)
                    k.step_rk4(dt, steps)
                    k.set_option("checkpoint_every", 0)
                    got["rec"] = k.adjoint_recorded(seed)
        gmax = max(np.abs(go[0]).max(), np.abs(go[1]).max())
        for key in (1, 0, "rec"):
            gt, gw, gk = got[key]
            assert np.abs(gt - go[0]).max() <= tol * np.abs(go[0]).max(), (key, scaling)
            assert np.abs(gw - go[1]).max() <= tol * np.abs(go[1]).max(), (key, scaling)
            assert abs(gk - go[2]) <= tol * max(abs(go[2]), gmax), (key, scaling)


def test_adjoint_complete_graph_long_run(need_gpu):
    """The one-workgroup adjoint over 70001 steps (two forward launches and two reverse
    launches of whole checkpoint segments): L = sum theta(T) gives dL/dtheta0 = 1, dL/domega = T
    and dL/dK = 0 (the linear invariant of the symmetric uniform model)."""
    rng = np.random.default_rng(9)
    n, dt, steps = 64, 0.001, 70001
    with Kuramoto("f64", device=0) as k:
        k.set_graph(gen.complete_graph(n))
        k.set_params(rng.standard_normal(n), 3.0)
        th0 = rng.uniform(0, 2 * np.pi, n)
        k.set_phases(th0)
        gt, gw, gk = k.adjoint_rk4(dt, steps, np.ones(n), theta0=th0, ckpt_every=1000)
    T = steps * dt
    assert np.abs(gt - 1).max() < 1e-9
    assert np.abs(gw - T).max() < 1e-9 * T
    assert abs(gk) < 1e-9 * T * n


def test_adjoint_exact_cases(need_gpu):
    """L = sum theta(T): dL/dtheta0 = 1, dL/domega = T, dL/dK = 0 (linear invariant, symmetric A,
    uniform scaling); K = 0: dL/dtheta0 = seed, dL/domega = T seed."""
    w = ragged_sbm(5)
    n, steps, dt = w.graph.n, 40, 0.02
    with ctx(w, "f64") as k:
        gt, gw, gk = k.adjoint_rk4(dt, steps, np.ones(n), theta0=w.theta0, ckpt_every=9)
        assert np.abs(gt - 1).max() < 1e-12 and np.abs(gw - steps * dt).max() < 1e-12 and abs(gk) < 1e-11
        seed = np.random.default_rng(1).standard_normal(n)
        k.set_params(w.omega, 0.0)
        gt, gw, gk = k.adjoint_rk4(dt, steps, seed, theta0=w.theta0, ckpt_every=40)
        assert np.abs(gt - seed).max() < 1e-13 and np.abs(gw - steps * dt * seed).max() < 1e-12
        # no steps: the seed comes back unchanged
        gt, gw, gk = k.adjoint_rk4(dt, 0, seed, theta0=w.theta0)
        assert np.array_equal(gt, seed) and not gw.any() and gk == 0.0


def test_adjoint_rejects_asymmetric_without_transpose(need_gpu):
    from paper_2102_07167_amd.kur import KurError, KUR_EINVAL
    rng = np.random.default_rng(2)
    g = gen.random_dense(40, 0.3, rng, symmetric=False)
    with Kuramoto("f64", device=0) as k:
        k.set_graph(g)
        k.set_params(np.zeros(40), 1.0)
        k.set_phases(np.zeros(40))
        assert k.graph_info()["symmetric"] == 0
        with pytest.raises(KurError) as ei:
            k.adjoint_rk4(0.1, 3, np.ones(40))
        assert ei.value.status == KUR_EINVAL


def asymmetric_workload(seed, weighted=False):
    """A ragged block graph made asymmetric: a random 30 % of its entries dropped one way, the
    block 0 -> 2 made dense (a dense off-diagonal block in one direction only, 2 -> 0 empty);
    weighted: value 2 on 80 % of the kept entries, else 1..3."""
    rng = np.random.default_rng(seed)
    sizes = [150, 1, 97, 260, 33]
    n = sum(sizes)
    V = np.zeros((5, 5), dtype=np.int32)
    for b in (0, 2, 3, 4):
        V[b, b] = 1
    A = gen.block_model(sizes, V, 0.1, 1, rng).dense().astype(np.int32)
    A[rng.random((n, n)) < 0.3] = 0
    A[:150, 151:248] = rng.random((150, 97)) < 0.9
    A[151:248, :150] = 0
    np.fill_diagonal(A, 0)
    if weighted:
        A = A * np.where(rng.random((n, n)) < 0.8, 2, rng.integers(1, 4, (n, n)))
    labels = np.repeat(np.arange(5), sizes).astype(np.int32)
    perm = rng.permutation(n)
    B = np.zeros_like(A)
    B[np.ix_(perm, perm)] = A
    lab = np.empty(n, dtype=np.int32)
    lab[perm] = labels
    g = gen.from_dense(B, lab)
    return gen.Workload("asym", g, rng.standard_normal(n), rng.uniform(0, 2 * np.pi, n), 2.5, 0.02, 30,
                        target=rng.uniform(0, 2 * np.pi, n))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("opts", [dict(), dict(chunk=64, tile_rows=64, flat_min_vec=0.5, ckpt=7),
                                  dict(scaling=1, threads=256), dict(weighted=True), dict(threads=128, chunk=64),
                                  dict(mask_min=0.0, chunk=512), dict(mask_min=0.0, chunk=512, weighted=True),
                                  dict(mask_min=0.0, chunk=512, mask_sub=128, mask_item=5000)])
def test_adjoint_asymmetric_with_transpose(need_gpu, dtype, opts):
    """Asymmetric A with the option "transpose": the gathers of J^T l run over the layout of A^T
    and match the oracle's discrete adjoint, which scatters the rows of A."""
    opts = dict(opts)
    w = asymmetric_workload(31, weighted=opts.pop("weighted", False))
    ckpt = opts.pop("ckpt", 100)
    scaling = opts.get("scaling", 0)
    if dtype == "f32":
        w.omega = w.omega.astype(np.float32).astype(np.float64)
        w.theta0 = w.theta0.astype(np.float32).astype(np.float64)
    thT, _, _ = oracle.rk4(w.graph, w.omega, w.K, w.theta0, w.dt, w.steps, scaling=scaling)
    _, seed = oracle.loss_and_seed(thT, w.target)
    gt_o, gw_o, gk_o = oracle.adjoint_rk4(w.graph, w.omega, w.K, w.theta0, w.dt, w.steps, seed, scaling=scaling)
    with ctx(w, dtype, transpose=1, **opts) as k:
        assert k.graph_info()["symmetric"] == 0
        gt, gw, gk = k.adjoint_rk4(w.dt, w.steps, seed, theta0=w.theta0, ckpt_every=ckpt)
        # the recorded variant gives the same gradients
        k.set_option("checkpoint_every", ckpt)
        k.set_phases(w.theta0)
        k.step_rk4(w.dt, w.steps)
        k.set_option("checkpoint_every", 0)
        gt2, gw2, gk2 = k.adjoint_recorded(seed)
    tol = 1e-10 if dtype == "f64" else 1e-3
    for a, b in ((gt, gt_o), (gw, gw_o)):
        assert np.abs(a - b).max() <= tol * np.abs(b).max(), (np.abs(a - b).max(), np.abs(b).max())
    assert abs(gk - gk_o) <= tol * max(abs(gk_o), np.abs(gw_o).max())
    assert np.array_equal(gt, gt2) and np.array_equal(gw, gw2) and gk == gk2


def _load_adjoint_fixture(name):
    """(L, dL/dK, rows, theta(T), dL/dtheta0, dL/domega) of a fixture written by
    tests/golden/make_sbm4x1024_adjoint.py (oracle only)."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)
    L = gk = None
    rows = []
    with open(path) as f:
        for line in f:
            p = line.split()
            if not p or p[0].startswith("#"):
                continue
            if p[0] == "L":
                L = float(p[1])
            elif p[0] == "gK":
                gk = float(p[1])
            elif p[0] == "row":
                rows.append([float(x) for x in p[1:]])
    a = np.array(rows)
    return L, gk, a[:, 0].astype(np.int64), a[:, 1], a[:, 2], a[:, 3]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_adjoint_sbm_4x1024_200_steps_matches_oracle(need_gpu, dtype):
    """The adjoint workload down-scaled to gen.sbm_equal(n_comm=4) (N = 4096), 200 steps,
    checkpoints every 32, the loss (1 - r(T))^2 + mean chordal distance: theta(T), L and the
    gradients of theta0 (seeded 1/4 of the rows), omega and K against the oracle's discrete
    adjoint stored in tests/golden/ (FP64 inputs: 1e-10 of the largest gradient, theta(T) at
    1e-12 max(1, |theta|); FP32-rounded inputs: 1e-3 and 1e-5). The seed dL/dtheta(T) is formed
    by the oracle's loss function from the GPU's own theta(T)."""
    w = gen.sbm_equal(n_comm=4, steps=200)
    tag = "f64in" if dtype == "f64" else "f32in"
    L_o, gk_o, rows, thT_o, gt_o, gw_o = _load_adjoint_fixture("sbm4x1024_adjoint_200_%s.txt" % tag)
    om, th0, K, dt = w.omega, w.theta0, w.K, w.dt
    if dtype == "f32":
        r32 = lambda x: np.asarray(x, dtype=np.float32).astype(np.float64)
        om, th0, K, dt = r32(om), r32(th0), float(np.float32(K)), float(np.float32(dt))
    with Kuramoto(dtype, device=0) as k:
        k.set_graph(w.graph)
        k.set_params(om, K)
        k.set_phases(th0)
        k.step_rk4(dt, w.steps)
        thT = k.get_phases(wrapped=False)
        L, seed = oracle.loss_and_seed(thT, w.target)
        gt, gw, gk = k.adjoint_rk4(dt, w.steps, seed, theta0=th0, ckpt_every=32)
    ptol = 1e-12 * max(1.0, np.abs(thT_o).max()) if dtype == "f64" else 1e-5
    assert np.abs(thT[rows] - thT_o).max() <= ptol
    assert abs(L - L_o) <= (1e-12 if dtype == "f64" else 1e-5) * abs(L_o)
    tol = 1e-10 if dtype == "f64" else 1e-3
    gmax = max(np.abs(gt_o).max(), np.abs(gw_o).max())
    assert np.abs(gt[rows] - gt_o).max() <= tol * np.abs(gt_o).max()
    assert np.abs(gw[rows] - gw_o).max() <= tol * np.abs(gw_o).max()
    assert abs(gk - gk_o) <= tol * max(abs(gk_o), gmax)


def _loss(k, w, th0, om, K, steps):
    k.set_params(om, K)
    k.set_phases(th0)
    k.step_rk4(w.dt, steps)
    return oracle.loss_and_seed(k.get_phases(), w.target)


def test_adjoint_sbm_64x1024_2000_steps_central_differences(need_gpu):
    """Equal-community SBM N = 65536 (64 x 1024), 2000 steps of dt 0.01, checkpoint every 32,
    loss (1 - r(T))^2 + mean chordal distance to seeded targets: 16 theta0, 15 omega coordinates
    and K against central differences of the GPU FP64 forward.

    Bound: |g - fd| <= 1e-6 max(|fd|, 1e-3 max|g|) + 2 eps |L| / h + h^2 / 6, with h = 1e-5. A
    central difference carries the rounding of two loss evaluations over 2h (measured at most
    0.4 eps |L| / h for h in [1e-7, 1e-5]) and the truncation h^2 |L3| / 6, L3 the third
    derivative along the coordinate (|L3| measured at most 0.44 where truncation dominates,
    h = 1e-3; 1 is used). h = 1e-5 balances the two; at h = 1e-6 the rounding alone (2.7e-10
    measured) exceeds 1e-9 of the largest gradient."""
    w = gen.sbm_equal(steps=2000, seed=1005)
    steps = w.steps
    with ctx(w, "f64") as k:
        L0, seed = _loss(k, w, w.theta0, w.omega, w.K, steps)
        gt, gw, gk = k.adjoint_rk4(w.dt, steps, seed, theta0=w.theta0, ckpt_every=32)
        rng = np.random.default_rng(55)
        h = 1e-5
        gmax = max(np.abs(gt).max(), np.abs(gw).max())
        noise = 2 * EPS * abs(L0) / h + h * h / 6

        def bound(fd):
            return 1e-6 * max(abs(fd), 1e-3 * gmax) + noise

        for j in rng.choice(w.graph.n, 16, replace=False):
            e = np.zeros(w.graph.n)
            e[j] = h
            fd = (_loss(k, w, w.theta0 + e, w.omega, w.K, steps)[0] - _loss(k, w, w.theta0 - e, w.omega, w.K, steps)[0]) / (2 * h)
            assert abs(gt[j] - fd) <= bound(fd), (j, gt[j], fd)
        for j in rng.choice(w.graph.n, 15, replace=False):
            e = np.zeros(w.graph.n)
            e[j] = h
            fd = (_loss(k, w, w.theta0, w.omega + e, w.K, steps)[0] - _loss(k, w, w.theta0, w.omega - e, w.K, steps)[0]) / (2 * h)
            assert abs(gw[j] - fd) <= bound(fd), (j, gw[j], fd)
        fd = (_loss(k, w, w.theta0, w.omega, w.K + h, steps)[0] - _loss(k, w, w.theta0, w.omega, w.K - h, steps)[0]) / (2 * h)
        assert abs(gk - fd) <= bound(fd), (gk, fd)


def test_adjoint_sbm_64x1024_2000_steps_fp32(need_gpu):
    """The same full-size adjoint in FP32 (central differences of an FP32 forward carry no
    signal at this step): its gradients against the FP64 adjoint on the same FP32-rounded
    inputs, within 1e-3 of the largest gradient (the FP32 bound of the smaller adjoint tests),
    for theta0, omega and K, with the loss and its seed formed from each run's own phases."""
    w = gen.sbm_equal(steps=2000, seed=1005)
    r32 = lambda x: np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)
    w.theta0, w.omega = r32(w.theta0), r32(w.omega)
    w.K, w.dt = float(np.float32(w.K)), float(np.float32(w.dt))
    grads = {}
    for dtype in ("f64", "f32"):
        with ctx(w, dtype) as k:
            L, seed = _loss(k, w, w.theta0, w.omega, w.K, w.steps)
            grads[dtype] = (L,) + tuple(k.adjoint_rk4(w.dt, w.steps, seed, theta0=w.theta0, ckpt_every=32))
    L64, gt64, gw64, gk64 = grads["f64"]
    L32, gt32, gw32, gk32 = grads["f32"]
    assert abs(L32 - L64) <= 1e-4 * abs(L64)
    assert np.isfinite(gt32).all() and np.isfinite(gw32).all() and np.isfinite(gk32)
    assert np.abs(gt32 - gt64).max() <= 1e-3 * np.abs(gt64).max()
    assert np.abs(gw32 - gw64).max() <= 1e-3 * np.abs(gw64).max()
    assert abs(gk32 - gk64) <= 1e-3 * max(abs(gk64), 1e-3 * np.abs(gw64).max())


@pytest.mark.parametrize("record_stages", [False, True])
@pytest.mark.parametrize("where", ["cuda", "cpu"])
def test_autograd_function(need_gpu, record_stages, where):
    """The loss of config 5, (1 - r(T))^2 + mean chordal distance to a target, through the
    autograd wrappers: theta(T) and r(T) both come from the library (device calls), and the
    gradients of theta0, omega and K match the oracle's discrete adjoint to 1e-10. Tensors on
    the GPU stay there; CPU tensors are moved to the device and their gradients moved back."""
    import torch
    from paper_2102_07167_amd.autograd import integrate, order_parameter
    w = ragged_sbm(9)
    with ctx(w, "f64") as k:
        th0 = torch.tensor(w.theta0, device=where, requires_grad=True)
        om = torch.tensor(w.omega, device=where, requires_grad=True)
        K = torch.tensor(w.K, dtype=torch.float64, device=where, requires_grad=True)
        thT = integrate(k, th0, om, K, w.dt, w.steps, ckpt_every=8, record_stages=record_stages)
        assert thT.device.type == where
        tgt = torch.tensor(w.target, device=where)
        r, _ = order_parameter(k, thT)
        loss = (1 - r) ** 2 + (2 * (1 - torch.cos(thT - tgt))).mean()
        loss.backward()
        thT_o, _, _ = oracle.rk4(w.graph, w.omega, w.K, w.theta0, w.dt, w.steps)
        L_o, seed = oracle.loss_and_seed(thT_o, w.target)
        assert abs(loss.item() - L_o) < 1e-12
        gt_o, gw_o, gk_o = oracle.adjoint_rk4(w.graph, w.omega, w.K, w.theta0, w.dt, w.steps, seed)
        assert th0.grad.device.type == where and om.grad.device.type == where
        assert np.abs(th0.grad.cpu().numpy() - gt_o).max() <= 1e-10 * np.abs(gt_o).max()
        assert np.abs(om.grad.cpu().numpy() - gw_o).max() <= 1e-10 * np.abs(gw_o).max()
        assert abs(K.grad.item() - gk_o) <= 1e-10 * max(abs(gk_o), 1e-3)


def test_autograd_fp32_and_psi(need_gpu):
    """FP32 model with float32 tensors: gradients within the FP32 bound (1e-3) of the oracle's
    FP64 adjoint; a loss on psi(T) differentiates through the library's order parameter."""
    import torch
    from paper_2102_07167_amd.autograd import integrate, order_parameter
    w = ragged_sbm(13)
    w.omega = w.omega.astype(np.float32).astype(np.float64)
    w.theta0 = w.theta0.astype(np.float32).astype(np.float64)
    with ctx(w, "f32") as k:
        th0 = torch.tensor(w.theta0, dtype=torch.float32, device="cuda", requires_grad=True)
        om = torch.tensor(w.omega, dtype=torch.float32, device="cuda", requires_grad=True)
        thT = integrate(k, th0, om, w.K, w.dt, w.steps, ckpt_every=8)
        r, psi = order_parameter(k, thT)
        (torch.sin(psi) + r).backward()
    thT_o, _, _ = oracle.rk4(w.graph, w.omega, w.K, w.theta0, w.dt, w.steps)
    ro, po = oracle.order_parameter(thT_o)
    n = w.graph.n
    # d(sin psi + r)/dtheta_m = cos(psi) cos(psi - theta_m)/(N r) + sin(psi - theta_m)/N
    seed = (np.cos(po) * np.cos(po - thT_o) / ro + np.sin(po - thT_o)) / n
    gt_o, gw_o, _ = oracle.adjoint_rk4(w.graph, w.omega, w.K, w.theta0, w.dt, w.steps, seed)
    assert np.abs(th0.grad.cpu().numpy() - gt_o).max() <= 1e-3 * np.abs(gt_o).max()
    assert np.abs(om.grad.cpu().numpy() - gw_o).max() <= 1e-3 * np.abs(gw_o).max()


def test_recorded_adjoint_matches_full_adjoint(need_gpu):
    """Checkpoints kept by kur_step_rk4 give bit for bit the gradients of the full adjoint, which
    repeats the forward pass; a change of omega or K invalidates the recording."""
    from paper_2102_07167_amd.kur import KurError, KUR_ESTATE
    w = ragged_sbm(7)
    seed = np.random.default_rng(3).standard_normal(w.graph.n)
    for dtype in ("f64", "f32"):
        with ctx(w, dtype) as k:
            with pytest.raises(KurError) as ei:
                k.adjoint_recorded(seed)
            assert ei.value.status == KUR_ESTATE
            k.set_option("checkpoint_every", 7)
            k.step_rk4(w.dt, 30)
            k.set_option("checkpoint_every", 0)
            serial, dt, ns = k.recorded_run()
            assert serial > 0 and dt == w.dt and ns == 30
            a = k.adjoint_recorded(seed)
            b = k.adjoint_rk4(w.dt, 30, seed, theta0=w.theta0, ckpt_every=7)
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]
            k.set_params(w.omega, w.K * 1.5)
            assert k.recorded_run()[0] == 0
            with pytest.raises(KurError):
                k.adjoint_recorded(seed)


@pytest.mark.parametrize("asym", [False, True])
def test_recorded_stages_adjoint(need_gpu, asym):
    """With option record_stages the recording run keeps every stage state and the recorded
    adjoint recomputes nothing: the gradients equal bit for bit those of the checkpoint path
    (both use the same stage states); the run itself, its r samples and the steps after it equal
    those of a plain run bit for bit."""
    w = asymmetric_workload(41) if asym else ragged_sbm(9)
    n = w.graph.n
    seed = np.random.default_rng(4).standard_normal(n)
    opts = dict(transpose=1) if asym else {}
    for dtype in ("f64", "f32"):
        with ctx(w, dtype, **opts) as k:
            r0, _ = k.step_rk4(w.dt, 30, r_every=5)
            th0 = k.get_phases(wrapped=False)
            k.step_rk4(w.dt, 7)
            th_a = k.get_phases(wrapped=False)
        with ctx(w, dtype, **opts) as k:
            k.set_option("checkpoint_every", 8)
            k.set_option("record_stages", 1)
            r1, _ = k.step_rk4(w.dt, 30, r_every=5)
            k.set_option("checkpoint_every", 0)
            assert np.array_equal(r0, r1)
            assert np.array_equal(k.get_phases(wrapped=False), th0)
            a = k.adjoint_recorded(seed)
            k.step_rk4(w.dt, 7)
            assert np.array_equal(k.get_phases(wrapped=False), th_a)
        with ctx(w, dtype, **opts) as k:
            k.set_option("checkpoint_every", 8)
            k.step_rk4(w.dt, 30)
            k.set_option("checkpoint_every", 0)
            b = k.adjoint_recorded(seed)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]
        if dtype == "f64":
            go = oracle.adjoint_rk4(w.graph, w.omega, w.K, w.theta0, w.dt, 30, seed)
            assert np.abs(a[0] - go[0]).max() <= 1e-10 * np.abs(go[0]).max()


def test_autograd_two_forwards(need_gpu):
    """Backward of an earlier forward after a later one on the same model still gets its own
    gradients (the recording belongs to the later run, so the adjoint repeats the forward)."""
    import torch
    from paper_2102_07167_amd.autograd import integrate
    w = ragged_sbm(11)
    with ctx(w, "f64") as k:
        th_a = torch.tensor(w.theta0, device="cuda", requires_grad=True)
        th_b = torch.tensor(w.theta0[::-1].copy(), device="cuda", requires_grad=True)
        om = torch.tensor(w.omega, device="cuda")
        K = torch.tensor(w.K, dtype=torch.float64, device="cuda")
        out_a = integrate(k, th_a, om, K, w.dt, 20, 8)
        out_b = integrate(k, th_b, om, K, w.dt, 20, 8)
        out_a.sum().backward()
        out_b.sum().backward()
    # L = sum theta(T): dL/dtheta0 = 1 (symmetric A, uniform scaling)
    assert np.abs(th_a.grad.cpu().numpy() - 1).max() < 1e-12 and np.abs(th_b.grad.cpu().numpy() - 1).max() < 1e-12
