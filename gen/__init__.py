"""Seeded synthetic inputs for the Kuramoto-on-graphs workloads.

Input infrastructure shared by the oracle, the tests and the benchmark. It produces graphs
(adjacency in user order plus planted community labels), intrinsic frequencies, initial phases
and target phases. It contains none of the method's arithmetic: no right-hand side, no order
parameters, no block split, no integrator.

Every workload is synthetic, as in the paper, whose experiments use random matrices and closed
form initial data (Sec. 2 "Numerical comparisons", Sec. 3 "Numerical comparisons", "Community
detection in graphs" and "Numerical integration").

Random streams: ``numpy.random.SeedSequence(seed).spawn(5)`` gives one PCG64 stream each for the
graph, the user permutation, omega, theta0 and the target phases. The graph stream only draws
community sizes, densities and a 64-bit key; pair decisions are counter-based hashes in
``kurgen.c`` so they are independent of thread count.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libkurgen.so")
_lib = None

TWO_PI = 2.0 * math.pi


def build(force: bool = True) -> str:
    """Compile kurgen.c with gcc (OpenMP) into gen/libkurgen.so."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp,
                               os.path.join(_HERE, "kurgen.c"), "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        i64, u64, f64 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
        lib.kg_inter_pairs.restype = i64
        lib.kg_inter_pairs.argtypes = [i64, P, i64, f64, u64, P, P]
        lib.kg_sbm_degrees.restype = None
        lib.kg_sbm_degrees.argtypes = [i64, P, i64, P, u64, P, P, P, P, P]
        lib.kg_sbm_fill.restype = None
        lib.kg_sbm_fill.argtypes = [i64, P, i64, P, u64, P, P, P, P, P, P, P, P]
        lib.kg_intra_edge.restype = ctypes.c_int
        lib.kg_intra_edge.argtypes = [u64, i64, ctypes.c_uint32, ctypes.c_uint32, f64]
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def streams(seed: int, k: int = 5):
    """PCG64 streams (graph, permutation, omega, theta0, target) spawned from one seed."""
    ss = np.random.SeedSequence(seed)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(k)]


@dataclass
class Graph:
    """A 0/1 symmetric adjacency in user order.

    ``row_ptr``/``col``: CSR (int64 / int32), columns ascending in every row, no self loops.
    ``labels``: planted community of every user node (int32).
    ``complete``: True for the all-to-all graph, whose CSR is not materialised (``row_ptr`` and
    ``col`` are None); every pair l != m is coupled.
    """
    n: int
    labels: np.ndarray
    row_ptr: np.ndarray | None = None
    col: np.ndarray | None = None
    complete: bool = False
    sizes: np.ndarray | None = None
    rho: np.ndarray | None = None
    p_out: float = 0.0
    uperm: np.ndarray | None = None       # planted index -> user index
    key: int = 0
    meta: dict = field(default_factory=dict)
    weight: np.ndarray | None = None      # int32 value A_ml of every CSR entry (None: all 1)

    @property
    def nnz(self) -> int:
        if self.complete:
            return self.n * (self.n - 1)
        return int(self.row_ptr[-1])

    def dense(self) -> np.ndarray:
        """Dense uint8 adjacency (tiny graphs only)."""
        if self.n > 8192:
            raise ValueError("dense() is for small graphs")
        A = np.zeros((self.n, self.n), dtype=np.uint8 if self.weight is None else np.int32)
        if self.complete:
            A[:] = 1
            np.fill_diagonal(A, 0)
            return A
        for m in range(self.n):
            sl = slice(self.row_ptr[m], self.row_ptr[m + 1])
            A[m, self.col[sl]] = 1 if self.weight is None else self.weight[sl]
        return A


def complete_graph(n: int) -> Graph:
    """All-to-all coupling of n oscillators (the classical model, one community)."""
    return Graph(n=n, labels=np.zeros(n, dtype=np.int32), complete=True,
                 sizes=np.array([n], dtype=np.int64), rho=np.array([1.0]), p_out=0.0,
                 uperm=np.arange(n, dtype=np.int32))


def sbm(sizes, rho, p_out: float, key: int, uperm: np.ndarray | None = None) -> Graph:
    """Symmetric stochastic block model.

    sizes[c]: community sizes (planted order); rho[c]: intra-pair edge probability; p_out:
    cross-community pair probability; key: 64-bit hash key; uperm[p]: user index of planted
    node p (identity when None).
    """
    lib = _load()
    sizes = np.ascontiguousarray(sizes, dtype=np.int64)
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    nc = len(sizes)
    cptr = np.zeros(nc + 1, dtype=np.int64)
    np.cumsum(sizes, out=cptr[1:])
    n = int(cptr[-1])
    if uperm is None:
        uperm = np.arange(n, dtype=np.int32)
    uperm = np.ascontiguousarray(uperm, dtype=np.int32)
    key = int(key) & ((1 << 64) - 1)
    ioff = np.zeros(n + 1, dtype=np.int64)
    ne = lib.kg_inter_pairs(n, _p(cptr), nc, float(p_out), key, _p(ioff), None)
    iq = np.zeros(max(ne, 1), dtype=np.int64)
    lib.kg_inter_pairs(n, _p(cptr), nc, float(p_out), key, _p(ioff), _p(iq))
    ideg = np.zeros(n, dtype=np.int64)
    deg = np.zeros(n, dtype=np.int64)
    lib.kg_sbm_degrees(n, _p(cptr), nc, _p(rho), key, _p(ioff), _p(iq), _p(uperm), _p(ideg), _p(deg))
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(deg, out=row_ptr[1:])
    col = np.empty(max(int(row_ptr[-1]), 1), dtype=np.int32)
    soff = np.zeros(n + 1, dtype=np.int64)
    snbr = np.zeros(max(2 * ne, 1), dtype=np.int64)
    by_user = np.concatenate([np.argsort(uperm[cptr[c]:cptr[c + 1]], kind="stable").astype(np.int32)
                              for c in range(nc)])
    lib.kg_sbm_fill(n, _p(cptr), nc, _p(rho), key, _p(ioff), _p(iq), _p(uperm), _p(by_user),
                    _p(row_ptr), _p(col), _p(soff), _p(snbr))
    labels = np.empty(n, dtype=np.int32)
    labels[uperm] = np.repeat(np.arange(nc, dtype=np.int32), sizes)
    return Graph(n=n, labels=labels, row_ptr=row_ptr, col=col[: int(row_ptr[-1])], sizes=sizes,
                 rho=rho, p_out=float(p_out), uperm=uperm, key=key,
                 meta={"inter_undirected_edges": int(ne)})


def intra_edge(key: int, c: int, i: int, j: int, rho: float) -> bool:
    """The generator's own decision for the intra pair (i, j) of community c."""
    return bool(_load().kg_intra_edge(int(key) & ((1 << 64) - 1), c, i, j, rho))


def random_dense(n: int, p_one: float, rng: np.random.Generator, symmetric: bool = True) -> Graph:
    """Unstructured random 0/1 matrix (the paper's threshold matrices of Sec. 3: an entry is one
    with probability p_one), no self loops; symmetric by mirroring the upper triangle."""
    A = (rng.random((n, n)) < p_one).astype(np.uint8)
    if symmetric:
        A = np.triu(A, 1)
        A = A + A.T
    np.fill_diagonal(A, 0)
    return from_dense(A)


def from_dense(A: np.ndarray, labels: np.ndarray | None = None) -> Graph:
    """CSR of the nonzero entries of A; integer values other than 0/1 are kept as weights."""
    n = A.shape[0]
    rows, cols = np.nonzero(A)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=row_ptr[1:])
    vals = A[rows, cols]
    weight = None if np.all(vals == 1) else vals.astype(np.int32)
    return Graph(n=n, labels=np.zeros(n, np.int32) if labels is None else labels.astype(np.int32),
                 row_ptr=row_ptr, col=cols.astype(np.int32), weight=weight)


def weighted_sbm(sizes, prevalent, exception: float, J: int, p_out: float, rng: np.random.Generator,
                 uperm: np.ndarray | None = None) -> Graph:
    """Symmetric integer-weighted block model (small graphs, dense construction): inside block c
    every pair takes the value prevalent[c] with probability 1 - exception, else a value drawn
    uniformly from {0..J} without prevalent[c]; pairs across blocks are 0, or with probability
    p_out a value drawn uniformly from {1..J}. uperm[p]: user index of planted node p."""
    sizes = np.asarray(sizes, dtype=np.int64)
    n = int(sizes.sum())
    lab = np.repeat(np.arange(len(sizes)), sizes)
    A = np.zeros((n, n), dtype=np.int32)
    iu = np.triu_indices(n, 1)
    same = lab[iu[0]] == lab[iu[1]]
    vals = np.zeros(len(iu[0]), dtype=np.int32)
    pv = np.asarray(prevalent)[lab[iu[0]]]
    exc = rng.random(len(vals)) < exception
    other = rng.integers(0, J, len(vals))  # uniform over {0..J} without the prevalent value
    other = other + (other >= pv)
    vals[same] = np.where(exc, other, pv)[same]
    cross = ~same & (rng.random(len(vals)) < p_out)
    vals[cross] = rng.integers(1, J + 1, int(cross.sum()))
    A[iu] = vals
    A = A + A.T
    if uperm is not None:
        B = np.zeros_like(A)
        B[np.ix_(uperm, uperm)] = A
        A = B
        labels = np.empty(n, dtype=np.int32)
        labels[uperm] = lab
    else:
        labels = lab.astype(np.int32)
    return from_dense(A, labels)


def block_model(sizes, V, exception: float, J: int, rng: np.random.Generator,
                uperm: np.ndarray | None = None) -> Graph:
    """Symmetric integer-valued block model with a prevalent value per pair of blocks (small
    graphs, dense construction): every pair of nodes (i, j) of blocks (a, c), i != j, takes the
    value V[a][c] with probability 1 - exception, else a value drawn uniformly from {0..J}
    without V[a][c]. V is a symmetric integer matrix with entries in {0..J}; with J = 1 the
    result is a 0/1 graph whose block (a, c) has density 1 - exception where V[a][c] = 1 and
    exception where it is 0. uperm[p]: user index of planted node p."""
    sizes = np.asarray(sizes, dtype=np.int64)
    V = np.asarray(V, dtype=np.int32)
    n = int(sizes.sum())
    lab = np.repeat(np.arange(len(sizes)), sizes)
    iu = np.triu_indices(n, 1)
    pv = V[lab[iu[0]], lab[iu[1]]]
    exc = rng.random(len(pv)) < exception
    other = rng.integers(0, J, len(pv))  # uniform over {0..J} without the prevalent value
    other = other + (other >= pv)
    A = np.zeros((n, n), dtype=np.int32)
    A[iu] = np.where(exc, other, pv)
    A = A + A.T
    if uperm is not None:
        B = np.zeros_like(A)
        B[np.ix_(uperm, uperm)] = A
        A = B
        labels = np.empty(n, dtype=np.int32)
        labels[uperm] = lab
    else:
        labels = lab.astype(np.int32)
    return from_dense(A, labels)


def paired_sbm(n_comm: int = 64, comm_size: int = 1024, rho_in: float = 0.97, rho_pair: float = 0.9,
               p_out: float = 2e-4, seed: int = 1008) -> Graph:
    """Equal communities coupled in pairs: community c is linked to community c xor 1 by a dense
    off-diagonal block (pair probability rho_pair); inside a community the pair probability is
    rho_in; other pairs of nodes are linked with probability p_out (the count drawn from the
    binomial law, the pairs uniformly, duplicates dropped). Planted order is the user order."""
    if n_comm % 2:
        raise ValueError("n_comm must be even")
    g_rng, b_rng = streams(seed, 2)
    s = int(comm_size)
    n = n_comm * s
    lab = np.repeat(np.arange(n_comm, dtype=np.int32), s)
    # background edges between unpaired communities (u < v)
    npairs = n * (n - 1) // 2
    m = int(b_rng.binomial(npairs, p_out))
    u = b_rng.integers(0, n, 2 * m + 16)
    v = b_rng.integers(0, n, 2 * m + 16)
    keep = (u < v) & (lab[u] != lab[v]) & ((lab[u] ^ 1) != lab[v])
    bg = np.unique(np.stack([u[keep], v[keep]], 1), axis=0)[:m]
    bg_rows = np.concatenate([bg[:, 0], bg[:, 1]])
    bg_cols = np.concatenate([bg[:, 1], bg[:, 0]])
    order = np.argsort(bg_rows, kind="stable")
    bg_rows, bg_cols = bg_rows[order], bg_cols[order]
    bg_ptr = np.searchsorted(bg_rows, np.arange(0, n + 1, s))
    # intra blocks (upper triangle mirrored) and pair blocks (drawn for a < c, transposed for c)
    intra = []
    for a in range(n_comm):
        U = np.triu(g_rng.random((s, s)) < rho_in, 1)
        intra.append(U | U.T)
    pair = {}
    for a in range(0, n_comm, 2):
        pair[a] = g_rng.random((s, s)) < rho_pair
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    cols = []
    for a in range(n_comm):
        # the pair (a, a xor 1) occupies the columns [lo, lo + 2s); row-major keys r n + column
        lo = (a & ~1) * s
        strip = np.zeros((s, 2 * s), dtype=bool)
        c = a ^ 1
        strip[:, a * s - lo:(a + 1) * s - lo] = intra[a]
        strip[:, c * s - lo:(c + 1) * s - lo] = pair[a] if a % 2 == 0 else pair[c].T
        r, cc = np.nonzero(strip)
        key = r.astype(np.int64) * n + cc + lo
        sl = slice(bg_ptr[a], bg_ptr[a + 1])
        keyb = np.sort((bg_rows[sl] - a * s).astype(np.int64) * n + bg_cols[sl])
        key = np.insert(key, np.searchsorted(key, keyb), keyb)
        row_ptr[a * s + 1:(a + 1) * s + 1] = np.bincount(key // n, minlength=s)
        cols.append((key % n).astype(np.int32))
    np.cumsum(row_ptr, out=row_ptr)
    col = np.concatenate(cols)
    return Graph(n=n, labels=lab, row_ptr=row_ptr, col=col, sizes=np.full(n_comm, s, dtype=np.int64),
                 rho=np.full(n_comm, rho_in), p_out=float(p_out), uperm=np.arange(n, dtype=np.int32),
                 meta={"rho_pair": rho_pair, "background_edges": int(len(bg))})


# ------------------------------------------------------------------------------------------------
# Frequencies and phases
# ------------------------------------------------------------------------------------------------

def special_omega(M: int, omega0: float) -> np.ndarray:
    """omega_m = 1 + omega0 (2m - M - 1)/(M - 1), m = 1..M (Sec. 2, special choices)."""
    m = np.arange(1, M + 1, dtype=np.float64)
    return 1.0 + omega0 * (2.0 * m - M - 1.0) / (M - 1.0)


def splay_theta(M: int) -> np.ndarray:
    """theta_m(0) = 2 pi m / M, m = 1..M (Sec. 2, special choices)."""
    return TWO_PI * np.arange(1, M + 1, dtype=np.float64) / M


def uniform_theta(rng: np.random.Generator, n: int) -> np.ndarray:
    return rng.uniform(0.0, TWO_PI, size=n)


# ------------------------------------------------------------------------------------------------
# The workloads
# ------------------------------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    graph: Graph
    omega: np.ndarray
    theta0: np.ndarray
    K: float
    dt: float
    steps: int
    target: np.ndarray | None = None
    r_every: int = 1
    meta: dict = field(default_factory=dict)


def _perm(rng: np.random.Generator, n: int) -> np.ndarray:
    return rng.permutation(n).astype(np.int32)


def all_to_all(n: int = 512, K: float = 2.0, dt: float = 0.01, steps: int = 200, seed: int = 1001) -> Workload:
    """Classical all-to-all model: omega ~ N(0,1), theta0 ~ U[0, 2 pi)."""
    g_rng, p_rng, w_rng, t_rng, x_rng = streams(seed)
    return Workload(name="all_to_all_n%d" % n, graph=complete_graph(n), omega=w_rng.standard_normal(n),
                    theta0=uniform_theta(t_rng, n), K=K, dt=dt, steps=steps, r_every=1)


def sbm_equal(n_comm: int = 64, comm_size: int = 1024, rho_in: float = 0.97, p_out: float = 2e-4,
              K: float = 4.0, dt: float = 0.01, steps: int = 1000, seed: int = 1002,
              permute: bool = True) -> Workload:
    """Equal-community SBM: nodes randomly permuted (user order), planted labels kept."""
    g_rng, p_rng, w_rng, t_rng, x_rng = streams(seed)
    n = n_comm * comm_size
    key = int(g_rng.integers(0, 2**63))
    uperm = _perm(p_rng, n) if permute else None
    g = sbm(np.full(n_comm, comm_size), np.full(n_comm, rho_in), p_out, key, uperm)
    return Workload(name="sbm_%dx%d" % (n_comm, comm_size), graph=g, omega=w_rng.standard_normal(n),
                    theta0=uniform_theta(t_rng, n), K=K, dt=dt, steps=steps,
                    target=uniform_theta(x_rng, n), r_every=10)


def sbm_paired_workload(n_comm: int = 64, comm_size: int = 1024, rho_in: float = 0.97, rho_pair: float = 0.9,
                        p_out: float = 2e-4, K: float = 4.0, dt: float = 0.01, steps: int = 1000,
                        seed: int = 1008) -> Workload:
    """Equal communities coupled in pairs by dense off-diagonal blocks (paired_sbm), with
    omega ~ N(0, 1) and theta0 ~ U[0, 2 pi)."""
    _, _, w_rng, t_rng, x_rng = streams(seed)
    g = paired_sbm(n_comm, comm_size, rho_in, rho_pair, p_out, seed)
    n = g.n
    return Workload(name="paired_%dx%d" % (n_comm, comm_size), graph=g, omega=w_rng.standard_normal(n),
                    theta0=uniform_theta(t_rng, n), K=K, dt=dt, steps=steps,
                    target=uniform_theta(x_rng, n), r_every=10)


def powerlaw_sizes(rng: np.random.Generator, n: int, smin: int = 256, smax: int = 16384) -> np.ndarray:
    """Community sizes with density proportional to s^-2 above smin, clipped at smax, summing to n.

    Draw s = floor(smin/(1-u)) clipped to smax until the total reaches n; the last size is cut
    to the remainder; a remainder below smin is merged into the previous community and a merged
    community above smax is split into two near-equal halves.
    """
    out = []
    tot = 0
    while tot < n:
        u = rng.random()
        s = int(min(smax, math.floor(smin / (1.0 - u))))
        s = min(s, n - tot)
        out.append(s)
        tot += s
    if len(out) > 1 and out[-1] < smin:
        last = out.pop()
        out[-1] += last
        if out[-1] > smax:
            merged = out.pop()
            out += [merged // 2, merged - merged // 2]
    return np.array(out, dtype=np.int64)


def sbm_heterogeneous(n: int = 1 << 20, K: float = 3.0, dt: float = 0.005, steps: int = 500,
                      seed: int = 1003, mean_inter_degree: float = 8.0, smin: int = 256,
                      smax: int = 16384, rho_lo: float = 0.3, rho_hi: float = 1.0) -> Workload:
    """Heterogeneous SBM: power-law community sizes, intra densities ~ U[rho_lo, rho_hi],
    Erdos-Renyi cross edges with the given mean degree, omega ~ Cauchy(0, 0.5)."""
    g_rng, p_rng, w_rng, t_rng, x_rng = streams(seed)
    sizes = powerlaw_sizes(g_rng, n, smin, smax)
    rho = g_rng.uniform(rho_lo, rho_hi, size=len(sizes))
    key = int(g_rng.integers(0, 2**63))
    p_out = mean_inter_degree / max(n - 1, 1)
    g = sbm(sizes, rho, p_out, key, _perm(p_rng, n))
    omega = 0.5 * w_rng.standard_cauchy(n)
    return Workload(name="sbm_het_n%d" % n, graph=g, omega=omega, theta0=uniform_theta(t_rng, n),
                    K=K, dt=dt, steps=steps, target=uniform_theta(x_rng, n), r_every=10)


def paper_four_communities(M: int = 4096, rho_in: float = 0.95, p_out: float = 0.05, K: float = 3.0,
                           dt: float = 0.01, T: float = 200.0, omega0: float = 2.0,
                           seed: int = 1006) -> Workload:
    """Four equal communities with the special omega and splay theta0 (Sec. 3, numerical
    integration); the densities are not stated in the text and are a stated guess."""
    g_rng, p_rng, w_rng, t_rng, x_rng = streams(seed)
    key = int(g_rng.integers(0, 2**63))
    g = sbm(np.full(4, M // 4), np.full(4, rho_in), p_out, key, _perm(p_rng, M))
    return Workload(name="paper_4comm_M%d" % M, graph=g, omega=special_omega(M, omega0),
                    theta0=splay_theta(M), K=K, dt=dt, steps=int(round(T / dt)), r_every=100)


def four_blocks_flip(M: int, p: float, seed: int = 1007) -> Graph:
    """Diagonal blocks of sizes (5-k)M/10, k=1..4, entries flipped with probability p (Sec. 3,
    community detection), symmetrised."""
    g_rng, p_rng, *_ = streams(seed)
    sizes = np.array([(5 - k) * M // 10 for k in range(1, 5)], dtype=np.int64)
    sizes[-1] += M - sizes.sum()
    key = int(g_rng.integers(0, 2**63))
    return sbm(sizes, np.full(4, 1.0 - p), p, key, _perm(p_rng, M))


def batch_instances_iter(n_inst: int = 256, nmin: int = 1024, nmax: int = 65536, Kmax: float = 6.0,
                         dt: float = 0.01, steps: int = 2000, seed: int = 1004):
    """Ensemble of independent instances, generated lazily: N log-uniform in [nmin, nmax],
    all-to-all or equal-community SBM (communities of about 1024, rho 0.97, p_out 2e-4) by a fair
    coin, K swept uniformly over [0, Kmax], omega ~ N(0,1), theta0 ~ U[0, 2 pi)."""
    ss = np.random.SeedSequence(seed)
    top = np.random.Generator(np.random.PCG64(ss.spawn(1)[0]))
    Ks = np.linspace(0.0, Kmax, n_inst)
    plan = []
    for i in range(n_inst):
        n = int(round(math.exp(top.uniform(math.log(nmin), math.log(nmax)))))
        kind = "a2a" if top.random() < 0.5 else "sbm"
        plan.append((n, kind, int(top.integers(0, 2**31))))
    for i, (n, kind, s_i) in enumerate(plan):
        g_rng, p_rng, w_rng, t_rng, x_rng = streams(s_i)
        if kind == "a2a":
            g = complete_graph(n)
        else:
            nb = max(1, int(round(n / 1024)))
            sizes = np.full(nb, n // nb, dtype=np.int64)
            sizes[: n - sizes.sum()] += 1
            key = int(g_rng.integers(0, 2**63))
            g = sbm(sizes, np.full(nb, 0.97), 2e-4, key, _perm(p_rng, n))
        yield Workload(name="inst%d_%s_n%d" % (i, kind, n), graph=g, omega=w_rng.standard_normal(n),
                       theta0=uniform_theta(t_rng, n), K=float(Ks[i]), dt=dt, steps=steps, r_every=10,
                       meta={"kind": kind})


def batch_instances(*args, **kw):
    """The ensemble of batch_instances_iter as a list."""
    return list(batch_instances_iter(*args, **kw))
