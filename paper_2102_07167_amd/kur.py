"""Thin ctypes binding of the C ABI in include/kur.h (argument marshalling only).

Every computation runs in the HIP kernels of ``libkur.so``; this module converts numpy arrays
and torch device tensors into pointers and status codes into exceptions. If the shared library
is missing it raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .buildlib import SO

KUR_OK, KUR_EINVAL, KUR_ENOMEM, KUR_EDEVICE, KUR_ESTATE, KUR_ENONFINITE = range(6)
KUR_F32, KUR_F64 = 1, 2
STATUS_NAMES = {0: "KUR_OK", 1: "KUR_EINVAL", 2: "KUR_ENOMEM", 3: "KUR_EDEVICE", 4: "KUR_ESTATE",
                5: "KUR_ENONFINITE"}

_lib = None

P = ctypes.c_void_p
I64 = ctypes.c_int64
I32 = ctypes.c_int32
F64 = ctypes.c_double
ST = ctypes.c_int

# name -> (restype, argtypes); the full exported surface of include/kur.h
SIGNATURES = {
    "kur_version": (ctypes.c_int, []),
    "kur_create": (ST, [ctypes.POINTER(P), ctypes.c_int, ctypes.c_int, P]),
    "kur_destroy": (None, [P]),
    "kur_last_error": (ctypes.c_char_p, [P]),
    "kur_set_option": (ST, [P, ctypes.c_char_p, F64]),
    "kur_set_graph_csr": (ST, [P, I64, P, P, P]),
    "kur_set_graph": (ST, [P, I64, I32, P, P, P, P, P, P, P]),
    "kur_set_graph_csr_w": (ST, [P, I64, P, P, P, P]),
    "kur_get_row_layers": (ST, [P, I64, P, P, P]),
    "kur_get_block_groups": (ST, [P, I32, P, P, P]),
    "kur_graph_pairs": (ST, [P, P]),
    "kur_graph_info": (ST, [P, P]),
    "kur_graph_masks": (ST, [P, P]),
    "kur_graph_mask_items": (ST, [P, P, P]),
    "kur_get_perm": (ST, [P, P]),
    "kur_get_blocks": (ST, [P, P, P]),
    "kur_get_row_lists": (ST, [P, I64, P, P, P, P]),
    "kur_set_params": (ST, [P, P, F64]),
    "kur_set_phases": (ST, [P, P]),
    "kur_eval_rhs": (ST, [P, P, P]),
    "kur_step_rk4": (ST, [P, F64, I64, I64, P, P]),
    "kur_get_phases": (ST, [P, P, ctypes.c_int]),
    "kur_order_parameter": (ST, [P, P, P]),
    "kur_get_state": (ST, [P, P, ctypes.POINTER(ctypes.c_size_t)]),
    "kur_set_state": (ST, [P, P, ctypes.c_size_t]),
    "kur_sync": (ST, [P]),
    "kur_kernel_time": (ST, [P, P, P]),
    "kur_adjoint_rk4": (ST, [P, P, F64, I64, I64, P, P, P, P]),
    "kur_set_graph_complete": (ST, [P, I64]),
    "kur_batch_begin": (ST, [P]),
    "kur_batch_add": (ST, [P, I64, ctypes.c_int, P, P, P, F64, P, P]),
    "kur_batch_commit": (ST, [P]),
    "kur_batch_info": (ST, [P, P, P]),
    "kur_batch_step": (ST, [P, F64, I64, I64, P, P]),
    "kur_read_bandwidth": (ST, [P, I64, I32, P]),
    "kur_adjoint_rk4_recorded": (ST, [P, P, P, P, P]),
    "kur_recorded_run": (ST, [P, P, P, P]),
    "kur_autotune_csr": (ST, [P, I64, P, P, P, I32, ctypes.c_char_p, P]),
    "kur_tune_tiles": (ST, [P, I32, P]),
    "kur_tune_key": (ST, [P, I64, P, P, ctypes.c_char_p, ctypes.c_size_t]),
    "kur_ens_set_graph_csr": (ST, [P, I64, P, P, P]),
    "kur_ens_set_params": (ST, [P, I32, P, P]),
    "kur_ens_set_phases": (ST, [P, P]),
    "kur_ens_eval_rhs": (ST, [P, P]),
    "kur_ens_step": (ST, [P, F64, I64, I64, P, P]),
    "kur_ens_get_phases": (ST, [P, P, ctypes.c_int]),
    "kur_ens_info": (ST, [P, P]),
    "kur_ens_block_modes": (ST, [P, P, P]),
    "kur_ens_get_perm": (ST, [P, P]),
    "kur_ens_row_pattern": (ST, [P, I64, P, P, P]),
    "kur_ens_kernel_time": (ST, [P, P]),
    "kur_ens_autotune_csr": (ST, [P, I64, P, P, P, I32, I32, P]),
    "kur_diagnostics": (ST, [P, P]),
    "kur_diagnostics_noalloc": (ST, [P, P]),
    "kur_step_midpoint": (ST, [P, F64, I64, I32, I64, P, P]),
    "kur_step_adaptive": (ST, [P, F64, F64, F64, I64, P]),
    "kur_stream": (ST, [P, ctypes.POINTER(P)]),
    "kur_set_params_dev": (ST, [P, P, F64]),
    "kur_set_phases_dev": (ST, [P, P]),
    "kur_eval_rhs_dev": (ST, [P, P, P]),
    "kur_get_phases_dev": (ST, [P, P, ctypes.c_int]),
    "kur_order_parameter_dev": (ST, [P, P, P]),
    "kur_order_parameter_vjp_dev": (ST, [P, P, P, P, P, ctypes.c_int]),
    "kur_adjoint_rk4_dev": (ST, [P, P, F64, I64, I64, P, P, P, P]),
    "kur_adjoint_rk4_recorded_dev": (ST, [P, P, P, P, P]),
}


class KurError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), message))
        self.status = status


def lib():
    """Load libkur.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(SO):
            raise RuntimeError("libkur.so is not built (run paper_2102_07167_amd.build.build())")
        L = ctypes.CDLL(SO)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(P)


def _f64(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and a.shape != (n,):
        raise ValueError("expected shape (%d,), got %s" % (n, a.shape))
    return a


class Kuramoto:
    """One library context: a graph, omega, K, the phase state, one device and one stream."""

    def __init__(self, dtype: str = "f32", device: int = 0, stream=None):
        self._L = lib()
        self.dtype = dtype
        h = P()
        code = KUR_F32 if dtype in ("f32", "float32") else KUR_F64
        st = None
        if stream is not None:
            st = P(int(getattr(stream, "cuda_stream", stream)))
        rc = self._L.kur_create(ctypes.byref(h), code, int(device), st)
        if rc != KUR_OK:
            raise KurError(rc, "kur_create(dtype=%s, device=%d) failed" % (dtype, device))
        self._h = h
        self.n = 0
        self.device = int(device)

    def close(self):
        if getattr(self, "_h", None):
            self._L.kur_destroy(self._h)
            self._h = None
        self._ext_stream = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _chk(self, rc):
        if rc != KUR_OK:
            raise KurError(rc, self._L.kur_last_error(self._h).decode())

    # -- configuration ----------------------------------------------------------------------
    def set_option(self, key: str, value: float):
        self._chk(self._L.kur_set_option(self._h, key.encode(), float(value)))

    def set_graph_csr(self, n, row_ptr, col, labels):
        row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int32)
        labels = np.ascontiguousarray(labels, dtype=np.int32)
        self._chk(self._L.kur_set_graph_csr(self._h, int(n), _ptr(row_ptr), _ptr(col), _ptr(labels)))
        self.n = int(n)

    def set_graph_blocks(self, n, block_ptr, mode, list_ptr, list_col, inter_ptr, inter_col, perm=None):
        block_ptr = np.ascontiguousarray(block_ptr, dtype=np.int64)
        mode = np.ascontiguousarray(mode, dtype=np.uint8)
        list_ptr = np.ascontiguousarray(list_ptr, dtype=np.int64)
        list_col = np.ascontiguousarray(list_col, dtype=np.uint16)
        inter_ptr = np.ascontiguousarray(inter_ptr, dtype=np.int64)
        inter_col = np.ascontiguousarray(inter_col, dtype=np.int32)
        perm = None if perm is None else np.ascontiguousarray(perm, dtype=np.int32)
        self._chk(self._L.kur_set_graph(self._h, int(n), len(block_ptr) - 1, _ptr(block_ptr), _ptr(mode),
                                        _ptr(list_ptr), _ptr(list_col), _ptr(inter_ptr), _ptr(inter_col),
                                        _ptr(perm)))
        self.n = int(n)

    def set_graph_complete(self, n):
        """All-to-all coupling: one dense block whose list of zeros is empty."""
        self._chk(self._L.kur_set_graph_complete(self._h, int(n)))
        self.n = int(n)

    def set_graph_csr_w(self, n, row_ptr, col, weight, labels):
        row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int32)
        weight = np.ascontiguousarray(weight, dtype=np.int32)
        labels = np.ascontiguousarray(labels, dtype=np.int32)
        self._chk(self._L.kur_set_graph_csr_w(self._h, int(n), _ptr(row_ptr), _ptr(col), _ptr(weight), _ptr(labels)))
        self.n = int(n)

    def set_graph(self, graph):
        """Any object with n, labels, row_ptr, col, complete and optionally integer weights."""
        if getattr(graph, "complete", False):
            self.set_graph_complete(graph.n)
        elif getattr(graph, "weight", None) is not None:
            self.set_graph_csr_w(graph.n, graph.row_ptr, graph.col, graph.weight, graph.labels)
        else:
            self.set_graph_csr(graph.n, graph.row_ptr, graph.col, graph.labels)

    def block_groups(self, b: int):
        """(column blocks, factors) whose localised order parameters enter the rows of block b."""
        cnt = I32(0)
        self._chk(self._L.kur_get_block_groups(self._h, int(b), None, None, ctypes.byref(cnt)))
        blk = np.empty(max(cnt.value, 1), dtype=np.int32)
        md = np.empty(max(cnt.value, 1), dtype=np.int32)
        self._chk(self._L.kur_get_block_groups(self._h, int(b), _ptr(blk), _ptr(md), ctypes.byref(cnt)))
        return blk[: cnt.value], md[: cnt.value]

    def graph_masks(self) -> dict:
        """Bitmask segments of the installed layout (option "mask_min"): their count and bytes."""
        out = np.zeros(2, dtype=np.int64)
        self._chk(self._L.kur_graph_masks(self._h, _ptr(out)))
        return {"mask_segments": int(out[0]), "mask_bytes": int(out[1])}

    def graph_mask_items(self) -> np.ndarray:
        """Bitmask work items of a host-only context's layout, one row per item in launch order:
        tile, block, segment, first sub-chunk, sub-chunks, rows, units per row, cells, first
        partial-sum row."""
        cnt = I64(0)
        self._chk(self._L.kur_graph_mask_items(self._h, ctypes.byref(cnt), None))
        out = np.zeros((max(cnt.value, 1), 9), dtype=np.int64)
        self._chk(self._L.kur_graph_mask_items(self._h, ctypes.byref(cnt), _ptr(out)))
        return out[: cnt.value]

    def graph_pairs(self) -> int:
        """Number of dense off-diagonal blocks of the installed graph."""
        v = I64(0)
        self._chk(self._L.kur_graph_pairs(self._h, ctypes.byref(v)))
        return int(v.value)

    def row_layers(self, m: int):
        """(block-order columns, layer) of the list entries of block-order row m (host-only)."""
        cnt = I64(0)
        self._chk(self._L.kur_get_row_layers(self._h, int(m), None, None, ctypes.byref(cnt)))
        cols = np.empty(cnt.value, dtype=np.int32)
        lay = np.empty(cnt.value, dtype=np.int32)
        self._chk(self._L.kur_get_row_layers(self._h, int(m), _ptr(cols), _ptr(lay), ctypes.byref(cnt)))
        return cols, lay

    def set_batch(self, instances):
        """instances: iterable of (graph, K, omega, theta0); graph as for set_graph."""
        self._chk(self._L.kur_batch_begin(self._h))
        total = 0
        for graph, K, omega, theta0 in instances:
            n = int(graph.n)
            om, th = _f64(omega, n), _f64(theta0, n)
            if getattr(graph, "complete", False):
                self._chk(self._L.kur_batch_add(self._h, n, 1, None, None, None, float(K), _ptr(om), _ptr(th)))
            else:
                rp = np.ascontiguousarray(graph.row_ptr, dtype=np.int64)
                cl = np.ascontiguousarray(graph.col, dtype=np.int32)
                lb = np.ascontiguousarray(graph.labels, dtype=np.int32)
                self._chk(self._L.kur_batch_add(self._h, n, 0, _ptr(rp), _ptr(cl), _ptr(lb), float(K), _ptr(om),
                                                _ptr(th)))
            total += n
        self._chk(self._L.kur_batch_commit(self._h))
        self.n = total

    def batch_info(self):
        ni = ctypes.c_int32(0)
        self._chk(self._L.kur_batch_info(self._h, ctypes.byref(ni), None))
        rf = np.empty(ni.value + 1, dtype=np.int64)
        self._chk(self._L.kur_batch_info(self._h, ctypes.byref(ni), _ptr(rf)))
        return rf

    def batch_step(self, dt: float, nsteps: int, r_every: int = 0):
        """Advance every instance; returns r and psi as (samples, instances) arrays (or None)."""
        ni = len(self.batch_info()) - 1
        ns = nsteps // r_every + 1 if r_every > 0 else 0
        r = np.empty((ns, ni)) if ns else None
        psi = np.empty((ns, ni)) if ns else None
        self._chk(self._L.kur_batch_step(self._h, float(dt), int(nsteps), int(r_every), _ptr(r), _ptr(psi)))
        return r, psi

    def graph_info(self) -> dict:
        out = np.zeros(10, dtype=np.int64)
        self._chk(self._L.kur_graph_info(self._h, _ptr(out)))
        keys = ["n", "blocks", "dense_blocks", "list_entries", "list_padded", "inter_entries", "tiles", "chunk",
                "symmetric", "max_block"]
        return {k: int(v) for k, v in zip(keys, out)}

    def perm(self) -> np.ndarray:
        p = np.empty(self.n, dtype=np.int32)
        self._chk(self._L.kur_get_perm(self._h, _ptr(p)))
        return p

    def blocks(self):
        nb = self.graph_info()["blocks"]
        bp = np.empty(nb + 1, dtype=np.int64)
        md = np.empty(nb, dtype=np.uint8)
        self._chk(self._L.kur_get_blocks(self._h, _ptr(bp), _ptr(md)))
        return bp, md

    def row_lists(self, row: int):
        nl, ni = I64(0), I64(0)
        self._chk(self._L.kur_get_row_lists(self._h, int(row), None, ctypes.byref(nl), None, ctypes.byref(ni)))
        lst = np.empty(max(nl.value, 1), dtype=np.int32)
        itr = np.empty(max(ni.value, 1), dtype=np.int32)
        self._chk(self._L.kur_get_row_lists(self._h, int(row), _ptr(lst), ctypes.byref(nl), _ptr(itr),
                                            ctypes.byref(ni)))
        return lst[: nl.value], itr[: ni.value]

    def set_params(self, omega, K: float):
        omega = _f64(omega, self.n)
        self._chk(self._L.kur_set_params(self._h, _ptr(omega), float(K)))

    def set_phases(self, theta):
        theta = _f64(theta, self.n)
        self._chk(self._L.kur_set_phases(self._h, _ptr(theta)))

    # -- computation --------------------------------------------------------------------------
    def eval_rhs(self, theta=None) -> np.ndarray:
        out = np.empty(self.n)
        th = None if theta is None else _f64(theta, self.n)
        self._chk(self._L.kur_eval_rhs(self._h, _ptr(th), _ptr(out)))
        return out

    def step_rk4(self, dt: float, nsteps: int, r_every: int = 0, want_r: bool = True):
        ns = nsteps // r_every + 1 if r_every > 0 else 0
        r = np.empty(ns) if (ns and want_r) else None
        psi = np.empty(ns) if (ns and want_r) else None
        self._chk(self._L.kur_step_rk4(self._h, float(dt), int(nsteps), int(r_every), _ptr(r), _ptr(psi)))
        return r, psi

    def get_phases(self, wrapped: bool = False) -> np.ndarray:
        out = np.empty(self.n)
        self._chk(self._L.kur_get_phases(self._h, _ptr(out), 1 if wrapped else 0))
        return out

    def order_parameter(self):
        r, psi = F64(), F64()
        self._chk(self._L.kur_order_parameter(self._h, ctypes.byref(r), ctypes.byref(psi)))
        return r.value, psi.value

    def get_state(self) -> bytes:
        nb = ctypes.c_size_t(0)
        self._chk(self._L.kur_get_state(self._h, None, ctypes.byref(nb)))
        buf = ctypes.create_string_buffer(nb.value)
        self._chk(self._L.kur_get_state(self._h, buf, ctypes.byref(nb)))
        return buf.raw[: nb.value]

    def set_state(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        self._chk(self._L.kur_set_state(self._h, buf, len(blob)))

    def adjoint_rk4(self, dt: float, nsteps: int, dl_dthetaT, theta0=None, ckpt_every: int = 32):
        """(dL/dtheta0, dL/domega, dL/dK) of a loss on theta(T) after nsteps RK4 steps from theta0."""
        seed = _f64(dl_dthetaT, self.n)
        th0 = None if theta0 is None else _f64(theta0, self.n)
        gt = np.empty(self.n)
        gw = np.empty(self.n)
        gk = F64()
        self._chk(self._L.kur_adjoint_rk4(self._h, _ptr(th0), float(dt), int(nsteps), int(ckpt_every), _ptr(seed),
                                          _ptr(gt), _ptr(gw), ctypes.byref(gk)))
        return gt, gw, gk.value

    def adjoint_recorded(self, dl_dthetaT):
        """Gradients for the last kur_step_rk4 run recorded with option checkpoint_every > 0."""
        seed = _f64(dl_dthetaT, self.n)
        gt = np.empty(self.n)
        gw = np.empty(self.n)
        gk = F64()
        self._chk(self._L.kur_adjoint_rk4_recorded(self._h, _ptr(seed), _ptr(gt), _ptr(gw), ctypes.byref(gk)))
        return gt, gw, gk.value

    def step_midpoint(self, dt: float, nsteps: int, iters: int = 4, r_every: int = 0):
        """Implicit midpoint rule with `iters` fixed-point iterations per step (kur_step_midpoint);
        returns r and psi samples like step_rk4."""
        if r_every > 0:
            ns = nsteps // r_every + 1
            r = np.empty(ns)
            psi = np.empty(ns)
            self._chk(self._L.kur_step_midpoint(self._h, float(dt), int(nsteps), int(iters), int(r_every), _ptr(r),
                                                _ptr(psi)))
            return r, psi
        self._chk(self._L.kur_step_midpoint(self._h, float(dt), int(nsteps), int(iters), 0, None, None))
        return None, None

    def step_adaptive(self, t_end: float, dt0: float, atol: float, max_steps: int = 1000000) -> dict:
        """Variable-step embedded RK pair over t_end (kur_step_adaptive)."""
        out = np.zeros(4)
        self._chk(self._L.kur_step_adaptive(self._h, float(t_end), float(dt0), float(atol), int(max_steps), _ptr(out)))
        return {"t": out[0], "dt": out[1], "accepted": int(out[2]), "rejected": int(out[3])}

    def diagnostics(self) -> dict:
        """Potential V, mean unwrapped phase and mean omega of the current state (kur_diagnostics)."""
        out = np.zeros(3)
        self._chk(self._L.kur_diagnostics(self._h, _ptr(out)))
        return {"V": out[0], "mean_theta": out[1], "mean_omega": out[2]}

    def diagnostics_noalloc(self) -> dict:
        """kur_diagnostics_noalloc: the diagnostics without any device allocation (fixed scratch)."""
        out = np.zeros(3)
        self._chk(self._L.kur_diagnostics_noalloc(self._h, _ptr(out)))
        return {"V": out[0], "mean_theta": out[1], "mean_omega": out[2]}

    def recorded_run(self):
        """(serial, dt, nsteps) of the run kept for adjoint_recorded (serial 0: none)."""
        sr, dt, ns = I64(0), F64(0), I64(0)
        self._chk(self._L.kur_recorded_run(self._h, ctypes.byref(sr), ctypes.byref(dt), ctypes.byref(ns)))
        return sr.value, dt.value, ns.value

    # -- layout autotuning -------------------------------------------------------------------
    _TUNE_FIELDS = ("tau", "chunk", "threads", "tile_rows", "tile_min_cost", "flat_min_vec", "ms_per_step",
                    "ms_per_step_start", "timed", "cache", "builds", "seconds", "xcds", "inter_gather")

    def _tune_report(self, rep):
        d = dict(zip(self._TUNE_FIELDS, (float(x) for x in rep)))
        for k in ("chunk", "threads", "tile_rows", "tile_min_cost", "timed", "cache", "builds", "xcds", "inter_gather"):
            d[k] = int(d[k])
        return d

    def autotune(self, graph, effort: int = 1, cache: str | None = None) -> dict:
        """Install `graph` (CSR with planted labels) in the layout that runs fastest on this device;
        see kur_autotune_csr. Returns the chosen options and timings."""
        rp = np.ascontiguousarray(graph.row_ptr, dtype=np.int64)
        cl = np.ascontiguousarray(graph.col, dtype=np.int32)
        lb = np.ascontiguousarray(graph.labels, dtype=np.int32)
        rep = np.zeros(14)
        self._chk(self._L.kur_autotune_csr(self._h, int(graph.n), _ptr(rp), _ptr(cl), _ptr(lb), int(effort),
                                           None if cache is None else os.fsencode(cache), _ptr(rep)))
        self.n = int(graph.n)
        return self._tune_report(rep)

    def tune_tiles(self, effort: int = 1) -> dict:
        """Re-tile the installed graph or batch with the fastest tile options (kur_tune_tiles)."""
        rep = np.zeros(14)
        self._chk(self._L.kur_tune_tiles(self._h, int(effort), _ptr(rep)))
        return self._tune_report(rep)

    def tune_key(self, graph) -> str:
        """The tuning-cache signature of `graph` for this context."""
        rp = np.ascontiguousarray(graph.row_ptr, dtype=np.int64)
        lb = np.ascontiguousarray(graph.labels, dtype=np.int32)
        buf = ctypes.create_string_buffer(256)
        self._chk(self._L.kur_tune_key(self._h, int(graph.n), _ptr(rp), _ptr(lb), buf, 256))
        return buf.value.decode()

    # -- shared-graph ensembles (FP32) ------------------------------------------------------
    _ENS_INFO = ("n", "blocks", "gemm_blocks", "gemm_rows", "gemm_pairs", "csr_entries", "B", "Bp", "gemm_items",
                 "symmetric", "offdiag_blocks", "gemm_cells_issued")

    def ens_set_graph(self, graph):
        """Install `graph` (CSR with planted labels) for replicas; see kur_ens_set_graph_csr."""
        rp = np.ascontiguousarray(graph.row_ptr, dtype=np.int64)
        cl = np.ascontiguousarray(graph.col, dtype=np.int32)
        lb = np.ascontiguousarray(graph.labels, dtype=np.int32)
        self._chk(self._L.kur_ens_set_graph_csr(self._h, int(graph.n), _ptr(rp), _ptr(cl), _ptr(lb)))
        self.ens_n = int(graph.n)

    def ens_set_params(self, K, omega):
        """K: (B,), omega: (B, n) per replica (user order)."""
        K = np.ascontiguousarray(np.atleast_1d(K), dtype=np.float64)
        om = np.ascontiguousarray(omega, dtype=np.float64).reshape(len(K), self.ens_n)
        self._chk(self._L.kur_ens_set_params(self._h, len(K), _ptr(K), _ptr(om)))
        self.ens_B = len(K)

    def ens_set_phases(self, theta):
        th = np.ascontiguousarray(theta, dtype=np.float64).reshape(self.ens_B, self.ens_n)
        self._chk(self._L.kur_ens_set_phases(self._h, _ptr(th)))

    def ens_eval_rhs(self):
        out = np.empty((self.ens_B, self.ens_n))
        self._chk(self._L.kur_ens_eval_rhs(self._h, _ptr(out)))
        return out

    def ens_step(self, dt: float, nsteps: int, r_every: int = 0):
        """Advance every replica; returns r and psi as (samples, B) arrays (or None)."""
        if r_every > 0:
            ns = nsteps // r_every + 1
            r = np.empty((ns, self.ens_B))
            psi = np.empty((ns, self.ens_B))
            self._chk(self._L.kur_ens_step(self._h, float(dt), int(nsteps), int(r_every), _ptr(r), _ptr(psi)))
            return r, psi
        self._chk(self._L.kur_ens_step(self._h, float(dt), int(nsteps), 0, None, None))
        return None, None

    def ens_get_phases(self, wrapped: bool = True):
        out = np.empty((self.ens_B, self.ens_n))
        self._chk(self._L.kur_ens_get_phases(self._h, _ptr(out), 1 if wrapped else 0))
        return out

    def ens_info(self) -> dict:
        out = np.zeros(12, dtype=np.int64)
        self._chk(self._L.kur_ens_info(self._h, _ptr(out)))
        return dict(zip(self._ENS_INFO, (int(x) for x in out)))

    def ens_block_modes(self):
        nb = self.ens_info()["blocks"]
        g = np.zeros(nb, dtype=np.uint8)
        d = np.zeros(nb)
        self._chk(self._L.kur_ens_block_modes(self._h, _ptr(g), _ptr(d)))
        return g, d

    def ens_perm(self):
        p = np.empty(self.ens_n, dtype=np.int32)
        self._chk(self._L.kur_ens_get_perm(self._h, _ptr(p)))
        return p

    def ens_row_pattern(self, m: int):
        """(CSR columns, dense 0/1 row or None) of block-order row m (host-only contexts)."""
        cnt = I64(0)
        self._chk(self._L.kur_ens_row_pattern(self._h, int(m), None, ctypes.byref(cnt), None))
        cols = np.empty(cnt.value, dtype=np.int32)
        cap = I64(cnt.value)
        dense = np.full(self.ens_n, 255, dtype=np.uint8)
        self._chk(self._L.kur_ens_row_pattern(self._h, int(m), _ptr(cols), ctypes.byref(cap), _ptr(dense)))
        return cols, dense

    def ens_kernel_time(self) -> dict:
        out = np.zeros(4)
        self._chk(self._L.kur_ens_kernel_time(self._h, _ptr(out)))
        return {"gemm_launches": int(out[0]), "gemm_ms": out[1], "rows_launches": int(out[2]), "rows_ms": out[3]}

    def ens_autotune(self, graph, B: int, effort: int = 1) -> dict:
        rp = np.ascontiguousarray(graph.row_ptr, dtype=np.int64)
        cl = np.ascontiguousarray(graph.col, dtype=np.int32)
        lb = np.ascontiguousarray(graph.labels, dtype=np.int32)
        rep = np.zeros(6)
        self._chk(self._L.kur_ens_autotune_csr(self._h, int(graph.n), _ptr(rp), _ptr(cl), _ptr(lb), int(B), int(effort),
                                               _ptr(rep)))
        self.ens_n = int(graph.n)
        return dict(zip(("ens_tau", "ms_per_step", "ms_all_gemm", "ms_no_gemm", "timed", "seconds"),
                        (float(x) for x in rep)))

    def read_bandwidth(self, nbytes: int = 4 << 30, repeats: int = 5) -> float:
        """GB/s of a plain streaming read on this context's device (roofline reference)."""
        g = F64()
        self._chk(self._L.kur_read_bandwidth(self._h, int(nbytes), int(repeats), ctypes.byref(g)))
        return g.value

    def sync(self):
        self._chk(self._L.kur_sync(self._h))

    def kernel_time(self):
        n, ms = I64(0), F64(0)
        self._chk(self._L.kur_kernel_time(self._h, ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value

    # -- device tensors (user order, context dtype) -----------------------------------------
    # The library enqueues on its own stream. Around every call the context stream waits for
    # the caller's current torch stream, and the caller's stream then waits for the context
    # stream; so work the caller enqueues later (including the reuse of a freed tensor's memory
    # by torch's caching allocator, which follows the allocating stream) runs after the call.
    # Tensors must therefore belong to the caller's current stream. (Tensors are not marked with
    # record_stream on the context stream: that stream ends with the context, and torch would
    # later record events on its stale handle.)
    def stream_handle(self) -> int:
        h = P()
        self._chk(self._L.kur_stream(self._h, ctypes.byref(h)))
        return int(h.value or 0)

    def _dev_args(self, tensors, n=None):
        import torch
        want = torch.float32 if self.dtype in ("f32", "float32") else torch.float64
        for t in tensors:
            if t is None:
                continue
            if not t.is_cuda or t.dtype != want or not t.is_contiguous():
                raise ValueError("device calls take contiguous %s tensors on the GPU" % want)
            if n is not None and t.numel() != n:
                raise ValueError("expected %d entries, got %d" % (n, t.numel()))
        return want

    def _dev_call(self, fn, tensors, *args):
        import torch
        ext = getattr(self, "_ext_stream", None)
        if ext is None:
            ext = torch.cuda.ExternalStream(self.stream_handle())
            self._ext_stream = ext
        cur = torch.cuda.current_stream()
        same = cur.cuda_stream == ext.cuda_stream
        if not same:
            ext.wait_stream(cur)
        self._chk(fn(self._h, *args))
        if not same:
            cur.wait_stream(ext)

    @staticmethod
    def _dp(t):
        return None if t is None else P(t.data_ptr())

    def set_params_dev(self, omega_t, K: float):
        self._dev_args([omega_t], self.n)
        self._dev_call(self._L.kur_set_params_dev, [omega_t], self._dp(omega_t), float(K))

    def set_phases_dev(self, theta_t):
        self._dev_args([theta_t], self.n)
        self._dev_call(self._L.kur_set_phases_dev, [theta_t], self._dp(theta_t))

    def eval_rhs_dev(self, theta_t, out_t):
        """F(theta) into out_t (theta_t None: the current phases)."""
        self._dev_args([theta_t, out_t], self.n)
        self._dev_call(self._L.kur_eval_rhs_dev, [theta_t, out_t], self._dp(theta_t), self._dp(out_t))

    def get_phases_dev(self, out_t, wrapped: bool = False):
        self._dev_args([out_t], self.n)
        self._dev_call(self._L.kur_get_phases_dev, [out_t], self._dp(out_t), 1 if wrapped else 0)

    def order_parameter_dev(self, theta_t, out_t):
        """out_t[0] = r, out_t[1] = psi of theta_t (None: the current phases)."""
        self._dev_args([theta_t], self.n)
        self._dev_args([out_t], 2)
        self._dev_call(self._L.kur_order_parameter_dev, [theta_t, out_t], self._dp(theta_t), self._dp(out_t))

    def order_parameter_vjp_dev(self, theta_t, rpsi_t, grad_t, out_t, accumulate: bool = False):
        """out_t (+)= g_r dr/dtheta + g_psi dpsi/dtheta at (r, psi) = rpsi_t, (g_r, g_psi) = grad_t."""
        self._dev_args([theta_t, out_t], self.n)
        self._dev_args([rpsi_t, grad_t], 2)
        self._dev_call(self._L.kur_order_parameter_vjp_dev, [theta_t, rpsi_t, grad_t, out_t], self._dp(theta_t),
                       self._dp(rpsi_t), self._dp(grad_t), self._dp(out_t), 1 if accumulate else 0)

    def adjoint_rk4_dev(self, dt: float, nsteps: int, seed_t, gt_t, gw_t, gk_t, theta0_t=None,
                        ckpt_every: int = 32):
        """kur_adjoint_rk4_dev: the gradients into gt_t, gw_t (n) and gk_t (1 entry); any output may
        be None."""
        self._dev_args([seed_t, gt_t, gw_t, theta0_t], self.n)
        self._dev_args([gk_t], 1)
        ts = [theta0_t, seed_t, gt_t, gw_t, gk_t]
        self._dev_call(self._L.kur_adjoint_rk4_dev, ts, self._dp(theta0_t), float(dt), int(nsteps), int(ckpt_every),
                       self._dp(seed_t), self._dp(gt_t), self._dp(gw_t), self._dp(gk_t))

    def adjoint_recorded_dev(self, seed_t, gt_t, gw_t, gk_t):
        """kur_adjoint_rk4_recorded_dev with device seed and gradients."""
        self._dev_args([seed_t, gt_t, gw_t], self.n)
        self._dev_args([gk_t], 1)
        self._dev_call(self._L.kur_adjoint_rk4_recorded_dev, [seed_t, gt_t, gw_t, gk_t], self._dp(seed_t),
                       self._dp(gt_t), self._dp(gw_t), self._dp(gk_t))
