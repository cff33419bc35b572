"""ctypes binding of libtn.so (include/tn.h): argument marshalling only.

Every step of the contraction runs in the library's HIP kernels; there is no
Python or CPU fallback.  Loading fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtn.so")

TN_OK, TN_EINVAL, TN_ESTATE, TN_ENOMEM, TN_EDEVICE, TN_ENUMERIC, TN_ZERO = range(7)
STATUS_NAMES = {0: "TN_OK", 1: "TN_EINVAL", 2: "TN_ESTATE", 3: "TN_ENOMEM", 4: "TN_EDEVICE",
                5: "TN_ENUMERIC", 6: "TN_ZERO"}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2}
R_FACTORS = {"gram": 0, "tsqr": 1}
KERNEL_KINDS = {"gemm": 0, "gram": 1, "copy": 2, "core_lds": 3, "core_global": 4, "scale": 5, "lanczos": 6,
                "bwd_gemm": 7, "bwd_core": 8, "recompute": 9}


class TNError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.message = message


class tn_tree_opts(C.Structure):
    _fields_ = [("chi", C.c_int32), ("cutoff", C.c_double), ("compress_late", C.c_int32),
                ("gauge_r", C.c_int32), ("precision", C.c_int32), ("jacobi_max_sweeps", C.c_int32),
                ("device_budget_bytes", C.c_int64), ("keep_intermediates", C.c_int32), ("grad", C.c_int32),
                ("plain", C.c_int32), ("checkpoint_segments", C.c_int32), ("r_factor", C.c_int32)]


_lib = None


def _init_torch_first() -> None:
    """PyTorch-ROCm carries its own HIP runtime; the library links the system one.  Both run
    in one process as long as torch's initialises the device first, so when torch is
    importable and sees a GPU it is initialised before the library is loaded.  Stream
    handles are never passed between the two runtimes (contexts use their own streams)."""
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.init()
    except Exception:
        pass


def load_library(path: Optional[str] = None) -> C.CDLL:
    """Load libtn.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"{p} is missing: run `python -m paper_2206_07044_amd.build` first")
    _init_torch_first()
    lib = C.CDLL(p)
    P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    pI32, pI64, pD = C.POINTER(I32), C.POINTER(I64), C.POINTER(D)
    sig = {
        "tn_create": ([C.c_int, P, C.POINTER(P)], C.c_int),
        "tn_destroy": ([P], None),
        "tn_last_error": ([P], C.c_char_p),
        "tn_load_graph": ([P, I32, I32, pI32, pI32, pI32, pI64, pD], C.c_int),
        "tn_update_values": ([P, pD], C.c_int),
        "tn_update_values_device": ([P, P], C.c_int),
        "tn_set_tree": ([P, I32, pI32, pI32, C.POINTER(tn_tree_opts)], C.c_int),
        "tn_plan_info": ([P, pI64, pD, pD, pI32], C.c_int),
        "tn_set_workspace": ([P, P, C.c_size_t], C.c_int),
        "tn_compress_pair": ([P, P, P, I64, I32, I64, I32, D, P, P, pI32], C.c_int),
        "tn_compress_pair_static": ([P, P, P, I64, I32, I64, I32, D, P, P, pI32], C.c_int),
        "tn_contract_compressed": ([P, pD, pD], C.c_int),
        "tn_result": ([P, pD, pD], C.c_int),
        "tn_enqueue": ([P], C.c_int),
        "tn_fetch": ([P], C.c_int),
        "tn_compress_stats": ([P, I32, pD, pI32, pI32, pI32], C.c_int),
        "tn_grad": ([P, pD], C.c_int),
        "tn_grad_device": ([P, P], C.c_int),
        "tn_grad_info": ([P, pD, pD, pI32], C.c_int),
        "tn_grad_checkpoint_info": ([P, pI32, pD, pI64], C.c_int),
        "tn_gemm_tiles_get": ([pI32], C.c_int),
        "tn_gemm_tiles_set": ([pI32], C.c_int),
        "tn_gemm_tune": ([C.c_int, I32, I32, pD], C.c_int),
        "tn_ising_values_device": ([P, D, P], C.c_int),
        "tn_sync": ([P], C.c_int),
        "tn_batch_create": ([I32, C.POINTER(P), C.POINTER(P)], C.c_int),
        "tn_batch_destroy": ([P], None),
        "tn_batch_last_error": ([P], C.c_char_p),
        "tn_batch_contract": ([P, pD, pD], C.c_int),
        "tn_batch_grad": ([P, C.POINTER(P)], C.c_int),
        "tn_ising_coupling_grad_device": ([P, D, P, P, P], C.c_int),
        "tn_read_tensor": ([P, I32, pD, I64, pI64], C.c_int),
        "tn_read_projectors": ([P, I32, pD, pD, I64, pI32, I32, pI32], C.c_int),
        "tn_profile": ([P, C.c_uint32], C.c_int),
        "tn_profile_read": ([P, I32, pD, pI64, pD, pD], C.c_int),
        "tn_plan_describe": ([I32, I32, pI32, pI32, pI32, I32, pI32, pI32, C.POINTER(tn_tree_opts), I64, pI64, pI64],
                             C.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def exported_symbols() -> List[str]:
    return ["tn_create", "tn_destroy", "tn_last_error", "tn_load_graph", "tn_update_values",
            "tn_update_values_device", "tn_set_workspace", "tn_set_tree", "tn_plan_info", "tn_contract_compressed", "tn_result",
            "tn_enqueue", "tn_fetch", "tn_compress_stats", "tn_read_tensor", "tn_read_projectors", "tn_profile", "tn_profile_read", "tn_grad",
            "tn_grad_device", "tn_grad_info", "tn_grad_checkpoint_info", "tn_ising_values_device", "tn_ising_coupling_grad_device", "tn_sync",
            "tn_batch_create", "tn_batch_destroy", "tn_batch_last_error", "tn_batch_contract", "tn_batch_grad",
            "tn_plan_describe", "tn_compress_pair", "tn_compress_pair_static", "tn_gemm_tiles_get",
            "tn_gemm_tiles_set", "tn_gemm_tune"]


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def make_opts(chi: int, precision: str = "fp64", cutoff: float = 0.0, max_sweeps: int = 0,
              budget: int = 0, keep: bool = False, grad: bool = False, plain: bool = False,
              late: bool = False, gauge_r: int = 0, segments: int = 0, r_factor: str = "gram") -> tn_tree_opts:
    if precision not in PRECISIONS:
        raise ValueError(f"precision must be one of {sorted(PRECISIONS)}")
    if r_factor not in R_FACTORS:
        raise ValueError(f"r_factor must be one of {sorted(R_FACTORS)}")
    return tn_tree_opts(int(chi), float(cutoff), int(bool(late)), int(gauge_r), PRECISIONS[precision],
                        int(max_sweeps), int(budget), int(bool(keep)), int(bool(grad)), int(bool(plain)),
                        int(segments), R_FACTORS[r_factor])


def tn_plan_describe(n: int, edge_u, edge_v, edge_dim, pair_i, pair_j, chi: int,
                     late: bool = False) -> List[Tuple[int, ...]]:
    """Host-only Algorithm 1 expansion: list of (kind, a, b, out, m, n, k, new_dim)."""
    lib = load_library()
    eu, ev, ed, pi, pj = map(_i32, (edge_u, edge_v, edge_dim, pair_i, pair_j))
    opts = make_opts(chi, late=late)
    n_ops = C.c_int64(0)
    st = lib.tn_plan_describe(n, eu.size, _ptr(eu, C.c_int32), _ptr(ev, C.c_int32), _ptr(ed, C.c_int32), pi.size,
                              _ptr(pi, C.c_int32), _ptr(pj, C.c_int32), C.byref(opts), 0, None, C.byref(n_ops))
    if st != TN_OK:
        raise TNError(st, "invalid graph or tree")
    buf = np.zeros((max(1, n_ops.value), 8), dtype=np.int64)
    st = lib.tn_plan_describe(n, eu.size, _ptr(eu, C.c_int32), _ptr(ev, C.c_int32), _ptr(ed, C.c_int32), pi.size,
                              _ptr(pi, C.c_int32), _ptr(pj, C.c_int32), C.byref(opts), n_ops.value,
                              _ptr(buf, C.c_int64), C.byref(n_ops))
    if st != TN_OK:
        raise TNError(st, "invalid graph or tree")
    return [tuple(int(x) for x in row) for row in buf[:n_ops.value]]


GEMM_CLASSES = 72
GEMM_TILES = ["64x64", "256x16", "16x256", "128x32", "32x128", "skinny_tall16", "skinny_tall32", "skinny_wide16",
              "skinny_wide32"]


def tn_gemm_tiles_get() -> np.ndarray:
    """The process-wide tile table (one tn_gemm_tile per class)."""
    t = np.zeros(GEMM_CLASSES, dtype=np.int32)
    st = load_library().tn_gemm_tiles_get(_ptr(t, C.c_int32))
    if st != TN_OK:
        raise TNError(st, "tn_gemm_tiles_get")
    return t


def tn_gemm_tiles_set(table: Optional[Sequence[int]]) -> None:
    """Install a tile table, or the built-in defaults with None."""
    if table is None:
        st = load_library().tn_gemm_tiles_set(None)
    else:
        t = _i32(table)
        if t.size != GEMM_CLASSES:
            raise ValueError(f"a tile table has {GEMM_CLASSES} entries")
        st = load_library().tn_gemm_tiles_set(_ptr(t, C.c_int32))
    if st != TN_OK:
        raise TNError(st, "a tile does not fit its class")


def tn_gemm_tune(klass: int, copies: int = 8, device: int = 0) -> np.ndarray:
    """Microseconds per grouped launch of every tile on the class's representative shape (-1: n/a)."""
    us = np.zeros(len(GEMM_TILES), dtype=np.float64)
    st = load_library().tn_gemm_tune(int(device), int(klass), int(copies), _ptr(us, C.c_double))
    if st != TN_OK:
        raise TNError(st, f"tn_gemm_tune(class {klass})")
    return us


class Context:
    """One tn_ctx: a graph, a planned tree and its device arena."""

    def __init__(self, device: int = 0, stream: Optional[int] = None):
        self._lib = load_library()
        self._h = C.c_void_p()
        # bumped by every call that changes the inputs or the last evaluation (values, trees,
        # evaluations): the autograd functions compare it to know whether the context still
        # holds the forward pass they are asked to differentiate
        self.state_id = 0
        st = self._lib.tn_create(int(device), C.c_void_p(stream) if stream else None, C.byref(self._h))
        if st != TN_OK:
            raise TNError(st, "tn_create failed (no HIP device?)")

    def last_error(self) -> str:
        msg = self._lib.tn_last_error(self._h) if self._h else None
        return msg.decode() if msg else ""

    def close(self) -> None:
        if self._h:
            self._lib.tn_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int) -> int:
        if st != TN_OK:
            msg = self._lib.tn_last_error(self._h)
            raise TNError(st, msg.decode() if msg else "")
        return st

    def tn_load_graph(self, n: int, edge_u, edge_v, edge_dim, offsets, data) -> None:
        eu, ev, ed = map(_i32, (edge_u, edge_v, edge_dim))
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        self._data = np.ascontiguousarray(data, dtype=np.float64)
        self._n_data = int(off[-1]) if off.size else 0
        self.state_id += 1
        self._check(self._lib.tn_load_graph(self._h, int(n), eu.size, _ptr(eu, C.c_int32), _ptr(ev, C.c_int32),
                                            _ptr(ed, C.c_int32), _ptr(off, C.c_int64),
                                            _ptr(self._data, C.c_double)))

    def tn_update_values(self, data) -> None:
        d = np.ascontiguousarray(data, dtype=np.float64)
        self.state_id += 1
        self._check(self._lib.tn_update_values(self._h, _ptr(d, C.c_double)))

    def tn_update_values_device(self, dev_ptr: int) -> None:
        self.state_id += 1
        self._check(self._lib.tn_update_values_device(self._h, C.c_void_p(dev_ptr)))

    def tn_set_tree(self, pair_i, pair_j, chi: int, precision: str = "fp64", cutoff: float = 0.0,
                    max_sweeps: int = 0, budget: int = 0, keep_intermediates: bool = False,
                    grad: bool = False, plain: bool = False, late: bool = False, gauge_r: int = 0,
                    checkpoint_segments: int = 0, r_factor: str = "gram") -> None:
        """checkpoint_segments (grad only): 0/1 keep every forward buffer the reverse pass reads;
        S >= 2 recompute forward segments in the reverse pass; -1 the S of smallest arena.
        r_factor: "gram" (Gram + pivoted Cholesky) or "tsqr" (Householder TSQR) for D <= 64."""
        pi, pj = _i32(pair_i), _i32(pair_j)
        opts = make_opts(chi, precision, cutoff, max_sweeps, budget, keep_intermediates, grad, plain, late,
                         gauge_r, checkpoint_segments, r_factor)
        self.state_id += 1
        self._check(self._lib.tn_set_tree(self._h, pi.size, _ptr(pi, C.c_int32), _ptr(pj, C.c_int32),
                                          C.byref(opts)))

    def tn_set_workspace(self, dev_ptr: Optional[int], nbytes: int) -> None:
        """Arena memory for later plans (device pointer, caller owned); None: library allocation."""
        self._check(self._lib.tn_set_workspace(self._h, C.c_void_p(dev_ptr) if dev_ptr else None, int(nbytes)))

    def tn_plan_info(self) -> dict:
        ab, ff, fb, ns = C.c_int64(), C.c_double(), C.c_double(), C.c_int32()
        self._check(self._lib.tn_plan_info(self._h, C.byref(ab), C.byref(ff), C.byref(fb), C.byref(ns)))
        return {"arena_bytes": ab.value, "fwd_flops": ff.value, "fwd_bytes": fb.value, "n_steps": ns.value}

    def tn_contract_compressed(self) -> Tuple[float, float]:
        m, e = C.c_double(), C.c_double()
        self.state_id += 1
        st = self._lib.tn_contract_compressed(self._h, C.byref(m), C.byref(e))
        if st == TN_ZERO:
            return 0.0, float("-inf")
        self._check(st)
        return m.value, e.value

    def tn_result(self) -> Tuple[float, float]:
        s, l = C.c_double(), C.c_double()
        self._check(self._lib.tn_result(self._h, C.byref(s), C.byref(l)))
        return s.value, l.value

    def tn_enqueue(self) -> None:
        self.state_id += 1
        self._check(self._lib.tn_enqueue(self._h))

    def tn_fetch(self) -> int:
        st = self._lib.tn_fetch(self._h)
        if st not in (TN_OK, TN_ZERO):
            self._check(st)
        return st

    def tn_compress_stats(self):
        n = C.c_int32()
        self._check(self._lib.tn_compress_stats(self._h, 0, None, None, None, C.byref(n)))
        k = max(1, n.value)
        disc = np.zeros(k)
        tie = np.zeros(k, dtype=np.int32)
        sw = np.zeros(k, dtype=np.int32)
        self._check(self._lib.tn_compress_stats(self._h, n.value, _ptr(disc, C.c_double), _ptr(tie, C.c_int32),
                                                _ptr(sw, C.c_int32), C.byref(n)))
        return disc[:n.value], tie[:n.value], sw[:n.value]

    def tn_profile(self, kinds) -> None:
        mask = 0
        for k in kinds:
            mask |= 1 << KERNEL_KINDS[k]
        self._check(self._lib.tn_profile(self._h, mask))

    def tn_profile_read(self, kind: str) -> dict:
        ms, n, f, b = C.c_double(), C.c_int64(), C.c_double(), C.c_double()
        self._check(self._lib.tn_profile_read(self._h, KERNEL_KINDS[kind], C.byref(ms), C.byref(n), C.byref(f),
                                              C.byref(b)))
        return {"ms": ms.value, "launches": n.value, "flops": f.value, "bytes": b.value}

    def tn_read_tensor(self, index: int) -> np.ndarray:
        n = C.c_int64()
        self._check(self._lib.tn_read_tensor(self._h, int(index), None, 0, C.byref(n)))
        out = np.zeros(max(1, n.value))
        self._check(self._lib.tn_read_tensor(self._h, int(index), _ptr(out, C.c_double), n.value, C.byref(n)))
        return out[:n.value]

    def tn_read_projectors(self, comp: int, values: bool = True) -> dict:
        """Compression `comp`'s bond (tree nodes a and b, bundled edges in P_L's row order, the new
        edge) and, with `values`, its projectors P_L (D x chi') and P_R (chi' x D) as float64."""
        info = np.zeros(6, dtype=np.int32)
        self._check(self._lib.tn_read_projectors(self._h, int(comp), None, None, 0, None, 0, _ptr(info, C.c_int32)))
        D, cn, e_new, a, b, ne = (int(x) for x in info)
        edges = np.zeros(max(1, ne), dtype=np.int32)
        out = {"D": D, "chi": cn, "new_edge": e_new, "a": a, "b": b}
        if values:
            pl = np.zeros(max(1, D * cn))
            pr = np.zeros(max(1, D * cn))
            self._check(self._lib.tn_read_projectors(self._h, int(comp), _ptr(pl, C.c_double), _ptr(pr, C.c_double),
                                                     D * cn, _ptr(edges, C.c_int32), ne, _ptr(info, C.c_int32)))
            out["p_left"] = pl[:D * cn].reshape(D, cn)
            out["p_right"] = pr[:D * cn].reshape(cn, D)
        else:
            self._check(self._lib.tn_read_projectors(self._h, int(comp), None, None, 0, _ptr(edges, C.c_int32), ne,
                                                     _ptr(info, C.c_int32)))
        out["edges"] = [int(e) for e in edges[:ne]]
        return out

    def tn_grad(self, out: Optional[np.ndarray] = None) -> np.ndarray:
        """d ln|Z| / d data (float64, the layout of the loaded data)."""
        g = np.zeros(self._n_data) if out is None else out
        self._check(self._lib.tn_grad(self._h, _ptr(g, C.c_double)))
        return g

    def tn_grad_device(self, dev_ptr: int) -> None:
        self._check(self._lib.tn_grad_device(self._h, C.c_void_p(dev_ptr)))

    def tn_sync(self) -> None:
        self._check(self._lib.tn_sync(self._h))

    def tn_ising_values_device(self, beta: float, J_ptr: int) -> None:
        self.state_id += 1
        self._check(self._lib.tn_ising_values_device(self._h, float(beta), C.c_void_p(J_ptr)))

    def tn_ising_coupling_grad_device(self, beta: float, J_ptr: int, dT_ptr: int, dJ_ptr: int) -> None:
        self._check(self._lib.tn_ising_coupling_grad_device(self._h, float(beta), C.c_void_p(J_ptr),
                                                            C.c_void_p(dT_ptr), C.c_void_p(dJ_ptr)))

    def tn_compress_pair(self, a_ptr: int, b_ptr: int, m_a: int, D: int, m_b: int, chi: int, cutoff: float,
                         a_out_ptr: int, b_out_ptr: int) -> int:
        """One bond compression of device float64 matrices A (m_a x D) and B (D x m_b); returns chi'."""
        nw = C.c_int32()
        self._check(self._lib.tn_compress_pair(self._h, C.c_void_p(a_ptr), C.c_void_p(b_ptr), int(m_a), int(D),
                                               int(m_b), int(chi), float(cutoff), C.c_void_p(a_out_ptr),
                                               C.c_void_p(b_out_ptr), C.byref(nw)))
        return nw.value

    def tn_compress_pair_static(self, a_ptr: int, b_ptr: int, m_a: int, D: int, m_b: int, chi: int,
                                cutoff: float, a_out_ptr: int, b_out_ptr: int) -> int:
        """tn_compress_pair on the library's fixed device scratch (allocates nothing); returns chi'."""
        nw = C.c_int32()
        self._check(self._lib.tn_compress_pair_static(self._h, C.c_void_p(a_ptr), C.c_void_p(b_ptr), int(m_a),
                                                      int(D), int(m_b), int(chi), float(cutoff),
                                                      C.c_void_p(a_out_ptr), C.c_void_p(b_out_ptr), C.byref(nw)))
        return nw.value

    def tn_grad_info(self) -> dict:
        f, b, n = C.c_double(), C.c_double(), C.c_int32()
        self._check(self._lib.tn_grad_info(self._h, C.byref(f), C.byref(b), C.byref(n)))
        return {"bwd_flops": f.value, "bwd_bytes": b.value, "n_levels": n.value}

    def tn_grad_checkpoint_info(self) -> dict:
        sg, f, b = C.c_int32(), C.c_double(), C.c_int64()
        self._check(self._lib.tn_grad_checkpoint_info(self._h, C.byref(sg), C.byref(f), C.byref(b)))
        return {"segments": sg.value, "recompute_flops": f.value, "checkpoint_bytes": b.value}


class Batch:
    """tn_batch: several planned contexts merged level by level and replayed from one hipGraph."""

    def __init__(self, contexts: Sequence["Context"]):
        self._lib = load_library()
        self.contexts = list(contexts)
        arr = (C.c_void_p * len(self.contexts))(*[c._h.value for c in self.contexts])
        self._h = C.c_void_p()
        st = self._lib.tn_batch_create(len(self.contexts), arr, C.byref(self._h))
        if st != TN_OK:
            msgs = [c.last_error() for c in self.contexts]
            raise TNError(st, "tn_batch_create failed: " + "; ".join(m for m in msgs if m))

    def _check(self, st: int) -> int:
        if st != TN_OK:
            msg = self._lib.tn_batch_last_error(self._h)
            raise TNError(st, msg.decode() if msg else "")
        return st

    def tn_batch_contract(self):
        n = len(self.contexts)
        m = np.zeros(n)
        e = np.zeros(n)
        for c in self.contexts:
            c.state_id += 1
        self._check(self._lib.tn_batch_contract(self._h, _ptr(m, C.c_double), _ptr(e, C.c_double)))
        return m, e

    def tn_batch_grad(self, dev_ptrs: Sequence[int]) -> None:
        arr = (C.c_void_p * len(dev_ptrs))(*[int(p) for p in dev_ptrs])
        self._check(self._lib.tn_batch_grad(self._h, arr))

    def close(self) -> None:
        if self._h:
            self._lib.tn_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
