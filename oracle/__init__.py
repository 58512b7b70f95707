"""Python front-end of the LCO oracle -- TEST INFRASTRUCTURE ONLY.

The oracle is the plain CPU definition of what the HIP library computes
(construction, permutation, contraction and addition of linearised-coordinate
sparse tensors), written in ``lco_oracle.cpp`` with coordinate lists, std::stable_sort
and std::map.  Only the tests, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package; the product library never does.

Every function returns numpy arrays; tensors are ``(dims, livs, vals)`` triples
with unsigned 64-bit LIVs in the default order (first mode least significant)
and FP64 values.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liblco_oracle.so")
_lib = None

STATUS = {0: "ok", 1: "bad argument", 2: "index overflow", 3: "shape mismatch", 4: "unsorted",
          5: "duplicate", 7: "unsupported"}


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle status {code}: {STATUS.get(code, '?')}")
        self.code = code


@dataclass
class Tensor:
    dims: np.ndarray   # uint64 (order,)
    livs: np.ndarray   # uint64 (nnz,)
    vals: np.ndarray   # float64 (nnz,)
    absum: np.ndarray | None = None  # float64 (nnz,), sum of |products| (contraction only)

    @property
    def order(self):
        return int(self.dims.shape[0])

    @property
    def nnz(self):
        return int(self.livs.shape[0])


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (plain -O2, no fused multiply-add)."""
    from .build import build_oracle
    return build_oracle(force=force)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    f64p = ctypes.POINTER(ctypes.c_double)
    i32p = ctypes.POINTER(ctypes.c_int)
    vp = ctypes.c_void_p
    lib.ora_status.argtypes = [vp]; lib.ora_status.restype = ctypes.c_int
    lib.ora_nnz.argtypes = [vp]; lib.ora_nnz.restype = ctypes.c_int64
    lib.ora_order.argtypes = [vp]; lib.ora_order.restype = ctypes.c_int
    lib.ora_copy.argtypes = [vp, u64p, u64p, f64p, f64p]; lib.ora_copy.restype = None
    lib.ora_free.argtypes = [vp]; lib.ora_free.restype = None
    lib.ora_linearise.argtypes = [ctypes.c_int, u64p, ctypes.c_int64, u64p, u64p]
    lib.ora_linearise.restype = ctypes.c_int
    lib.ora_delinearise.argtypes = [ctypes.c_int, u64p, ctypes.c_int64, u64p, u64p]
    lib.ora_delinearise.restype = ctypes.c_int
    lib.ora_create.argtypes = [ctypes.c_int, u64p, ctypes.c_int64, u64p, f64p, ctypes.c_int]
    lib.ora_create.restype = vp
    lib.ora_permute.argtypes = [ctypes.c_int, u64p, ctypes.c_int64, u64p, f64p, i32p]
    lib.ora_permute.restype = vp
    lib.ora_contract.argtypes = [ctypes.c_int, u64p, ctypes.c_int64, u64p, f64p, i32p,
                                 ctypes.c_int, u64p, ctypes.c_int64, u64p, f64p, i32p,
                                 ctypes.c_int, i32p, ctypes.c_int]
    lib.ora_contract.restype = vp
    lib.ora_add.argtypes = [ctypes.c_int, u64p, ctypes.c_int64, u64p, f64p, i32p,
                            u64p, ctypes.c_int64, u64p, f64p, i32p, i32p, ctypes.c_double, ctypes.c_double]
    lib.ora_add.restype = vp
    _lib = lib
    return lib


def _u64(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.uint64))
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def _f64(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i32(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.int32))
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _take(h, with_absum=False) -> Tensor:
    lib = _load()
    try:
        st = lib.ora_status(h)
        if st != 0:
            raise OracleError(st)
        n = lib.ora_nnz(h)
        order = lib.ora_order(h)
        dims = np.zeros(order, np.uint64)
        livs = np.zeros(n, np.uint64)
        vals = np.zeros(n, np.float64)
        absum = np.zeros(n, np.float64) if with_absum else None
        f64p = ctypes.POINTER(ctypes.c_double)
        lib.ora_copy(h, _u64(dims)[1], _u64(livs)[1], _f64(vals)[1],
                     absum.ctypes.data_as(f64p) if with_absum else None)
        return Tensor(dims, livs, vals, absum)
    finally:
        lib.ora_free(h)


def linearise(dims, coords) -> np.ndarray:
    """LIVs of coordinate rows in the default order (Section 3.1)."""
    dims, dp = _u64(dims)
    coords, cp = _u64(np.asarray(coords, dtype=np.uint64).reshape(-1, max(len(dims), 1))
                       if len(dims) else np.zeros((len(coords), 0), np.uint64))
    n = coords.shape[0]
    out = np.zeros(n, np.uint64)
    st = _load().ora_linearise(len(dims), dp, n, cp, _u64(out)[1])
    if st:
        raise OracleError(st)
    return out


def delinearise(dims, livs) -> np.ndarray:
    dims, dp = _u64(dims)
    livs, lp = _u64(livs)
    out = np.zeros((livs.shape[0], len(dims)), np.uint64)
    st = _load().ora_delinearise(len(dims), dp, livs.shape[0], lp, _u64(out)[1])
    if st:
        raise OracleError(st)
    return out


def create(dims, coords, vals, sum_duplicates: bool = False) -> Tensor:
    """Sorted LCO tensor from unsorted coordinates (stable sort; duplicates summed in input order)."""
    dims, dp = _u64(dims)
    order = len(dims)
    coords = np.ascontiguousarray(np.asarray(coords, dtype=np.uint64).reshape(-1, order) if order
                                  else np.zeros((len(vals), 0), np.uint64))
    coords, cp = _u64(coords)
    vals, vp = _f64(vals)
    h = _load().ora_create(order, dp, vals.shape[0], cp, vp, int(sum_duplicates))
    return _take(h)


def permute(t: Tensor, perm) -> Tensor:
    """Permute modes: output mode r is input mode perm[r] (Section 4)."""
    dims, dp = _u64(t.dims)
    livs, lp = _u64(t.livs)
    vals, vp = _f64(t.vals)
    perm, pp = _i32(perm)
    h = _load().ora_permute(len(dims), dp, livs.shape[0], lp, vp, pp)
    return _take(h)


def contract(a: Tensor, a_labels, b: Tensor, b_labels, c_labels, mode: str = "map") -> Tensor:
    """Einstein-notation product of two LCO tensors (Sections 2 and 5.2).

    ``mode='map'`` accumulates in a std::map; ``mode='sort'`` sorts the product
    list (same products, same order of summation).  The result carries
    ``absum`` (sum of |products| per entry) for cancellation-aware tolerances.
    """
    da, dap = _u64(a.dims); la, lap = _u64(a.livs); va, vap = _f64(a.vals); laa, laap = _i32(a_labels)
    db, dbp = _u64(b.dims); lb, lbp = _u64(b.livs); vb, vbp = _f64(b.vals); lbb, lbbp = _i32(b_labels)
    lc, lcp = _i32(c_labels)
    h = _load().ora_contract(len(da), dap, la.shape[0], lap, vap, laap,
                             len(db), dbp, lb.shape[0], lbp, vbp, lbbp,
                             len(lc), lcp, 0 if mode == "map" else 1)
    return _take(h, with_absum=True)


def add(a: Tensor, a_labels, b: Tensor, b_labels, c_labels, alpha: float = 1.0, beta: float = 1.0) -> Tensor:
    """c = alpha*a + beta*b over the same labelled modes (Section 2; Section 3.2's
    sum of the two Laplacian terms): b's and c's labels are permutations of a's."""
    if a.order != b.order or len(a_labels) != a.order or len(b_labels) != a.order or len(c_labels) != a.order:
        raise OracleError(1)
    da, dap = _u64(a.dims); la, lap = _u64(a.livs); va, vap = _f64(a.vals); laa, laap = _i32(a_labels)
    db, dbp = _u64(b.dims); lb, lbp = _u64(b.livs); vb, vbp = _f64(b.vals); lbb, lbbp = _i32(b_labels)
    lc, lcp = _i32(c_labels)
    h = _load().ora_add(len(da), dap, la.shape[0], lap, vap, laap, dbp, lb.shape[0], lbp, vbp, lbbp, lcp,
                        float(alpha), float(beta))
    return _take(h)
