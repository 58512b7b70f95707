"""ctypes binding of ``liblco.so`` (the C-ABI of ``include/lco.h``).

Marshalling only.  Device arrays are torch CUDA (HIP) tensors; the library's
allocations go through the torch caching allocator on the context's stream, so
the LIV / value arrays of a result can be viewed as torch tensors without a copy.

If the compiled library is missing this module raises ImportError: there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading

__all__ = [
    "LcoError", "Context", "Tensor", "Plan", "RpPlan", "load_library", "library_path",
    "lco_ctx_create", "lco_ctx_destroy", "lco_ctx_synchronize", "lco_create", "lco_destroy", "lco_permute",
    "lco_permute_noalloc", "LCO_NOALLOC_MAX_NNZ",
    "lco_contract", "lco_add", "lco_contract_batch", "lco_batch_stats", "ContractDesc", "Server", "lco_read",
    "BatchPlan", "lco_plan_info", "lco_plan_contract", "lco_plan_permute", "lco_classify", "lco_select",
    "lco_fastdiv_host", "lco_timing_enable", "lco_timing_only", "lco_timing_reset", "lco_timing_query", "lco_timing_kernels",
    "lco_ctx_set_crossovers", "lco_ctx_get_crossovers", "MI355X_CROSSOVERS", "PAPER_CROSSOVERS",
    "lco_ctx_set_index_algorithm", "lco_ctx_get_index_algorithm", "lco_ctx_use_paper_selector",
    "lco_ctx_use_mi355x_selector", "MI355X_INDEX_ALGORITHM",
    "lco_version", "LCO_SORTED", "LCO_COORDS", "LCO_SUM_DUPLICATES", "ALGOS", "ALGO_IDS", "CLASSES",
    "LCO_ALG_AUTO", "LCO_ALG_CSC", "LCO_ALG_CSR", "LCO_ALG_DCSC", "LCO_ALG_DCSR", "LCO_ALG_CSCNA",
    "LCO_ALG_CSRNA", "LCO_ALG_SOP", "LCO_SPARSE", "LCO_ROW_SPARSE", "LCO_COL_SPARSE", "LCO_INDEX_SPARSE",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liblco.so")

LCO_SORTED = 0x1
LCO_COORDS = 0x2
LCO_SUM_DUPLICATES = 0x4

LCO_ALG_AUTO, LCO_ALG_CSC, LCO_ALG_CSR, LCO_ALG_DCSC, LCO_ALG_DCSR, LCO_ALG_CSCNA, LCO_ALG_CSRNA, LCO_ALG_SOP = range(8)
ALGOS = {0: "auto", 1: "CSC", 2: "CSR", 3: "DCSC", 4: "DCSR", 5: "CSCNA", 6: "CSRNA", 7: "SOP"}
ALGO_IDS = {v: k for k, v in ALGOS.items()}
LCO_SPARSE, LCO_ROW_SPARSE, LCO_COL_SPARSE, LCO_INDEX_SPARSE = range(4)
CLASSES = {0: "sparse", 1: "row-sparse", 2: "column-sparse", 3: "index-sparse"}

_STATUS = {0: "ok", 1: "bad argument", 2: "index overflow", 3: "shape mismatch", 4: "unsorted input",
           5: "duplicate entry", 6: "out of memory", 7: "unsupported", 8: "HIP runtime error"}


class LcoError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


class Plan(ctypes.Structure):
    _fields_ = [("m", ctypes.c_uint64), ("k", ctypes.c_uint64), ("n", ctypes.c_uint64),
                ("nnz_a", ctypes.c_int64), ("nnz_b", ctypes.c_int64),
                ("a_class", ctypes.c_int), ("b_class", ctypes.c_int), ("algo", ctypes.c_int),
                ("permute_a", ctypes.c_int), ("permute_b", ctypes.c_int), ("permute_c", ctypes.c_int),
                ("num_contracted", ctypes.c_int), ("num_entrywise", ctypes.c_int)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["algo_name"] = ALGOS[self.algo]
        d["a_class_name"] = CLASSES[self.a_class]
        d["b_class_name"] = CLASSES[self.b_class]
        return d


class RpPlan(ctypes.Structure):
    _fields_ = [("identity", ctypes.c_int), ("prefix", ctypes.c_int), ("suffix", ctypes.c_int),
                ("rearrangement", ctypes.c_uint32), ("key_bits", ctypes.c_int), ("seg_bits", ctypes.c_int),
                ("full_bits", ctypes.c_int), ("method", ctypes.c_int), ("passes", ctypes.c_int),
                ("digit_bits", ctypes.c_int), ("key_div", ctypes.c_uint64), ("key_range", ctypes.c_uint64),
                ("seg_div", ctypes.c_uint64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ServerConfig(ctypes.Structure):
    _fields_ = [("workers", ctypes.c_int), ("max_batch", ctypes.c_int), ("plain", ctypes.c_int),
                ("solo_nnz", ctypes.c_int64), ("hbm_budget", ctypes.c_uint64)]


class ServerResult(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_int64), ("status", ctypes.c_int), ("out", ctypes.c_void_p),
                ("latency_ms", ctypes.c_double), ("queue_ms", ctypes.c_double), ("batch_size", ctypes.c_int)]


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)

_lib = None
_lock = threading.Lock()


def library_path() -> str:
    return _LIB_PATH


def load_library():
    """Load liblco.so (ImportError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is not None:
            return _lib
        # One HIP runtime per process: torch ships its own libamdhip64 (same soname); importing torch
        # first makes the dynamic loader bind liblco.so to that already-loaded runtime.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"{_LIB_PATH} is missing: build it with paper_1802_02619_amd/build.py "
                              "(or __graft_entry__.build()); there is no CPU fallback")
        L = ctypes.CDLL(_LIB_PATH)
        vp, i32, i64, u32, u64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
        pi32 = ctypes.POINTER(ctypes.c_int)
        pu64 = ctypes.POINTER(ctypes.c_uint64)
        pvp = ctypes.POINTER(ctypes.c_void_p)
        sig = {
            "lco_ctx_create": (i32, [i32, vp, _ALLOC_FN, _FREE_FN, vp, pvp]),
            "lco_ctx_destroy": (i32, [vp]),
            "lco_ctx_set_stream": (i32, [vp, vp]),
            "lco_ctx_synchronize": (i32, [vp]),
            "lco_timing_enable": (i32, [vp, i32]),
            "lco_timing_only": (i32, [vp, ctypes.c_char_p]),
            "lco_timing_reset": (i32, [vp]),
            "lco_timing_query": (i32, [vp, ctypes.c_char_p, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double)]),
            "lco_timing_kernel_name": (ctypes.c_char_p, [vp, i32]),
            "lco_create": (i32, [vp, i32, pu64, i64, vp, vp, u32, pvp]),
            "lco_destroy": (i32, [vp]),
            "lco_read": (i32, [vp, vp, vp]),
            "lco_batch_plan_create": (i32, [vp, i32, ctypes.POINTER(ContractDesc), pvp]),
            "lco_batch_plan_output": (vp, [vp, i32]),
            "lco_batch_plan_execute": (i32, [vp, vp]),
            "lco_batch_plan_graph_launch": (i32, [vp, vp]),
            "lco_batch_plan_launch_info": (i32, [vp, i32] + [ctypes.POINTER(i32)] * 4 +
                                           [ctypes.POINTER(ctypes.c_double)]),
            "lco_batch_plan_destroy": (i32, [vp]),
            "lco_server_create": (i32, [i32, ctypes.POINTER(ServerConfig), pvp]),
            "lco_server_submit": (i32, [vp, ctypes.POINTER(ContractDesc), ctypes.POINTER(i64)]),
            "lco_server_poll": (i32, [vp, ctypes.POINTER(ServerResult), i32, ctypes.POINTER(i32)]),
            "lco_server_drain": (i32, [vp]),
            "lco_server_destroy": (i32, [vp]),
            "lco_nnz": (i64, [vp]),
            "lco_order": (i32, [vp]),
            "lco_dims": (pu64, [vp]),
            "lco_livs": (vp, [vp]),
            "lco_vals": (vp, [vp]),
            "lco_permute": (i32, [vp, vp, pi32, pvp]),
            "lco_permute_noalloc": (i32, [vp, vp, pi32, vp, vp, pu64]),
            "lco_contract": (i32, [vp, vp, pi32, vp, pi32, i32, pi32, u32, pvp]),
            "lco_add": (i32, [vp, ctypes.c_double, vp, pi32, ctypes.c_double, vp, pi32, pi32, pvp]),
            "lco_ctx_set_crossovers": (i32, [vp, ctypes.c_double, ctypes.c_double, ctypes.c_double]),
            "lco_ctx_get_crossovers": (i32, [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(ctypes.c_double)]),
            "lco_ctx_set_index_algorithm": (i32, [vp, i32]),
            "lco_ctx_get_index_algorithm": (i32, [vp, pi32]),
            "lco_plan_info": (i32, [vp, vp, pi32, vp, pi32, i32, pi32, u32, ctypes.POINTER(Plan)]),
            "lco_contract_batch": (i32, [vp, i32, ctypes.POINTER(ContractDesc), ctypes.POINTER(ctypes.c_void_p)]),
            "lco_batch_stats": (i32, [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)]),
            "lco_classify": (i32, [u64, u64, i64, ctypes.POINTER(i32)]),
            "lco_select": (i32, [i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]),
            "lco_plan_contract": (i32, [i32, pu64, pi32, i64, i32, pu64, pi32, i64, i32, pi32, u32,
                                        ctypes.POINTER(Plan)]),
            "lco_plan_permute": (i32, [i32, pu64, pi32, i64, ctypes.POINTER(RpPlan)]),
            "lco_fastdiv_host": (i32, [u64, i64, pu64, pu64, pu64]),
            "lco_status_str": (ctypes.c_char_p, [i32]),
            "lco_last_error": (ctypes.c_char_p, []),
            "lco_version": (ctypes.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
        return L


def _check(st: int):
    if st != 0:
        raise LcoError(st, load_library().lco_last_error().decode())


def _u64arr(xs):
    xs = [int(x) for x in xs]
    return (ctypes.c_uint64 * max(1, len(xs)))(*xs)


def _i32arr(xs):
    xs = [int(x) for x in xs]
    return (ctypes.c_int * max(1, len(xs)))(*xs)


# Label and permutation lists repeat from call to call: their int arrays are
# kept (the library only reads them during a call), bounded in number.
_LABEL_ARRAYS = {}


def _labels(xs):
    k = tuple(xs)
    a = _LABEL_ARRAYS.get(k)
    if a is None:
        if len(_LABEL_ARRAYS) >= 4096:
            _LABEL_ARRAYS.clear()
        a = _LABEL_ARRAYS[k] = _i32arr(k)
    return a


def lco_version() -> str:
    return load_library().lco_version().decode()


# ------------------------------------------------------------------ context
class Context:
    """A library context on one device and stream.  With allocator="torch" (the default) device memory
    comes from torch's caching allocator and livs()/vals() are torch views; with allocator="library"
    the library allocates itself (hipMalloc, with released blocks reused in stream order) and tensors
    are read with to_numpy()."""

    def __init__(self, device: int = 0, stream=None, allocator: str = "torch"):
        import torch
        if allocator not in ("torch", "library"):
            raise ValueError("allocator must be 'torch' or 'library'")
        L = load_library()
        self._torch = torch
        self.device = int(device)
        self._dev = torch.device("cuda", self.device)
        if stream is None:
            stream = torch.cuda.current_stream(self._dev)
        self.stream = stream
        self._allocs = {}
        if allocator == "library":
            h = ctypes.c_void_p()
            _check(L.lco_ctx_create(self.device, ctypes.c_void_p(stream.cuda_stream), ctypes.cast(None, _ALLOC_FN),
                                    ctypes.cast(None, _FREE_FN), None, ctypes.byref(h)))
            self.handle = h
            return

        self._stream_handle = int(stream.cuda_stream)

        def _alloc(user, nbytes, strm):
            try:
                # torch's allocator ties a block to the current stream: allocate on the context's stream
                # (entering a stream context only when another stream is current)
                if torch.cuda.current_stream(self._dev).cuda_stream == self._stream_handle:
                    t = torch.empty(int(nbytes), dtype=torch.uint8, device=self._dev)
                else:
                    with torch.cuda.stream(self.stream):
                        t = torch.empty(int(nbytes), dtype=torch.uint8, device=self._dev)
                p = t.data_ptr()
                self._allocs[p] = t
                return p
            except Exception:  # reported to the caller as LCO_E_OOM
                return None

        def _free(user, ptr, nbytes, strm):
            self._allocs.pop(ptr, None)

        self._alloc_cb = _ALLOC_FN(_alloc)
        self._free_cb = _FREE_FN(_free)
        h = ctypes.c_void_p()
        _check(L.lco_ctx_create(self.device, ctypes.c_void_p(stream.cuda_stream), self._alloc_cb, self._free_cb,
                                None, ctypes.byref(h)))
        self.handle = h

    def synchronize(self):
        _check(load_library().lco_ctx_synchronize(self.handle))

    def set_stream(self, stream):
        """Move the context's later work to another torch stream of its device (waits for the old one)."""
        _check(load_library().lco_ctx_set_stream(self.handle, ctypes.c_void_p(stream.cuda_stream)))
        self.stream = stream
        self._stream_handle = int(stream.cuda_stream)

    def destroy(self):
        if self.handle:
            _check(load_library().lco_ctx_destroy(self.handle))
            self.handle = None

    def view(self, ptr: int, nbytes: int, dtype):
        """torch view of `nbytes` at device pointer `ptr` inside one of this context's allocations
        (torch-allocating contexts only)."""
        t = self._allocs.get(ptr)
        if t is not None:
            return t[:nbytes].view(dtype)
        for start, buf in self._allocs.items():  # inside a shared allocation (batch outputs)
            if start <= ptr and ptr + nbytes <= start + buf.numel():
                off = ptr - start
                return buf[off:off + nbytes].view(dtype)
        raise KeyError("pointer is not inside a torch allocation of this context (library-allocating contexts: "
                       "read tensors with to_numpy())")


def lco_ctx_create(device: int = 0, stream=None, allocator: str = "torch") -> Context:
    return Context(device, stream, allocator)


def lco_ctx_destroy(ctx: Context):
    ctx.destroy()


def lco_ctx_synchronize(ctx: Context):
    ctx.synchronize()


# ------------------------------------------------------------------ tensors
class Tensor:
    """Handle of an LCO tensor owned by the library (release with destroy())."""

    def __init__(self, ctx: Context, handle):
        self.ctx = ctx
        self.handle = handle

    @property
    def nnz(self) -> int:
        return int(load_library().lco_nnz(self.handle))

    @property
    def order(self) -> int:
        return int(load_library().lco_order(self.handle))

    @property
    def dims(self):
        L = load_library()
        p = L.lco_dims(self.handle)
        return [int(p[i]) for i in range(self.order)]

    def livs(self):
        """torch int64 view (bit pattern of the unsigned LIVs) on the device; no copy."""
        import torch
        n = self.nnz
        if n == 0:
            return torch.zeros(0, dtype=torch.int64, device=self.ctx._dev)
        p = load_library().lco_livs(self.handle)
        return self.ctx.view(p, n * 8, torch.uint8).view(torch.int64)

    def vals(self):
        import torch
        n = self.nnz
        if n == 0:
            return torch.zeros(0, dtype=torch.float64, device=self.ctx._dev)
        p = load_library().lco_vals(self.handle)
        return self.ctx.view(p, n * 8, torch.uint8).view(torch.float64)

    def to_numpy(self):
        """(dims, livs uint64, vals float64) copied to the host (lco_read)."""
        import numpy as np
        n = self.nnz
        livs = np.empty(n, dtype=np.uint64)
        vals = np.empty(n, dtype=np.float64)
        if n:
            _check(load_library().lco_read(self.handle, livs.ctypes.data_as(ctypes.c_void_p),
                                           vals.ctypes.data_as(ctypes.c_void_p)))
        return np.array(self.dims, dtype=np.uint64), livs, vals

    def destroy(self):
        if self.handle:
            _check(load_library().lco_destroy(self.handle))
            self.handle = None


def lco_create(ctx: Context, dims, idx, vals, flags: int = 0) -> Tensor:
    """Build a tensor from device arrays: `idx` (int64/uint64 torch tensor of LIVs, or of
    nnz*order coordinates with LCO_COORDS) and `vals` (float64)."""
    import torch
    L = load_library()
    nnz = int(vals.numel())
    if idx.dtype not in (torch.int64, torch.uint64) or vals.dtype != torch.float64:
        raise TypeError("idx must be int64/uint64 and vals float64")
    idx = idx.contiguous()
    vals = vals.contiguous()
    h = ctypes.c_void_p()
    _check(L.lco_create(ctx.handle, len(dims), _u64arr(dims), nnz, ctypes.c_void_p(idx.data_ptr() if nnz else 0),
                        ctypes.c_void_p(vals.data_ptr() if nnz else 0), int(flags), ctypes.byref(h)))
    return Tensor(ctx, h)


def lco_destroy(t: Tensor):
    t.destroy()


def lco_read(t: Tensor):
    """(livs uint64, vals float64) of a tensor, copied to the host."""
    _, livs, vals = t.to_numpy()
    return livs, vals


def lco_permute(ctx: Context, t: Tensor, perm) -> Tensor:
    L = load_library()
    h = ctypes.c_void_p()
    _check(L.lco_permute(ctx.handle, t.handle, _labels(perm), ctypes.byref(h)))
    return Tensor(ctx, h)


LCO_NOALLOC_MAX_NNZ = 1 << 20  # include/lco.h


def lco_permute_noalloc(ctx: Context, t: Tensor, perm, out_livs, out_vals):
    """lco_permute into caller-owned device tensors (int64 / float64, t.nnz entries each), with no device
    allocation by the library; returns the output dimensions."""
    L = load_library()
    dims = (ctypes.c_uint64 * max(1, t.order))()
    _check(L.lco_permute_noalloc(ctx.handle, t.handle, _i32arr(perm), ctypes.c_void_p(out_livs.data_ptr()),
                                 ctypes.c_void_p(out_vals.data_ptr()), dims))
    return [int(dims[r]) for r in range(t.order)]


def lco_contract(ctx: Context, a: Tensor, a_labels, b: Tensor, b_labels, c_labels, flags: int = 0) -> Tensor:
    L = load_library()
    h = ctypes.c_void_p()
    _check(L.lco_contract(ctx.handle, a.handle, _labels(a_labels), b.handle, _labels(b_labels), len(c_labels),
                          _labels(c_labels), int(flags), ctypes.byref(h)))
    return Tensor(ctx, h)


# selector crossovers (doubly compressed, no accumulator, index cell): the paper's table as is, and
# those measured on MI355X (LCO_MI355X_* in include/lco.h), a new context's default
PAPER_CROSSOVERS = (3.0, 3.0, 3.0)
MI355X_CROSSOVERS = (10.0, 3.0, 30.0)
MI355X_INDEX_ALGORITHM = "DCSC"


def lco_ctx_set_crossovers(ctx: Context, doubly_compressed: float, no_accumulator: float, outer_product: float):
    _check(load_library().lco_ctx_set_crossovers(ctx.handle, float(doubly_compressed), float(no_accumulator),
                                                 float(outer_product)))


def lco_ctx_get_crossovers(ctx: Context):
    d, n, o = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(load_library().lco_ctx_get_crossovers(ctx.handle, ctypes.byref(d), ctypes.byref(n), ctypes.byref(o)))
    return (d.value, n.value, o.value)


def lco_ctx_set_index_algorithm(ctx: Context, algo):
    """The index-sparse x index-sparse cell's algorithm above its crossover: "SOP" or "DCSC"/"DCSR"."""
    _check(load_library().lco_ctx_set_index_algorithm(ctx.handle, ALGO_IDS[algo] if isinstance(algo, str) else
                                                      int(algo)))


def lco_ctx_get_index_algorithm(ctx: Context) -> str:
    a = ctypes.c_int()
    _check(load_library().lco_ctx_get_index_algorithm(ctx.handle, ctypes.byref(a)))
    return ALGOS[a.value]


def lco_ctx_use_paper_selector(ctx: Context):
    """The paper's table unchanged: crossovers of 3 and SOP in the index-sparse cell."""
    lco_ctx_set_crossovers(ctx, *PAPER_CROSSOVERS)
    lco_ctx_set_index_algorithm(ctx, "SOP")


def lco_ctx_use_mi355x_selector(ctx: Context):
    """The selector measured on MI355X (a new context's default)."""
    lco_ctx_set_crossovers(ctx, *MI355X_CROSSOVERS)
    lco_ctx_set_index_algorithm(ctx, MI355X_INDEX_ALGORITHM)


def lco_add(ctx: Context, a: Tensor, a_labels, b: Tensor, b_labels, c_labels, alpha: float = 1.0,
            beta: float = 1.0) -> Tensor:
    """c = alpha*a + beta*b over the same labelled modes (output mode order: c_labels)."""
    L = load_library()
    h = ctypes.c_void_p()
    _check(L.lco_add(ctx.handle, float(alpha), a.handle, _labels(a_labels), float(beta), b.handle,
                     _labels(b_labels), _labels(c_labels), ctypes.byref(h)))
    return Tensor(ctx, h)


class ContractDesc(ctypes.Structure):
    _fields_ = [("a", ctypes.c_void_p), ("a_labels", ctypes.POINTER(ctypes.c_int)),
                ("b", ctypes.c_void_p), ("b_labels", ctypes.POINTER(ctypes.c_int)),
                ("c_order", ctypes.c_int), ("c_labels", ctypes.POINTER(ctypes.c_int)),
                ("flags", ctypes.c_uint32)]


def _handle_value(h) -> int:
    return (h.value or 0) if isinstance(h, ctypes.c_void_p) else int(h)


def _desc_array(items):
    """lco_contract_desc records of `items` (a, a_labels, b, b_labels, c_labels[, flags]) as a numpy
    array laid out like ContractDesc, and the label arrays it points to (one per distinct list)."""
    import numpy as np
    n = len(items)
    dt = np.dtype({"names": [f for f, _ in ContractDesc._fields_],
                   "formats": ["u8", "u8", "u8", "u8", "i4", "u8", "u4"],
                   "offsets": [getattr(ContractDesc, f).offset for f, _ in ContractDesc._fields_],
                   "itemsize": ctypes.sizeof(ContractDesc)})
    rec = np.zeros(max(1, n), dtype=dt)
    labels = {}

    def lab(x):
        k = tuple(x)
        a = labels.get(k)
        if a is None:
            a = labels[k] = _i32arr(k)
        return ctypes.addressof(a)

    if n:
        rec["a"][:n] = [_handle_value(it[0].handle) for it in items]
        rec["a_labels"][:n] = [lab(it[1]) for it in items]
        rec["b"][:n] = [_handle_value(it[2].handle) for it in items]
        rec["b_labels"][:n] = [lab(it[3]) for it in items]
        rec["c_order"][:n] = [len(it[4]) for it in items]
        rec["c_labels"][:n] = [lab(it[4]) for it in items]
        rec["flags"][:n] = [int(it[5]) if len(it) > 5 else 0 for it in items]
    return rec, labels


def lco_contract_batch(ctx: Context, items):
    """Batched products; `items` is a list of (a, a_labels, b, b_labels, c_labels[, flags]).
    Returns the list of result tensors (bit-identical to lco_contract on each item)."""
    L = load_library()
    n = len(items)
    rec, labels = _desc_array(items)
    outs = (ctypes.c_void_p * max(1, n))()
    _check(L.lco_contract_batch(ctx.handle, n, ctypes.cast(rec.ctypes.data, ctypes.POINTER(ContractDesc)), outs))
    del labels  # the label arrays live until the call has returned
    return [Tensor(ctx, h) for h in outs[:n]]  # plain integer handles


class _Borrowed(Tensor):
    """A tensor owned by something else (a batch plan): destroy() does nothing."""

    def destroy(self):
        self.handle = None


def _descs(items):
    rec, labels = _desc_array(items)
    return ctypes.cast(rec.ctypes.data, ctypes.POINTER(ContractDesc)), (rec, labels)


class BatchPlan:
    """lco_batch_plan_*: a batch planned once, re-executed (or replayed as a HIP graph) on demand.
    `items` as for lco_contract_batch.  outputs() are owned by the plan."""

    def __init__(self, ctx: Context, items):
        L = load_library()
        self.ctx = ctx
        descs, self._keep = _descs(items)
        h = ctypes.c_void_p()
        _check(L.lco_batch_plan_create(ctx.handle, len(items), descs, ctypes.byref(h)))
        self.handle = h
        self.count = len(items)

    def outputs(self):
        L = load_library()
        return [_Borrowed(self.ctx, ctypes.c_void_p(L.lco_batch_plan_output(self.handle, i)))
                for i in range(self.count)]

    def execute(self):
        _check(load_library().lco_batch_plan_execute(self.ctx.handle, self.handle))

    def graph_launch(self):
        _check(load_library().lco_batch_plan_graph_launch(self.ctx.handle, self.handle))

    def launches(self):
        """Per size bucket: bucket, instances, branch, 64-row chunks per work item, tuned time (ms)."""
        L = load_library()
        out = []
        i = 0
        while True:
            b, n, a, g = (ctypes.c_int() for _ in range(4))
            ms = ctypes.c_double()
            st = L.lco_batch_plan_launch_info(self.handle, i, ctypes.byref(b), ctypes.byref(n), ctypes.byref(a),
                                              ctypes.byref(g), ctypes.byref(ms))
            if st != 0:
                return out
            out.append({"bucket": b.value, "instances": n.value, "branch": ALGOS[a.value],
                        "chunks_per_item": g.value, "tuned_ms": ms.value})
            i += 1

    def destroy(self):
        if self.handle:
            _check(load_library().lco_batch_plan_destroy(self.handle))
            self.handle = None


class Server:
    """Continuous-batching request server (lco_server_*).  Result tensors have no Python
    context: read them with to_numpy() and release them with destroy()."""

    def __init__(self, device: int = 0, workers: int = 3, max_batch: int = 256, plain: bool = False,
                 solo_nnz: int = 1 << 22, hbm_budget: int = 64 << 30):
        L = load_library()
        cfg = ServerConfig(int(workers), int(max_batch), int(bool(plain)), int(solo_nnz), int(hbm_budget))
        h = ctypes.c_void_p()
        _check(L.lco_server_create(int(device), ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h
        self._buf = (ServerResult * 256)()

    def submit(self, a: Tensor, a_labels, b: Tensor, b_labels, c_labels, flags: int = 0) -> int:
        arrs = (_i32arr(a_labels), _i32arr(b_labels), _i32arr(c_labels))
        d = ContractDesc(a.handle, arrs[0], b.handle, arrs[1], len(c_labels), arrs[2], int(flags))
        t = ctypes.c_int64()
        _check(load_library().lco_server_submit(self.handle, ctypes.byref(d), ctypes.byref(t)))
        return t.value

    def poll(self):
        """Completed requests: list of dicts (ticket, status, out Tensor or None, latency_ms,
        queue_ms, batch_size)."""
        L = load_library()
        res = []
        while True:
            n = ctypes.c_int()
            _check(L.lco_server_poll(self.handle, self._buf, len(self._buf), ctypes.byref(n)))
            for i in range(n.value):
                r = self._buf[i]
                res.append({"ticket": r.ticket, "status": r.status,
                            "out": Tensor(None, ctypes.c_void_p(r.out)) if r.out else None,
                            "latency_ms": r.latency_ms, "queue_ms": r.queue_ms, "batch_size": r.batch_size})
            if n.value < len(self._buf):
                return res

    def drain(self):
        _check(load_library().lco_server_drain(self.handle))

    def destroy(self):
        if self.handle:
            _check(load_library().lco_server_destroy(self.handle))
            self.handle = None


def lco_batch_stats(ctx: Context):
    """(batched, per_call, persistent) instance counts of the last lco_contract_batch call."""
    b, p, q = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(load_library().lco_batch_stats(ctx.handle, ctypes.byref(b), ctypes.byref(p), ctypes.byref(q)))
    return b.value, p.value, q.value


def lco_plan_info(ctx: Context, a: Tensor, a_labels, b: Tensor, b_labels, c_labels, flags: int = 0) -> Plan:
    L = load_library()
    p = Plan()
    _check(L.lco_plan_info(ctx.handle, a.handle, _i32arr(a_labels), b.handle, _i32arr(b_labels), len(c_labels),
                           _i32arr(c_labels), int(flags), ctypes.byref(p)))
    return p


# ------------------------------------------------------------------ host-only planning
def lco_plan_contract(a_dims, a_labels, a_nnz, b_dims, b_labels, b_nnz, c_labels, flags: int = 0) -> Plan:
    L = load_library()
    p = Plan()
    _check(L.lco_plan_contract(len(a_dims), _u64arr(a_dims), _i32arr(a_labels), int(a_nnz), len(b_dims),
                               _u64arr(b_dims), _i32arr(b_labels), int(b_nnz), len(c_labels), _i32arr(c_labels),
                               int(flags), ctypes.byref(p)))
    return p


def lco_plan_permute(dims, perm, nnz: int) -> RpPlan:
    L = load_library()
    p = RpPlan()
    _check(L.lco_plan_permute(len(dims), _u64arr(dims), _i32arr(perm), int(nnz), ctypes.byref(p)))
    return p


def lco_classify(rows: int, cols: int, nnz: int) -> int:
    c = ctypes.c_int()
    _check(load_library().lco_classify(int(rows), int(cols), int(nnz), ctypes.byref(c)))
    return c.value


def lco_select(a_class: int, b_class: int):
    f, s = ctypes.c_int(), ctypes.c_int()
    _check(load_library().lco_select(int(a_class), int(b_class), ctypes.byref(f), ctypes.byref(s)))
    return f.value, s.value


def lco_fastdiv_host(d: int, nums):
    import numpy as np
    nums = np.ascontiguousarray(np.asarray(nums, dtype=np.uint64))
    q = np.zeros_like(nums)
    r = np.zeros_like(nums)
    p = ctypes.POINTER(ctypes.c_uint64)
    _check(load_library().lco_fastdiv_host(int(d), nums.shape[0], nums.ctypes.data_as(p), q.ctypes.data_as(p),
                                           r.ctypes.data_as(p)))
    return q, r


# ------------------------------------------------------------------ timing
def lco_timing_enable(ctx: Context, on: bool = True):
    _check(load_library().lco_timing_enable(ctx.handle, int(on)))


def lco_timing_only(ctx: Context, kernel=None):
    """Time only launches of `kernel` (None: every kernel)."""
    _check(load_library().lco_timing_only(ctx.handle, kernel.encode() if kernel else None))


def lco_timing_reset(ctx: Context):
    _check(load_library().lco_timing_reset(ctx.handle))


def lco_timing_query(ctx: Context, kernel: str):
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    _check(load_library().lco_timing_query(ctx.handle, kernel.encode(), ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


def lco_timing_kernels(ctx: Context):
    L = load_library()
    out = []
    i = 0
    while True:
        s = L.lco_timing_kernel_name(ctx.handle, i)
        if not s:
            return out
        out.append(s.decode())
        i += 1
