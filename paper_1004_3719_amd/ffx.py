"""ctypes binding of libffx.so: the C ABI of include/ffx.h with the same names.

Only argument marshalling happens here: device tensors are passed as raw
pointers with their leading dimension and the current HIP stream; every step
of a product runs in the library's kernels. There is no fallback: if the
library is missing or does not load, every call raises.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libffx.so")

FFX_OK, FFX_EINVAL, FFX_EBOUND, FFX_ENOMEM, FFX_EDEVICE, FFX_EUNSUPPORTED = range(6)
FFX_I32, FFX_I64 = 0, 1
ACC = {"auto": 0, "int64": 1, "fp64": 2, "fp32": 3, "fp64c": 4, "fp32c": 5}  # fp64c, fp32c: centered residues
SEL = {"heuristic": 0, "learned": 1, "fixed": 2}
FORMATS = ["STREAM", "SELL", "SELL_SORTED", "BAND_STREAM", "BAND_SELL", "BAND_SELL_SORTED"]
NUM_FORMATS = len(FORMATS)


class FfxError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


STATUS_NAMES = {0: "FFX_OK", 1: "FFX_EINVAL", 2: "FFX_EBOUND", 3: "FFX_ENOMEM", 4: "FFX_EDEVICE", 5: "FFX_EUNSUPPORTED"}


class BuildOpts(ctypes.Structure):
    _fields_ = [("size", ctypes.c_uint32), ("acc", ctypes.c_int32), ("selector", ctypes.c_int32),
                ("fixed_format", ctypes.c_int32), ("split_pm1", ctypes.c_int32), ("block_rows", ctypes.c_int32),
                ("build_transpose", ctypes.c_int32), ("tile_entries", ctypes.c_int32),
                ("compact_x", ctypes.c_int32), ("model_path", ctypes.c_char_p), ("reorder", ctypes.c_int32),
                ("col_sorted", ctypes.c_int32)]


class MatrixInfo(ctypes.Structure):
    _fields_ = [("nrows", ctypes.c_int64), ("ncols", ctypes.c_int64), ("m", ctypes.c_uint32), ("acc", ctypes.c_int32),
                ("nnz_input", ctypes.c_int64), ("nnz", ctypes.c_int64), ("n_plus", ctypes.c_int64),
                ("n_minus", ctypes.c_int64), ("n_band", ctypes.c_int64), ("nblocks", ctypes.c_int64),
                ("ntiles", ctypes.c_int64), ("max_row_terms", ctypes.c_int64), ("reduce_every", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("stream_bytes", ctypes.c_int64),
                ("has_transpose", ctypes.c_int32), ("value_bytes", ctypes.c_int32),
                ("format_blocks", ctypes.c_int64 * NUM_FORMATS), ("reordered", ctypes.c_int32),
                ("bandwidth_input", ctypes.c_int64), ("bandwidth_stored", ctypes.c_int64),
                ("sg_groups", ctypes.c_int64), ("sg_stream_bytes", ctypes.c_int64)]


class TrainOpts(ctypes.Structure):
    _fields_ = [("size", ctypes.c_uint32), ("epochs", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("lr", ctypes.c_float), ("seed", ctypes.c_uint64), ("n_val", ctypes.c_int64),
                ("n_margins", ctypes.c_int32), ("margins", ctypes.c_void_p)]


class TrainReport(ctypes.Structure):
    _fields_ = [("train_loss", ctypes.c_double), ("val_loss", ctypes.c_double), ("margin", ctypes.c_float),
                ("val_cost", ctypes.c_double), ("val_cost_stream", ctypes.c_double),
                ("val_cost_heuristic", ctypes.c_double), ("steps", ctypes.c_int32)]


class BatchParams(ctypes.Structure):
    _fields_ = [("wg_per_cu", ctypes.c_int32), ("order", ctypes.c_int32), ("max_chunk", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("xcd", ctypes.c_int32), ("compact_x", ctypes.c_int32)]


_lib = None

_SIGS = {
    "ffx_build_opts_default": (None, [ctypes.POINTER(BuildOpts)]),
    "ffx_matrix_create_csr": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_int, ctypes.c_uint32,
                                             ctypes.POINTER(BuildOpts), ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "ffx_matrix_create_coo": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_uint32,
                                             ctypes.POINTER(BuildOpts), ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "ffx_matrix_info_get": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(MatrixInfo)]),
    "ffx_matrix_block_formats": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64]),
    "ffx_matrix_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "ffx_spmv": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p,
                                ctypes.c_int, ctypes.c_void_p]),
    "ffx_spmv_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_uint32,
                                        ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    "ffx_spmv_t": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p,
                                  ctypes.c_int, ctypes.c_void_p]),
    "ffx_spmm": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_int64,
                                ctypes.c_uint32, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p]),
    "ffx_spmm_t": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_int64,
                                  ctypes.c_uint32, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p]),
    "ffx_power": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
                                 ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p]),
    "ffx_set_sequence_graph_batch": (ctypes.c_int, [ctypes.c_int32]),
    "ffx_sequence_gf2": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
                                        ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p]),
    "ffx_spmm_gf2": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                    ctypes.c_int64, ctypes.c_void_p]),
    "ffx_check_block": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64,
                                       ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "ffx_sequence": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                    ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                    ctypes.c_void_p]),
    "ffx_batch_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(BatchParams),
                                        ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "ffx_batch_spmm": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    "ffx_batch_tune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_int, ctypes.c_int32, ctypes.c_char_p, ctypes.c_void_p,
                                      ctypes.POINTER(BatchParams)]),
    "ffx_batch_get_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(BatchParams)]),
    "ffx_batch_set_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(BatchParams)]),
    "ffx_batch_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "ffx_selector_create": (ctypes.c_int, [ctypes.c_uint64, ctypes.POINTER(ctypes.c_void_p)]),
    "ffx_selector_set_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "ffx_selector_get_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "ffx_selector_predict": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                            ctypes.c_void_p]),
    "ffx_selector_gradient": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_int64, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                             ctypes.c_void_p]),
    "ffx_selector_train_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_int64, ctypes.c_float, ctypes.POINTER(ctypes.c_double),
                                               ctypes.c_void_p]),
    "ffx_selector_save": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p]),
    "ffx_selector_load": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_void_p)]),
    "ffx_selector_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "ffx_sigma_basis": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                       ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]),
    "ffx_sequence_rank": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p,
                                         ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p]),
    "ffx_reorder_rcm": (ctypes.c_int, [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "ffx_block_features": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_int, ctypes.c_uint32, ctypes.POINTER(BuildOpts),
                                          ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
    "ffx_matrix_block_times": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                              ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "ffx_selector_label": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_int, ctypes.c_uint32, ctypes.POINTER(BuildOpts),
                                          ctypes.c_int32, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int64,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.POINTER(ctypes.c_int64)]),
    "ffx_train_opts_default": (None, [ctypes.c_void_p]),
    "ffx_selector_train": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_int64, ctypes.c_void_p, ctypes.c_char_p,
                                          ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p, ctypes.c_void_p]),
    "ffx_gather_rate": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                       ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "ffx_set_ntt_threshold": (ctypes.c_int, [ctypes.c_int64]),
    "ffx_tune_tile_entries": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_int, ctypes.c_uint32,
                                             ctypes.POINTER(BuildOpts), ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_uint64, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                             ctypes.c_void_p]),
    "ffx_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "ffx_last_error": (ctypes.c_char_p, []),
    "ffx_version": (ctypes.c_char_p, []),
}


def lib():
    """The loaded library; raises if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libffx.so is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(st):
    if st != FFX_OK:
        raise FfxError(st, lib().ffx_last_error().decode())


def _stream(stream, current=True):
    """A HIP stream handle: the given one, else torch's current stream (or NULL, the null stream)."""
    if stream is None:
        if not current:
            return ctypes.c_void_p(None)
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _dt(t):
    import torch
    if t.dtype == torch.int32:
        return FFX_I32
    if t.dtype == torch.int64:
        return FFX_I64
    raise TypeError("vectors must be int32 or int64 tensors, got %s" % t.dtype)


def _block(t, rows, name):
    """(pointer, s, ld) of a device tensor holding rows x s residues, row-major with unit column stride."""
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if t.dim() == 1:
        if t.shape[0] != rows or (rows > 1 and t.stride(0) != 1):
            raise ValueError("%s: expected %d contiguous entries" % (name, rows))
        return t.data_ptr(), 1, 1
    if t.dim() != 2 or t.shape[0] != rows or (t.shape[1] > 1 and t.stride(1) != 1):
        raise ValueError("%s: expected a %d x s tensor with unit column stride" % (name, rows))
    return t.data_ptr(), t.shape[1], max(t.stride(0), t.shape[1])


PACKAGED_MODEL = os.path.join(os.path.dirname(os.path.abspath(__file__)), "models", "selector.bin")


def build_opts(acc="auto", selector="heuristic", fixed_format=None, split_pm1=True, block_rows=4096,
               build_transpose=False, tile_entries=0, compact_x=-1, model_path=None, reorder=False, col_sorted=-1):
    o = BuildOpts()
    lib().ffx_build_opts_default(ctypes.byref(o))
    o.acc = ACC[acc]
    if fixed_format is not None:
        selector = "fixed"
        o.fixed_format = FORMATS.index(fixed_format) if isinstance(fixed_format, str) else int(fixed_format)
    o.selector = SEL[selector]
    o.split_pm1 = int(bool(split_pm1))
    o.block_rows = int(block_rows)
    o.build_transpose = int(bool(build_transpose))
    o.tile_entries = int(tile_entries)
    o.compact_x = int(compact_x)
    if selector == "learned" and not model_path:
        model_path = PACKAGED_MODEL  # the network trained for this GPU, shipped with the package
    o.model_path = model_path.encode() if model_path else None
    o.reorder = int(bool(reorder))
    o.col_sorted = int(col_sorted)
    return o


class Matrix:
    """An encoded matrix over Z/mZ on the device (ffx_matrix)."""

    def __init__(self, handle):
        self._h = ctypes.c_void_p(handle)
        self._dims = None  # (nrows, ncols), read once: a handle's shape never changes

    @classmethod
    def from_csr(cls, nrows, ncols, rowptr, col, val, m, stream=None, **opts):
        rp = np.ascontiguousarray(rowptr, dtype=np.int64)
        rp = rp - rp[0]
        c = np.ascontiguousarray(col, dtype=np.int32)
        v = np.ascontiguousarray(val)
        vt = FFX_I32 if v.dtype == np.int32 else FFX_I64
        if vt == FFX_I64:
            v = np.ascontiguousarray(v, dtype=np.int64)
        o = build_opts(**opts)
        h = ctypes.c_void_p()
        _check(lib().ffx_matrix_create_csr(int(nrows), int(ncols), rp.ctypes.data, c.ctypes.data, v.ctypes.data, vt,
                                           int(m), ctypes.byref(o), _stream(stream, False), ctypes.byref(h)))
        return cls(h.value)

    @classmethod
    def from_coo(cls, nrows, ncols, row, col, val, m, stream=None, **opts):
        r = np.ascontiguousarray(row, dtype=np.int32)
        c = np.ascontiguousarray(col, dtype=np.int32)
        v = np.ascontiguousarray(val)
        vt = FFX_I32 if v.dtype == np.int32 else FFX_I64
        if vt == FFX_I64:
            v = np.ascontiguousarray(v, dtype=np.int64)
        o = build_opts(**opts)
        h = ctypes.c_void_p()
        _check(lib().ffx_matrix_create_coo(int(nrows), int(ncols), len(r), r.ctypes.data, c.ctypes.data,
                                           v.ctypes.data, vt, int(m), ctypes.byref(o), _stream(stream, False),
                                           ctypes.byref(h)))
        return cls(h.value)

    @classmethod
    def from_synth(cls, A, stream=None, **opts):
        """From a synth.Csr (raw values, any int64)."""
        return cls.from_csr(A.nrows, A.ncols, A.rowptr, A.col, A.val, A.m, stream=stream, **opts)

    def close(self):
        if self._h is not None and self._h.value:
            _check(lib().ffx_matrix_destroy(self._h))
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def info(self):
        I = MatrixInfo()
        _check(lib().ffx_matrix_info_get(self._h, ctypes.byref(I)))
        d = {k: getattr(I, k) for k, _ in MatrixInfo._fields_ if k != "format_blocks"}
        d["format_blocks"] = {FORMATS[f]: int(I.format_blocks[f]) for f in range(NUM_FORMATS)}
        return d

    def block_times(self, x, reps=4, y=None, stream=None):
        """Microseconds per product of each row block in its stored format (ffx_matrix_block_times)."""
        import torch
        inf = self.info()
        px, _, _ = _block(x, inf["ncols"], "x")
        if y is None:
            y = torch.empty(inf["nrows"], dtype=x.dtype, device=x.device)
        py, _, _ = _block(y, inf["nrows"], "y")
        out = np.zeros(max(1, inf["nblocks"]), np.float32)
        _check(lib().ffx_matrix_block_times(self._h, ctypes.c_void_p(px), ctypes.c_void_p(py), _dt(x), int(reps),
                                            out.ctypes.data, _stream(stream)))
        return out[:inf["nblocks"]]

    def block_formats(self, transpose=False):
        n = self.info()["nblocks"]
        out = np.zeros(max(1, n), np.int32)
        _check(lib().ffx_matrix_block_formats(self._h, int(transpose), out.ctypes.data, n))
        return out[:n]

    # ----- products -----
    def shape(self):
        """(nrows, ncols) of the matrix."""
        if self._dims is None:
            inf = self.info()
            self._dims = (inf["nrows"], inf["ncols"])
        return self._dims

    def _prod(self, fn, trans, X, alpha, beta, Y, stream):
        import torch
        nrows, ncols = self.shape()
        nin, nout = (nrows, ncols) if trans else (ncols, nrows)
        px, s, ldx = _block(X, nin, "x")
        if Y is None:
            Y = torch.empty((nout,) if X.dim() == 1 else (nout, s), dtype=X.dtype, device=X.device)
            beta = 0
        if Y.dtype != X.dtype:
            raise TypeError("x and y dtypes differ")
        py, sy, ldy = _block(Y, nout, "y")
        if sy != s:
            raise ValueError("x has %d columns, y has %d" % (s, sy))
        if X.dim() == 1 and fn in ("ffx_spmv", "ffx_spmv_t", "ffx_spmv_noalloc"):
            _check(getattr(lib(), fn)(self._h, int(alpha), ctypes.c_void_p(px), int(beta), ctypes.c_void_p(py),
                                      _dt(X), _stream(stream)))
        else:
            f = "ffx_spmm_t" if trans else "ffx_spmm"
            _check(getattr(lib(), f)(self._h, s, int(alpha), ctypes.c_void_p(px), ldx, int(beta), ctypes.c_void_p(py),
                                     ldy, _dt(X), _stream(stream)))
        return Y

    def spmv(self, x, alpha=1, beta=0, y=None, stream=None):
        return self._prod("ffx_spmv", False, x, alpha, beta, y, stream)

    def spmv_noalloc(self, x, alpha=1, beta=0, y=None, stream=None):
        """As spmv, through ffx_spmv_noalloc (the library allocates nothing; y must be given for that)."""
        if x.dim() != 1:
            raise ValueError("spmv_noalloc takes one vector")
        return self._prod("ffx_spmv_noalloc", False, x, alpha, beta, y, stream)

    def spmv_t(self, x, alpha=1, beta=0, y=None, stream=None):
        return self._prod("ffx_spmv_t", True, x, alpha, beta, y, stream)

    def spmm(self, X, alpha=1, beta=0, Y=None, stream=None):
        return self._prod("ffx_spmm", False, X, alpha, beta, Y, stream)

    def spmm_t(self, X, alpha=1, beta=0, Y=None, stream=None):
        return self._prod("ffx_spmm_t", True, X, alpha, beta, Y, stream)

    def spmm_gf2(self, X, Y=None, stream=None):
        """Y = A X over GF(2) for a matrix built with m = 2; X is an int32 tensor of ncols x w packed words
        (bit b of word c of row j = entry j of vector 32c + b)."""
        import torch
        inf = self.info()
        if X.dtype != torch.int32:
            raise TypeError("GF(2) blocks are int32 tensors of packed words")
        px, w, ldx = _block(X, inf["ncols"], "X")
        if Y is None:
            Y = torch.empty((inf["nrows"], w) if X.dim() == 2 else (inf["nrows"],), dtype=torch.int32, device=X.device)
        py, wy, ldy = _block(Y, inf["nrows"], "Y")
        if wy != w:
            raise ValueError("X and Y have different word counts")
        _check(lib().ffx_spmm_gf2(self._h, w, ctypes.c_void_p(px), ldx, ctypes.c_void_p(py), ldy, _stream(stream)))
        return Y

    def sequence_gf2(self, U, V, L, want_last=False, stream=None):
        """S_i = U^T A^i V over GF(2), i < L, for int32 tensors U, V of n x w packed words; returns S as an
        L x 32w x w int32 tensor (and A^L V)."""
        import torch
        n = self.shape()[0]
        for t in (U, V):
            if t.dtype != torch.int32:
                raise TypeError("GF(2) blocks are int32 tensors of packed words")
        pu, w, ldu = _block(U, n, "U")
        pv, wv, ldv = _block(V, n, "V")
        if wv != w:
            raise ValueError("U and V have different word counts")
        S = torch.empty((int(L), 32 * w, w), dtype=torch.int32, device=V.device)
        W = torch.empty((n, w), dtype=torch.int32, device=V.device) if want_last else None
        _check(lib().ffx_sequence_gf2(self._h, w, ctypes.c_void_p(pu), ldu, ctypes.c_void_p(pv), ldv, int(L),
                                      ctypes.c_void_p(S.data_ptr()), ctypes.c_void_p(W.data_ptr() if W is not None else 0),
                                      _stream(stream)))
        return (S, W) if want_last else S

    def power(self, k, V, W=None, stream=None):
        import torch
        n = self.shape()[0]
        pv, s, ldv = _block(V, n, "V")
        if W is None:
            W = torch.empty_like(V)
        pw, sw, ldw = _block(W, n, "W")
        _check(lib().ffx_power(self._h, int(k), s, ctypes.c_void_p(pv), ldv, ctypes.c_void_p(pw), ldw, _dt(V),
                               _stream(stream)))
        return W

    def sequence(self, U, V, L, want_last=False, stream=None):
        import torch
        n = self.shape()[0]
        pu, s, ldu = _block(U, n, "U")
        pv, sv, ldv = _block(V, n, "V")
        if sv != s or U.dtype != V.dtype:
            raise ValueError("U and V must have the same width and dtype")
        S = torch.empty((int(L), s, s), dtype=U.dtype, device=U.device)
        W = torch.empty((n, s), dtype=U.dtype, device=U.device) if want_last else None
        _check(lib().ffx_sequence(self._h, s, ctypes.c_void_p(pu), ldu, ctypes.c_void_p(pv), ldv, int(L),
                                  ctypes.c_void_p(S.data_ptr()), ctypes.c_void_p(W.data_ptr() if W is not None else 0),
                                  _dt(U), _stream(stream)))
        return (S, W) if want_last else S


def check_block(X, m, stream=None):
    """Checked mode: -1 when every entry of the device tensor X (n or n x s, int32/int64) is a residue
    in [0, m-1], else the smallest flat index k*ld + c of an entry outside it. Bad arguments raise."""
    n = X.shape[0]
    p, s, ld = _block(X, n, "X")
    bad = ctypes.c_int64(-1)
    st = lib().ffx_check_block(int(m), ctypes.c_void_p(p), n, s, ld, _dt(X), _stream(stream), ctypes.byref(bad))
    if st == 1 and bad.value >= 0:  # FFX_EINVAL naming an entry: the block is not canonical
        return bad.value
    _check(st)
    return -1


def set_sequence_graph_batch(batch):
    """Iterations per hipGraph replay in Matrix.sequence (0: one direct launch per iteration)."""
    _check(lib().ffx_set_sequence_graph_batch(int(batch)))


def version():
    return lib().ffx_version().decode()


class Batch:
    """Many matrices (same modulus) with their own numbers of right-hand sides, one launch (ffx_batch)."""

    def __init__(self, mats, s, wg_per_cu=0, order=0, max_chunk=8, use_graph=True, xcd=1, compact_x=-1):
        self.mats = list(mats)  # the handles must outlive the batch
        self.s = [int(v) for v in s]
        n = len(self.mats)
        hs = (ctypes.c_void_p * n)(*[m.handle.value for m in self.mats])
        ss = (ctypes.c_int32 * n)(*self.s)
        p = BatchParams(int(wg_per_cu), int(order), int(max_chunk), int(bool(use_graph)), int(xcd), int(compact_x))
        h = ctypes.c_void_p()
        _check(lib().ffx_batch_create(n, hs, ss, ctypes.byref(p), None, ctypes.byref(h)))
        self._h = h

    def _operands(self, Xs, Ys):
        n = len(self.mats)
        if len(Xs) != n or len(Ys) != n:
            raise ValueError("one X and one Y per matrix")
        xp, yp, lx, ly = [], [], [], []
        for k, (X, Y, M) in enumerate(zip(Xs, Ys, self.mats)):
            inf = M.info()
            px, sx, ldx = _block(X, inf["ncols"], "X[%d]" % k)
            py, sy, ldy = _block(Y, inf["nrows"], "Y[%d]" % k)
            if sx != self.s[k] or sy != self.s[k]:
                raise ValueError("matrix %d: expected %d right-hand sides" % (k, self.s[k]))
            xp.append(px)
            yp.append(py)
            lx.append(ldx)
            ly.append(ldy)
        return ((ctypes.c_void_p * n)(*xp), (ctypes.c_int64 * n)(*lx), (ctypes.c_void_p * n)(*yp),
                (ctypes.c_int64 * n)(*ly), _dt(Xs[0]))

    def spmm(self, Xs, Ys, stream=None):
        X, lx, Y, ly, dt = self._operands(Xs, Ys)
        _check(lib().ffx_batch_spmm(self._h, X, lx, Y, ly, dt, _stream(stream)))
        return Ys

    def tune(self, Xs, Ys, reps=3, cache_path=None, stream=None):
        X, lx, Y, ly, dt = self._operands(Xs, Ys)
        p = BatchParams()
        _check(lib().ffx_batch_tune(self._h, X, lx, Y, ly, dt, int(reps),
                                    cache_path.encode() if cache_path else None, _stream(stream), ctypes.byref(p)))
        return {k: getattr(p, k) for k, _ in BatchParams._fields_}

    def params(self):
        p = BatchParams()
        _check(lib().ffx_batch_get_params(self._h, ctypes.byref(p)))
        return {k: getattr(p, k) for k, _ in BatchParams._fields_}

    def set_params(self, wg_per_cu=0, order=0, max_chunk=8, use_graph=True, xcd=1, compact_x=-1):
        p = BatchParams(int(wg_per_cu), int(order), int(max_chunk), int(bool(use_graph)), int(xcd), int(compact_x))
        _check(lib().ffx_batch_set_params(self._h, ctypes.byref(p)))

    def close(self):
        if self._h is not None and self._h.value:
            _check(lib().ffx_batch_destroy(self._h))
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


NFEAT, NPARAM = 32, 6662


def block_features(nrows, ncols, rowptr, col, val, m, **opts):
    """The builder's 32 features of every row block (ffx_block_features), as an (nblocks, 32) array."""
    rp = np.ascontiguousarray(rowptr, dtype=np.int64)
    rp = rp - rp[0]
    c = np.ascontiguousarray(col, dtype=np.int32)
    v = np.ascontiguousarray(val, dtype=np.int64)
    o = build_opts(**opts)
    nb = ctypes.c_int64()
    _check(lib().ffx_block_features(int(nrows), int(ncols), rp.ctypes.data, c.ctypes.data, v.ctypes.data, FFX_I64,
                                    int(m), ctypes.byref(o), None, 0, ctypes.byref(nb)))
    out = np.zeros((max(1, nb.value), NFEAT), np.float32)
    _check(lib().ffx_block_features(int(nrows), int(ncols), rp.ctypes.data, c.ctypes.data, v.ctypes.data, FFX_I64,
                                    int(m), ctypes.byref(o), out.ctypes.data, nb.value, None))
    return out[:nb.value]


def selector_label(nrows, ncols, rowptr, col, val, m, reps=6, seed=0, stream=None, **opts):
    """Features, log2 microseconds per block of each format and the heuristic's formats of one training
    window, measured by the library (ffx_selector_label): arrays (nb x 32), (nb x 6), (nb)."""
    rp = np.ascontiguousarray(rowptr, dtype=np.int64)
    rp = rp - rp[0]
    c = np.ascontiguousarray(col, dtype=np.int32)
    v = np.ascontiguousarray(val, dtype=np.int64)
    o = build_opts(**opts)
    nb = ctypes.c_int64()
    _check(lib().ffx_block_features(int(nrows), int(ncols), rp.ctypes.data, c.ctypes.data, v.ctypes.data, FFX_I64,
                                    int(m), ctypes.byref(o), None, 0, ctypes.byref(nb)))
    n = nb.value
    F = np.zeros((max(1, n), NFEAT), np.float32)
    T = np.zeros((max(1, n), NUM_FORMATS), np.float32)
    H = np.zeros(max(1, n), np.int32)
    _check(lib().ffx_selector_label(int(nrows), int(ncols), rp.ctypes.data, c.ctypes.data, v.ctypes.data, FFX_I64,
                                    int(m), ctypes.byref(o), int(reps), int(seed) & (2**64 - 1),
                                    _stream(stream), n, F.ctypes.data, T.ctypes.data, H.ctypes.data, None))
    return F[:n], T[:n], H[:n]


def selector_train(X, T, mask=None, heur=None, epochs=60, batch=512, lr=2e-3, seed=0, n_val=-1, margins=None,
                   out_model=None, stream=None):
    """Trains a selector in the library (ffx_selector_train) on labelled blocks: (Selector, report dict).
    The first n_val samples (default n/10) are held out for the validation loss and the decision margin."""
    X = np.ascontiguousarray(X, np.float32)
    T = np.ascontiguousarray(T, np.float32)
    M = None if mask is None else np.ascontiguousarray(mask, np.float32)
    H = None if heur is None else np.ascontiguousarray(heur, np.int32)
    o = TrainOpts()
    lib().ffx_train_opts_default(ctypes.byref(o))
    o.epochs, o.batch, o.lr, o.seed, o.n_val = int(epochs), int(batch), float(lr), int(seed) & (2**64 - 1), int(n_val)
    mg = None
    if margins is not None:
        mg = np.ascontiguousarray(margins, np.float32)
        o.n_margins, o.margins = len(mg), mg.ctypes.data
    rep = TrainReport()
    h = ctypes.c_void_p()
    _check(lib().ffx_selector_train(X.ctypes.data, T.ctypes.data, None if M is None else M.ctypes.data,
                                    None if H is None else H.ctypes.data, X.shape[0], ctypes.byref(o),
                                    out_model.encode() if out_model else None, ctypes.byref(h), ctypes.byref(rep),
                                    _stream(stream)))
    return Selector(handle=h), {k: getattr(rep, k) for k, _ in TrainReport._fields_}


def gather_rate(table_bytes, row_bytes, count, window=0, reps=5, stream=None):
    """Random gathers per second of row_bytes-byte rows from a table_bytes table (ffx_gather_rate)."""
    r = ctypes.c_double()
    _check(lib().ffx_gather_rate(int(table_bytes), int(row_bytes), int(count), int(window), int(reps),
                                 _stream(stream), ctypes.byref(r)))
    return r.value


def set_ntt_threshold(min_length):
    """Smallest operand length at which order-basis products use the NTT (ffx_set_ntt_threshold)."""
    _check(lib().ffx_set_ntt_threshold(int(min_length)))


def tune_tile_entries(nrows, ncols, rowptr, col, val, m, s=1, reps=5, seed=0, stream=None, **opts):
    """(best tile_entries, {candidate: median microseconds}) of the s-vector product (ffx_tune_tile_entries)."""
    rp = np.ascontiguousarray(rowptr, dtype=np.int64)
    rp = rp - rp[0]
    c = np.ascontiguousarray(col, dtype=np.int32)
    v = np.ascontiguousarray(val, dtype=np.int64)
    o = build_opts(**opts)
    best = ctypes.c_int32()
    us = np.zeros(4, np.float32)
    _check(lib().ffx_tune_tile_entries(int(nrows), int(ncols), rp.ctypes.data, c.ctypes.data, v.ctypes.data, FFX_I64,
                                       int(m), ctypes.byref(o), int(s), int(reps), int(seed) & (2**64 - 1),
                                       _stream(stream), ctypes.byref(best), us.ctypes.data))
    return best.value, {k: float(t) for k, t in zip((512, 1024, 2048, 4096), us)}


def sigma_basis(G, p, shift, stream=None):
    """Order basis of the power series G (device int32 tensor m x n x sigma, residues mod the prime
    p) to order sigma with the given shifted degrees (ffx_sigma_basis): (M, d) with M a device int32
    tensor m x m x (sigma + 1) and d the final shifted degrees."""
    import torch
    if G.dtype != torch.int32 or G.dim() != 3:
        raise TypeError("sigma_basis takes an m x n x sigma int32 tensor of residues (got %s, %d dims)"
                        % (G.dtype, G.dim()))
    m, n, sigma = (int(v) for v in G.shape)
    G = G.contiguous()
    M = torch.empty((m, m, sigma + 1), dtype=torch.int32, device=G.device)
    sh = np.ascontiguousarray(shift, dtype=np.int32)
    d = np.zeros(m, np.int32)
    _check(lib().ffx_sigma_basis(int(p), m, n, sigma, ctypes.c_void_p(G.data_ptr()), sigma, sh.ctypes.data,
                                 ctypes.c_void_p(M.data_ptr()), sigma + 1, d.ctypes.data, _stream(stream)))
    return M, [int(v) for v in d]


def sequence_rank(S, p, stream=None):
    """Block Wiedemann steps 2-3 on a sequence S (device tensor L x s x s, int32 or int64, as
    Matrix.sequence returns it; ffx_sequence_rank): (rank, deg det F, codeg det F, row degrees of F)."""
    L, s = int(S.shape[0]), int(S.shape[1])
    S = S.contiguous()
    deg = np.zeros(s, np.int32)
    r, D, e = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib().ffx_sequence_rank(int(p), s, L, ctypes.c_void_p(S.data_ptr()), _dt(S), deg.ctypes.data,
                                   ctypes.byref(r), ctypes.byref(D), ctypes.byref(e), _stream(stream)))
    return r.value, D.value, e.value, [int(v) for v in deg]


def reorder_rcm(n, rowptr, col):
    """The reverse Cuthill-McKee order of a square pattern (ffx_reorder_rcm, host only): perm[new] = old."""
    rp = np.ascontiguousarray(rowptr, dtype=np.int64)
    rp = rp - rp[0]
    c = np.ascontiguousarray(col, dtype=np.int32)
    perm = np.empty(max(int(n), 1), np.int32)
    _check(lib().ffx_reorder_rcm(int(n), rp.ctypes.data, c.ctypes.data, perm.ctypes.data))
    return perm[:int(n)]


class Selector:
    """The format-selection network on the device (ffx_selector)."""

    def __init__(self, seed=0, handle=None):
        if handle is None:
            h = ctypes.c_void_p()
            _check(lib().ffx_selector_create(int(seed) & (2**64 - 1), ctypes.byref(h)))
            handle = h
        self._h = handle

    @classmethod
    def load(cls, path):
        h = ctypes.c_void_p()
        _check(lib().ffx_selector_load(path.encode(), ctypes.byref(h)))
        return cls(handle=h)

    def save(self, path):
        _check(lib().ffx_selector_save(self._h, path.encode()))

    def get_params(self):
        th = np.zeros(NPARAM, np.float32)
        mu = np.zeros(NFEAT, np.float32)
        sc = np.zeros(NFEAT, np.float32)
        _check(lib().ffx_selector_get_params(self._h, th.ctypes.data, mu.ctypes.data, sc.ctypes.data))
        return th, mu, sc

    def set_params(self, theta=None, mean=None, scale=None):
        arrs = [None if a is None else np.ascontiguousarray(a, np.float32) for a in (theta, mean, scale)]
        _check(lib().ffx_selector_set_params(self._h, *[None if a is None else a.ctypes.data for a in arrs]))

    def predict(self, X, stream=None):
        import torch
        out = torch.empty((X.shape[0], 6), dtype=torch.float32, device=X.device)
        _check(lib().ffx_selector_predict(self._h, ctypes.c_void_p(X.data_ptr()), X.shape[0],
                                          ctypes.c_void_p(out.data_ptr()), _stream(stream)))
        return out

    def gradient(self, X, T, M, stream=None):
        import torch
        g = torch.empty(NPARAM, dtype=torch.float32, device=X.device)
        loss = ctypes.c_double()
        _check(lib().ffx_selector_gradient(self._h, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(T.data_ptr()),
                                           ctypes.c_void_p(M.data_ptr()), X.shape[0], ctypes.c_void_p(g.data_ptr()),
                                           ctypes.byref(loss), _stream(stream)))
        return loss.value, g

    def train_step(self, X, T, M, lr=1e-3, want_loss=False, stream=None):
        loss = ctypes.c_double()
        _check(lib().ffx_selector_train_step(self._h, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(T.data_ptr()),
                                             ctypes.c_void_p(M.data_ptr()), X.shape[0], float(lr),
                                             ctypes.byref(loss) if want_loss else None, _stream(stream)))
        return loss.value if want_loss else None

    def close(self):
        if self._h is not None and self._h.value:
            _check(lib().ffx_selector_destroy(self._h))
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
