"""Python binding of the gfx950 two-phase SpGEMM library (libspgemm_mi355x.so).

Argument marshalling only: every step of the product runs in the HIP kernels
behind the C ABI declared in include/spgemm.h.  PyTorch supplies device memory
(tensors) and the stream.  If the compiled library is missing, the first call
into it raises ImportError: there is no CPU fallback.

    h = Handle()                                   # spg_create
    rp, nnz = spgemm_symbolic(h, A, B)             # C.row_ptr (device), nnz(C)
    C = spgemm_numeric(h, A, B, rp, nnz)           # DeviceCsr with sorted columns
    spgemm_numeric(h, A2, B2, rp, nnz, out=C)      # reuse: new values, same structure
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch  # imported first so the library binds to torch's HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspgemm_mi355x.so")

_lib = None


def lib():
    """The loaded C library; raises if it was not built (no CPU fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1801_03065_amd.build` "
                              "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _sigs.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


# ----------------------------------------------------------------- C types
SPG_OK, SPG_ERR_INVALID_ARG, SPG_ERR_DIM_MISMATCH, SPG_ERR_INDEX_OVERFLOW = 0, 1, 2, 3
SPG_ERR_OUT_OF_MEMORY, SPG_ERR_NOT_READY, SPG_ERR_STRUCTURE_MISMATCH = 4, 5, 6
SPG_ERR_HIP, SPG_ERR_UNSUPPORTED, SPG_ERR_INTERNAL = 7, 8, 9
SPG_F64, SPG_F32 = 0, 1
SPG_I32, SPG_I64 = 0, 1
ACC_AUTO, ACC_DENSE, ACC_HASH, ACC_HASH_L2, ACC_LL = 0, 1, 2, 3, 4
FP32_PLAIN, FP32_COMPENSATED, FP32_WIDE = 0, 1, 2
KIND_NAMES = ("empty", "dense_wave", "hash_wave", "dense_wg", "hash_two_level", "word_hash_wave", "short_rows",
              "planned_wave")


class spg_csr(ctypes.Structure):
    _fields_ = [("nrows", ctypes.c_int64), ("ncols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("rp_type", ctypes.c_int), ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p),
                ("values", ctypes.c_void_p), ("dtype", ctypes.c_int)]


class spg_csr_out(ctypes.Structure):
    _fields_ = spg_csr._fields_


class spg_options(ctypes.Structure):
    _fields_ = [("compression", ctypes.c_int32), ("cf_threshold", ctypes.c_double),
                ("accumulator", ctypes.c_int32), ("fp32_mode", ctypes.c_int32),
                ("fp64_heavy_row_flops", ctypes.c_int64), ("l1_hash_slots", ctypes.c_int32),
                ("autotune", ctypes.c_int32), ("fp32_terms_max", ctypes.c_int32),
                ("verify_structure", ctypes.c_int32), ("sorted_output", ctypes.c_int32)]


class spg_stats(ctypes.Structure):
    _fields_ = [("flops", ctypes.c_int64), ("flops_compressed", ctypes.c_int64),
                ("max_row_flops", ctypes.c_int64), ("max_row_flops_compressed", ctypes.c_int64),
                ("nnz_c", ctypes.c_int64), ("max_row_nnz", ctypes.c_int64),
                ("nnz_b_compressed", ctypes.c_int64), ("compressed", ctypes.c_int32),
                ("n_kinds", ctypes.c_int32), ("rows_symbolic", ctypes.c_int64 * 8),
                ("rows_numeric", ctypes.c_int64 * 8), ("l2_spill_rows", ctypes.c_int32),
                ("tuned_policy", ctypes.c_int32), ("tuned_lanes", ctypes.c_int32),
                ("fp64_rows", ctypes.c_int32), ("reserved", ctypes.c_int32 * 4)]


_P = ctypes.c_void_p
_S = ctypes.c_int
_sigs = {
    "spg_default_options": (None, [ctypes.POINTER(spg_options)]),
    "spg_create": (_S, [ctypes.POINTER(_P), _P, ctypes.POINTER(spg_options)]),
    "spg_destroy": (_S, [_P]),
    "spg_set_stream": (_S, [_P, _P]),
    "spg_set_options": (_S, [_P, ctypes.POINTER(spg_options)]),
    "spgemm_symbolic": (_S, [_P, ctypes.POINTER(spg_csr), ctypes.POINTER(spg_csr), _P, _S,
                             ctypes.POINTER(ctypes.c_int64)]),
    "spgemm_numeric": (_S, [_P, ctypes.POINTER(spg_csr), ctypes.POINTER(spg_csr), ctypes.POINTER(spg_csr_out)]),
    "spgemm_numeric_values": (_S, [_P, ctypes.POINTER(spg_csr), ctypes.POINTER(spg_csr), ctypes.POINTER(spg_csr_out)]),
    "spgemm_batch_numeric_values": (_S, [_P, ctypes.c_int32, ctypes.POINTER(spg_csr), ctypes.POINTER(spg_csr),
                                         ctypes.POINTER(spg_csr_out)]),
    "spgemm_numeric_noalloc": (_S, [_P, ctypes.POINTER(spg_csr), ctypes.POINTER(spg_csr),
                                    ctypes.POINTER(spg_csr_out)]),
    "spgemm_masked": (_S, [_P, ctypes.POINTER(spg_csr), ctypes.POINTER(spg_csr), ctypes.POINTER(spg_csr), _P,
                           ctypes.c_int]),
    "spg_batch_choices": (_S, [_P, ctypes.c_int32, _P, _P]),
    "spg_check_errors": (_S, [_P]),
    "spgemm_numeric_rows": (_S, [_P, ctypes.POINTER(spg_csr), ctypes.POINTER(spg_csr), ctypes.c_int64,
                                 ctypes.c_int64, _P, _P]),
    "spgemm_batch_symbolic": (_S, [_P, ctypes.c_int32, ctypes.POINTER(spg_csr), ctypes.POINTER(spg_csr),
                                   ctypes.POINTER(_P), _S, ctypes.POINTER(ctypes.c_int64)]),
    "spgemm_batch_numeric": (_S, [_P, ctypes.c_int32, ctypes.POINTER(spg_csr), ctypes.POINTER(spg_csr),
                                  ctypes.POINTER(spg_csr_out)]),
    "spgemm_backward": (_S, [_P, ctypes.POINTER(spg_csr), ctypes.POINTER(spg_csr), ctypes.POINTER(spg_csr), _P, _P]),
    "spg_get_stats": (_S, [_P, ctypes.POINTER(spg_stats)]),
    "spg_status_string": (ctypes.c_char_p, [_S]),
    "spg_last_error": (ctypes.c_char_p, [_P]),
    "spg_version": (ctypes.c_char_p, []),
}


class SpgemmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{lib().spg_status_string(status).decode()} ({status}): {msg}")
        self.status = status


def version() -> str:
    return lib().spg_version().decode()


# ----------------------------------------------------------------- operands
@dataclass
class DeviceCsr:
    """CSR on the GPU: row_ptr int32/int64, col_idx int32, values float64/float32."""

    nrows: int
    ncols: int
    row_ptr: torch.Tensor
    col_idx: torch.Tensor
    values: torch.Tensor | None

    @property
    def nnz(self) -> int:
        return int(self.col_idx.numel())

    @staticmethod
    def from_arrays(nrows, ncols, row_ptr, col_idx, values, device="cuda", rp_dtype=torch.int32,
                    dtype=torch.float64) -> "DeviceCsr":
        rp = torch.as_tensor(row_ptr).to(device=device, dtype=rp_dtype)
        ci = torch.as_tensor(col_idx).to(device=device, dtype=torch.int32)
        va = None if values is None else torch.as_tensor(values).to(device=device, dtype=dtype)
        return DeviceCsr(int(nrows), int(ncols), rp.contiguous(), ci.contiguous(),
                         None if va is None else va.contiguous())

    def with_values(self, values: torch.Tensor) -> "DeviceCsr":
        return DeviceCsr(self.nrows, self.ncols, self.row_ptr, self.col_idx, values.contiguous())


def _itype(t: torch.Tensor) -> int:
    if t.dtype == torch.int32:
        return SPG_I32
    if t.dtype == torch.int64:
        return SPG_I64
    raise TypeError(f"row_ptr must be int32 or int64, got {t.dtype}")


def _dtype(t: torch.Tensor | None) -> int:
    if t is None:
        return SPG_F64
    if t.dtype == torch.float64:
        return SPG_F64
    if t.dtype == torch.float32:
        return SPG_F32
    raise TypeError(f"values must be float64 or float32, got {t.dtype}")


def _check_dev(t: torch.Tensor | None, what: str):
    if t is not None and (not t.is_cuda or not t.is_contiguous()):
        raise ValueError(f"{what} must be a contiguous GPU tensor")


def _csr(M: DeviceCsr) -> spg_csr:
    _check_dev(M.row_ptr, "row_ptr")
    _check_dev(M.col_idx, "col_idx")
    _check_dev(M.values, "values")
    if M.col_idx.dtype != torch.int32:
        raise TypeError("col_idx must be int32")
    return spg_csr(M.nrows, M.ncols, M.nnz, _itype(M.row_ptr), M.row_ptr.data_ptr(),
                   M.col_idx.data_ptr() if M.nnz else None,
                   M.values.data_ptr() if (M.values is not None and M.nnz) else None, _dtype(M.values))


def options(**kw) -> spg_options:
    o = spg_options()
    lib().spg_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


# ----------------------------------------------------------------- handle
class Handle:
    """spg_create / spg_destroy; holds the symbolic plan for reuse."""

    def __init__(self, stream: torch.cuda.Stream | None = None, **opts):
        torch.cuda.init()
        s = (stream or torch.cuda.current_stream()).cuda_stream
        self._h = _P()
        o = options(**opts)
        rc = lib().spg_create(ctypes.byref(self._h), _P(s), ctypes.byref(o))
        if rc != SPG_OK:
            raise SpgemmError(rc, "spg_create")

    def _raise(self, rc: int):
        raise SpgemmError(rc, lib().spg_last_error(self._h).decode())

    @property
    def ptr(self):
        return self._h

    def set_options(self, **opts):
        o = options(**opts)
        rc = lib().spg_set_options(self._h, ctypes.byref(o))
        if rc != SPG_OK:
            self._raise(rc)

    def set_stream(self, stream: torch.cuda.Stream):
        rc = lib().spg_set_stream(self._h, _P(stream.cuda_stream))
        if rc != SPG_OK:
            self._raise(rc)

    def stats(self) -> dict:
        st = spg_stats()
        rc = lib().spg_get_stats(self._h, ctypes.byref(st))
        if rc != SPG_OK:
            self._raise(rc)
        d = {k: getattr(st, k) for k, _ in spg_stats._fields_ if k not in ("reserved",)}
        d["rows_symbolic"] = dict(zip(KIND_NAMES, list(st.rows_symbolic)[:st.n_kinds]))
        d["rows_numeric"] = dict(zip(KIND_NAMES, list(st.rows_numeric)[:st.n_kinds]))
        return d

    def batch_choices(self, count: int):
        """Per product of the batch plan: (accumulator policy, lanes per B row)."""
        import numpy as np

        pol = np.zeros(count, dtype=np.int32)
        lanes = np.zeros(count, dtype=np.int32)
        rc = lib().spg_batch_choices(self._h, count, pol.ctypes.data_as(_P), lanes.ctypes.data_as(_P))
        if rc != SPG_OK:
            self._raise(rc)
        return pol, lanes

    def check_errors(self):
        rc = lib().spg_check_errors(self._h)
        if rc != SPG_OK:
            self._raise(rc)

    def close(self):
        if self._h:
            lib().spg_destroy(self._h)
            self._h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def spgemm_symbolic(h: Handle, A: DeviceCsr, B: DeviceCsr, rp_dtype=torch.int32):
    """spgemm_symbolic: returns (C.row_ptr device tensor of rp_dtype, nnz(C))."""
    rp = torch.empty(A.nrows + 1, dtype=rp_dtype, device=A.row_ptr.device)
    nnz = ctypes.c_int64(0)
    a, b = _csr(A), _csr(B)
    rc = lib().spgemm_symbolic(h.ptr, ctypes.byref(a), ctypes.byref(b), _P(rp.data_ptr()), _itype(rp),
                              ctypes.byref(nnz))
    if rc != SPG_OK:
        h._raise(rc)
    return rp, int(nnz.value)


def spgemm_numeric(h: Handle, A: DeviceCsr, B: DeviceCsr, C_row_ptr: torch.Tensor, nnz: int,
                   out: DeviceCsr | None = None) -> DeviceCsr:
    """spgemm_numeric: writes (or allocates) C's columns and values; never blocks the host."""
    if A.values is None or B.values is None:
        raise ValueError("numeric phase needs values")
    if out is None:
        ci = torch.empty(nnz, dtype=torch.int32, device=A.values.device)
        va = torch.empty(nnz, dtype=A.values.dtype, device=A.values.device)
        out = DeviceCsr(A.nrows, B.ncols, C_row_ptr, ci, va)
    c = spg_csr_out(out.nrows, out.ncols, out.nnz, _itype(out.row_ptr), out.row_ptr.data_ptr(),
                    out.col_idx.data_ptr() if out.nnz else None,
                    out.values.data_ptr() if out.nnz else None, _dtype(out.values))
    a, b = _csr(A), _csr(B)
    rc = lib().spgemm_numeric(h.ptr, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
    if rc != SPG_OK:
        h._raise(rc)
    return out


def spgemm_numeric_values(h: Handle, A: DeviceCsr, B: DeviceCsr, out: DeviceCsr) -> DeviceCsr:
    """spgemm_numeric_values: new values on a known structure; out.col_idx must hold the
    columns an earlier spgemm_numeric on this plan wrote, only out.values is written."""
    if A.values is None or B.values is None:
        raise ValueError("numeric phase needs values")
    c = spg_csr_out(out.nrows, out.ncols, out.nnz, _itype(out.row_ptr), out.row_ptr.data_ptr(),
                    out.col_idx.data_ptr() if out.nnz else None,
                    out.values.data_ptr() if out.nnz else None, _dtype(out.values))
    a, b = _csr(A), _csr(B)
    rc = lib().spgemm_numeric_values(h.ptr, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
    if rc != SPG_OK:
        h._raise(rc)
    return out


def spgemm_numeric_noalloc(h: Handle, A: DeviceCsr, B: DeviceCsr, out: DeviceCsr) -> DeviceCsr:
    """spgemm_numeric_noalloc: the numeric phase into caller-allocated C, with no
    device allocation inside the call (scratch from the library's static array)."""
    if A.values is None or B.values is None:
        raise ValueError("numeric phase needs values")
    c = spg_csr_out(out.nrows, out.ncols, out.nnz, _itype(out.row_ptr), out.row_ptr.data_ptr(),
                    out.col_idx.data_ptr() if out.nnz else None,
                    out.values.data_ptr() if out.nnz else None, _dtype(out.values))
    a, b = _csr(A), _csr(B)
    rc = lib().spgemm_numeric_noalloc(h.ptr, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
    if rc != SPG_OK:
        h._raise(rc)
    return out


def spgemm_masked(h: Handle, A: DeviceCsr, B: DeviceCsr, M: DeviceCsr, structural: bool = False,
                  dtype: torch.dtype | None = None) -> torch.Tensor:
    """spgemm_masked: (A*B) on M's stored entries (M's entry order), or with
    structural=True the number of paths i -> k -> j per entry.  Returns a tensor of
    nnz(M) values (A's dtype; in structural mode A's values may be None, dtype names
    the output type, float64 by default)."""
    out_dtype = dtype or (A.values.dtype if A.values is not None else torch.float64)
    out = torch.empty(M.nnz, dtype=out_dtype, device=M.col_idx.device)
    a, b, mm = _csr(A), _csr(B), _csr(M)
    a.dtype = _dtype(out)
    rc = lib().spgemm_masked(h.ptr, ctypes.byref(a), ctypes.byref(b), ctypes.byref(mm),
                             _P(out.data_ptr()) if M.nnz else None, 1 if structural else 0)
    if rc != SPG_OK:
        h._raise(rc)
    return out


def spgemm(A: DeviceCsr, B: DeviceCsr, handle: Handle | None = None, rp_dtype=torch.int32) -> DeviceCsr:
    """Both phases; the product with sorted columns."""
    h = handle or Handle()
    rp, nnz = spgemm_symbolic(h, A, B, rp_dtype)
    return spgemm_numeric(h, A, B, rp, nnz)


def spgemm_backward(h: Handle, A: DeviceCsr, B: DeviceCsr, G: DeviceCsr, need_dA: bool = True,
                    need_dB: bool = True):
    """spgemm_backward: (dA on pattern(A), dB on pattern(B)) for dL/dC = G (C's structure)."""
    dA = torch.empty_like(A.values) if need_dA else None
    dB = torch.empty_like(B.values) if need_dB else None
    a, b, g = _csr(A), _csr(B), _csr(G)
    rc = lib().spgemm_backward(h.ptr, ctypes.byref(a), ctypes.byref(b), ctypes.byref(g),
                               _P(dA.data_ptr()) if (dA is not None and A.nnz) else None,
                               _P(dB.data_ptr()) if (dB is not None and B.nnz) else None)
    if rc != SPG_OK:
        h._raise(rc)
    return dA, dB


class _SpGEMMFunction(torch.autograd.Function):
    """C.values = numeric(A.values, B.values) on a fixed symbolic plan."""

    @staticmethod
    def forward(ctx, a_values, b_values, prod):
        A = prod.A.with_values(a_values)
        B = prod.B.with_values(b_values)
        C = spgemm_numeric(prod.handle, A, B, prod.row_ptr, prod.nnz)
        if prod.check:
            prod.handle.check_errors()
        ctx.prod = prod
        ctx.save_for_backward(a_values, b_values, C.col_idx)
        return C.values

    @staticmethod
    def backward(ctx, grad_c):
        a_values, b_values, c_col = ctx.saved_tensors
        prod = ctx.prod
        A = prod.A.with_values(a_values)
        B = prod.B.with_values(b_values)
        G = DeviceCsr(A.nrows, B.ncols, prod.row_ptr, c_col, grad_c.contiguous())
        dA, dB = spgemm_backward(prod.handle, A, B, G, ctx.needs_input_grad[0], ctx.needs_input_grad[1])
        if prod.check:
            prod.handle.check_errors()
        return dA, dB, None


class SparseProduct:
    """A differentiable C = A * B on a fixed structure.

    The symbolic phase runs once at construction; calling the object runs the
    numeric phase on new values (the reuse case) and returns C's values as an
    autograd-tracked tensor; C's row_ptr / col_idx are in .row_ptr / .col_idx
    after the first call.

    The numeric and backward kernels never block the host, so a structure
    changed in place behind the plan (same pointers and sizes, other columns)
    is only reported by handle.check_errors().  With check=True the handle
    fingerprints A's and B's structure at the symbolic phase
    (verify_structure), and every forward and backward call compares the
    fingerprint on the device and then runs that check (one stream
    synchronisation each), raising SpgemmError (STRUCTURE_MISMATCH) instead
    of returning values or gradients computed on the wrong structure.  A
    handle passed in keeps its own options.
    """

    def __init__(self, A: DeviceCsr, B: DeviceCsr, handle: Handle | None = None, rp_dtype=torch.int32,
                 check: bool = False):
        self.A, self.B = A, B
        self.check = check
        self.handle = handle or Handle(verify_structure=1 if check else 0)
        self.row_ptr, self.nnz = spgemm_symbolic(self.handle, A, B, rp_dtype)
        self.col_idx = None

    def __call__(self, a_values: torch.Tensor, b_values: torch.Tensor) -> torch.Tensor:
        out = _SpGEMMFunction.apply(a_values, b_values, self)
        return out

    def structure(self) -> DeviceCsr:
        """C's structure (runs one numeric pass on the stored values if needed)."""
        C = spgemm_numeric(self.handle, self.A, self.B, self.row_ptr, self.nnz)
        self.col_idx = C.col_idx
        return C


# ----------------------------------------------------------------- batch
def spgemm_batch_symbolic(h: Handle, As: list, Bs: list, rp_dtype=torch.int32):
    """spgemm_batch_symbolic: returns ([C_i.row_ptr], [nnz(C_i)])."""
    n = len(As)
    if n != len(Bs) or n == 0:
        raise ValueError("need equal, non-empty lists")
    a = (spg_csr * n)(*[_csr(M) for M in As])
    b = (spg_csr * n)(*[_csr(M) for M in Bs])
    rps = [torch.empty(M.nrows + 1, dtype=rp_dtype, device=M.row_ptr.device) for M in As]
    ptrs = (_P * n)(*[r.data_ptr() for r in rps])
    nnz = (ctypes.c_int64 * n)()
    rc = lib().spgemm_batch_symbolic(h.ptr, n, a, b, ptrs, _itype(rps[0]), nnz)
    if rc != SPG_OK:
        h._raise(rc)
    return rps, [int(v) for v in nnz]


def batch_outputs(As, Bs, rps, nnzs, dtype):
    """C_i laid out back to back in one allocation (the zero-copy layout)."""
    dev = rps[0].device
    tot = sum(nnzs)
    ci = torch.empty(max(tot, 1), dtype=torch.int32, device=dev)
    va = torch.empty(max(tot, 1), dtype=dtype, device=dev)
    out, off = [], 0
    for A, B, rp, nz in zip(As, Bs, rps, nnzs):
        out.append(DeviceCsr(A.nrows, B.ncols, rp, ci[off:off + nz], va[off:off + nz]))
        off += nz
    return out


def spgemm_batch_numeric(h: Handle, As: list, Bs: list, Cs: list):
    """spgemm_batch_numeric into the given outputs (see batch_outputs)."""
    n = len(As)
    a = (spg_csr * n)(*[_csr(M) for M in As])
    b = (spg_csr * n)(*[_csr(M) for M in Bs])
    c = (spg_csr_out * n)(*[spg_csr_out(C.nrows, C.ncols, C.nnz, _itype(C.row_ptr), C.row_ptr.data_ptr(),
                                        C.col_idx.data_ptr() if C.nnz else None,
                                        C.values.data_ptr() if C.nnz else None, _dtype(C.values))
                            for C in Cs])
    rc = lib().spgemm_batch_numeric(h.ptr, n, a, b, c)
    if rc != SPG_OK:
        h._raise(rc)
    return Cs


def spgemm_batch_numeric_values(h: Handle, As: list, Bs: list, Cs: list):
    """spgemm_batch_numeric_values: new values on the batch's known structure (Cs back to
    back, holding the columns an earlier spgemm_batch_numeric wrote)."""
    n = len(As)
    a = (spg_csr * n)(*[_csr(M) for M in As])
    b = (spg_csr * n)(*[_csr(M) for M in Bs])
    c = (spg_csr_out * n)(*[spg_csr_out(C.nrows, C.ncols, C.nnz, _itype(C.row_ptr), C.row_ptr.data_ptr(),
                                        C.col_idx.data_ptr() if C.nnz else None,
                                        C.values.data_ptr() if C.nnz else None, _dtype(C.values))
                            for C in Cs])
    rc = lib().spgemm_batch_numeric_values(h.ptr, n, a, b, c)
    if rc != SPG_OK:
        h._raise(rc)
    return Cs


def pack_batch(mats, device="cuda", dtype=torch.float64, rp_dtype=torch.int32):
    """Device operands with all values (and column indices) back to back in one allocation each."""
    import numpy as np

    ci = torch.as_tensor(np.concatenate([M.col_idx for M in mats]) if mats else np.zeros(0, np.int32)).to(device)
    va = torch.as_tensor(np.concatenate([M.values for M in mats])).to(device=device, dtype=dtype)
    out, off = [], 0
    for M in mats:
        nz = int(M.row_ptr[-1])
        rp = torch.as_tensor(M.row_ptr).to(device=device, dtype=rp_dtype)
        out.append(DeviceCsr(M.nrows, M.ncols, rp, ci[off:off + nz], va[off:off + nz]))
        off += nz
    return out


def spgemm_numeric_rows(h: Handle, A: DeviceCsr, B: DeviceCsr, row_begin: int, row_end: int,
                        col_panel: torch.Tensor, val_panel: torch.Tensor):
    """spgemm_numeric_rows: rows [row_begin, row_end) of C into the panel buffers."""
    a, b = _csr(A), _csr(B)
    rc = lib().spgemm_numeric_rows(h.ptr, ctypes.byref(a), ctypes.byref(b), row_begin, row_end,
                                   _P(col_panel.data_ptr()) if col_panel.numel() else None,
                                   _P(val_panel.data_ptr()) if val_panel.numel() else None)
    if rc != SPG_OK:
        h._raise(rc)
