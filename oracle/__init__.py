"""Python face of the plain CPU SpGEMM oracle (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package. It wraps `spgemm_oracle.c` (sequential C, IEEE double, products
rounded before each add) through ctypes and never touches the GPU library.

Functions (each cites the passage of the paper it follows in the C source):
  flops(A, B)             -> (f_m, max_row_flops, row_flops)    Background section
  block_counts(B, width)  -> distinct col//width per row of B    Compression subsection
  symbolic(A, B)          -> C.row_ptr                          Algorithm 2, line "symbolic"
  spgemm(A, B, with_abs)  -> C (sorted columns) [, S]           Algorithm 1
  rows(A, B, rows)        -> selected rows of C (+ S) by the same definition
  grad(A, B, C, G)        -> (dA on pattern(A), dB on pattern(B))
  masked(A, B, M)         -> (A*B) on pattern(M), or path counts       Background (graph analytics)
  rows_check(...)         -> compares candidate rows with the definition (comparison helper)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from synth import Csr

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spgemm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I = ctypes.c_int64
        lib.spo_flops.restype = ctypes.c_int64
        lib.spo_flops.argtypes = [I, I, P, P, P, P, P]
        lib.spo_block_counts.restype = ctypes.c_int
        lib.spo_block_counts.argtypes = [I, I, P, P, ctypes.c_int32, P]
        lib.spo_symbolic.restype = ctypes.c_int
        lib.spo_symbolic.argtypes = [I, I, I, P, P, P, P, P]
        lib.spo_numeric.restype = ctypes.c_int
        lib.spo_numeric.argtypes = [I, I, I, P, P, P, P, P, P, P, P, P, P]
        lib.spo_rows.restype = ctypes.c_int
        lib.spo_rows.argtypes = [I, I, I, P, P, P, P, P, P, I, P, P, P, P, P]
        lib.spo_rows_check.restype = ctypes.c_int
        lib.spo_rows_check.argtypes = [I, I, I, P, P, P, P, P, P, I, P, P, P, P, ctypes.c_double, ctypes.c_int,
                                       P, I, P, I, P]
        lib.spo_masked.restype = ctypes.c_int
        lib.spo_masked.argtypes = [I, I, I, P, P, P, P, P, P, P, P, ctypes.c_int, P, P]
        lib.spo_grad.restype = ctypes.c_int
        lib.spo_grad.argtypes = [I, I, I, P, P, P, P, P, P, P, P, P, P, P]
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _norm(A: Csr):
    rp = np.ascontiguousarray(A.row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(A.col_idx, dtype=np.int32)
    va = np.ascontiguousarray(A.values, dtype=np.float64)  # float32 widens exactly
    return rp, ci, va


def _check_dims(A: Csr, B: Csr):
    if A.ncols != B.nrows:
        raise ValueError(f"dimension mismatch: A is {A.nrows}x{A.ncols}, B is {B.nrows}x{B.ncols}")


def flops(A: Csr, B: Csr):
    _check_dims(A, B)
    arp, aci, _ = _norm(A)
    brp, _, _ = _norm(B)
    rf = np.zeros(max(A.nrows, 1), dtype=np.int64)
    mx = ctypes.c_int64(0)
    fm = _load().spo_flops(A.nrows, A.ncols, _p(arp), _p(aci), _p(brp), _p(rf), ctypes.byref(mx))
    if fm < 0:
        raise ValueError("bad CSR input")
    return int(fm), int(mx.value), rf[: A.nrows]


def block_counts(B: Csr, width: int = 32) -> np.ndarray:
    brp, bci, _ = _norm(B)
    out = np.zeros(max(B.nrows, 1), dtype=np.int64)
    rc = _load().spo_block_counts(B.nrows, B.ncols, _p(brp), _p(bci), width, _p(out))
    if rc:
        raise ValueError(f"spo_block_counts rc={rc}")
    return out[: B.nrows]


def symbolic(A: Csr, B: Csr) -> np.ndarray:
    _check_dims(A, B)
    arp, aci, _ = _norm(A)
    brp, bci, _ = _norm(B)
    crp = np.zeros(A.nrows + 1, dtype=np.int64)
    rc = _load().spo_symbolic(A.nrows, A.ncols, B.ncols, _p(arp), _p(aci), _p(brp), _p(bci), _p(crp))
    if rc:
        raise ValueError(f"spo_symbolic rc={rc}")
    return crp


def spgemm(A: Csr, B: Csr, with_abs: bool = False):
    """C = A*B in float64 with sorted columns; optionally S(i,j) = sum |a*b|."""
    crp = symbolic(A, B)
    arp, aci, ava = _norm(A)
    brp, bci, bva = _norm(B)
    nnz = int(crp[-1])
    cci = np.zeros(max(nnz, 1), dtype=np.int32)
    cva = np.zeros(max(nnz, 1), dtype=np.float64)
    cab = np.zeros(max(nnz, 1), dtype=np.float64) if with_abs else None
    rc = _load().spo_numeric(A.nrows, A.ncols, B.ncols, _p(arp), _p(aci), _p(ava),
                             _p(brp), _p(bci), _p(bva), _p(crp), _p(cci), _p(cva),
                             _p(cab) if with_abs else None)
    if rc:
        raise ValueError(f"spo_numeric rc={rc}")
    C = Csr(A.nrows, B.ncols, crp, cci[:nnz], cva[:nnz])
    return (C, cab[:nnz]) if with_abs else C


def grad(A: Csr, B: Csr, C: Csr, G: np.ndarray):
    """(dA, dB) of L = sum(G * C) over pattern(C); C must have sorted columns."""
    _check_dims(A, B)
    arp, aci, ava = _norm(A)
    brp, bci, bva = _norm(B)
    crp = np.ascontiguousarray(C.row_ptr, dtype=np.int64)
    cci = np.ascontiguousarray(C.col_idx, dtype=np.int32)
    g = np.ascontiguousarray(G, dtype=np.float64)
    dA = np.zeros(max(A.nnz, 1))
    dB = np.zeros(max(B.nnz, 1))
    rc = _load().spo_grad(A.nrows, A.ncols, B.ncols, _p(arp), _p(aci), _p(ava),
                          _p(brp), _p(bci), _p(bva), _p(crp), _p(cci), _p(g), _p(dA), _p(dB))
    if rc:
        raise ValueError(f"spo_grad rc={rc}")
    return dA[: A.nnz], dB[: B.nnz]


def rows(A: Csr, B: Csr, sel):
    """Rows `sel` of C = A*B: (row_ptr over the selection, col_idx, values, S)."""
    _check_dims(A, B)
    arp, aci, ava = _norm(A)
    brp, bci, bva = _norm(B)
    sel = np.ascontiguousarray(sel, dtype=np.int64)
    rp = np.zeros(sel.shape[0] + 1, dtype=np.int64)
    L = _load()
    rc = L.spo_rows(A.nrows, A.ncols, B.ncols, _p(arp), _p(aci), _p(ava), _p(brp), _p(bci), _p(bva),
                    sel.shape[0], _p(sel), _p(rp), None, None, None)
    if rc:
        raise ValueError(f"spo_rows rc={rc}")
    nnz = int(rp[-1])
    ci = np.zeros(max(nnz, 1), dtype=np.int32)
    va = np.zeros(max(nnz, 1))
    ab = np.zeros(max(nnz, 1))
    rc = L.spo_rows(A.nrows, A.ncols, B.ncols, _p(arp), _p(aci), _p(ava), _p(brp), _p(bci), _p(bva),
                    sel.shape[0], _p(sel), _p(rp), _p(ci), _p(va), _p(ab))
    if rc:
        raise ValueError(f"spo_rows rc={rc}")
    return rp, ci[:nnz], va[:nnz], ab[:nnz]


def masked(A: Csr, B: Csr, M: Csr, structural: bool = False, with_abs: bool = False):
    """(A*B) on the stored entries of M (M's entry order); structural: path counts."""
    _check_dims(A, B)
    if M.nrows != A.nrows or M.ncols != B.ncols:
        raise ValueError("mask must be A.nrows x B.ncols")
    arp, aci, ava = _norm(A)
    brp, bci, bva = _norm(B)
    mrp, mci, _ = _norm(M)
    out = np.zeros(max(M.nnz, 1))
    ab = np.zeros(max(M.nnz, 1)) if with_abs else None
    rc = _load().spo_masked(A.nrows, A.ncols, B.ncols, _p(arp), _p(aci), _p(ava), _p(brp), _p(bci), _p(bva),
                            _p(mrp), _p(mci), 1 if structural else 0, _p(out), _p(ab) if with_abs else None)
    if rc:
        raise ValueError(f"spo_masked rc={rc}")
    return (out[: M.nnz], ab[: M.nnz]) if with_abs else out[: M.nnz]


def rows_check(A: Csr, B: Csr, sel, grp, gci, gval, tol: float, rel_mode: int, stride: int = 101,
               sub_cap: int = 1 << 20):
    """Compare candidate rows (grp offsets over `sel`, columns gci, values gval as
    float64) with the definition; returns dict(max_rel_S, bad, entries, bad_rows,
    sub = sampled |g-c|/S).  A comparison helper of the tests, not a method."""
    _check_dims(A, B)
    arp, aci, ava = _norm(A)
    brp, bci, bva = _norm(B)
    sel = np.ascontiguousarray(sel, dtype=np.int64)
    grp = np.ascontiguousarray(grp, dtype=np.int64)
    gci = np.ascontiguousarray(gci, dtype=np.int32)
    gval = np.ascontiguousarray(gval, dtype=np.float64)
    stats = np.zeros(4)
    sub = np.zeros(max(sub_cap, 1), dtype=np.float32)
    ns = ctypes.c_int64(0)
    rc = _load().spo_rows_check(A.nrows, A.ncols, B.ncols, _p(arp), _p(aci), _p(ava), _p(brp), _p(bci), _p(bva),
                                sel.shape[0], _p(sel), _p(grp), _p(gci), _p(gval), tol, rel_mode, _p(stats),
                                stride, _p(sub), sub_cap, ctypes.byref(ns))
    if rc:
        raise ValueError(f"spo_rows_check rc={rc}")
    return {"max_rel_S": float(stats[0]), "bad": int(stats[1]), "entries": int(stats[2]),
            "bad_rows": int(stats[3]), "sub": sub[: ns.value]}
