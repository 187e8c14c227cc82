"""Shared helpers of the GPU tests: marshal synthetic CSR onto the GPU, run the
library through its C ABI binding, compare with the oracle."""
from __future__ import annotations

import numpy as np

import oracle
import synth


def dev(M: synth.Csr, dtype="f64", rp="i32"):
    import torch

    import paper_1801_03065_amd as spg

    return spg.DeviceCsr.from_arrays(M.nrows, M.ncols, M.row_ptr, M.col_idx, M.values,
                                     rp_dtype=torch.int32 if rp == "i32" else torch.int64,
                                     dtype=torch.float64 if dtype == "f64" else torch.float32)


def run(A: synth.Csr, B: synth.Csr, dtype="f64", rp="i32", crp="i32", handle=None, **opts):
    """Both phases on the GPU; returns (row_ptr, col_idx, values) as numpy and the handle."""
    import torch

    import paper_1801_03065_amd as spg

    h = handle or spg.Handle(**opts)
    dA, dB = dev(A, dtype, rp), dev(B, dtype, rp)
    r, nnz = spg.spgemm_symbolic(h, dA, dB, torch.int32 if crp == "i32" else torch.int64)
    C = spg.spgemm_numeric(h, dA, dB, r, nnz)
    h.check_errors()
    torch.cuda.synchronize()
    return (r.cpu().numpy().astype(np.int64), C.col_idx.cpu().numpy(), C.values.cpu().numpy()), h


def check_structure(ref: synth.Csr, got):
    rp, ci, _ = got
    assert rp.shape == ref.row_ptr.shape
    bad = np.nonzero(rp != ref.row_ptr)[0]
    assert bad.size == 0, f"row_ptr differs first at row {bad[:5]}"
    diff = np.nonzero(ci != ref.col_idx)[0]
    assert diff.size == 0, f"col_idx differs at {diff.size} entries, first {diff[:5]}"


def check_f64(ref: synth.Csr, S: np.ndarray, got, rel=1e-12):
    """|gpu - oracle| <= rel * max(|oracle|, sum |a*b|) per entry (summation order differs)."""
    check_structure(ref, got)
    v = got[2]
    err = np.abs(v - ref.values)
    bound = rel * np.maximum(np.abs(ref.values), S)
    worst = np.argmax(err - bound) if err.size else 0
    assert np.all(err <= bound), f"value error {err[worst]:.3e} > {bound[worst]:.3e} at {worst}"
    return float(err.max()) if err.size else 0.0


def check_f32(ref: synth.Csr, S: np.ndarray, got, rel=1e-5):
    """FP32 result vs the FP64 oracle on the FP32-rounded inputs: |err| <= rel * S."""
    check_structure(ref, got)
    v = got[2].astype(np.float64)
    err = np.abs(v - ref.values)
    bound = rel * S
    ok = err <= bound
    worst = np.argmax(err - bound) if err.size else 0
    assert np.all(ok), f"value error {err[worst]:.3e} > {bound[worst]:.3e} at {worst}"
    rel_err = err / np.maximum(S, 1e-300)
    return float(rel_err.max()) if err.size else 0.0, float(np.median(rel_err)) if err.size else 0.0


def oracle_ref(A, B):
    return oracle.spgemm(A, B, with_abs=True)


def f32_inputs(A: synth.Csr):
    """The matrix with values rounded to FP32 (held as float64 for the oracle)."""
    return A.with_values(A.values.astype(np.float32).astype(np.float64))
