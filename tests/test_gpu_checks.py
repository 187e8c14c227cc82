"""GPU tests of the statistics and guards around the two phases.

* FP32 default accuracy: rows whose entries may sum more products than FP32
  can add within 1e-5 * sum |a*b| accumulate in FP64 (the term limit derived
  from gamma_n), and the default FP32 product meets that bound.
* Compression statistics (Compression subsection): the pairs of compressed B
  and the compressed flop count equal the oracle's column-set word counts.
* Unsorted rows of B wider than the word-count bitmap are accepted (the
  analysis skips compression for them).
* Structure fingerprint: a structure changed in place behind unchanged
  pointers and sizes is reported as STRUCTURE_MISMATCH.
"""
import numpy as np
import pytest

import oracle
import synth
from helpers import check_f32, check_f64, dev, f32_inputs, oracle_ref, run

pytestmark = pytest.mark.gpu


def _long_rows_pair(seed=4):
    """Rows of A with 20 or 400 entries (above and below the FP32 term limit
    of 167) into a B whose rows overlap heavily, so entries of C sum up to
    hundreds of products of random sign."""
    rng = np.random.default_rng(seed)
    m, n, k = 600, 2000, 300
    lens = np.where(rng.random(m) < 0.3, 400, 20)
    A = synth.random_csr(m, n, lens, seed)
    B = synth.random_csr(n, k, rng.integers(10, 60, n), seed + 1)
    return A, B, int((lens > 167).sum())


@pytest.mark.parametrize("mode,limit", [(0, 167), (1, 52730), (2, 0)])
def test_fp32_default_term_limit(mode, limit):
    A, B, nlong = _long_rows_pair()
    ref, S = oracle_ref(f32_inputs(A), f32_inputs(B))
    got, h = run(A, B, dtype="f32", fp32_mode=mode)
    mx, med = check_f32(ref, S, got)
    st = h.stats()
    want = nlong if mode == 0 else 0
    assert st["fp64_rows"] == want, (st["fp64_rows"], want)
    print(f"fp32 mode {mode} (term limit {limit}): fp64 rows {st['fp64_rows']}, max {mx:.3e} median {med:.3e}")


def test_fp32_term_limit_off_and_explicit():
    A, B, nlong = _long_rows_pair(7)
    ref, S = oracle_ref(f32_inputs(A), f32_inputs(B))
    got, h = run(A, B, dtype="f32", fp32_mode=0, fp32_terms_max=0)
    assert h.stats()["fp64_rows"] == 0
    check_f32(ref, S, got, rel=1e-4)  # plain FP32 throughout: gamma_400 bound
    got, h = run(A, B, dtype="f32", fp32_mode=0, fp32_terms_max=19)
    assert h.stats()["fp64_rows"] == A.nrows  # every row has more than 19 entries
    check_f32(ref, S, got)
    # FP64 values take the same kind lists (one launch set more), same results
    ref64, S64 = oracle_ref(A, B)
    got, h = run(A, B, fp32_terms_max=19)
    check_f64(ref64, S64, got)


@pytest.mark.parametrize("case", ["27pt", "5pt", "galerkin", "random"])
def test_compressed_counts_equal_oracle(case):
    if case == "27pt":
        A = synth.stencil27(24)
        B = A
    elif case == "5pt":
        A = B = synth.laplace2d_5pt(64, 64)
    elif case == "galerkin":
        A0 = synth.stencil27(24)
        P, A = synth.aggregation_2x2x2(24)
        B = oracle.spgemm(A0, P)
    else:
        A, B = synth.tiny_random(400, 300, 0.05, 3), synth.shuffle_columns(synth.tiny_random(300, 900, 0.2, 4), 5)
    bc = oracle.block_counts(B, 32)
    want_fmc = int(bc[A.col_idx].sum())
    _, h = run(A, B, compression=1)
    st = h.stats()
    assert st["compressed"] == 1
    assert st["nnz_b_compressed"] == int(bc.sum())
    assert st["flops_compressed"] == want_fmc
    assert st["flops"] == int(np.diff(B.row_ptr)[A.col_idx].sum())
    _, h = run(A, B, compression=0)
    assert h.stats()["nnz_b_compressed"] == 0 and h.stats()["flops_compressed"] == want_fmc


def test_compressed_counts_27pt_100():
    A = synth.stencil27(100)
    _, h = run(A, A)
    st = h.stats()
    assert st["compressed"] == 1
    assert st["nnz_b_compressed"] == 9_413_224
    assert st["flops_compressed"] == 250_303_600 and st["flops"] == 704_969_000


@pytest.mark.parametrize("acc", [0, 1, 2])
def test_wide_unsorted_b_row(acc):
    """A row of B with unsorted columns spanning more than 2^19 columns."""
    rng = np.random.default_rng(11)
    n, k, m = 64, (1 << 20) + 77, 300
    B = synth.random_csr(n, k, rng.integers(0, 30, n), 12)
    cols = [list(B.col_idx[B.row_ptr[r]:B.row_ptr[r + 1]]) for r in range(n)]
    cols[5] = [k - 1, 3, 700_000, 12, 524_300, 1 << 19]
    cols[9] = [900_000, 2]
    rp = np.zeros(n + 1, dtype=np.int64)
    rp[1:] = np.cumsum([len(c) for c in cols])
    B = synth.Csr(n, k, rp, np.concatenate([np.asarray(c, np.int32) for c in cols]),
                  rng.standard_normal(int(rp[-1])))
    A = synth.random_csr(m, n, rng.integers(0, 12, m), 13)
    ref, S = oracle_ref(A, B)
    got, h = run(A, B, accumulator=acc)
    check_f64(ref, S, got)
    assert h.stats()["compressed"] == 0


def test_structure_change_in_place_detected():
    import torch

    import paper_1801_03065_amd as spg

    A = synth.stencil27(6)
    dA = dev(A)
    h = spg.Handle(verify_structure=1)
    rp, nnz = spg.spgemm_symbolic(h, dA, dA)
    C = spg.spgemm_numeric(h, dA, dA, rp, nnz)
    h.check_errors()
    # same sizes, other columns: swap two column indices of different rows
    ci = dA.col_idx
    a, b = int(A.row_ptr[3]), int(A.row_ptr[40])
    va, vb = ci[a].item(), ci[b].item()
    ci[a], ci[b] = vb, va
    spg.spgemm_numeric(h, dA, dA, rp, nnz, out=C)
    with pytest.raises(spg.SpgemmError) as e:
        h.check_errors()
    assert e.value.status == spg.SPG_ERR_STRUCTURE_MISMATCH
    # restored: the digest matches again
    ci[a], ci[b] = va, vb
    spg.spgemm_numeric(h, dA, dA, rp, nnz, out=C)
    h.check_errors()
    torch.cuda.synchronize()


def test_sparse_product_check_raises():
    import torch

    import paper_1801_03065_amd as spg

    A = synth.laplace7(6)
    B = synth.fixed_row_random(A.ncols, A.ncols, 5, 3)
    dA, dB = dev(A), dev(B)
    prod = spg.SparseProduct(dA, dB, check=True)
    av = dA.values.clone().requires_grad_(True)
    bv = dB.values.clone().requires_grad_(True)
    out = prod(av, bv)
    out.sum().backward()
    row0 = set(B.col_idx[:5].tolist())
    dB.col_idx[0] = next(c for c in range(B.ncols) if c not in row0)  # same sizes, another column
    with pytest.raises(spg.SpgemmError):
        prod(av, bv)
    torch.cuda.synchronize()
