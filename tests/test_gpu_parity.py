"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Structure (row_ptr, col_idx) must match bit for bit; FP64 values within
1e-12 * max(|c|, sum |a*b|) per entry (summation order differs); integer-valued
stencil products are exact in any order, so there they must match exactly.
"""
import numpy as np
import pytest

import oracle
import synth
from helpers import check_f32, check_f64, check_structure, dev, f32_inputs, oracle_ref, run

pytestmark = pytest.mark.gpu


def _exact(A, B, **kw):
    ref = oracle.spgemm(A, B)
    got, h = run(A, B, **kw)
    check_structure(ref, got)
    assert np.array_equal(got[2], ref.values)
    return h


def test_5pt_square_64x64():
    A = synth.laplace2d_5pt(64, 64)
    h = _exact(A, A)
    st = h.stats()
    assert st["flops"] == 100104 and st["nnz_c"] == 51972 and st["max_row_flops"] == 25


@pytest.mark.parametrize("acc", [0, 1, 2, 3])
@pytest.mark.parametrize("g", [2, 3, 7, 20])
def test_27pt_square_small(g, acc):
    A = synth.stencil27(g)
    h = _exact(A, A, accumulator=acc, l1_hash_slots=64 if acc == 3 else 0)
    used = {k for k, v in h.stats()["rows_numeric"].items() if v}
    if acc == 0:
        # at g = 2 every row has 8 * 8 = 64 multiplications (short-row teams);
        # from g = 3 on even a corner row has 125, and at most 50 touched
        # words: the numeric phase runs on the stored structure
        assert used == ({"short_rows"} if g == 2 else {"planned_wave"}), used
    else:
        want = {1: "dense_wave", 2: "hash_wave", 3: "hash_two_level"}[acc]
        assert used == {want}, used


@pytest.mark.parametrize("g", [4, 10])
def test_galerkin_small(g):
    A = synth.stencil27(g)
    P, Pt = synth.aggregation_2x2x2(g)
    AP = oracle.spgemm(A, P)
    _exact(A, P)
    _exact(Pt, AP)


@pytest.mark.parametrize("seed", range(6))
def test_random_unsorted_rectangular(seed):
    rng = np.random.default_rng(seed)
    m, n, k = int(rng.integers(50, 700)), int(rng.integers(50, 700)), int(rng.integers(1, 5000))
    A = synth.shuffle_columns(synth.random_csr(m, n, rng.integers(0, 20, m), seed), seed)
    B = synth.shuffle_columns(synth.random_csr(n, k, rng.integers(0, 30, n), seed + 9), seed + 1)
    ref, S = oracle_ref(A, B)
    got, _ = run(A, B)
    check_f64(ref, S, got)


@pytest.mark.parametrize("acc", [0, 1, 2, 3])
@pytest.mark.parametrize("comp", [-1, 0, 1])
def test_forced_paths_agree(acc, comp):
    rng = np.random.default_rng(7)
    A = synth.shuffle_columns(synth.random_csr(400, 300, rng.integers(0, 25, 400), 1), 2)
    B = synth.random_csr(300, 3000, rng.integers(0, 40, 300), 3)
    ref, S = oracle_ref(A, B)
    got, h = run(A, B, accumulator=acc, compression=comp,
                 l1_hash_slots=64 if acc == 3 else 0)
    check_f64(ref, S, got)
    st = h.stats()
    if acc == 3:
        assert st["rows_numeric"]["hash_two_level"] > 0
    if comp == 1:
        assert st["compressed"] == 1
    if comp == 0:
        assert st["compressed"] == 0


def test_heavy_rows_dense_workgroup():
    """A few rows with tens of thousands of entries in C: workgroup-per-row kernels."""
    rng = np.random.default_rng(11)
    counts = rng.integers(0, 6, 500)
    counts[[3, 77, 400]] = [1500, 900, 2500]
    A = synth.random_csr(500, 2000, counts, 5)
    B = synth.random_csr(2000, 200000, rng.integers(5, 60, 2000), 6)
    ref, S = oracle_ref(A, B)
    got, h = run(A, B)
    check_f64(ref, S, got)
    assert h.stats()["rows_numeric"]["dense_wg"] >= 3


def test_wide_window_two_level_hash():
    """Rows whose column window exceeds the LDS bit window and are large: level-2 hash."""
    rng = np.random.default_rng(12)
    counts = rng.integers(0, 4, 300)
    counts[[5, 100]] = [400, 700]
    A = synth.random_csr(300, 1000, counts, 8)
    B = synth.random_csr(1000, 1 << 23, rng.integers(1, 12, 1000), 9)
    ref, S = oracle_ref(A, B)
    got, h = run(A, B)
    check_f64(ref, S, got)
    assert h.stats()["rows_numeric"]["hash_two_level"] >= 2


@pytest.mark.parametrize("shape", [(0, 5, 7), (5, 0, 7), (5, 7, 0), (1, 1, 1), (64, 64, 1)])
def test_degenerate_shapes(shape):
    m, n, k = shape
    A = synth.tiny_random(m, n, 0.5, 1)
    B = synth.tiny_random(n, k, 0.5, 2)
    ref, S = oracle_ref(A, B)
    got, _ = run(A, B)
    check_f64(ref, S, got)


def test_empty_rows_and_structural_zeros():
    A0 = synth.tiny_random(60, 50, 0.15, 3, zero_frac=0.3)
    rows = np.repeat(np.arange(60), A0.row_lengths())
    sel = (rows < 10) | (rows >= 20)
    counts = np.bincount(rows[sel], minlength=60)
    rp = np.zeros(61, np.int64)
    np.cumsum(counts, out=rp[1:])
    A = synth.Csr(60, 50, rp, A0.col_idx[sel], A0.values[sel])
    B = synth.tiny_random(50, 40, 0.2, 4, zero_frac=0.3)
    ref, S = oracle_ref(A, B)
    got, _ = run(A, B)
    check_f64(ref, S, got)


def test_int64_row_ptrs():
    A = synth.stencil27(6)
    ref = oracle.spgemm(A, A)
    got, _ = run(A, A, rp="i64", crp="i64")
    check_structure(ref, got)
    assert np.array_equal(got[2], ref.values)


@pytest.mark.parametrize("widths", [("i64", "i32"), ("i32", "i64")])
def test_mixed_row_ptr_widths(widths):
    """A and B with row pointers of different widths (one launch copies both)."""
    import torch

    import paper_1801_03065_amd as spg

    A = synth.stencil27(7)
    B = synth.random_csr(A.ncols, 500, np.random.default_rng(8).integers(0, 6, A.ncols), 9)
    ref, S = oracle_ref(A, B)
    h = spg.Handle()
    dA, dB = dev(A, rp=widths[0]), dev(B, rp=widths[1])
    rp, nnz = spg.spgemm_symbolic(h, dA, dB, torch.int64)
    C = spg.spgemm_numeric(h, dA, dB, rp, nnz)
    h.check_errors()
    torch.cuda.synchronize()
    check_f64(ref, S, (rp.cpu().numpy(), C.col_idx.cpu().numpy(), C.values.cpu().numpy()))


def test_scan_over_many_blocks():
    """2.2M rows: the row-size scan has more than 1024 blocks of 2048 entries
    and takes its one-workgroup top scan."""
    rng = np.random.default_rng(12)
    m = n = 2_200_000
    A = synth.random_csr(m, n, rng.integers(0, 3, m), 13)
    B = synth.random_csr(n, 3000, rng.integers(0, 4, n), 14)
    ref, S = oracle_ref(A, B)
    got, _ = run(A, B)
    check_f64(ref, S, got)


@pytest.mark.parametrize("acc", [0, 1, 2, 3])
def test_row_panels_equal_whole_product(acc):
    """spgemm_numeric_rows over panels reproduces the whole numeric result."""
    import torch

    import paper_1801_03065_amd as spg
    from helpers import dev

    rng = np.random.default_rng(21)
    counts = rng.integers(0, 20, 700)
    counts[[10, 400]] = [900, 1300]  # heavy rows land in the workgroup kinds
    A = synth.random_csr(700, 2500, counts, 4)
    B = synth.random_csr(2500, 60000, rng.integers(0, 30, 2500), 5)
    ref, S = oracle_ref(A, B)
    h = spg.Handle(accumulator=acc, l1_hash_slots=64 if acc == 3 else 0)
    dA, dB = dev(A), dev(B)
    rp, nnz = spg.spgemm_symbolic(h, dA, dB, torch.int64)
    rph = rp.cpu().numpy()
    cuts = [0, 1, 10, 11, 300, 401, 700]
    ci = np.zeros(nnz, np.int32)
    va = np.zeros(nnz)
    for rb, re_ in zip(cuts[:-1], cuts[1:]):
        n = int(rph[re_] - rph[rb])
        pc = torch.full((max(n, 1),), -7, dtype=torch.int32, device="cuda")
        pv = torch.zeros(max(n, 1), dtype=torch.float64, device="cuda")
        spg.spgemm_numeric_rows(h, dA, dB, rb, re_, pc, pv)
        h.check_errors()
        torch.cuda.synchronize()
        ci[rph[rb]:rph[re_]] = pc.cpu().numpy()[:n]
        va[rph[rb]:rph[re_]] = pv.cpu().numpy()[:n]
    check_f64(ref, S, (rph, ci, va))


def test_heavy_rows_window_away_from_zero():
    """Workgroup-kind rows whose column window starts far from column 0."""
    rng = np.random.default_rng(13)
    counts = rng.integers(0, 6, 300)
    counts[[7, 150]] = [1200, 1700]
    A = synth.random_csr(300, 1500, counts, 6)
    B0 = synth.random_csr(1500, 90000, rng.integers(5, 40, 1500), 7)
    B = synth.Csr(1500, 250000, B0.row_ptr, (B0.col_idx + 150000).astype(np.int32), B0.values)
    ref, S = oracle_ref(A, B)
    got, h = run(A, B)
    check_f64(ref, S, got)
    assert h.stats()["rows_numeric"]["dense_wg"] >= 2


@pytest.mark.parametrize("fmax", [4, 12, 30, 64])
def test_short_rows_teams(fmax):
    """Rows with at most 64 multiplications: several rows per wavefront, team
    size the next power of two of the largest row (8 to 64 lanes)."""
    rng = np.random.default_rng(fmax)
    m, n, k = 3000, 900, 2500
    nb = rng.integers(0, 5, n)
    B = synth.shuffle_columns(synth.random_csr(n, k, nb, 31), 3)
    A = synth.random_csr(m, n, rng.integers(0, 12, m), 32)
    # keep entries of each row of A while its multiplications stay within fmax
    lens = np.diff(B.row_ptr)
    rp, ci, va = [0], [], []
    for i in range(m):
        tot = 0
        for e in range(A.row_ptr[i], A.row_ptr[i + 1]):
            if tot + lens[A.col_idx[e]] <= fmax:
                ci.append(A.col_idx[e])
                va.append(A.values[e])
                tot += lens[A.col_idx[e]]
        rp.append(len(ci))
    A = synth.Csr(m, n, np.array(rp, np.int64), np.array(ci, np.int32), np.array(va))
    ref, S = oracle_ref(A, B)
    got, h = run(A, B)
    check_f64(ref, S, got)
    st = h.stats()
    assert st["rows_numeric"]["short_rows"] > 0 and st["rows_symbolic"]["short_rows"] > 0
    assert st["max_row_flops"] <= fmax


def test_short_rows_many_empty_b_rows():
    """Short rows whose A row is longer than the team (most B rows are empty):
    the team walks its A row in chunks."""
    rng = np.random.default_rng(5)
    n, k = 4000, 700
    nb = np.where(rng.random(n) < 0.1, rng.integers(1, 3, n), 0)
    B = synth.random_csr(n, k, nb, 41)
    A = synth.random_csr(400, n, rng.integers(60, 200, 400), 42)
    fl = oracle.flops(A, B)[2]
    ref, S = oracle_ref(A, B)
    got, h = run(A, B)
    check_f64(ref, S, got)
    assert h.stats()["rows_numeric"]["short_rows"] == int(np.count_nonzero((fl > 0) & (fl <= 64)))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_short_rows_unit_b_rows(dtype):
    """B rows of zero or one entry (an injection with many repeated
    columns): every A entry makes at most one product, and the teams form
    them without the expansion; A rows of 1-150 entries (several chunks per
    team), one B row of two entries in a few of them."""
    rng = np.random.default_rng(71)
    n, k = 3000, 40
    nb = (rng.random(n) < 0.8).astype(np.int64)
    nb[rng.integers(0, n, 3)] = 2
    B = synth.random_csr(n, k, nb, 72)
    A = synth.random_csr(2500, n, rng.integers(0, 150, 2500), 73)
    if dtype == "f32":
        A, B = f32_inputs(A), f32_inputs(B)
    ref, S = oracle_ref(A, B)
    got, h = run(A, B, dtype=dtype)
    (check_f64 if dtype == "f64" else check_f32)(ref, S, got)
    assert h.stats()["rows_numeric"]["short_rows"] > 0


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_short_rows_fp32(mode):
    A = synth.stencil27(6)
    P, _ = synth.aggregation_2x2x2(6)
    A32, P32 = f32_inputs(A), f32_inputs(P)
    ref, S = oracle_ref(A32, P32)
    got, h = run(A, P, dtype="f32", fp32_mode=mode)
    check_f32(ref, S, got)
    assert set(k for k, v in h.stats()["rows_numeric"].items() if v) == {"short_rows"}


def test_stored_structure_and_word_hash_mix():
    """Rows with at most 64 touched words run on the structure the symbolic
    phase stored; rows with more rebuild it with the word hash."""
    rng = np.random.default_rng(21)
    A = synth.shuffle_columns(synth.random_csr(2000, 3000, rng.integers(3, 40, 2000), 51), 4)
    B = synth.random_csr(3000, 60000, rng.integers(1, 30, 3000), 52)
    ref, S = oracle_ref(A, B)
    got, h = run(A, B)
    check_f64(ref, S, got)
    st = h.stats()
    assert st["rows_numeric"]["planned_wave"] > 0 and st["rows_numeric"]["word_hash_wave"] > 0, st
    # Reuse: new values on the same plan
    import torch

    import paper_1801_03065_amd as spg
    from helpers import dev

    A2 = A.with_values(rng.standard_normal(A.nnz))
    dA2, dB = dev(A2), dev(B)
    rp = torch.as_tensor(got[0].astype(np.int32), device="cuda")
    spg.spgemm_symbolic(h, dA2, dB)
    C = spg.spgemm_numeric(h, dA2, dB, rp, int(got[0][-1]))
    h.check_errors()
    ref2, S2 = oracle_ref(A2, B)
    check_f64(ref2, S2, (got[0], C.col_idx.cpu().numpy(), C.values.cpu().numpy()))


def _malformed_cases():
    """Operands a caller could pass by mistake; each must be rejected with
    SPG_ERR_INVALID_ARG (the analysis before the check reads row ranges
    clamped to the arrays and skips out-of-range columns)."""
    A = synth.random_csr(40, 30, np.full(40, 3), 1)
    B = synth.random_csr(30, 50, np.full(30, 4), 2)
    cases = {}
    rp = A.row_ptr.copy(); rp[5], rp[6] = rp[6], rp[5] + 100      # not monotone, past nnz
    cases["row_ptr_not_monotone"] = (synth.Csr(A.nrows, A.ncols, rp, A.col_idx, A.values), B)
    rp = A.row_ptr.copy(); rp[-1] = A.nnz - 2                      # last != nnz
    cases["row_ptr_end"] = (synth.Csr(A.nrows, A.ncols, rp, A.col_idx, A.values), B)
    ci = A.col_idx.copy(); ci[7] = 10 ** 6                         # column of A >= rows of B
    cases["a_col_too_large"] = (synth.Csr(A.nrows, A.ncols, A.row_ptr, ci, A.values), B)
    ci = A.col_idx.copy(); ci[3] = -5                              # negative column
    cases["a_col_negative"] = (synth.Csr(A.nrows, A.ncols, A.row_ptr, ci, A.values), B)
    ci = B.col_idx.copy(); ci[9] = 50                              # column of B >= its columns
    cases["b_col_too_large"] = (A, synth.Csr(B.nrows, B.ncols, B.row_ptr, ci, B.values))
    return A, B, cases


@pytest.mark.parametrize("case", ["row_ptr_not_monotone", "row_ptr_end", "a_col_too_large", "a_col_negative",
                                  "b_col_too_large"])
def test_malformed_input_rejected_then_handle_reusable(case):
    import paper_1801_03065_amd as spg
    from helpers import dev

    A, B, cases = _malformed_cases()
    bA, bB = cases[case]
    h = spg.Handle()
    with pytest.raises(spg.SpgemmError) as ei:
        spg.spgemm_symbolic(h, dev(bA), dev(bB))
    assert ei.value.status == spg.SPG_ERR_INVALID_ARG
    got, _ = run(A, B, handle=h)  # the same handle, valid operands
    ref, S = oracle_ref(A, B)
    check_f64(ref, S, got)


@pytest.mark.parametrize("comp", [-1, 1])
@pytest.mark.parametrize("acc", [0, 1])
def test_short_unsorted_b_rows(acc, comp):
    """B whose rows hold 0-6 entries (one lane per B row in the analysis and
    in the compression) with shuffled columns: sortedness found per row, heavy
    rows without segments; compression by the rule and forced."""
    rng = np.random.default_rng(41)
    m, n, k = 2000, 3000, 5000
    B = synth.shuffle_columns(synth.random_csr(n, k, rng.integers(0, 7, n), 42), 43)
    counts = rng.integers(0, 30, m)
    counts[[5, 900]] = [2500, 1800]  # rows with thousands of entries in C
    A = synth.random_csr(m, n, counts, 44)
    ref, S = oracle_ref(A, B)
    got, h = run(A, B, accumulator=acc, compression=comp)
    check_f64(ref, S, got)
    if comp == 1:
        assert h.stats()["compressed"] == 1


def test_handle_reused_across_products():
    """One handle through products of different shapes and kinds, growing and
    shrinking: each plan replaces the previous one completely."""
    import paper_1801_03065_amd as spg

    A = synth.stencil27(6)
    P, Pt = synth.aggregation_2x2x2(6)
    AP = oracle.spgemm(A, P)
    rng = np.random.default_rng(21)
    R = synth.random_csr(5000, A.ncols, rng.integers(0, 40, 5000), 22)
    big = synth.stencil27(12)
    h = spg.Handle()
    for L, Rm in ((A, A), (A, P), (Pt, AP), (R, A), (big, big), (A, A)):
        ref, S = oracle_ref(L, Rm)
        got, _ = run(L, Rm, handle=h)
        check_f64(ref, S, got)


def test_numeric_rejects_missing_or_different_plan():
    """Numeric before any symbolic phase, with operands other than the plan's,
    or with C of another size: clear errors, and the handle still works."""
    import torch

    import paper_1801_03065_amd as spg

    A = synth.stencil27(4)
    A2 = synth.stencil27(5)
    h = spg.Handle()
    dA, dA2 = dev(A), dev(A2)
    rp0 = torch.zeros(A.nrows + 1, dtype=torch.int32, device="cuda")
    with pytest.raises(spg.SpgemmError) as ei:
        spg.spgemm_numeric(h, dA, dA, rp0, 1)
    assert ei.value.status == spg.SPG_ERR_NOT_READY
    rp, nnz = spg.spgemm_symbolic(h, dA, dA)
    with pytest.raises(spg.SpgemmError) as ei:
        spg.spgemm_numeric(h, dA2, dA2, rp, nnz)
    assert ei.value.status in (spg.SPG_ERR_STRUCTURE_MISMATCH, spg.SPG_ERR_DIM_MISMATCH)
    with pytest.raises(spg.SpgemmError) as ei:
        spg.spgemm_numeric(h, dA, dA, rp, nnz - 1)
    assert ei.value.status == spg.SPG_ERR_STRUCTURE_MISMATCH
    C = spg.spgemm_numeric(h, dA, dA, rp, nnz)
    h.check_errors()
    torch.cuda.synchronize()
    ref, S = oracle_ref(A, A)
    check_f64(ref, S, (rp.cpu().numpy().astype(np.int64), C.col_idx.cpu().numpy(), C.values.cpu().numpy()))


def _runs_matrix(m, n, seed):
    """Rows made of runs of consecutive columns (1..12 long, up to 70 entries
    per row): their B rows lie back to back in B's storage."""
    rng = np.random.default_rng(seed)
    rows = []
    for _ in range(m):
        cols = set()
        for _ in range(int(rng.integers(0, 8))):
            s0, ln = int(rng.integers(0, n - 12)), int(rng.integers(1, 13))
            cols.update(range(s0, s0 + ln))
        rows.append(sorted(cols)[:70])
    rp = np.zeros(m + 1, dtype=np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    ci = np.array([c for r in rows for c in r], dtype=np.int32)
    return synth.Csr(m, n, rp, ci, rng.standard_normal(ci.size))


@pytest.mark.parametrize("comp", [-1, 0, 1])
def test_bit_window_rows_of_column_runs(comp):
    """Bit-window kernels on rows made of runs of consecutive columns (B rows
    back to back in B's storage), with empty B rows inside the runs, B rows
    longer than a lane group, rows beyond the fast path's slots and rows of
    more than 64 entries; compression by the rule, off and on."""
    rng = np.random.default_rng(21)
    n = 2500
    A = _runs_matrix(500, n, 22)
    lens = np.where(rng.random(n) < 0.2, 0, rng.integers(1, 40, n))
    B = synth.random_csr(n, 3000, lens, 23)
    ref, S = oracle_ref(A, B)
    got, h = run(A, B, accumulator=1, compression=comp)
    check_f64(ref, S, got)
    st = h.stats()
    assert st["rows_symbolic"]["dense_wave"] > 0
