"""Heavy rows of C in column segments (one workgroup per row, LDS segments cut
by the symbolic phase) against the oracle, element by element.

The cases aim at each step of the segmented path: rows whose A entries fit one
chunk of 512 (a cursor per B row moves from segment to segment) and rows with
several chunks (cursors kept in scratch between segments; these rows, longer
than FP32's term limit, share the launch of the others and are taken first),
dense words (a cut falls inside a run of full words), wide windows with few
entries (segments cut only at the aligned word groups), windows far from
column 0, the FP32 forms, row panels, and B with unsorted rows (the
window-wide kernel instead).
"""
import numpy as np
import pytest

import synth
from helpers import check_f32, check_f64, check_structure, dev, f32_inputs, oracle_ref, run

pytestmark = pytest.mark.gpu


def _heavy(counts_a, rows, n, k, b_lo, b_hi, seed):
    rng = np.random.default_rng(seed)
    counts = rng.integers(0, 4, rows)
    for r, c in counts_a.items():
        counts[r] = c
    A = synth.random_csr(rows, n, counts, seed + 1)
    B = synth.random_csr(n, k, rng.integers(b_lo, b_hi, n), seed + 2)
    return A, B


def _contiguous_rows(n, k, lens, starts, seed):
    """n x k matrix whose row r holds columns starts[r] .. starts[r]+lens[r]-1."""
    rng = np.random.default_rng(seed)
    rp = np.zeros(n + 1, np.int64)
    np.cumsum(lens, out=rp[1:])
    ci = np.concatenate([np.arange(s, s + L, dtype=np.int32) for s, L in zip(starts, lens)])
    return synth.Csr(n, k, rp, ci, rng.standard_normal(ci.shape[0]))


def test_one_chunk_many_segments():
    """Heavy rows of one chunk (<= 512 A entries) over long B rows: tens of segments."""
    A, B = _heavy({3: 200, 40: 120, 41: 256, 99: 60}, 120, 700, 1 << 20, 300, 3000, 101)
    ref, S = oracle_ref(A, B)
    got, h = run(A, B)
    check_f64(ref, S, got)
    st = h.stats()
    assert st["rows_numeric"]["dense_wg"] >= 4
    assert st["max_row_nnz"] > 20 * 4096  # many segments


def test_many_chunks_many_segments():
    """Heavy rows of exactly one chunk (512 A entries) and of several (513, 900, 2000)."""
    A, B = _heavy({0: 512, 5: 513, 17: 900, 50: 2000}, 80, 3000, 1 << 20, 20, 400, 202)
    ref, S = oracle_ref(A, B)
    got, h = run(A, B)
    check_f64(ref, S, got)
    assert h.stats()["rows_numeric"]["dense_wg"] >= 3


def test_dense_words_cut_inside_runs():
    """B rows are contiguous column blocks: C rows are dense runs of full words,
    so segment cuts fall inside them."""
    rng = np.random.default_rng(303)
    n, k = 400, 300000
    lens = rng.integers(200, 6000, n)
    starts = rng.integers(0, k - 6000, n)
    B = _contiguous_rows(n, k, lens, starts, 304)
    counts = rng.integers(0, 3, 64)
    counts[[1, 30, 63]] = [40, 150, 300]
    A = synth.random_csr(64, n, counts, 305)
    ref, S = oracle_ref(A, B)
    got, h = run(A, B)
    check_f64(ref, S, got)
    assert h.stats()["rows_numeric"]["dense_wg"] >= 3


def test_wide_window_few_entries_group_cuts():
    """Rows of 1100-3000 entries spread over 2^20 columns: one segment would
    hold them, but their words span several aligned groups."""
    A, B = _heavy({2: 60, 9: 90, 33: 150}, 40, 500, 1 << 20, 15, 25, 404)
    ref, S = oracle_ref(A, B)
    got, h = run(A, B)
    check_f64(ref, S, got)
    assert h.stats()["rows_numeric"]["dense_wg"] >= 1


def test_window_far_from_zero_dense_policy():
    """Heavy rows whose window starts at column 2^20 + 12345; the dense policy
    sends every row it can to the bit-window kinds."""
    A, B0 = _heavy({5: 180, 6: 700}, 30, 800, 600000, 100, 900, 505)
    B = synth.Csr(B0.nrows, 1700000, B0.row_ptr, (B0.col_idx + (1 << 20) + 12345).astype(np.int32), B0.values)
    ref, S = oracle_ref(A, B)
    for acc in (0, 1):
        got, h = run(A, B, accumulator=acc)
        check_f64(ref, S, got)
        assert h.stats()["rows_numeric"]["dense_wg"] >= 2


@pytest.mark.parametrize("mode", ["plain", "compensated", "wide", "heavy_fp64"])
def test_fp32_forms_on_segments(mode):
    A, B = _heavy({3: 200, 40: 700}, 60, 900, 1 << 20, 100, 1500, 606)
    A32, B32 = f32_inputs(A), f32_inputs(B)
    ref, S = oracle_ref(A32, B32)
    opts = {"plain": {}, "compensated": {"fp32_mode": 1}, "wide": {"fp32_mode": 2},
            "heavy_fp64": {"fp64_heavy_row_flops": 1 << 14}}[mode]
    got, h = run(A32, B32, dtype="f32", **opts)
    check_f32(ref, S, got, rel=1e-5 if mode == "plain" else 1e-6)
    assert h.stats()["rows_numeric"]["dense_wg"] >= 2 or mode == "heavy_fp64"


def test_fp32_rows_past_term_limit_accumulate_in_fp64():
    """FP32 values: segmented rows longer than the FP32 term limit (167 A
    entries) share the other rows' launch but accumulate in FP64.  About 40
    terms meet in each entry of C, so FP32 accumulation shows (the plain mode
    exceeds 1e-7 S somewhere) while FP64 accumulation leaves only the final
    rounding to FP32 (below 1e-7 S on every entry of those rows)."""
    rng = np.random.default_rng(909)
    counts = rng.integers(20, 120, 6)
    counts[[1, 4]] = 900
    A = synth.random_csr(6, 2000, counts, 910)
    B = synth.random_csr(2000, 70000, np.full(2000, 3000), 911)
    A32, B32 = f32_inputs(A), f32_inputs(B)
    ref, S = oracle_ref(A32, B32)
    heavy = np.concatenate([np.arange(ref.row_ptr[i], ref.row_ptr[i + 1]) for i in (1, 4)])

    def rel_err(got):
        check_structure(ref, got)
        return np.abs(got[2].astype(np.float64) - ref.values) / np.maximum(S, 1e-300)

    plain, _ = run(A32, B32, dtype="f32", fp32_terms_max=0)
    got, h = run(A32, B32, dtype="f32")
    st = h.stats()
    assert st["rows_numeric"]["dense_wg"] >= 2 and st["fp64_rows"] >= 2
    assert rel_err(plain)[heavy].max() > 1e-7
    e = rel_err(got)
    assert e[heavy].max() <= 1e-7
    assert e.max() <= 1e-5


def test_panels_through_segmented_rows():
    """spgemm_numeric_rows with panel edges next to and around heavy rows."""
    import torch

    import paper_1801_03065_amd as spg

    A, B = _heavy({4: 230, 5: 600, 20: 90}, 40, 900, 1 << 20, 100, 1200, 707)
    ref, S = oracle_ref(A, B)
    h = spg.Handle()
    dA, dB = dev(A), dev(B)
    rp, nnz = spg.spgemm_symbolic(h, dA, dB, torch.int64)
    rph = rp.cpu().numpy()
    ci = np.zeros(nnz, np.int32)
    va = np.zeros(nnz)
    cuts = [0, 4, 5, 6, 20, 21, 40]
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


def test_unsorted_b_heavy_rows_window_kernel():
    """B with unsorted rows: heavy rows take the window-wide kernel."""
    A, B0 = _heavy({3: 300, 8: 60}, 20, 600, 200000, 50, 400, 808)
    B = synth.shuffle_columns(B0, 809)
    ref, S = oracle_ref(A, B)
    got, h = run(A, B)
    check_f64(ref, S, got)
    assert h.stats()["rows_numeric"]["dense_wg"] >= 1


def test_rmat13_square_reuse():
    """R-MAT scale 13 squared (hub rows of B, power-law A rows), twice with
    fresh values on the same plan."""
    import torch

    import paper_1801_03065_amd as spg

    A = synth.rmat_symmetric(13, 16, seed=4)
    h = spg.Handle()
    dA = dev(A)
    rp, nnz = spg.spgemm_symbolic(h, dA, dA, torch.int64)
    assert h.stats()["rows_numeric"]["dense_wg"] > 0
    for seed in (0, 1):
        A2 = A if seed == 0 else synth.revalue(A, 77)
        d2 = dA.with_values(torch.as_tensor(A2.values, device="cuda"))  # the plan's structure tensors
        C = spg.spgemm_numeric(h, d2, d2, rp, nnz)
        h.check_errors()
        torch.cuda.synchronize()
        ref, S = oracle_ref(A2, A2)
        check_f64(ref, S, (rp.cpu().numpy().astype(np.int64), C.col_idx.cpu().numpy(), C.values.cpu().numpy()))
