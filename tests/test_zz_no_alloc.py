"""spgemm_numeric_noalloc against spgemm_numeric and the oracle.

The allocation-free numeric entry point takes its heavy-row scratch from the
library's static device array.  Each case runs two products in a row on one
handle, the second smaller than the first, and checks the allocation-free
result against the allocating entry point's (same kernels: structure equal,
values within the FP64 tolerance) and against the oracle.  The cases use the
kinds that need scratch: heavy rows of unsorted B (value windows), the
two-level hash with a tiny level 1 (level-2 tables), heavy rows in segments
with long rows of A (per-entry cursors).
"""
import numpy as np
import pytest

import oracle
import synth
from helpers import check_f64, dev, oracle_ref

pytestmark = pytest.mark.gpu


def _heavy_unsorted(m, seed):
    rng = np.random.default_rng(seed)
    n, k = 3000, 40000
    B = synth.shuffle_columns(synth.random_csr(n, k, rng.integers(20, 80, n), seed), seed + 1)
    A = synth.random_csr(m, n, rng.integers(100, 400, m), seed + 2)
    return A, B


def _long_a_rows(m, seed):
    rng = np.random.default_rng(seed)
    n, k = 4000, 200000
    B = synth.random_csr(n, k, rng.integers(50, 200, n), seed)
    A = synth.random_csr(m, n, rng.integers(300, 1200, m), seed + 1)
    return A, B


CASES = {
    "unsorted_heavy": (_heavy_unsorted, {}),
    "two_level_hash": (_heavy_unsorted, {"accumulator": 3, "l1_hash_slots": 64}),
    "segments_long_a": (_long_a_rows, {}),
}


def _both(h, A, B):
    import torch

    import paper_1801_03065_amd as spg

    dA, dB = dev(A), dev(B)
    rp, nnz = spg.spgemm_symbolic(h, dA, dB)
    C1 = spg.spgemm_numeric(h, dA, dB, rp, nnz)
    h.check_errors()
    C2 = spg.DeviceCsr(A.nrows, B.ncols, rp, torch.full_like(C1.col_idx, -1), torch.full_like(C1.values, np.nan))
    spg.spgemm_numeric_noalloc(h, dA, dB, C2)
    h.check_errors()
    torch.cuda.synchronize()
    r = rp.cpu().numpy().astype(np.int64)
    return (r, C1.col_idx.cpu().numpy(), C1.values.cpu().numpy()), (r, C2.col_idx.cpu().numpy(), C2.values.cpu().numpy())


@pytest.mark.parametrize("case", sorted(CASES))
def test_noalloc_matches_numeric(case):
    import paper_1801_03065_amd as spg

    make, opts = CASES[case]
    h = spg.Handle(**opts)
    for m, seed in ((900, 5), (250, 8)):  # the second product is smaller
        A, B = make(m, seed)
        ref, S = oracle_ref(A, B)
        got_alloc, got_free = _both(h, A, B)
        assert np.array_equal(got_free[1], got_alloc[1])
        scale = np.maximum(np.abs(got_alloc[2]), S)
        assert np.all(np.abs(got_free[2] - got_alloc[2]) <= 1e-12 * scale)
        check_f64(ref, S, got_free)
        used = {k for k, v in h.stats()["rows_numeric"].items() if v}
        print(f"{case} m={m}: kinds {sorted(used)}")
        if case == "two_level_hash":
            assert "hash_two_level" in used
        else:
            assert used & {"dense_wg"}, used
