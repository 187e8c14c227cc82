"""GPU parity of the masked product (A*B on a mask's pattern) and its
structural form (path counts), against the oracle's plain definition.
Counts are integers: exact.  Values: FP64 within 1e-12 * max(|c|, S), FP32
(accumulated in FP64, rounded once) within 1e-5 * S."""
import numpy as np
import pytest

import oracle
import synth
from helpers import dev, f32_inputs

pytestmark = pytest.mark.gpu


def _lower(A):
    rows = np.repeat(np.arange(A.nrows), A.row_lengths())
    keep = A.col_idx < rows
    r, c = rows[keep], A.col_idx[keep]
    rp = np.zeros(A.nrows + 1, dtype=np.int64)
    np.add.at(rp, r + 1, 1)
    return synth.Csr(A.nrows, A.ncols, np.cumsum(rp), c.astype(np.int32), np.ones(c.size))


def _gpu(A, B, M, structural=False, dtype="f64"):
    import torch

    import paper_1801_03065_amd as spg

    h = spg.Handle()
    dA, dB, dM = dev(A, dtype), dev(B, dtype), dev(M, dtype)
    if structural:
        dA, dB = dA.with_values(dA.values), dB.with_values(dB.values)
    out = spg.spgemm_masked(h, dA, dB, dM, structural=structural)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_masked_random(seed, dtype):
    rng = np.random.default_rng(seed)
    m, n, k = 600, 500, 4000
    lens_m = np.where(rng.random(m) < 0.05, 1500, rng.integers(0, 60, m))  # some rows of the workgroup kind
    A = synth.shuffle_columns(synth.random_csr(m, n, rng.integers(0, 40, m), seed), seed + 1)
    B = synth.shuffle_columns(synth.random_csr(n, k, rng.integers(0, 50, n), seed + 2), seed + 3)
    M = synth.shuffle_columns(synth.random_csr(m, k, lens_m, seed + 4), seed + 5)
    A0, B0 = (A, B) if dtype == "f64" else (f32_inputs(A), f32_inputs(B))
    want, S = oracle.masked(A0, B0, M, with_abs=True)
    got = _gpu(A, B, M, dtype=dtype)
    tol = 1e-12 * np.maximum(np.abs(want), S) if dtype == "f64" else 1e-5 * S
    assert np.all(np.abs(got - want) <= tol)
    cnt = oracle.masked(A, B, M, structural=True)
    assert np.array_equal(_gpu(A, B, M, structural=True, dtype=dtype), cnt)


@pytest.mark.parametrize("scale", [10, 13])
def test_triangle_counts_rmat(scale):
    G = synth.rmat_symmetric(scale, 16, seed=scale)
    L = _lower(G)
    want = oracle.masked(L, L, L, structural=True)
    got = _gpu(L, L, L, structural=True)
    assert np.array_equal(got, want)
    # the full adjacency as the mask (hub rows take the workgroup kind):
    # every triangle is counted six times
    want6 = oracle.masked(G, G, G, structural=True)
    got6 = _gpu(G, G, G, structural=True)
    assert np.array_equal(got6, want6)
    assert got6.sum() == 6 * got.sum()
    print(f"R-MAT scale {scale}: {int(got.sum())} triangles, longest mask row {G.row_lengths().max()}")


def test_masked_degenerate():
    A = synth.tiny_random(5, 4, 0.5, 1)
    B = synth.tiny_random(4, 6, 0.5, 2)
    empty = synth.Csr(5, 6, np.zeros(6, dtype=np.int64), np.zeros(0, np.int32), np.zeros(0))
    assert _gpu(A, B, empty).size == 0
    full = synth.Csr(5, 6, np.arange(0, 31, 6, dtype=np.int64), np.tile(np.arange(6, dtype=np.int32), 5),
                     np.ones(30))
    Az = synth.Csr(5, 4, np.zeros(6, dtype=np.int64), np.zeros(0, np.int32), np.zeros(0))  # A with no entries
    assert np.array_equal(_gpu(Az, B, full), np.zeros(30))
    assert np.allclose(_gpu(A, B, full), oracle.masked(A, B, full), rtol=1e-13, atol=1e-13)
