"""GPU parity of the FP32 forms and of the backward against the FP64 oracle.

FP32: the oracle runs on the FP32-rounded inputs in FP64, so only the GPU's
accumulation error is measured: |err| <= 1e-5 * S (S = sum |a*b| per entry).
Compensated pairs (Dot2) and FP64 accumulation must also meet their own
bounds: about one rounding of the result, u*|c| with u = 2^-24, plus a
second-order term.
Backward: dA = (G B^T) on pattern(A), dB = (A^T G) on pattern(B) against the
oracle gradient (FP64: 1e-12 relative to sum |terms|) and against central
finite differences of the GPU's own forward.
"""
import numpy as np
import pytest

import oracle
import synth
from helpers import check_f32, dev, f32_inputs, oracle_ref, run

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def _random_pair(seed, m=500, n=400, k=3000, ra=20, rb=30):
    rng = np.random.default_rng(seed)
    A = synth.shuffle_columns(synth.random_csr(m, n, rng.integers(0, ra, m), seed), seed)
    B = synth.random_csr(n, k, rng.integers(0, rb, n), seed + 5)
    return A, B


@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("acc", [0, 1, 2, 3])
def test_fp32_modes(mode, acc):
    A, B = _random_pair(3)
    A32, B32 = f32_inputs(A), f32_inputs(B)
    ref, S = oracle_ref(A32, B32)
    got, _ = run(A, B, dtype="f32", fp32_mode=mode, accumulator=acc, l1_hash_slots=64 if acc == 3 else 0)
    mx, med = check_f32(ref, S, got)
    err = np.abs(got[2].astype(np.float64) - ref.values)
    print(f"fp32 mode {mode} acc {acc}: max rel-to-S {mx:.3e} median {med:.3e}")
    if mode in (1, 2):
        assert np.all(err <= U32 * np.abs(ref.values) + 1e-9 * S)


def test_fp32_compensated_beats_plain_on_cancellation():
    """Rows whose terms cancel: the compensated pair keeps the small result."""
    rng = np.random.default_rng(9)
    m, n, k = 300, 64, 50
    A = synth.random_csr(m, n, np.full(m, 16), 1)
    A = A.with_values(np.ones(A.nnz))
    big = rng.choice([-1.0, 1.0], size=(n, k)) * 4096.0
    small = rng.standard_normal((n, k)) * 1e-3
    dense = (big + small).astype(np.float32).astype(np.float64)
    rp = np.arange(0, n * k + 1, k, dtype=np.int64)
    B = synth.Csr(n, k, rp, np.tile(np.arange(k, dtype=np.int32), n), dense.reshape(-1))
    ref, S = oracle_ref(A, B)
    errs = {}
    for mode in (0, 1):
        got, _ = run(A, B, dtype="f32", fp32_mode=mode)
        errs[mode] = np.abs(got[2].astype(np.float64) - ref.values)
    assert errs[1].max() <= U32 * np.abs(ref.values).max() + 1e-9 * S.max()
    assert errs[1].max() < errs[0].max()
    print(f"cancellation: plain max err {errs[0].max():.3e}, compensated {errs[1].max():.3e}")


def test_fp32_integer_stencil_exact():
    A = synth.stencil27(7)
    ref = oracle.spgemm(A, A)
    for mode in (0, 1, 2):
        got, _ = run(A, A, dtype="f32", fp32_mode=mode)
        assert np.array_equal(got[1], ref.col_idx)
        assert np.array_equal(got[2].astype(np.float64), ref.values)


# ---------------------------------------------------------------- backward
def _grad_gpu(A, B, G, dtype="f64"):
    import torch

    import paper_1801_03065_amd as spg

    h = spg.Handle()
    dA_, dB_ = dev(A, dtype), dev(B, dtype)
    rp, nnz = spg.spgemm_symbolic(h, dA_, dB_)
    C = spg.spgemm_numeric(h, dA_, dB_, rp, nnz)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    Gd = spg.DeviceCsr(C.nrows, C.ncols, rp, C.col_idx, torch.as_tensor(G, dtype=tdt, device="cuda"))
    dA, dB = spg.spgemm_backward(h, dA_, dB_, Gd)
    h.check_errors()
    torch.cuda.synchronize()
    return dA.cpu().numpy().astype(np.float64), dB.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("seed", range(4))
def test_backward_matches_oracle_gradient(seed):
    A, B = _random_pair(seed, m=300, n=200, k=900)
    C = oracle.spgemm(A, B)
    G = np.random.default_rng(seed + 100).standard_normal(C.nnz)
    rdA, rdB = oracle.grad(A, B, C, G)
    sA, sB = oracle.grad(A.with_values(np.abs(A.values)), B.with_values(np.abs(B.values)), C, np.abs(G))
    dA, dB = _grad_gpu(A, B, G)
    assert np.all(np.abs(dA - rdA) <= 1e-12 * np.maximum(sA, 1e-300))
    assert np.all(np.abs(dB - rdB) <= 1e-12 * np.maximum(sB, 1e-300))


def test_backward_fp32_and_stencil_times_random():
    """The differentiation workload's shape at 12^3: 7-point Laplacian times 16 random columns per row."""
    A = synth.laplace7(12)
    B = synth.fixed_row_random(A.ncols, A.ncols, 16, 7)
    A32, B32 = f32_inputs(A), f32_inputs(B)
    C = oracle.spgemm(A32, B32)
    G = np.random.default_rng(1).standard_normal(C.nnz).astype(np.float32).astype(np.float64)
    rdA, rdB = oracle.grad(A32, B32, C, G)
    sA, sB = oracle.grad(A32.with_values(np.abs(A32.values)), B32.with_values(np.abs(B32.values)), C, np.abs(G))
    dA, dB = _grad_gpu(A, B, G, "f32")
    assert np.all(np.abs(dA - rdA) <= 1e-5 * sA)
    assert np.all(np.abs(dB - rdB) <= 1e-5 * sB)


def test_backward_finite_differences_and_autograd():
    """L = sum(G * C) is bilinear: central differences of the GPU forward are exact up to rounding."""
    import torch

    import paper_1801_03065_amd as spg

    A = synth.laplace7(6)
    B = synth.fixed_row_random(A.ncols, A.ncols, 16, 3)
    dA_, dB_ = dev(A), dev(B)
    prod = spg.SparseProduct(dA_, dB_)
    a = dA_.values.clone().requires_grad_(True)
    b = dB_.values.clone().requires_grad_(True)
    cvals = prod(a, b)
    G = torch.randn(cvals.shape, dtype=torch.float64, device="cuda")
    loss = (cvals * G).sum()
    loss.backward()
    rng = np.random.default_rng(0)
    h = 1e-6

    def L(av, bv):
        return float((prod(av, bv) * G).sum())

    with torch.no_grad():
        for e in rng.integers(0, A.nnz, 40):
            ap, am = a.detach().clone(), a.detach().clone()
            ap[e] += h
            am[e] -= h
            fd = (L(ap, b.detach()) - L(am, b.detach())) / (2 * h)
            assert abs(fd - float(a.grad[e])) <= 1e-6 * (1 + abs(fd))
        for f in rng.integers(0, B.nnz, 40):
            bp, bm = b.detach().clone(), b.detach().clone()
            bp[f] += h
            bm[f] -= h
            fd = (L(a.detach(), bp) - L(a.detach(), bm)) / (2 * h)
            assert abs(fd - float(b.grad[f])) <= 1e-6 * (1 + abs(fd))
    # and against the oracle gradient
    C = oracle.spgemm(A, B)
    rdA, rdB = oracle.grad(A, B, C, G.cpu().numpy())
    assert np.allclose(a.grad.cpu().numpy(), rdA, rtol=1e-12, atol=1e-12)
    assert np.allclose(b.grad.cpu().numpy(), rdB, rtol=1e-12, atol=1e-12)


def test_fp32_heaviest_rows_in_fp64():
    """Rows at or above the flop threshold accumulate in FP64 (error about one rounding of the
    result); the rest keep plain FP32 accumulation."""
    rng = np.random.default_rng(17)
    counts = rng.integers(1, 8, 400)
    counts[[3, 200, 399]] = [300, 250, 400]
    A = synth.random_csr(400, 500, counts, 2)
    B = synth.random_csr(500, 800, rng.integers(1, 25, 500), 3)
    A32, B32 = f32_inputs(A), f32_inputs(B)
    ref, S = oracle_ref(A32, B32)
    thr = 2000
    got, h = run(A, B, dtype="f32", fp32_mode=0, fp64_heavy_row_flops=thr)
    check_f32(ref, S, got)
    fl = oracle.flops(A32, B32)[2]
    heavy = np.nonzero(fl >= thr)[0]
    assert heavy.size >= 3
    err = np.abs(got[2].astype(np.float64) - ref.values)
    for i in heavy:
        s, e = ref.row_ptr[i], ref.row_ptr[i + 1]
        assert np.all(err[s:e] <= U32 * np.abs(ref.values[s:e]) + 1e-12 * S[s:e])
