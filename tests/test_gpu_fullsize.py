"""GPU parity at the full sizes of the benchmark and form workloads, in the
launch configurations bench.py times.

* 27-point A*A on 100^3 and the Galerkin chain P^T*(A*P): every entry against
  the oracle (the oracle finishes the 705M multiplications in seconds).
* R-MAT scale 20 squared (C has 2.37e10 entries): row sizes on sampled rows,
  values on row panels (the heaviest rows, a random band, the last rows) in
  FP64, FP32 with FP64 accumulation of the heaviest rows, and compensated FP32.
* 512-product batch: one batched symbolic and numeric launch over all of them,
  sampled products checked in full.
* Differentiation on the 7-point 64^3 Laplacian times a 16-per-row random
  matrix: forward and backward against the oracle gradient on every entry, and
  FP64 central differences on 1,000 sampled entries.
"""
import numpy as np
import pytest

import oracle
import synth
from helpers import check_f32, check_f64, check_structure, dev, f32_inputs, oracle_ref, run

pytestmark = pytest.mark.gpu


def test_27pt_100_square_and_galerkin_every_entry():
    A = synth.stencil27(100)
    P, Pt = synth.aggregation_2x2x2(100)
    ref, S = oracle_ref(A, A)
    got, h = run(A, A)
    assert ref.nnz == 494 ** 3 and h.stats()["flops"] == 890 ** 3
    check_f64(ref, S, got)
    del ref, S, got
    AP, SAP = oracle_ref(A, P)
    got, _ = run(A, P)
    check_f64(AP, SAP, got)
    R, SR = oracle_ref(Pt, AP)
    got, _ = run(Pt, AP)
    assert R.nnz == 148 ** 3
    check_f64(R, SR, got)


def _panel(h, dA, rp, rb, re, dtype):
    import torch

    import paper_1801_03065_amd as spg

    n = int(rp[re] - rp[rb])
    ci = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    va = torch.empty(max(n, 1), dtype=dtype, device="cuda")
    spg.spgemm_numeric_rows(h, dA, dA, rb, re, ci, va)
    h.check_errors()
    torch.cuda.synchronize()
    lrp = (rp[rb:re + 1] - rp[rb]).astype(np.int64)
    return lrp, ci[:n].cpu().numpy(), va[:n].cpu().numpy()


@pytest.mark.timeout(600)
def test_rmat20_square_sampled_rows_and_panels():
    import torch

    import paper_1801_03065_amd as spg

    A = synth.rmat_symmetric(20, 16, seed=1)
    fm, maxrf, fl = oracle.flops(A, A)
    rng = np.random.default_rng(3)
    heavy = np.argsort(fl)[-8:]
    band = int(rng.integers(0, A.nrows - 2048))
    panels = [(int(i), int(i) + 1) for i in heavy] + [(band, band + 2048), (A.nrows - 512, A.nrows)]
    A32 = f32_inputs(A)
    for dtype, opts in ((torch.float64, {}), (torch.float32, {"fp64_heavy_row_flops": 1 << 16}),
                        (torch.float32, {"fp32_mode": 1})):
        h = spg.Handle(**opts)
        dA = dev(A, "f64" if dtype == torch.float64 else "f32")
        rp_t, nnz = spg.spgemm_symbolic(h, dA, dA, torch.int64)
        st = h.stats()
        assert st["flops"] == fm and st["max_row_flops"] == maxrf
        rp = rp_t.cpu().numpy().astype(np.int64)
        if dtype == torch.float64:
            sel = np.unique(np.concatenate([heavy, rng.integers(0, A.nrows, 5000)]))
            orp = oracle.rows(A, A, sel)[0]
            assert np.array_equal(np.diff(orp), rp[sel + 1] - rp[sel])
        for rb, re in panels:
            got = _panel(h, dA, rp, rb, re, dtype)
            Ain = A if dtype == torch.float64 else A32
            orp, oci, oval, oS = oracle.rows(Ain, Ain, np.arange(rb, re))
            ref = synth.Csr(re - rb, A.ncols, orp, oci, oval)
            if dtype == torch.float64:
                check_f64(ref, oS, got)
            else:
                check_f32(ref, oS, got)
        h.close()
        del dA
        torch.cuda.empty_cache()


@pytest.mark.timeout(600)
def test_batch_512_one_launch_sampled_products():
    import torch

    import paper_1801_03065_amd as spg

    specs = synth.batch_specs(512, 42)
    pairs = synth.batch_matrices(specs)  # in-process: no child processes beside the GPU
    As = spg.pack_batch([p[0] for p in pairs])
    Bs = spg.pack_batch([p[1] for p in pairs])
    h = spg.Handle(autotune=1)
    rps, nnzs = spg.spgemm_batch_symbolic(h, As, Bs)
    Cs = spg.batch_outputs(As, Bs, rps, nnzs, torch.float64)
    spg.spgemm_batch_numeric(h, As, Bs, Cs)
    torch.cuda.synchronize()
    h.check_errors()
    ns = np.array([s.n for s in specs])
    rng = np.random.default_rng(9)
    sample = np.unique(np.concatenate([[0, 511, int(np.argmax(ns)), int(np.argmin(ns))],
                                       rng.integers(0, 512, 4)]))
    for i in sample:
        A, B = pairs[i]
        ref, S = oracle_ref(A, B)
        assert nnzs[i] == ref.nnz
        C = Cs[i]
        check_f64(ref, S, (C.row_ptr.cpu().numpy().astype(np.int64), C.col_idx.cpu().numpy(),
                           C.values.cpu().numpy()))
    assert sum(nnzs) == h.stats()["nnz_c"]


def test_backward_7pt_64_every_entry_and_finite_differences():
    import torch

    import paper_1801_03065_amd as spg

    A = synth.laplace7(64)
    B = synth.fixed_row_random(A.ncols, A.ncols, 16, 5)
    A32, B32 = f32_inputs(A), f32_inputs(B)
    # FP32 forward + backward through the autograd Function
    dA32, dB32 = dev(A, "f32"), dev(B, "f32")
    prod = spg.SparseProduct(dA32, dB32)
    a = dA32.values.clone().requires_grad_(True)
    b = dB32.values.clone().requires_grad_(True)
    c = prod(a, b)
    C = oracle.spgemm(A32, B32)
    Cs = prod.structure()
    check_structure(C, (Cs.row_ptr.cpu().numpy().astype(np.int64), Cs.col_idx.cpu().numpy(), None))
    G = np.random.default_rng(1).standard_normal(C.nnz).astype(np.float32)
    c.backward(torch.as_tensor(G, device="cuda"))
    torch.cuda.synchronize()
    G64 = G.astype(np.float64)
    rdA, rdB = oracle.grad(A32, B32, C, G64)
    sA, sB = oracle.grad(A32.with_values(np.abs(A32.values)), B32.with_values(np.abs(B32.values)), C, np.abs(G64))
    dA, dB = a.grad.cpu().numpy().astype(np.float64), b.grad.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(dA - rdA) <= 1e-5 * sA)
    assert np.all(np.abs(dB - rdB) <= 1e-5 * sB)
    # FP64 central differences of L = sum(G * C) on 1,000 sampled entries (L is
    # bilinear: no truncation error; tolerance = rounding noise of L over 2h)
    dA64, dB64 = dev(A32), dev(B32)
    p64 = spg.SparseProduct(dA64, dB64)
    Gd = torch.as_tensor(G64, device="cuda")
    a64, b64 = dA64.values.clone(), dB64.values.clone()
    with torch.no_grad():
        noise = float((p64(a64, b64) * Gd).abs().sum()) * 2.0 ** -52
        hstep = 1e-6
        tol = 4 * noise / (2 * hstep)
        rng = np.random.default_rng(2)
        for which, n, ref in (("a", A.nnz, rdA), ("b", B.nnz, rdB)):
            for e in rng.integers(0, n, 500):
                xp, xm = (a64.clone(), a64.clone()) if which == "a" else (b64.clone(), b64.clone())
                xp[e] += hstep
                xm[e] -= hstep
                if which == "a":
                    lp, lm = float((p64(xp, b64) * Gd).sum()), float((p64(xm, b64) * Gd).sum())
                else:
                    lp, lm = float((p64(a64, xp) * Gd).sum()), float((p64(a64, xm) * Gd).sum())
                fd = (lp - lm) / (2 * hstep)
                assert abs(fd - ref[e]) <= tol + 1e-12 * abs(ref[e]), (which, e, fd, ref[e], tol)
