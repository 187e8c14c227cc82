"""The three forms beside the plain FP64 method, measured on one MI355X
(used by `bench.py --forms precision,batch,backward`).

precision: symmetric R-MAT square (scale --rmat-scale, edge factor 16,
    (0.57, 0.19, 0.19, 0.05)); one symbolic, then numeric in FP64, FP32,
    FP32 + compensated pairs, FP32 with FP64 accumulation, and FP32 with FP64
    accumulation for the rows of at least 2^16 multiplications only.  Errors are stated
    against the FP64 oracle on sampled rows (the 200 heaviest rows and 2000
    uniform rows), relative to S = sum |a*b| per entry: max and median.
batch: --batch-count products (n_i ~ U[1000, 65536], Poisson(lambda_i) rows,
    lambda_i ~ U[4, 32]); one batched symbolic, then 10 numeric recomputations
    on fresh seeded values, each replayed from a captured HIP graph (the value
    refresh is not timed), FP64 and FP32; baseline = the same
    products as separate plain FP64 numeric calls.
backward: C = A*B, A = 7-point Laplacian on g^3 (--diff-grid), B random with 16
    columns per row, FP32; forward + backward vs the plain FP64 products
    G*B^T and A^T*G that the masked gradients are taken from.
"""
from __future__ import annotations

import time

import numpy as np


def _ev():
    import torch

    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def _time(fn, reps, stream):
    import torch

    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a, b = _ev()
        a.record(stream)
        fn()
        b.record(stream)
        ts.append((a, b))
    torch.cuda.synchronize()
    return float(np.mean([a.elapsed_time(b) for a, b in ts]))


def precision(args, log):
    import torch

    import oracle
    import paper_1801_03065_amd as spg
    import synth

    A = synth.rmat_symmetric(args.rmat_scale, 16, seed=1)
    log(f"[precision] R-MAT scale {args.rmat_scale}: n={A.nrows} nnz={A.nnz}")
    s = torch.cuda.Stream()
    res = {"workload": f"R-MAT scale {args.rmat_scale} squared", "n": A.nrows, "nnz_A": A.nnz}
    d64 = spg.DeviceCsr.from_arrays(A.nrows, A.ncols, A.row_ptr, A.col_idx, A.values)
    d32 = spg.DeviceCsr.from_arrays(A.nrows, A.ncols, A.row_ptr, A.col_idx, A.values, dtype=torch.float32)
    h = spg.Handle(stream=s)
    t0 = time.perf_counter()
    rp, nnz = spg.spgemm_symbolic(h, d64, d64, torch.int64)
    tsym = (time.perf_counter() - t0) * 1e3
    st = h.stats()
    fm = st["flops"]
    res.update({"flops_m": fm, "nnz_c": nnz, "symbolic_ms": round(tsym, 3),
                "rows_numeric": {k: v for k, v in st["rows_numeric"].items() if v}})
    # sampled rows for the error statement
    rf = np.diff(oracle.symbolic(A, A)) if A.nrows <= (1 << 16) else None
    rng = np.random.default_rng(0)
    fl = oracle.flops(A, A)[2]
    sel = np.unique(np.concatenate([np.argsort(fl)[-200:], rng.integers(0, A.nrows, 2000)]))
    A32 = A.with_values(A.values.astype(np.float32).astype(np.float64))
    orp, oci, oval, oS = oracle.rows(A32, A32, sel)
    _, _, oval64, oS64 = oracle.rows(A, A, sel)
    log(f"[precision] oracle: {sel.size} sampled rows")
    rp_h = rp.cpu().numpy()
    idx = np.concatenate([np.arange(rp_h[i], rp_h[i + 1]) for i in sel])
    idx_t = torch.as_tensor(idx, device="cuda")
    heavy = 1 << 16  # rows with at least this many multiplications
    modes = {"fp64": (d64, torch.float64, 0, 0), "fp32": (d32, torch.float32, 0, 0),
             "fp32_compensated": (d32, torch.float32, 1, 0), "fp32_wide": (d32, torch.float32, 2, 0),
             "fp32_heavy_rows_fp64": (d32, torch.float32, 0, heavy)}
    for name, (D, dt, mode, thr) in modes.items():
        hm = spg.Handle(stream=s, fp32_mode=mode, fp64_heavy_row_flops=thr)
        rpm, nnzm = spg.spgemm_symbolic(hm, D, D, torch.int64)
        ci = torch.empty(nnzm, dtype=torch.int32, device="cuda")
        va = torch.empty(nnzm, dtype=dt, device="cuda")
        C = spg.DeviceCsr(D.nrows, D.ncols, rpm, ci, va)
        ms = _time(lambda: spg.spgemm_numeric(hm, D, D, rpm, nnzm, out=C), 3, s)
        hm.check_errors()
        got_ci = C.col_idx[idx_t].cpu().numpy()
        got = C.values[idx_t].cpu().numpy().astype(np.float64)
        assert np.array_equal(got_ci, oci), name
        ref = oval if dt == torch.float32 else oval64
        S = oS if dt == torch.float32 else oS64
        rel = np.abs(got - ref) / np.maximum(S, 1e-300)
        res[name] = {"numeric_ms": round(ms, 3), "gflops": round(2 * fm / (ms * 1e-3) / 1e9, 1),
                     "err_rel_S_max": float(rel.max()), "err_rel_S_median": float(np.median(rel)),
                     "sampled_entries": int(idx.size)}
        log(f"[precision] {name}: {ms:.3f} ms, max err {rel.max():.3g} S")
        del C, ci, va
        hm.close()
        torch.cuda.empty_cache()
    res["fp32_heavy_rows_fp64"]["heavy_row_flops"] = heavy
    for k in ("fp32", "fp32_compensated", "fp32_wide", "fp32_heavy_rows_fp64"):
        res[k]["speedup_vs_fp64"] = round(res["fp64"]["numeric_ms"] / res[k]["numeric_ms"], 3)
    return res


def batch(args, log):
    import torch

    import paper_1801_03065_amd as spg
    import synth

    specs = synth.batch_specs(args.batch_count, 42)
    pairs = synth.batch_matrices(specs)
    log(f"[batch] {len(pairs)} products generated")
    s = torch.cuda.Stream()
    res = {"workload": f"{len(pairs)} products, n_i~U[1000,65536], Poisson rows lambda~U[4,32]"}
    for name, dt in (("fp64", torch.float64), ("fp32", torch.float32)):
        h = spg.Handle(stream=s, autotune=1)
        As = spg.pack_batch([p[0] for p in pairs], dtype=dt)
        Bs = spg.pack_batch([p[1] for p in pairs], dtype=dt)
        t0 = time.perf_counter()
        rps, nnzs = spg.spgemm_batch_symbolic(h, As, Bs)
        tsym = (time.perf_counter() - t0) * 1e3
        Cs = spg.batch_outputs(As, Bs, rps, nnzs, dt)
        with torch.cuda.stream(s):
            spg.spgemm_batch_numeric(h, As, Bs, Cs)  # first call: tuning + allocation
        s.synchronize()
        st = h.stats()
        fm = st["flops"]
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            spg.spgemm_batch_numeric(h, As, Bs, Cs)
        torch.cuda.synchronize()
        # 10 recomputations, each on fresh seeded values of the same structure
        # (written into the packed value arrays outside the timed replay)
        bases = [X[0].values._base if X[0].values._base is not None else X[0].values for X in (As, Bs)]
        gen = torch.Generator(device="cuda")
        ms = 0.0
        for r in range(10):
            with torch.cuda.stream(s):
                for t, base in enumerate(bases):
                    gen.manual_seed(1000 + 2 * r + t)
                    base.copy_(torch.randn(base.shape, generator=gen, device="cuda", dtype=dt))
                a, b = _ev()
                a.record(s)
                g.replay()
                b.record(s)
            torch.cuda.synchronize()
            ms += a.elapsed_time(b) / 10
        h.check_errors()
        res[name] = {"symbolic_ms": round(tsym, 3), "numeric_ms": round(ms, 3), "flops_m": fm,
                     "nnz_c": int(sum(nnzs)), "gflops": round(2 * fm / (ms * 1e-3) / 1e9, 1),
                     "tuned_policy": st["tuned_policy"], "tuned_lanes": st["tuned_lanes"],
                     "rows_numeric": {k: v for k, v in st["rows_numeric"].items() if v}}
        del Cs, As, Bs, g
        h.close()
        torch.cuda.empty_cache()
    # baseline: each product alone, plain FP64 numeric calls
    hs, ops = [], []
    for A, B in pairs:
        dA = spg.DeviceCsr.from_arrays(A.nrows, A.ncols, A.row_ptr, A.col_idx, A.values)
        dB = spg.DeviceCsr.from_arrays(B.nrows, B.ncols, B.row_ptr, B.col_idx, B.values)
        h = spg.Handle(stream=s)
        rp, nz = spg.spgemm_symbolic(h, dA, dB)
        C = spg.spgemm_numeric(h, dA, dB, rp, nz)
        hs.append(h)
        ops.append((dA, dB, rp, nz, C))
    torch.cuda.synchronize()
    a, b = _ev()
    a.record(s)
    for h, (dA, dB, rp, nz, C) in zip(hs, ops):
        spg.spgemm_numeric(h, dA, dB, rp, nz, out=C)
    b.record(s)
    torch.cuda.synchronize()
    tseq = a.elapsed_time(b)
    res["sequential_fp64_ms"] = round(tseq, 3)
    res["speedup_batched_fp64_vs_sequential"] = round(tseq / res["fp64"]["numeric_ms"], 3)
    res["speedup_batched_fp32_vs_sequential_fp64"] = round(tseq / res["fp32"]["numeric_ms"], 3)
    for h in hs:
        h.close()
    return res


def backward(args, log):
    import torch

    import paper_1801_03065_amd as spg
    import synth

    g = args.diff_grid
    A = synth.laplace7(g)
    B = synth.fixed_row_random(A.ncols, A.ncols, 16, 5)
    s = torch.cuda.Stream()
    res = {"workload": f"7-point {g}^3 times random 16 per row, FP32", "n": A.nrows}
    dA = spg.DeviceCsr.from_arrays(A.nrows, A.ncols, A.row_ptr, A.col_idx, A.values, dtype=torch.float32)
    dB = spg.DeviceCsr.from_arrays(B.nrows, B.ncols, B.row_ptr, B.col_idx, B.values, dtype=torch.float32)
    h = spg.Handle(stream=s)
    prod = spg.SparseProduct(dA, dB, handle=h)
    a = dA.values.clone().requires_grad_(True)
    bv = dB.values.clone().requires_grad_(True)
    with torch.cuda.stream(s):
        c = prod(a, bv)
        G = torch.randn_like(c)
    s.synchronize()

    def fwd_bwd():
        with torch.cuda.stream(s):
            cc = prod(a, bv)
            cc.backward(G)

    ms = _time(fwd_bwd, 5, s)
    Gc = spg.DeviceCsr(A.nrows, B.ncols, prod.row_ptr, prod.structure().col_idx, G)
    ms_b = _time(lambda: spg.spgemm_backward(h, dA.with_values(a.detach()), dB.with_values(bv.detach()), Gc), 5, s)
    ms_f = _time(lambda: spg.spgemm_numeric(h, dA.with_values(a.detach()), dB.with_values(bv.detach()),
                                            prod.row_ptr, prod.nnz), 5, s)
    res.update({"forward_ms": round(ms_f, 3), "backward_ms": round(ms_b, 3), "forward_backward_ms": round(ms, 3),
                "flops_m": h.stats()["flops"]})
    # baseline: plain FP64 products G*B^T and A^T*G (both phases), masking not counted
    Cst = prod.structure()
    rp = Cst.row_ptr.cpu().numpy().astype(np.int64)
    Gh = synth.Csr(A.nrows, B.ncols, rp, Cst.col_idx.cpu().numpy(), G.double().cpu().numpy())

    def transpose(M):
        rows = np.repeat(np.arange(M.nrows), M.row_lengths())
        order = np.lexsort((rows, M.col_idx))
        cnt = np.bincount(M.col_idx, minlength=M.ncols)
        trp = np.zeros(M.ncols + 1, np.int64)
        np.cumsum(cnt, out=trp[1:])
        return synth.Csr(M.ncols, M.nrows, trp, rows[order].astype(np.int32), M.values[order])

    Bt, At = transpose(B), transpose(A)
    t64 = 0.0
    for L, R in ((Gh, Bt), (At, Gh)):
        dL = spg.DeviceCsr.from_arrays(L.nrows, L.ncols, L.row_ptr, L.col_idx, L.values)
        dR = spg.DeviceCsr.from_arrays(R.nrows, R.ncols, R.row_ptr, R.col_idx, R.values)
        hb = spg.Handle(stream=s)

        def both():
            r_, n_ = spg.spgemm_symbolic(hb, dL, dR)
            spg.spgemm_numeric(hb, dL, dR, r_, n_)

        t64 += _time(both, 3, s)
        hb.close()
    res["plain_fp64_products_ms"] = round(t64, 3)
    res["speedup_masked_backward_vs_plain_fp64"] = round(t64 / ms_b, 3)
    return res
