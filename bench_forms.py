"""The workloads beside the headline step, measured on one MI355X by
`bench.py` (each one's inputs are built on the host before the first GPU
call; their oracle timings use host threads, since the oracle's C calls
release the interpreter lock).

c1: 5-point Laplacian on 64x64 squared (n = 4096): symbolic and numeric time
    of a product too small to fill the GPU (latency).
precision: symmetric R-MAT square (scale --rmat-scale, edge factor 16,
    (0.57, 0.19, 0.19, 0.05)); one symbolic, then numeric in FP64, FP32 (the
    default: rows whose entries may sum more than 167 products accumulate in
    FP64), FP32 in FP32 everywhere, FP32 + compensated pairs, FP32 with FP64
    accumulation.  Errors against the FP64 oracle (on the FP32-rounded inputs
    for FP32) on sampled rows (the 200 heaviest rows by multiplications and
    2000 uniform rows), relative to S = sum |a*b| per entry: max and median.
batch: --batch-count products (n_i ~ U[1000, 65536], Poisson(lambda_i) rows,
    lambda_i ~ U[4, 32]); one batched symbolic with the per-class autotuner,
    then 10 numeric recomputations on fresh seeded values of the same
    structure, each replayed from a captured HIP graph (the value refresh is
    not timed), FP64 and FP32; the same recomputations on the known structure
    (position maps, values only); baseline = the same products as 512
    separate plain FP64 numeric calls.
backward: C = A*B, A = 7-point Laplacian on g^3 (--diff-grid), B random with 16
    columns per row, FP32; forward + backward vs the plain FP64 products
    G*B^T and A^T*G that the masked gradients are taken from.
Each form also times the CPU oracle on a stated sample of its work
(sequential C per row or per product, P host threads), in GFLOP/s.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
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


def host_threads():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rows_parallel(A, B, sel, threads):
    """oracle.rows over `sel` split across threads; returns the concatenated
    rows and (wall seconds, summed per-thread seconds)."""
    import oracle

    chunks = [c for c in np.array_split(sel, max(1, min(len(sel), 4 * threads))) if c.size]

    def one(c):
        t = time.perf_counter()
        r = oracle.rows(A, B, c)
        return r, time.perf_counter() - t

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(threads) as ex:
        res = list(ex.map(one, chunks))
    wall = time.perf_counter() - t0
    rps, cis, vas, abss = [], [], [], []
    off = 0
    for (rp, ci, va, ab), _ in res:
        rps.append(rp[:-1] + off)
        off += int(rp[-1])
        cis.append(ci)
        vas.append(va)
        abss.append(ab)
    rp = np.concatenate(rps + [np.array([off])])
    return (rp, np.concatenate(cis), np.concatenate(vas), np.concatenate(abss)), wall, sum(t for _, t in res)


# ---------------------------------------------------------------- c1
def prepare_c1(args):
    import synth

    return {"A": synth.laplace2d_5pt(64, 64)}


def run_c1(args, data, log):
    import torch

    import oracle
    import paper_1801_03065_amd as spg

    A = data["A"]
    s = torch.cuda.Stream()
    d = spg.DeviceCsr.from_arrays(A.nrows, A.ncols, A.row_ptr, A.col_idx, A.values)
    h = spg.Handle(stream=s)
    box = {}

    def sym():
        box["rp"], box["nnz"] = spg.spgemm_symbolic(h, d, d)

    tsym = _time(sym, 20, s)
    C = spg.spgemm_numeric(h, d, d, box["rp"], box["nnz"])
    tnum = _time(lambda: spg.spgemm_numeric(h, d, d, box["rp"], box["nnz"], out=C), 20, s)
    h.check_errors()
    fm = h.stats()["flops"]
    t = time.perf_counter()
    reps = 50
    for _ in range(reps):
        oracle.spgemm(A, A)
    tc = (time.perf_counter() - t) / reps
    h.close()
    return {"workload": "5-point Laplacian 64x64 squared, FP64", "flops_m": fm, "nnz_c": box["nnz"],
            "symbolic_ms": round(tsym, 4), "numeric_ms": round(tnum, 4),
            "gflops": round(2 * fm / ((tsym + tnum) * 1e-3) / 1e9, 2),
            "cpu_oracle": {"ms": round(tc * 1e3, 3), "gflops": round(2 * fm / tc / 1e9, 3), "threads": 1,
                           "sample": f"the whole product, mean of {reps}"}}


# ---------------------------------------------------------------- precision
def prepare_precision(args):
    import oracle
    import synth

    A = synth.rmat_symmetric(args.rmat_scale, 16, seed=1)
    fl = oracle.flops(A, A)[2]
    rng = np.random.default_rng(0)
    sel = np.unique(np.concatenate([np.argsort(fl, kind="stable")[-200:], rng.integers(0, A.nrows, 2000)]))
    A32 = A.with_values(A.values.astype(np.float32).astype(np.float64))
    th = host_threads()
    ref32, w32, s32 = _oracle_rows_parallel(A32, A32, sel, th)
    ref64, w64, s64 = _oracle_rows_parallel(A, A, sel, th)
    sfl = int(fl[sel].sum())
    return {"A": A, "sel": sel, "ref32": ref32, "ref64": ref64, "flops_sample": sfl,
            "cpu": {"gflops_one_core": round(2 * 2 * sfl / (s32 + s64) / 1e9, 3),
                    "gflops_wall": round(2 * 2 * sfl / (w32 + w64) / 1e9, 3), "threads": th,
                    "summed_core_s": round(s32 + s64, 2), "wall_s": round(w32 + w64, 2),
                    "sample": f"{sel.size} rows (200 heaviest + 2000 uniform), FP64 and FP32-rounded inputs"}}


def run_precision(args, data, log):
    import torch

    import paper_1801_03065_amd as spg

    A, sel = data["A"], data["sel"]
    s = torch.cuda.Stream()
    res = {"workload": f"R-MAT scale {args.rmat_scale} squared", "n": A.nrows, "nnz_A": A.nnz}
    d64 = spg.DeviceCsr.from_arrays(A.nrows, A.ncols, A.row_ptr, A.col_idx, A.values)
    d32 = spg.DeviceCsr.from_arrays(A.nrows, A.ncols, A.row_ptr, A.col_idx, A.values, dtype=torch.float32)
    modes = {"fp64": (d64, torch.float64, {}),
             "fp32": (d32, torch.float32, {}),
             "fp32_plain_everywhere": (d32, torch.float32, {"fp32_terms_max": 0}),
             "fp32_compensated": (d32, torch.float32, {"fp32_mode": 1}),
             "fp32_wide": (d32, torch.float32, {"fp32_mode": 2})}
    idx_t = None
    for name, (D, dt, opts) in modes.items():
        hm = spg.Handle(stream=s, **opts)
        a, b = _ev()
        a.record(s)
        rpm, nnzm = spg.spgemm_symbolic(hm, D, D, torch.int64)
        b.record(s)
        torch.cuda.synchronize()
        tsym = a.elapsed_time(b)
        st = hm.stats()
        if idx_t is None:
            rp_h = rpm.cpu().numpy()
            idx = np.concatenate([np.arange(rp_h[i], rp_h[i + 1]) for i in sel])
            idx_t = torch.as_tensor(idx, device="cuda")
            res.update({"flops_m": st["flops"], "nnz_c": nnzm, "symbolic_ms": round(tsym, 3),
                        "cf": round(st["flops_compressed"] / max(1, st["flops"]), 4),
                        "cmrf": round(st["max_row_flops_compressed"] / max(1, st["max_row_flops"]), 4),
                        "rows_numeric": {k: v for k, v in st["rows_numeric"].items() if v}})
        ci = torch.empty(nnzm, dtype=torch.int32, device="cuda")
        va = torch.empty(nnzm, dtype=dt, device="cuda")
        C = spg.DeviceCsr(D.nrows, D.ncols, rpm, ci, va)
        ms = _time(lambda: spg.spgemm_numeric(hm, D, D, rpm, nnzm, out=C), 3, s)
        hm.check_errors()
        got_ci = C.col_idx[idx_t].cpu().numpy()
        got = C.values[idx_t].cpu().numpy().astype(np.float64)
        ref = data["ref32"] if dt == torch.float32 else data["ref64"]
        assert np.array_equal(got_ci, ref[1]), name
        rel = np.abs(got - ref[2]) / np.maximum(ref[3], 1e-300)
        res[name] = {"numeric_ms": round(ms, 3), "gflops": round(2 * st["flops"] / (ms * 1e-3) / 1e9, 1),
                     "err_rel_S_max": float(rel.max()), "err_rel_S_median": float(np.median(rel)),
                     "within_bound": bool(rel.max() <= (1e-12 if dt == torch.float64 else 1e-5)),
                     "fp64_rows": st["fp64_rows"], "sampled_entries": int(idx_t.numel())}
        log(f"[precision] {name}: {ms:.3f} ms, max err {rel.max():.3g} S, median {np.median(rel):.3g} S")
        del C, ci, va
        hm.close()
        torch.cuda.empty_cache()
    for k in ("fp32", "fp32_plain_everywhere", "fp32_compensated", "fp32_wide"):
        res[k]["speedup_vs_fp64"] = round(res["fp64"]["numeric_ms"] / res[k]["numeric_ms"], 3)
    res["cpu_oracle"] = data["cpu"]
    return res


# ---------------------------------------------------------------- batch
def prepare_batch(args):
    import oracle
    import synth

    specs = synth.batch_specs(args.batch_count, 42)
    pairs = synth.batch_matrices(specs, host_threads())
    # oracle on a sample of products (every 32nd), in host threads
    sample = list(range(0, len(pairs), 32))
    th = host_threads()

    def one(i):
        t = time.perf_counter()
        A, B = pairs[i]
        fm = oracle.flops(A, B)[0]
        oracle.spgemm(A, B)
        return fm, time.perf_counter() - t

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(th) as ex:
        res = list(ex.map(one, sample))
    wall = time.perf_counter() - t0
    fm = sum(f for f, _ in res)
    core = sum(t for _, t in res)
    return {"pairs": pairs, "cpu": {"gflops_one_core": round(2 * fm / core / 1e9, 3),
                                    "gflops_wall": round(2 * fm / wall / 1e9, 3), "threads": th,
                                    "summed_core_s": round(core, 2), "wall_s": round(wall, 2),
                                    "sample": f"{len(sample)} of {len(pairs)} products (every 32nd), both phases"}}


def run_batch(args, data, log):
    import torch

    import paper_1801_03065_amd as spg

    pairs = data["pairs"]
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
            spg.spgemm_batch_numeric(h, As, Bs, Cs)  # first call: per-class tuning + allocation
        s.synchronize()
        st = h.stats()
        fm = st["flops"]
        pol, lanes = h.batch_choices(len(pairs))
        choices = {}
        for p_, l_ in zip(pol.tolist(), lanes.tolist()):
            choices[f"policy {p_}, {l_} lanes"] = choices.get(f"policy {p_}, {l_} lanes", 0) + 1
        bases = [X[0].values._base if X[0].values._base is not None else X[0].values for X in (As, Bs)]
        gen = torch.Generator(device="cuda")

        def refresh(r):
            with torch.cuda.stream(s):
                for t, base in enumerate(bases):
                    gen.manual_seed(1000 + 2 * r + t)
                    base.copy_(torch.randn(base.shape, generator=gen, device="cuda", dtype=dt))

        out = {}
        for path, fn in (("numeric", spg.spgemm_batch_numeric), ("values", spg.spgemm_batch_numeric_values)):
            with torch.cuda.stream(s):
                fn(h, As, Bs, Cs)  # values: the first call takes the position maps
            s.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=s):
                fn(h, As, Bs, Cs)
            torch.cuda.synchronize()
            ms = 0.0
            for r in range(10):  # 10 recomputations, each on fresh seeded values of the same structure
                refresh(r)
                a, b = _ev()
                with torch.cuda.stream(s):
                    a.record(s)
                    g.replay()
                    b.record(s)
                torch.cuda.synchronize()
                ms += a.elapsed_time(b) / 10
            h.check_errors()
            out[path] = ms
            del g
        nnzc = int(sum(nnzs))
        vb = 8 if dt == torch.float64 else 4
        res[name] = {"symbolic_ms": round(tsym, 3), "numeric_ms": round(out["numeric"], 3),
                     "values_numeric_ms": round(out["values"], 3), "flops_m": fm, "nnz_c": nnzc,
                     "gflops": round(2 * fm / (out["numeric"] * 1e-3) / 1e9, 1),
                     "values_gflops": round(2 * fm / (out["values"] * 1e-3) / 1e9, 1),
                     "c_write_gbps": round((4 + vb) * nnzc / (out["numeric"] * 1e-3) / 1e9, 1),
                     "choices": choices,
                     "rows_numeric": {k: v for k, v in st["rows_numeric"].items() if v}}
        log(f"[batch] {name}: numeric {out['numeric']:.2f} ms, values {out['values']:.2f} ms, choices {choices}")
        del Cs, As, Bs
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
    res["speedup_values_fp64_vs_sequential"] = round(tseq / res["fp64"]["values_numeric_ms"], 3)
    for h in hs:
        h.close()
    res["cpu_oracle"] = data["cpu"]
    return res


# ---------------------------------------------------------------- backward
def prepare_backward(args):
    import synth

    g = args.diff_grid
    A = synth.laplace7(g)
    B = synth.fixed_row_random(A.ncols, A.ncols, 16, 5)
    return {"A": A, "B": B}


def run_backward(args, data, log):
    import torch

    import oracle
    import paper_1801_03065_amd as spg
    import synth

    A, B = data["A"], data["B"]
    s = torch.cuda.Stream()
    res = {"workload": f"7-point {args.diff_grid}^3 times random 16 per row, FP32", "n": A.nrows}
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
    fm = h.stats()["flops"]
    res.update({"forward_ms": round(ms_f, 3), "backward_ms": round(ms_b, 3), "forward_backward_ms": round(ms, 3),
                "flops_m": fm})
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
    # CPU oracle: gradient of the whole product, one thread
    Ah, Bh = A.with_values(a.detach().double().cpu().numpy()), B.with_values(bv.detach().double().cpu().numpy())
    t = time.perf_counter()
    C = oracle.spgemm(Ah, Bh)
    oracle.grad(Ah, Bh, C, Gh.values)
    tc = time.perf_counter() - t
    res["cpu_oracle"] = {"s": round(tc, 3), "gflops": round(2 * 3 * fm / tc / 1e9, 3), "threads": 1,
                         "sample": "the whole forward (oracle product) and gradient (2 * f_m multiply-adds)"}
    return res


FORMS = {"c1": (prepare_c1, run_c1), "precision": (prepare_precision, run_precision),
         "batch": (prepare_batch, run_batch), "backward": (prepare_backward, run_backward)}
