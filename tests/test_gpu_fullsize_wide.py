"""GPU parity at full size on wide samples, in every floating-point mode.

* R-MAT scale 20 squared (C has 2.37e10 entries, more than fits at once):
  the product is computed in row panels of about 2^30 entries; the 1,000
  heaviest rows by multiplications and 100,000 seeded uniform rows are
  compared with the oracle row by row (columns exact, values within the
  FP64 / FP32 bounds) in FP64, FP32 (the default: rows past the term limit
  accumulate in FP64), compensated FP32 and FP32 with FP64 accumulation; the
  max and the median of |err| / S are printed per mode.
* 512-product batch: every product's row pointers against the oracle's
  symbolic phase; values of 64 products (the widest windows among them) in
  FP64 and FP32; two graph replays on fresh values, each checked.
"""
import concurrent.futures as cf
import os

import numpy as np
import pytest

import oracle
import synth
from helpers import check_f32, check_f64, dev, f32_inputs

pytestmark = pytest.mark.gpu


def _threads():
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:
        return 4


def _check_rows_parallel(A, B, sel, grp, gci, gval, tol, rel_mode):
    """oracle.rows_check over `sel` in host threads (the C call releases the GIL)."""
    th = _threads()
    parts = np.array_split(np.arange(sel.size), max(1, min(sel.size, 4 * th)))

    def one(ix):
        if ix.size == 0:
            return None
        lo, hi = ix[0], ix[-1] + 1
        o0 = grp[lo]
        return oracle.rows_check(A, B, sel[lo:hi], grp[lo:hi + 1] - o0, gci[o0:grp[hi]], gval[o0:grp[hi]],
                                 tol, rel_mode, stride=97)

    with cf.ThreadPoolExecutor(th) as ex:
        res = [r for r in ex.map(one, parts) if r is not None]
    return {"max_rel_S": max(r["max_rel_S"] for r in res), "bad": sum(r["bad"] for r in res),
            "entries": sum(r["entries"] for r in res), "bad_rows": sum(r["bad_rows"] for r in res),
            "sub": np.concatenate([r["sub"] for r in res])}


@pytest.mark.timeout(900)
def test_rmat20_heavy_and_uniform_rows_every_mode():
    import torch

    import paper_1801_03065_amd as spg

    A = synth.rmat_symmetric(20, 16, seed=1)
    fl = oracle.flops(A, A)[2]
    rng = np.random.default_rng(20)
    sel = np.unique(np.concatenate([np.argsort(fl, kind="stable")[-1000:], rng.integers(0, A.nrows, 100_000)]))
    A32 = f32_inputs(A)
    modes = [("fp64", "f64", {}, A, 1e-12, 0), ("fp32", "f32", {}, A32, 1e-5, 1),
             ("fp32_compensated", "f32", {"fp32_mode": 1}, A32, 1e-5, 1),
             ("fp32_wide", "f32", {"fp32_mode": 2}, A32, 1e-5, 1)]
    for name, dt, opts, Aref, tol, relm in modes:
        h = spg.Handle(**opts)
        dA = dev(A, dt)
        rp_t, nnz = spg.spgemm_symbolic(h, dA, dA, torch.int64)
        rp = rp_t.cpu().numpy().astype(np.int64)
        tdt = torch.float64 if dt == "f64" else torch.float32
        # row panels of about 2^30 entries, one buffer pair reused
        cap = 1 << 30
        bounds = [0]
        while bounds[-1] < A.nrows:
            r0 = bounds[-1]
            r1 = int(np.searchsorted(rp, rp[r0] + cap, side="right")) - 1
            bounds.append(min(A.nrows, max(r1, r0 + 1)))
        width = max(int(rp[b1] - rp[b0]) for b0, b1 in zip(bounds[:-1], bounds[1:]))
        ci = torch.empty(width, dtype=torch.int32, device="cuda")
        va = torch.empty(width, dtype=tdt, device="cuda")
        tot = {"max_rel_S": 0.0, "bad": 0, "entries": 0, "bad_rows": 0, "sub": []}
        for b0, b1 in zip(bounds[:-1], bounds[1:]):
            s = sel[(sel >= b0) & (sel < b1)]
            if s.size == 0:
                continue
            spg.spgemm_numeric_rows(h, dA, dA, b0, b1, ci, va)
            lens = rp[s + 1] - rp[s]
            grp = np.zeros(s.size + 1, dtype=np.int64)
            np.cumsum(lens, out=grp[1:])
            lens_t = torch.as_tensor(lens, device="cuda")
            shift = torch.as_tensor(rp[s] - rp[b0] - grp[:-1], device="cuda")
            idx = torch.repeat_interleave(shift, lens_t) + torch.arange(int(grp[-1]), device="cuda")
            gci = ci[idx].cpu().numpy()
            gval = va[idx].cpu().numpy().astype(np.float64)
            r = _check_rows_parallel(Aref, Aref, s, grp, gci, gval, tol, relm)
            tot["max_rel_S"] = max(tot["max_rel_S"], r["max_rel_S"])
            for k in ("bad", "entries", "bad_rows"):
                tot[k] += r[k]
            tot["sub"].append(r["sub"])
        h.check_errors()
        med = float(np.median(np.concatenate(tot["sub"])))
        print(f"R-MAT 20 {name}: {sel.size} rows, {tot['entries']} entries, max |err|/S {tot['max_rel_S']:.3e}, "
              f"median {med:.3e}, fp64 rows {h.stats()['fp64_rows']}")
        assert tot["bad_rows"] == 0, name
        assert tot["bad"] == 0, (name, tot["bad"], tot["max_rel_S"])
        h.close()
        del dA, ci, va
        torch.cuda.empty_cache()


@pytest.mark.timeout(900)
def test_batch_512_every_row_ptr_64_products_and_replays():
    import torch

    import paper_1801_03065_amd as spg

    specs = synth.batch_specs(512, 42)
    pairs = synth.batch_matrices(specs)
    th = _threads()
    with cf.ThreadPoolExecutor(th) as ex:
        sym = list(ex.map(lambda p: oracle.symbolic(p[0], p[1]), pairs))
    ns = np.array([s.n for s in specs])
    rng = np.random.default_rng(11)
    widest = list(np.argsort(ns)[-16:])
    sample = sorted(set(widest) | set(rng.choice(512, 64, replace=False).tolist()))[:64]
    for dt in ("f64", "f32"):
        tdt = torch.float64 if dt == "f64" else torch.float32
        As = spg.pack_batch([p[0] for p in pairs], dtype=tdt)
        Bs = spg.pack_batch([p[1] for p in pairs], dtype=tdt)
        s = torch.cuda.Stream()
        h = spg.Handle(stream=s, autotune=1)
        rps, nnzs = spg.spgemm_batch_symbolic(h, As, Bs)
        for i in range(512):
            assert np.array_equal(rps[i].cpu().numpy().astype(np.int64), sym[i]), i
        Cs = spg.batch_outputs(As, Bs, rps, nnzs, tdt)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            spg.spgemm_batch_numeric(h, As, Bs, Cs)  # tuning + allocation
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            spg.spgemm_batch_numeric(h, As, Bs, Cs)
        torch.cuda.synchronize()
        bases = [X[0].values._base if X[0].values._base is not None else X[0].values for X in (As, Bs)]
        for r in range(2):  # two replays on fresh values of the same structure
            fresh = synth.batch_revalue(pairs, r + 1, 500)
            va = np.concatenate([p[0].values for p in fresh])
            vb = np.concatenate([p[1].values for p in fresh])
            bases[0].copy_(torch.as_tensor(va).to(device="cuda", dtype=tdt))
            bases[1].copy_(torch.as_tensor(vb).to(device="cuda", dtype=tdt))
            torch.cuda.synchronize()
            with torch.cuda.stream(s):
                g.replay()
            torch.cuda.synchronize()
            h.check_errors()

            def one(i):
                A2, B2 = fresh[i]
                if dt == "f32":
                    A2, B2 = f32_inputs(A2), f32_inputs(B2)
                ref, S = oracle.spgemm(A2, B2, with_abs=True)
                return i, ref, S

            with cf.ThreadPoolExecutor(th) as ex:
                refs = list(ex.map(one, sample))
            for i, ref, S in refs:
                C = Cs[i]
                got = (C.row_ptr.cpu().numpy().astype(np.int64), C.col_idx.cpu().numpy(),
                       C.values.cpu().numpy())
                if dt == "f64":
                    check_f64(ref, S, got)
                else:
                    check_f32(ref, S, got)
        print(f"batch 512 {dt}: row pointers of all 512, values of {len(sample)} products after 2 replays")
        del g, Cs, As, Bs
        h.close()
        torch.cuda.empty_cache()
