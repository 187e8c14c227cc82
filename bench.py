"""Benchmark of the two-phase SpGEMM on one MI355X.

Workload (one step = both phases of every product, NoReuse): the multigrid
setup shapes on a 100^3 grid, FP64 values, int32 indices:
    C  = A * A          A = 27-point operator (diag 26, off -1), n = 1e6
    AP = A * P          P = 2x2x2 piecewise-constant aggregation (1e6 x 125000)
    R  = P^T * (A P)    the Galerkin coarse operator
Reported `value`: whole-step GFLOP/s = 2 * sum f_m / step time (a multiply and
an add per multiplication).  Symbolic and numeric phases are also reported
separately per product, with achieved HBM GB/s from algorithmic bytes
(numeric: A, B and C once plus C's row pointers; symbolic: A's and B's
structure, compressed B written and read once, C's row pointers), the
compression factors CF (compressed / raw flops) and CMRF (the same for the
longest row), the numeric-only (Reuse) rate and the rate on the known
structure (position maps, values only).  The `roofline` object covers the
dominant kernel, the numeric kernel of A*A, timed with HIP events on its own
stream.  `forms` holds the other workloads (bench_forms.py): the 5-point
latency case, R-MAT precision forms, the 512-product batch and the backward.
Inputs of every workload are built on the host before the first GPU call.

    python bench.py [--gpus 1] [--steps 5] [--warmup 1] [--no-cpu] [--forms c1,precision,batch,backward]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0

# HBM bytes per launch of the dominant kernel, from two rocprofv3 counter
# passes (FETCH_SIZE, WRITE_SIZE) over `bench.py --forms "" --steps 1 --warmup 0 --no-cpu`,
# each scaled by what the counter reads for the bench's 2 GiB device copy
# (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0).  Valid only for the kernel sources they
# were taken on: reported as null once those sources change.
TRAFFIC = {
    "kernel": "k_num_pl",
    "sources": ["paper_1801_03065_amd/csrc/spg_plan.hip", "paper_1801_03065_amd/csrc/spg_internal.hpp",
                "paper_1801_03065_amd/csrc/spg_accum.hpp"],
    "sha256": "4c45b3afc98c22126d6833664bd1d6381f35cb2efb3f81e45ebc5e462adf7e84",
    "read_bytes": 3.7433e9,
    "write_bytes": 1.5278e9,
}


def measured_traffic(kernel):
    import hashlib

    if not kernel.startswith(TRAFFIC["kernel"]):
        return None
    h = hashlib.sha256()
    try:
        for f in TRAFFIC["sources"]:
            with open(os.path.join(ROOT, f), "rb") as fh:
                h.update(fh.read())
    except OSError:
        return None
    if h.hexdigest() != TRAFFIC["sha256"]:
        return None
    return TRAFFIC["read_bytes"] + TRAFFIC["write_bytes"]


# numeric kernel that processes each row kind
KERNEL_OF_KIND = {"empty": "none", "dense_wave": "k_num_dw", "hash_wave": "k_num_hw", "dense_wg": "k_num_dg",
                  "hash_two_level": "k_num_hl", "word_hash_wave": "k_num_wh", "short_rows": "k_sr",
                  "planned_wave": "k_num_pl"}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def csr_bytes(M, vbytes=8, rp_bytes=4):
    return rp_bytes * (M.nrows + 1) + (4 + vbytes) * M.nnz


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--grid", type=int, default=100)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--forms", default="c1,precision,batch,backward",
                    help="comma list of extra workloads: c1,precision,batch,backward ('' for none)")
    ap.add_argument("--rmat-scale", type=int, default=20)
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--diff-grid", type=int, default=64)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); "
              "the library runs one product per GPU and has no multi-GPU sharding", file=sys.stderr)
        sys.exit(2)

    import synth
    import bench_forms

    g = args.grid
    log(f"[bench] building inputs, grid {g}^3")
    A = synth.stencil27(g)
    P, Pt = synth.aggregation_2x2x2(g)
    forms = [f for f in args.forms.split(",") if f]
    form_data = {}
    for f in forms:  # host-side inputs (and oracle samples) before any GPU call
        log(f"[bench] preparing {f}")
        form_data[f] = bench_forms.FORMS[f][0](args)

    import torch

    import paper_1801_03065_amd as spg

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")

    def to_dev(M):
        return spg.DeviceCsr.from_arrays(M.nrows, M.ncols, M.row_ptr, M.col_idx, M.values)

    dA, dP, dPt = to_dev(A), to_dev(P), to_dev(Pt)
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()

    # device copy bandwidth (for context beside the published peak)
    x = torch.empty(1 << 28, dtype=torch.float64, device=dev)  # 2 GiB
    y = torch.empty_like(x)
    for _ in range(2):
        y.copy_(x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    copy_gbps = 5 * 2 * x.numel() * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del x, y
    torch.cuda.empty_cache()

    names = ["AxA", "AxP", "PtxAP"]
    handles = {k: spg.Handle(stream=stream) for k in names}

    pool = []  # timing events made before the timed region (their HIP events are created on first record)

    def events():
        if len(pool) >= 2:
            return pool.pop(), pool.pop()
        return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    rec = {k: {"sym": [], "num": []} for k in names}
    last = {}

    def product(name, L, R, timing):
        h = handles[name]
        es, ee = events()
        es.record(stream)
        rp, nnz = spg.spgemm_symbolic(h, L, R)
        ee.record(stream)
        ns, ne = events()
        with torch.cuda.stream(stream):
            ci = torch.empty(nnz, dtype=torch.int32, device=dev)
            va = torch.empty(nnz, dtype=torch.float64, device=dev)
        C = spg.DeviceCsr(L.nrows, R.ncols, rp, ci, va)
        ns.record(stream)
        spg.spgemm_numeric(h, L, R, rp, nnz, out=C)
        ne.record(stream)
        if timing:
            rec[name]["sym"].append((es, ee))
            rec[name]["num"].append((ns, ne))
        last[name] = (L, R, rp, nnz, C)
        return C

    def step(timing):
        product("AxA", dA, dA, timing)
        AP = product("AxP", dA, dP, timing)
        product("PtxAP", dPt, AP, timing)

    log(f"[bench] warmup {args.warmup}")
    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    for k in names:
        handles[k].check_errors()

    log(f"[bench] timing {args.steps} steps")
    pool[:] = [torch.cuda.Event(enable_timing=True) for _ in range(4 * len(names) * args.steps)]
    for e in pool:
        e.record(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for k in names:
        handles[k].check_errors()
    ms_per_step = (t1 - t0) * 1e3 / args.steps

    # Reuse case: numeric phase only, same structure (timed separately), then
    # on the known structure (position maps taken at the first call, values only)
    reuse_ms, values_ms = {}, {}
    for k in names:
        L, R, rp, nnz, C = last[k]
        h = handles[k]
        for dst, fn in ((reuse_ms, lambda: spg.spgemm_numeric(h, L, R, rp, nnz, out=C)),
                        (values_ms, lambda: spg.spgemm_numeric_values(h, L, R, C))):
            fn()
            torch.cuda.synchronize()
            ts = []
            for _ in range(args.steps):
                a, b = events()
                a.record(stream)
                fn()
                b.record(stream)
                ts.append((a, b))
            torch.cuda.synchronize()
            h.check_errors()
            dst[k] = float(np.mean([a.elapsed_time(b) for a, b in ts]))

    stats = {k: handles[k].stats() for k in names}
    fm = {k: stats[k]["flops"] for k in names}
    total_fm = sum(fm.values())

    shapes = {
        "AxA": (A, A, stats["AxA"]["nnz_c"], A.nrows),
        "AxP": (A, P, stats["AxP"]["nnz_c"], A.nrows),
        "PtxAP": (Pt, None, stats["PtxAP"]["nnz_c"], Pt.nrows),
    }
    nnz_ap = stats["AxP"]["nnz_c"]
    ap_bytes = 4 * (P.nrows + 1) + 12 * nnz_ap
    phases = {}
    for k in names:
        L, R, nnzc, m = shapes[k]
        rb = csr_bytes(R) if R is not None else ap_bytes
        rstruct = (4 * (R.nrows + 1) + 4 * R.nnz) if R is not None else (4 * (P.nrows + 1) + 4 * nnz_ap)
        num_bytes = csr_bytes(L) + rb + 4 * (m + 1) + 12 * nnzc
        # numeric on the known structure: A and B values, A's structure, C's values
        rvals = (8 * R.nnz) if R is not None else 8 * nnz_ap
        val_bytes = csr_bytes(L) + rvals + 4 * (m + 1) + 8 * nnzc
        # compressed B: one (word, bits) record per pair plus its int64 row offsets
        nbr = R.nrows if R is not None else P.nrows
        bc_bytes = (8 * stats[k]["nnz_b_compressed"] + 8 * (nbr + 1)) if stats[k]["compressed"] else 0
        sym_bytes = (4 * (L.nrows + 1) + 4 * L.nnz) + rstruct + 2 * bc_bytes + 4 * (m + 1)
        tsym = float(np.mean([a.elapsed_time(b) for a, b in rec[k]["sym"]]))
        tnum = float(np.mean([a.elapsed_time(b) for a, b in rec[k]["num"]]))
        phases[k] = {
            "flops_m": fm[k], "nnz_c": nnzc, "compressed": bool(stats[k]["compressed"]),
            "cf": round(stats[k]["flops_compressed"] / max(1, fm[k]), 4),
            "cmrf": round(stats[k]["max_row_flops_compressed"] / max(1, stats[k]["max_row_flops"]), 4),
            "nnz_b_compressed": stats[k]["nnz_b_compressed"],
            "symbolic_ms": round(tsym, 4), "numeric_ms": round(tnum, 4), "reuse_numeric_ms": round(reuse_ms[k], 4),
            "values_numeric_ms": round(values_ms[k], 4),
            "values_hbm_gbps": round(val_bytes / (values_ms[k] * 1e-3) / 1e9, 1),
            "symbolic_gflops": round(2 * fm[k] / (tsym * 1e-3) / 1e9, 2),
            "numeric_gflops": round(2 * fm[k] / (tnum * 1e-3) / 1e9, 2),
            "numeric_hbm_gbps": round(num_bytes / (tnum * 1e-3) / 1e9, 1),
            "numeric_alg_bytes": int(num_bytes),
            "symbolic_hbm_gbps": round(sym_bytes / (tsym * 1e-3) / 1e9, 1),
            "symbolic_alg_bytes": int(sym_bytes),
            "rows_numeric": {kk: v for kk, v in stats[k]["rows_numeric"].items() if v},
        }

    # roofline: numeric kernel of A*A (one launch on `stream`), HIP events per launch
    dom = phases["AxA"]
    dom_kind = max(dom["rows_numeric"].items(), key=lambda kv: kv[1])[0]
    t_dom = dom["numeric_ms"] * 1e-3
    achieved = dom["numeric_alg_bytes"] / t_dom / 1e9
    kname = f"{KERNEL_OF_KIND[dom_kind]}<double>"
    traffic = measured_traffic(kname)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4),
                "traffic": None if traffic is None else round(traffic / 1e9, 3),
                "traffic_unit": "GB per launch", "algorithmic": round(dom["numeric_alg_bytes"] / 1e9, 3),
                "kernel": f"{kname} (27-point A*A, FP64)",
                "frac_of_measured_copy": round(achieved / copy_gbps, 4)}

    cpu = None
    if not args.no_cpu:
        import oracle

        log("[bench] CPU oracle baseline (full step, sequential C)")
        reps = 5
        t = time.perf_counter()
        for _ in range(reps):
            oracle.spgemm(A, A)
            APo = oracle.spgemm(A, P)
            oracle.spgemm(Pt, APo)
        tc = (time.perf_counter() - t) / reps
        cpu = {"value": round(2 * total_fm / tc / 1e9, 3), "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
               "sample": f"the full step (A*A, A*P, P^T*(AP) on 100^3, both phases), {reps} repetitions, "
                         f"{tc:.2f} s each on one host core",
               "cpu_model": bench_forms.cpu_model(), "host_threads": bench_forms.host_threads()}

    value = 2 * total_fm / (ms_per_step * 1e-3) / 1e9
    out = {
        "metric": "SpGEMM GFLOP/s (two-phase, symbolic+numeric, FP64), with per-phase GFLOP/s and HBM GB/s",
        "value": round(value, 2), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"27-point stencil squared on {g}^3 plus Galerkin P^T(AP) with 2x2x2 aggregation",
                   "n": A.nrows, "nnz_A": A.nnz, "flops_m_total": total_fm, "index": "int32",
                   "parallelism": "single GPU"},
        "phases": phases,
        "device_copy_gbps": round(copy_gbps, 1),
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    for k in names:
        handles[k].close()
    del last
    torch.cuda.empty_cache()
    if forms:
        out["forms"] = {}
        for f in forms:
            log(f"[bench] form {f}")
            out["forms"][f] = bench_forms.FORMS[f][1](args, form_data.pop(f), log)
            torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
