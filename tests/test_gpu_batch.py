"""GPU parity of the batched form: one plan for many independent products,
numeric reuse with fresh values, zero-copy and staged layouts, and a replay
captured in a HIP graph."""
import numpy as np
import pytest

import oracle
import synth
from helpers import check_f64

pytestmark = pytest.mark.gpu


def _batch(count, seed, n_lo=50, n_hi=900):
    specs = synth.batch_specs(count, seed, n_lo=n_lo, n_hi=n_hi, lam_lo=1.0, lam_hi=12.0)
    return specs, synth.batch_matrices(specs)


def _check(pairs, Cs, rel=1e-12):
    for (A, B), C in zip(pairs, Cs):
        ref, S = oracle.spgemm(A, B, with_abs=True)
        got = (C.row_ptr.cpu().numpy().astype(np.int64), C.col_idx.cpu().numpy(), C.values.cpu().numpy())
        check_f64(ref, S, got, rel)


@pytest.mark.parametrize("contiguous", [True, False])
def test_batch_matches_oracle_and_reuses(contiguous):
    import torch

    import paper_1801_03065_amd as spg

    specs, pairs = _batch(24, 5)
    pairs[3] = (synth.tiny_random(7, 9, 0.0, 1), synth.tiny_random(9, 4, 0.5, 2))  # an empty product
    h = spg.Handle()
    if contiguous:
        As = spg.pack_batch([p[0] for p in pairs])
        Bs = spg.pack_batch([p[1] for p in pairs])
    else:
        from helpers import dev

        As = [dev(p[0]) for p in pairs]
        Bs = [dev(p[1]) for p in pairs]
    rps, nnzs = spg.spgemm_batch_symbolic(h, As, Bs)
    for (A, B), nz in zip(pairs, nnzs):
        assert nz == oracle.symbolic(A, B)[-1]
    if contiguous:
        Cs = spg.batch_outputs(As, Bs, rps, nnzs, torch.float64)
    else:
        Cs = [spg.DeviceCsr(A.nrows, B.ncols, rp, torch.empty(nz, dtype=torch.int32, device="cuda"),
                            torch.empty(nz, dtype=torch.float64, device="cuda"))
              for A, B, rp, nz in zip(As, Bs, rps, nnzs)]
    spg.spgemm_batch_numeric(h, As, Bs, Cs)
    h.check_errors()
    torch.cuda.synchronize()
    _check(pairs, Cs)
    # reuse: fresh values, same structure
    pairs2 = synth.batch_revalue(pairs, 1, 77)
    for D, (A2, _) in zip(As, pairs2):
        D.values.copy_(torch.as_tensor(A2.values, device="cuda"))
    for D, (_, B2) in zip(Bs, pairs2):
        D.values.copy_(torch.as_tensor(B2.values, device="cuda"))
    spg.spgemm_batch_numeric(h, As, Bs, Cs)
    h.check_errors()
    torch.cuda.synchronize()
    _check(pairs2, Cs)


def test_batch_graph_replay():
    import torch

    import paper_1801_03065_amd as spg

    specs, pairs = _batch(16, 8)
    s = torch.cuda.Stream()
    h = spg.Handle(stream=s)
    As = spg.pack_batch([p[0] for p in pairs])
    Bs = spg.pack_batch([p[1] for p in pairs])
    rps, nnzs = spg.spgemm_batch_symbolic(h, As, Bs)
    Cs = spg.batch_outputs(As, Bs, rps, nnzs, torch.float64)
    with torch.cuda.stream(s):
        spg.spgemm_batch_numeric(h, As, Bs, Cs)  # first call allocates what it needs
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        spg.spgemm_batch_numeric(h, As, Bs, Cs)
    for r in range(3):
        pr = synth.batch_revalue(pairs, r + 2, 11)
        for D, (A2, _) in zip(As, pr):
            D.values.copy_(torch.as_tensor(A2.values, device="cuda"))
        for D, (_, B2) in zip(Bs, pr):
            D.values.copy_(torch.as_tensor(B2.values, device="cuda"))
        torch.cuda.synchronize()
        for C in Cs:
            C.values.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        h.check_errors()
        _check(pr, Cs)


def test_batch_fp32():
    import torch

    import paper_1801_03065_amd as spg
    from helpers import check_f32, f32_inputs

    specs, pairs = _batch(10, 3)
    h = spg.Handle(fp32_mode=1)
    As = spg.pack_batch([p[0] for p in pairs], dtype=torch.float32)
    Bs = spg.pack_batch([p[1] for p in pairs], dtype=torch.float32)
    rps, nnzs = spg.spgemm_batch_symbolic(h, As, Bs)
    Cs = spg.batch_outputs(As, Bs, rps, nnzs, torch.float32)
    spg.spgemm_batch_numeric(h, As, Bs, Cs)
    h.check_errors()
    torch.cuda.synchronize()
    for (A, B), C in zip(pairs, Cs):
        ref, S = oracle.spgemm(f32_inputs(A), f32_inputs(B), with_abs=True)
        got = (C.row_ptr.cpu().numpy().astype(np.int64), C.col_idx.cpu().numpy(), C.values.cpu().numpy())
        check_f32(ref, S, got)


def test_batch_with_degenerate_members():
    """Members with no rows, a 1x1 product, a single output column and an
    all-empty A among ordinary products, in one batched plan."""
    import torch

    import paper_1801_03065_amd as spg

    specs, pairs = _batch(6, 31)
    empty_rows = synth.Csr(0, 9, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    pairs[1] = (empty_rows, synth.tiny_random(9, 4, 0.5, 3))
    pairs[2] = (synth.Csr(1, 1, np.array([0, 1]), np.array([0], np.int32), np.array([2.5])),
                synth.Csr(1, 1, np.array([0, 1]), np.array([0], np.int32), np.array([-3.0])))
    pairs[3] = (synth.tiny_random(40, 30, 0.3, 4), synth.tiny_random(30, 1, 0.6, 5))
    pairs[4] = (synth.tiny_random(25, 12, 0.0, 6), synth.tiny_random(12, 8, 0.4, 7))
    h = spg.Handle()
    As = spg.pack_batch([p[0] for p in pairs])
    Bs = spg.pack_batch([p[1] for p in pairs])
    rps, nnzs = spg.spgemm_batch_symbolic(h, As, Bs)
    Cs = spg.batch_outputs(As, Bs, rps, nnzs, torch.float64)
    spg.spgemm_batch_numeric(h, As, Bs, Cs)
    torch.cuda.synchronize()
    h.check_errors()
    assert nnzs[1] == 0 and nnzs[2] == 1 and nnzs[4] == 0
    _check(pairs, Cs)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batch_autotune_per_class(dtype):
    """Products of very different shapes get their own (policy, lanes) choices.
    C_i rows of under 16 entries over B rows of ~3 fall into the first class
    (average C row size <= 16), rows of several hundred over B rows of ~26
    into the third (<= 1024); their lanes-per-B-row candidates (the rounded
    average B row length and its neighbours: 4-8 against 16-64) do not
    overlap, so the two groups must differ.  Every product still equals the
    oracle."""
    import torch

    import paper_1801_03065_amd as spg
    from helpers import check_f32, f32_inputs

    small = synth.batch_specs(6, 11, n_lo=2000, n_hi=4000, lam_lo=2.5, lam_hi=3.0)
    big = synth.batch_specs(6, 12, n_lo=2000, n_hi=4000, lam_lo=24.0, lam_hi=28.0)
    specs = [s for pair in zip(small, big) for s in pair]
    pairs = synth.batch_matrices(specs)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    As = spg.pack_batch([p[0] for p in pairs], dtype=tdt)
    Bs = spg.pack_batch([p[1] for p in pairs], dtype=tdt)
    h = spg.Handle(autotune=1)
    rps, nnzs = spg.spgemm_batch_symbolic(h, As, Bs)
    Cs = spg.batch_outputs(As, Bs, rps, nnzs, tdt)
    spg.spgemm_batch_numeric(h, As, Bs, Cs)
    h.check_errors()
    pol, lanes = h.batch_choices(len(pairs))
    print("per-product policy", pol.tolist(), "lanes", lanes.tolist())
    avg_c = np.array([int(n) / A.nrows for n, (A, _) in zip(nnzs, pairs)])
    assert np.all(avg_c[0::2] <= 16) and np.all((avg_c[1::2] > 128) & (avg_c[1::2] <= 1024)), avg_c
    for grp in (slice(0, None, 2), slice(1, None, 2)):  # one choice per class
        assert len(set(zip(pol[grp].tolist(), lanes[grp].tolist()))) == 1
    assert set(lanes[0::2].tolist()).isdisjoint(set(lanes[1::2].tolist()))
    assert len(set(zip(pol.tolist(), lanes.tolist()))) >= 2
    for r in range(2):  # a second call reuses the tuned classes
        torch.cuda.synchronize()
        for (A, B), C in zip(pairs, Cs):
            got = (C.row_ptr.cpu().numpy().astype(np.int64), C.col_idx.cpu().numpy(), C.values.cpu().numpy())
            if dtype == "f64":
                ref, S = oracle.spgemm(A, B, with_abs=True)
                check_f64(ref, S, got)
            else:
                ref, S = oracle.spgemm(f32_inputs(A), f32_inputs(B), with_abs=True)
                check_f32(ref, S, got)
        for C in Cs:
            C.values.fill_(float("nan"))
        spg.spgemm_batch_numeric(h, As, Bs, Cs)
        h.check_errors()
