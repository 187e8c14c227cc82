"""Pins for the CPU oracle, independent of the oracle's own code.

Each test checks the oracle against something the mathematics fixes:
closed forms of stencil products (derived from grid coordinates, never by
multiplying), brute-force dense products on tiny inputs, counting identities
and invariants. A dropped term, a wrong sign, a transposed operand, a lost
structural zero or an unsorted row fails at least one of them.
"""
import numpy as np
import pytest

import oracle
import synth


# ---------------------------------------------------------------- closed forms
def closed_form_5pt_square(nx, ny):
    """(4I - Adj)^2 = 16I - 8Adj + Adj^2 on the 5-point grid graph.

    Adj^2(p,p) = deg(p); Adj^2(p,q) = 2 for diagonal neighbours (two paths),
    1 for axial distance-2 neighbours. Built from coordinates only.
    """
    rows = []
    for y in range(ny):
        for x in range(nx):
            ent = {}
            deg = (x > 0) + (x < nx - 1) + (y > 0) + (y < ny - 1)
            for dy in range(-2, 3):
                for dx in range(-2, 3):
                    qx, qy = x + dx, y + dy
                    if not (0 <= qx < nx and 0 <= qy < ny):
                        continue
                    d1 = abs(dx) + abs(dy)
                    q = qy * nx + qx
                    if d1 == 0:
                        ent[q] = 16.0 + deg
                    elif d1 == 1:
                        ent[q] = -8.0
                    elif abs(dx) == 1 and abs(dy) == 1:
                        ent[q] = 2.0
                    elif d1 == 2:
                        ent[q] = 1.0
            rows.append(sorted(ent.items()))
    return rows


def assert_rows_equal(C, rows):
    assert C.nrows == len(rows)
    for i, r in enumerate(rows):
        s, e = C.row_ptr[i], C.row_ptr[i + 1]
        assert list(C.col_idx[s:e]) == [q for q, _ in r], f"row {i} pattern"
        assert list(C.values[s:e]) == [v for _, v in r], f"row {i} values"


@pytest.mark.parametrize("nx,ny", [(1, 1), (2, 3), (7, 5), (16, 16)])
def test_5pt_square_closed_form_small(nx, ny):
    A = synth.laplace2d_5pt(nx, ny)
    assert_rows_equal(oracle.spgemm(A, A), closed_form_5pt_square(nx, ny))


def test_5pt_square_64x64_counts_and_values():
    A = synth.laplace2d_5pt(64, 64)
    C = oracle.spgemm(A, A)
    fm, maxrf, _ = oracle.flops(A, A)
    assert A.nnz == 5 * 64 * 64 - 2 * 128 == 20224
    assert fm == 100104 and maxrf == 25
    assert C.nnz == 51972 and np.diff(C.row_ptr).max() == 13
    assert_rows_equal(C, closed_form_5pt_square(64, 64))
    # diagonal value classes: 20 interior, 19 edge, 18 corner
    diag = np.array([C.values[C.row_ptr[i] + np.searchsorted(C.col_idx[C.row_ptr[i]:C.row_ptr[i + 1]], i)]
                     for i in range(C.nrows)])
    assert (diag == 20).sum() == 62 * 62 and (diag == 19).sum() == 4 * 62 and (diag == 18).sum() == 4


def closed_form_27pt_square_row(g, p):
    """Row p of (27I - J)^2 = 729I - 54J + K^2 (x) K^2 (x) K^2, K = tridiag(1,1,1).

    K^2(x,y) on a line of g points: deg1(x) (2 or 3) on the diagonal, 2 at
    distance 1, 1 at distance 2.
    """
    x, y, z = p % g, (p // g) % g, p // (g * g)

    def k2(a, b):
        d = abs(a - b)
        if d == 0:
            return 1 + (a > 0) + (a < g - 1)
        return {1: 2, 2: 1}.get(d, 0)

    out = []
    for dz in range(-2, 3):
        for dy in range(-2, 3):
            for dx in range(-2, 3):
                qx, qy, qz = x + dx, y + dy, z + dz
                if not (0 <= qx < g and 0 <= qy < g and 0 <= qz < g):
                    continue
                q = qz * g * g + qy * g + qx
                jv = 1 if max(abs(dx), abs(dy), abs(dz)) <= 1 else 0
                v = 729 * (q == p) - 54 * jv + k2(x, qx) * k2(y, qy) * k2(z, qz)
                out.append((q, float(v)))
    return out


@pytest.mark.parametrize("g", [1, 2, 3, 6])
def test_27pt_square_closed_form_small(g):
    A = synth.stencil27(g)
    C = oracle.spgemm(A, A)
    assert_rows_equal(C, [closed_form_27pt_square_row(g, p) for p in range(g ** 3)])
    if g >= 2:
        fm, maxrf, _ = oracle.flops(A, A)
        assert fm == (9 * g - 10) ** 3 or g < 2
        assert C.nnz == (5 * g - 6) ** 3


@pytest.mark.slow
def test_27pt_square_100cubed():
    """Full config: nnz = 494^3, f_m = 890^3, maxrs 125, maxrf 729; sampled rows exact."""
    g = 100
    A = synth.stencil27(g)
    assert A.nnz == 26463592
    fm, maxrf, _ = oracle.flops(A, A)
    assert fm == 890 ** 3 == 704969000 and maxrf == 729
    C = oracle.spgemm(A, A)
    assert C.nnz == 494 ** 3 == 120553784
    assert np.diff(C.row_ptr).max() == 125
    assert C.values.min() == -46.0 and C.values.max() == 702.0 and not (C.values == 0).any()
    rng = np.random.default_rng(5)
    for p in list(rng.integers(0, g ** 3, 300)) + [0, g ** 3 - 1, 505050]:
        s, e = C.row_ptr[p], C.row_ptr[p + 1]
        ref = closed_form_27pt_square_row(g, int(p))
        assert list(C.col_idx[s:e]) == [q for q, _ in ref]
        assert list(C.values[s:e]) == [v for _, v in ref]


def galerkin_coarse_closed_form(h):
    """P^T A P for the 27-point operator and 2x2x2 aggregation on (2h)^3.

    Sum over fine pairs factorises per dimension: aggregate pair (a,b) on one
    axis contributes 4 fine neighbour pairs if a == b, 1 if |a-b| == 1, else 0;
    so the coarse entry is 27*8*[I==J] - prod_d s_d = 152 / -16 / -4 / -1.
    """
    rows = []
    for p in range(h ** 3):
        x, y, z = p % h, (p // h) % h, p // (h * h)
        r = []
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    qx, qy, qz = x + dx, y + dy, z + dz
                    if not (0 <= qx < h and 0 <= qy < h and 0 <= qz < h):
                        continue
                    s = 1
                    for d in (dx, dy, dz):
                        s *= 4 if d == 0 else 1
                    v = 27 * 8 * ((dx, dy, dz) == (0, 0, 0)) - s
                    r.append((qz * h * h + qy * h + qx, float(v)))
        rows.append(r)
    return rows


@pytest.mark.parametrize("g", [2, 4, 8])
def test_galerkin_closed_form_and_association(g):
    A = synth.stencil27(g)
    P, Pt = synth.aggregation_2x2x2(g)
    AP = oracle.spgemm(A, P)
    assert AP.nnz == (2 * g - 2) ** 3  # per axis: 2 aggregates reached, 1 at the two ends
    fm_ap, _, _ = oracle.flops(A, P)
    assert fm_ap == A.nnz  # P has one entry per row
    R = oracle.spgemm(Pt, AP)
    assert_rows_equal(R, galerkin_coarse_closed_form(g // 2))
    # association: (P^T A) P has the identical pattern and values
    PtA = oracle.spgemm(Pt, A)
    R2 = oracle.spgemm(PtA, P)
    assert np.array_equal(R.row_ptr, R2.row_ptr)
    assert np.array_equal(R.col_idx, R2.col_idx)
    assert np.array_equal(R.values, R2.values)
    # f_m(R*A) == f_m(A*P) for symmetric A, R = P^T (paired multigrid rows of Table 3)
    assert oracle.flops(Pt, A)[0] == oracle.flops(A, P)[0]


@pytest.mark.slow
def test_galerkin_100cubed_counts():
    g = 100
    A = synth.stencil27(g)
    P, Pt = synth.aggregation_2x2x2(g)
    AP = oracle.spgemm(A, P)
    assert AP.nnz == 198 ** 3 == 7762392
    R = oracle.spgemm(Pt, AP)
    assert R.nnz == 148 ** 3 == 3241792
    vals = set(np.unique(R.values).tolist())
    assert vals == {152.0, -16.0, -4.0, -1.0}
    rs = np.add.reduceat(R.values, R.row_ptr[:-1])
    h = 50
    c = np.arange(h ** 3)
    cx, cy, cz = c % h, (c // h) % h, c // (h * h)
    interior = (cx > 0) & (cx < h - 1) & (cy > 0) & (cy < h - 1) & (cz > 0) & (cz < h - 1)
    assert interior.sum() == 110592 and np.all(rs[interior] == 0)


# ---------------------------------------------------------------- brute force
def _cases():
    rng = np.random.default_rng(1234)
    out = []
    for t in range(160):
        m, n, k = (int(v) for v in rng.integers(0, 41, 3))
        if t % 17 == 0:
            k = 1
        dA, dB = float(rng.uniform(0, 0.6)), float(rng.uniform(0, 0.6))
        out.append((m, n, k, dA, dB, t))
    out += [(0, 0, 0, 0.5, 0.5, 1001), (5, 0, 7, 0.5, 0.5, 1002), (0, 4, 3, 0.5, 0.5, 1003),
            (6, 6, 6, 0.0, 0.5, 1004), (6, 6, 6, 1.0, 1.0, 1005), (40, 40, 40, 1.0, 1.0, 1006)]
    return out


@pytest.mark.parametrize("m,n,k,dA,dB,seed", _cases())
def test_bruteforce_dense(m, n, k, dA, dB, seed):
    A = synth.shuffle_columns(synth.tiny_random(m, n, dA, seed, "int", zero_frac=0.2), seed)
    B = synth.shuffle_columns(synth.tiny_random(n, k, dB, seed + 7, "int", zero_frac=0.2), seed + 1)
    C = oracle.spgemm(A, B)
    pat = (synth.pattern_dense(A) @ synth.pattern_dense(B)) > 0
    assert C.nnz == int(pat.sum())
    assert np.array_equal(synth.pattern_dense(C).astype(bool), pat)
    for i in range(C.nrows):  # strictly increasing columns
        assert np.all(np.diff(C.col_idx[C.row_ptr[i]:C.row_ptr[i + 1]]) > 0)
    # small integers: every partial sum is exact, so dense equality is exact
    assert np.array_equal(synth.to_dense(C), synth.to_dense(A) @ synth.to_dense(B))
    fm, maxrf, rf = oracle.flops(A, B)
    # f_m counted column-wise: B(j,:) is read once per stored A(:,j)
    colcnt = np.bincount(A.col_idx, minlength=n) if A.nnz else np.zeros(n, np.int64)
    assert fm == int((colcnt * B.row_lengths()).sum()) if n else fm == 0
    assert C.nnz <= fm
    assert np.array_equal(np.diff(oracle.symbolic(A, B)), C.row_lengths())


def test_structural_zeros_kept():
    # A = [1 1], B = [[1],[-1]] -> C = [0] stored
    A = synth.Csr(1, 2, np.array([0, 2]), np.array([0, 1], np.int32), np.array([1.0, 1.0]))
    B = synth.Csr(2, 1, np.array([0, 1, 2]), np.array([0, 0], np.int32), np.array([1.0, -1.0]))
    C = oracle.spgemm(A, B)
    assert C.nnz == 1 and C.values[0] == 0.0


def test_rows_with_nothing():
    A = synth.tiny_random(30, 20, 0.3, 3)
    B = synth.tiny_random(20, 25, 0.0, 4)  # B has no entries at all
    C = oracle.spgemm(A, B)
    assert C.nnz == 0 and np.all(C.row_ptr == 0)


def test_row_sum_invariant_normal_values():
    A = synth.random_csr(300, 200, np.random.default_rng(0).integers(0, 30, 300), 11)
    B = synth.random_csr(200, 500, np.random.default_rng(1).integers(0, 30, 200), 12)
    C, S = oracle.spgemm(A, B, with_abs=True)
    ones = np.ones(500)
    lhs = np.add.reduceat(np.append(C.values, 0), C.row_ptr[:-1])[:300] * (np.diff(C.row_ptr) > 0)
    Bd = synth.to_dense(B)
    rhs = synth.to_dense(A) @ (Bd @ ones)
    scale = synth.to_dense(A.with_values(np.abs(A.values))) @ (np.abs(Bd) @ ones)
    assert np.all(np.abs(lhs - rhs) <= 1e-12 * np.maximum(scale, 1e-300))
    assert np.all(S >= np.abs(C.values))


def test_transpose_pattern_identity():
    A = synth.tiny_random(25, 30, 0.2, 8)
    B = synth.tiny_random(30, 35, 0.2, 9)

    def T(M):
        D = synth.to_dense(M).T
        pd = synth.pattern_dense(M).T
        rows, cols = np.nonzero(pd)
        rp = np.zeros(D.shape[0] + 1, np.int64)
        np.cumsum(np.bincount(rows, minlength=D.shape[0]), out=rp[1:])
        return synth.Csr(D.shape[0], D.shape[1], rp, cols.astype(np.int32), D[rows, cols])

    C = oracle.spgemm(A, B)
    Ct = oracle.spgemm(T(B), T(A))
    assert np.array_equal(synth.pattern_dense(C).T, synth.pattern_dense(Ct))
    assert np.array_equal(synth.to_dense(C).T, synth.to_dense(Ct))


def test_block_counts():
    B = synth.shuffle_columns(synth.tiny_random(40, 300, 0.1, 21), 2)
    for w in (1, 8, 32, 64):
        want = [len({int(c) // w for c in B.col_idx[B.row_ptr[r]:B.row_ptr[r + 1]]}) for r in range(40)]
        assert list(oracle.block_counts(B, w)) == want
    assert np.array_equal(oracle.block_counts(B, 1), B.row_lengths())


def test_dimension_mismatch_raises():
    A = synth.tiny_random(3, 4, 0.5, 1)
    B = synth.tiny_random(5, 2, 0.5, 2)
    with pytest.raises(ValueError):
        oracle.spgemm(A, B)


# ---------------------------------------------------------------- gradient
@pytest.mark.parametrize("seed", range(12))
def test_grad_matches_dense_formula(seed):
    rng = np.random.default_rng(seed)
    m, n, k = (int(v) for v in rng.integers(1, 30, 3))
    A = synth.shuffle_columns(synth.tiny_random(m, n, 0.3, seed, "int"), seed)
    B = synth.tiny_random(n, k, 0.3, seed + 50, "int")
    C = oracle.spgemm(A, B)
    G = rng.integers(-3, 4, C.nnz).astype(np.float64)
    dA, dB = oracle.grad(A, B, C, G)
    Gd = synth.to_dense(C.with_values(G))
    ref_dA = Gd @ synth.to_dense(B).T
    ref_dB = synth.to_dense(A).T @ Gd
    ra = np.repeat(np.arange(m), A.row_lengths())
    rb = np.repeat(np.arange(n), B.row_lengths())
    assert np.array_equal(dA, ref_dA[ra, A.col_idx])
    assert np.array_equal(dB, ref_dB[rb, B.col_idx])


def test_grad_finite_difference():
    """L(A,B) = sum(G*C) is bilinear, so central differences are exact up to rounding."""
    rng = np.random.default_rng(3)
    A = synth.random_csr(20, 15, rng.integers(1, 6, 20), 1)
    B = synth.random_csr(15, 25, rng.integers(1, 6, 15), 2)
    C = oracle.spgemm(A, B)
    G = rng.standard_normal(C.nnz)
    dA, dB = oracle.grad(A, B, C, G)

    def L(Av, Bv):
        Cv = oracle.spgemm(A.with_values(Av), B.with_values(Bv))
        return float(np.dot(Cv.values, G))

    h = 1e-6
    for e in rng.integers(0, A.nnz, 10):
        ap, am = A.values.copy(), A.values.copy()
        ap[e] += h
        am[e] -= h
        assert abs((L(ap, B.values) - L(am, B.values)) / (2 * h) - dA[e]) < 1e-7
    for f in rng.integers(0, B.nnz, 10):
        bp, bm = B.values.copy(), B.values.copy()
        bp[f] += h
        bm[f] -= h
        assert abs((L(A.values, bp) - L(A.values, bm)) / (2 * h) - dB[f]) < 1e-7


def test_rows_agree_with_the_whole_product():
    """Selected rows by the sampled entry point equal the same rows of the full product."""
    rng = np.random.default_rng(4)
    A = synth.shuffle_columns(synth.random_csr(200, 150, rng.integers(0, 12, 200), 1), 3)
    B = synth.random_csr(150, 400, rng.integers(0, 15, 150), 2)
    C, S = oracle.spgemm(A, B, with_abs=True)
    sel = np.array([0, 199, 5, 5, 77, 120], dtype=np.int64)
    rp, ci, va, ab = oracle.rows(A, B, sel)
    for t, i in enumerate(sel):
        s, e = C.row_ptr[i], C.row_ptr[i + 1]
        assert np.array_equal(ci[rp[t]:rp[t + 1]], C.col_idx[s:e])
        assert np.array_equal(va[rp[t]:rp[t + 1]], C.values[s:e])
        assert np.array_equal(ab[rp[t]:rp[t + 1]], S[s:e])


# ---------------------------------------------------------------- column-set words (Compression subsection)
def _run_words(c0, c1):
    """Words of 32 columns spanned by the contiguous column run [c0, c1]."""
    return (c1 >> 5) - (c0 >> 5) + 1


def geometric_words_27pt(g):
    """Column-set words per row of the 27-point operator on g^3, from grid
    coordinates: each row reads, per neighbour line (y+dy, z+dz), the column
    run x-1..x+1 (clipped) at offset g*(y+dy) + g^2*(z+dz).  Lines lie g > 35
    columns apart, so no two share a word."""
    p = np.arange(g ** 3, dtype=np.int64)
    x, y, z = p % g, (p // g) % g, p // (g * g)
    lo, hi = np.maximum(x - 1, 0), np.minimum(x + 1, g - 1)
    out = np.zeros(p.size, dtype=np.int64)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            ok = (y + dy >= 0) & (y + dy < g) & (z + dz >= 0) & (z + dz < g)
            base = g * (y + dy) + g * g * (z + dz)
            out += np.where(ok, _run_words(base + lo, base + hi), 0)
    return out


def geometric_words_5pt(g):
    """The same for the 5-point operator on g^2 (g > 35): lines y-1 and y+1
    hold one column, line y the run x-1..x+1."""
    p = np.arange(g * g, dtype=np.int64)
    x, y = p % g, p // g
    lo, hi = np.maximum(x - 1, 0), np.minimum(x + 1, g - 1)
    return (y > 0).astype(np.int64) + (y < g - 1) + _run_words(g * y + lo, g * y + hi)


def geometric_words_ap(g):
    """Rows of A*P (27-point operator times 2x2x2 aggregation, h = g/2 > 35
    aggregates per line): fine point (x, y, z) reaches the aggregates of its
    neighbours, i.e. per distinct aggregate line (Y, Z) among
    ((y+dy)//2, (z+dz)//2) the aggregate run (x-1)//2 .. (x+1)//2 (clipped)."""
    h = g // 2
    p = np.arange(g ** 3, dtype=np.int64)
    x, y, z = p % g, (p // g) % g, p // (g * g)
    lo, hi = np.maximum(x - 1, 0) // 2, np.minimum(x + 1, g - 1) // 2
    # distinct aggregate lines: Y in {(y-1)//2, (y+1)//2} (clipped), same for Z
    ylo, yhi = np.maximum(y - 1, 0) // 2, np.minimum(y + 1, g - 1) // 2
    zlo, zhi = np.maximum(z - 1, 0) // 2, np.minimum(z + 1, g - 1) // 2
    out = np.zeros(p.size, dtype=np.int64)
    for zsel in (0, 1):
        for ysel in (0, 1):
            Z = np.where(zsel == 0, zlo, zhi)
            Y = np.where(ysel == 0, ylo, yhi)
            ok = ((zsel == 0) | (zhi != zlo)) & ((ysel == 0) | (yhi != ylo))
            base = h * Y + h * h * Z
            out += np.where(ok, _run_words(base + lo, base + hi), 0)
    return out


def test_block_counts_27pt_geometric():
    A = synth.stencil27(100)
    want = geometric_words_27pt(100)
    got = oracle.block_counts(A, 32)
    assert np.array_equal(got, want)
    # 9,413,224 pairs; compressed flops 250,303,600 of 704,969,000 (CF 0.355)
    assert int(got.sum()) == 9_413_224
    assert int(got[A.col_idx].sum()) == 250_303_600


def test_block_counts_5pt_geometric():
    A = synth.laplace2d_5pt(64, 64)
    got = oracle.block_counts(A, 32)
    assert np.array_equal(got, geometric_words_5pt(64))
    assert int(got.sum()) == 12_288  # CF 0.607 over A*A's 100,104 flops
    assert abs(got[A.col_idx].sum() / 100_104 - 0.607) < 5e-4


def test_block_counts_galerkin_geometric():
    A = synth.stencil27(100)
    P, Pt = synth.aggregation_2x2x2(100)
    AP = oracle.spgemm(A, P)
    got = oracle.block_counts(AP, 32)
    assert np.array_equal(got, geometric_words_ap(100))
    # P^T reads every row of A*P once: compressed flops = pairs of compressed AP,
    # f_m = nnz(A*P) = 198^3; CF 0.520
    assert int(got[Pt.col_idx].sum()) == int(got.sum()) == 4_038_012
    assert AP.nnz == 198 ** 3
    assert abs(got.sum() / 198 ** 3 - 0.520) < 5e-4


def test_block_counts_invariants():
    rng = np.random.default_rng(5)
    B = synth.shuffle_columns(synth.tiny_random(60, 1000, 0.05, 23), 4)
    lens = B.row_lengths()
    prev = oracle.block_counts(B, 1)
    for w in (2, 4, 8, 16, 32, 64, 1000):
        c = oracle.block_counts(B, w)
        # at most one word per entry and at most ceil(k / w) words; coarser
        # words never split a finer word
        assert np.all(c <= lens) and np.all(c <= -(-1000 // w))
        assert np.all(c <= prev)
        assert np.all((c > 0) == (lens > 0))
        prev = c
    assert np.array_equal(oracle.block_counts(B, 1000), (lens > 0).astype(np.int64))
    # a dense row of k columns has ceil(k / w) words
    D = synth.Csr(1, 77, np.array([0, 77]), rng.permutation(77).astype(np.int32), np.ones(77))
    for w in (1, 5, 32, 77):
        assert oracle.block_counts(D, w)[0] == -(-77 // w)


# ---------------------------------------------------------------- masked product
def _graph_lower(nv, edges):
    """Strictly lower triangle L of an undirected graph's adjacency (sorted rows)."""
    rows = [[] for _ in range(nv)]
    for a, b in edges:
        if a != b:
            hi, lo = max(a, b), min(a, b)
            if lo not in rows[hi]:
                rows[hi].append(lo)
    rp = np.zeros(nv + 1, dtype=np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    ci = np.array([c for r in rows for c in sorted(r)], dtype=np.int32)
    return synth.Csr(nv, nv, rp, ci, np.ones(ci.size))


def _triangles(nv, edges):
    L = _graph_lower(nv, edges)
    return float(oracle.masked(L, L, L, structural=True).sum())


def test_masked_triangle_counts_known_graphs():
    from itertools import combinations
    for n in (3, 4, 7, 12):  # complete graph: C(n, 3) triangles
        assert _triangles(n, list(combinations(range(n), 2))) == n * (n - 1) * (n - 2) / 6
    for n in (4, 5, 9):  # wheel: hub 0 joined to a cycle of n vertices: n triangles
        cyc = [(1 + i, 1 + (i + 1) % n) for i in range(n)]
        assert _triangles(n + 1, cyc + [(0, 1 + i) for i in range(n)]) == n
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    assert _triangles(10, outer + spokes + inner) == 0  # Petersen graph
    assert _triangles(7, [(a, b) for a in range(3) for b in range(3, 7)]) == 0  # K_{3,4}
    octa = [(a, b) for a, b in combinations(range(6), 2) if (a, b) not in ((0, 3), (1, 4), (2, 5))]
    assert _triangles(6, octa) == 8  # octahedron K_{2,2,2}


def test_masked_triangles_match_trace():
    A = synth.rmat_symmetric(8, 8, seed=3)
    D = (synth.to_dense(A) != 0).astype(np.float64)
    want = np.trace(D @ D @ D) / 6
    lower = np.tril(D, -1)
    rr, cc = np.nonzero(lower)
    rp = np.zeros(A.nrows + 1, dtype=np.int64)
    np.add.at(rp, rr + 1, 1)
    rp = np.cumsum(rp)
    L = synth.Csr(A.nrows, A.nrows, rp, cc.astype(np.int32), np.ones(cc.size))
    assert oracle.masked(L, L, L, structural=True).sum() == want


@pytest.mark.parametrize("seed", range(10))
def test_masked_brute_force(seed):
    rng = np.random.default_rng(seed)
    m, n, k = (int(x) for x in rng.integers(1, 30, 3))
    A = synth.shuffle_columns(synth.tiny_random(m, n, rng.uniform(0, 0.6), seed), seed + 1)
    B = synth.shuffle_columns(synth.tiny_random(n, k, rng.uniform(0, 0.6), seed + 2), seed + 3)
    M = synth.shuffle_columns(synth.tiny_random(m, k, rng.uniform(0, 0.7), seed + 4), seed + 5)
    Da, Db = synth.to_dense(A), synth.to_dense(B)
    full = Da @ Db
    cnt = synth.pattern_dense(A).astype(float) @ synth.pattern_dense(B).astype(float)  # stored zeros count
    ab = np.abs(Da) @ np.abs(Db)
    rows = np.repeat(np.arange(m), M.row_lengths())
    got, S = oracle.masked(A, B, M, with_abs=True)
    assert np.allclose(got, full[rows, M.col_idx], rtol=1e-13, atol=1e-13)
    assert np.allclose(S, ab[rows, M.col_idx], rtol=1e-13, atol=1e-13)
    assert np.array_equal(oracle.masked(A, B, M, structural=True), cnt[rows, M.col_idx])
    # the mask equal to C's own pattern gives C's values in C's order
    C = oracle.spgemm(A, B)
    assert np.array_equal(oracle.masked(A, B, C), C.values)


def test_rows_check_helper_agrees_with_rows():
    """The comparison helper accepts the oracle's own rows and flags a changed
    value and a changed column."""
    A = synth.shuffle_columns(synth.tiny_random(60, 50, 0.2, 31, dist="normal"), 32)
    B = synth.tiny_random(50, 70, 0.2, 33, dist="normal")
    sel = np.array([0, 5, 17, 59, 5])
    rp, ci, va, ab = oracle.rows(A, B, sel)
    ok = oracle.rows_check(A, B, sel, rp, ci, va, 1e-12, 0)
    assert ok["bad"] == 0 and ok["bad_rows"] == 0 and ok["entries"] == rp[-1] and ok["max_rel_S"] == 0.0
    va2 = va.copy()
    va2[3] += 1e-3 * max(ab[3], 1.0)
    r2 = oracle.rows_check(A, B, sel, rp, ci, va2, 1e-12, 0)
    assert r2["bad"] == 1
    ci2 = ci.copy()
    ci2[0] = ci2[0] + 1000
    assert oracle.rows_check(A, B, sel, rp, ci2, va, 1e-12, 0)["bad_rows"] == 1
