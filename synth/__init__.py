"""Seeded synthetic inputs for the two-phase SpGEMM tests and benchmark.

This module only *builds* input matrices (CSR, 32-bit column indices). It holds
none of the product's arithmetic, so the CPU oracle and the GPU library can both
be fed from it without sharing any step of the method.

Workload shapes follow the problem classes the paper measures in its
experiments section (Table 3): stencil squares A*A, multigrid triple products
R*A*P with R = P^T, and Kronecker/R-MAT graph squares; plus the batched and
differentiation forms. Every generator takes an explicit seed.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Csr:
    """Host CSR matrix: row_ptr int64[m+1], col_idx int32[nnz], values float64/32[nnz]."""

    nrows: int
    ncols: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    values: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1]) if self.nrows > 0 else 0

    def astype(self, dtype) -> "Csr":
        return Csr(self.nrows, self.ncols, self.row_ptr, self.col_idx,
                   self.values.astype(dtype))

    def with_values(self, values: np.ndarray) -> "Csr":
        assert values.shape == self.col_idx.shape
        return Csr(self.nrows, self.ncols, self.row_ptr, self.col_idx, values)

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.row_ptr)


def _from_dense_slots(cols: np.ndarray, vals: np.ndarray, ncols: int) -> Csr:
    """Rows given as fixed-width slot arrays, col < 0 marks an unused slot."""
    valid = cols >= 0
    counts = valid.sum(axis=1)
    rp = np.zeros(cols.shape[0] + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    return Csr(cols.shape[0], ncols, rp, cols[valid].astype(np.int32),
               vals[valid].astype(np.float64))


def laplace2d_5pt(nx: int, ny: int, diag: float = 4.0, off: float = -1.0) -> Csr:
    """2D 5-point Laplacian on an nx-by-ny grid, point (x, y) -> row y*nx + x.

    Columns are sorted per row. nnz = 5*nx*ny - 2*(nx+ny).
    """
    n = nx * ny
    p = np.arange(n, dtype=np.int64)
    x, y = p % nx, p // nx
    offs = [(0, -1), (-1, 0), (0, 0), (1, 0), (0, 1)]  # increasing column order
    cols = np.full((n, 5), -1, dtype=np.int64)
    vals = np.zeros((n, 5))
    for s, (dx, dy) in enumerate(offs):
        ok = (x + dx >= 0) & (x + dx < nx) & (y + dy >= 0) & (y + dy < ny)
        cols[ok, s] = p[ok] + dy * nx + dx
        vals[ok, s] = diag if (dx, dy) == (0, 0) else off
    return _from_dense_slots(cols, vals, n)


def stencil3d(g: int, points: int, diag: float, off: float) -> Csr:
    """3D 7- or 27-point stencil on a g^3 grid, point (x,y,z) -> z*g*g + y*g + x."""
    assert points in (7, 27)
    n = g ** 3
    p = np.arange(n, dtype=np.int64)
    x, y, z = p % g, (p // g) % g, p // (g * g)
    offs = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    if points == 7:
        offs = [o for o in offs if sum(abs(t) for t in o) <= 1]
    cols = np.full((n, len(offs)), -1, dtype=np.int64)
    vals = np.zeros((n, len(offs)))
    for s, (dx, dy, dz) in enumerate(offs):  # lexicographic (dz,dy,dx) = sorted columns
        ok = ((x + dx >= 0) & (x + dx < g) & (y + dy >= 0) & (y + dy < g)
              & (z + dz >= 0) & (z + dz < g))
        cols[ok, s] = p[ok] + dz * g * g + dy * g + dx
        vals[ok, s] = diag if (dx, dy, dz) == (0, 0, 0) else off
    return _from_dense_slots(cols, vals, n)


def stencil27(g: int) -> Csr:
    """27-point operator on g^3: diagonal 26, off-diagonal -1."""
    return stencil3d(g, 27, 26.0, -1.0)


def laplace7(g: int) -> Csr:
    """7-point Laplacian on g^3: diagonal 6, off-diagonal -1."""
    return stencil3d(g, 7, 6.0, -1.0)


def aggregation_2x2x2(g: int) -> tuple[Csr, Csr]:
    """Piecewise-constant prolongator P (g^3 x (g/2)^3, one 1.0 per row) and P^T.

    Fine point (x,y,z) belongs to aggregate (x//2, y//2, z//2). P^T is built
    directly (each aggregate lists its 8 fine points in increasing order).
    """
    assert g % 2 == 0
    h = g // 2
    n, nc = g ** 3, h ** 3
    p = np.arange(n, dtype=np.int64)
    x, y, z = p % g, (p // g) % g, p // (g * g)
    agg = (z // 2) * h * h + (y // 2) * h + (x // 2)
    P = Csr(n, nc, np.arange(n + 1, dtype=np.int64), agg.astype(np.int32), np.ones(n))
    c = np.arange(nc, dtype=np.int64)
    cx, cy, cz = c % h, (c // h) % h, c // (h * h)
    members = np.empty((nc, 8), dtype=np.int64)
    s = 0
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                members[:, s] = (2 * cz + dz) * g * g + (2 * cy + dy) * g + (2 * cx + dx)
                s += 1
    Pt = Csr(nc, n, np.arange(0, 8 * nc + 1, 8, dtype=np.int64),
             members.reshape(-1).astype(np.int32), np.ones(8 * nc))
    return P, Pt


def _csr_from_sorted_keys(keys: np.ndarray, nrows: int, ncols: int, vals: np.ndarray) -> Csr:
    rows = keys // ncols
    counts = np.bincount(rows, minlength=nrows)
    rp = np.zeros(nrows + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    return Csr(nrows, ncols, rp, (keys % ncols).astype(np.int32), vals)


def rmat_symmetric(scale: int, edge_factor: int = 16,
                   abcd=(0.57, 0.19, 0.19, 0.05), seed: int = 0) -> Csr:
    """Symmetric R-MAT graph as a sparse matrix.

    edge_factor * 2^scale directed edges, each by a recursive quadrant choice per
    bit with fixed (a, b, c, d) (no noise, no vertex permutation). Self-loops are
    dropped, the edge set is symmetrised by union and deduplicated. Each
    undirected edge gets one U[-1, 1) value, so the matrix is numerically
    symmetric. Columns are sorted per row.
    """
    rng = np.random.default_rng(seed)
    n = 1 << scale
    ne = edge_factor * n
    a, b, c, _ = abcd
    u = np.zeros(ne, dtype=np.int64)
    v = np.zeros(ne, dtype=np.int64)
    for bit in range(scale):
        r = rng.random(ne)
        ubit = r >= a + b              # quadrants c, d set the row bit
        vbit = ((r >= a) & (r < a + b)) | (r >= a + b + c)  # quadrants b, d set the column bit
        u |= ubit.astype(np.int64) << bit
        v |= vbit.astype(np.int64) << bit
    keep = u != v
    u, v = u[keep], v[keep]
    lo, hi = np.minimum(u, v), np.maximum(u, v)
    und = np.unique(lo * n + hi)
    w = rng.uniform(-1.0, 1.0, size=und.shape[0])
    lo, hi = und // n, und % n
    keys = np.concatenate([lo * n + hi, hi * n + lo])
    vals = np.concatenate([w, w])
    order = np.argsort(keys, kind="stable")
    return _csr_from_sorted_keys(keys[order], n, n, vals[order])


def _distinct_columns(rng, counts: np.ndarray, ncols: int) -> tuple[np.ndarray, np.ndarray]:
    """Per row r, counts[r] distinct uniform columns in [0, ncols), sorted.

    Returns (row_ptr, col_idx). Duplicates are redrawn until none remain.
    """
    counts = np.minimum(counts.astype(np.int64), ncols)
    m = counts.shape[0]
    rp = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    rows = np.repeat(np.arange(m, dtype=np.int64), counts)
    cols = rng.integers(0, ncols, size=rows.shape[0], dtype=np.int64)
    while True:
        ks = np.sort(rows * ncols + cols)
        dup = np.zeros(ks.shape[0], dtype=bool)
        dup[1:] = ks[1:] == ks[:-1]
        if not dup.any():
            return rp, (ks % ncols).astype(np.int32)
        cols = ks % ncols
        rows = ks // ncols
        cols[dup] = rng.integers(0, ncols, size=int(dup.sum()), dtype=np.int64)


def random_csr(m: int, k: int, counts: np.ndarray, seed: int, dist: str = "normal") -> Csr:
    """m x k matrix; row r has counts[r] distinct uniform columns (sorted)."""
    rng = np.random.default_rng(seed)
    rp, ci = _distinct_columns(rng, np.asarray(counts), k)
    return Csr(m, k, rp, ci, draw_values(rng, ci.shape[0], dist))


def draw_values(rng, size: int, dist: str) -> np.ndarray:
    if dist == "normal":
        return rng.standard_normal(size)
    if dist == "uniform":
        return rng.uniform(-1.0, 1.0, size)
    if dist == "ones":
        return np.ones(size)
    if dist == "int":  # small integers: exact in any summation order
        return rng.integers(-3, 4, size).astype(np.float64)
    raise ValueError(dist)


def revalue(A: Csr, seed: int, dist: str = "normal") -> Csr:
    """Same structure, fresh seeded values (the reuse case)."""
    rng = np.random.default_rng(seed)
    return A.with_values(draw_values(rng, A.nnz, dist).astype(A.values.dtype))


def fixed_row_random(n: int, k: int, per_row: int, seed: int) -> Csr:
    """n x k, exactly per_row distinct uniform columns per row, N(0,1) values."""
    return random_csr(n, k, np.full(n, per_row), seed, "normal")


def poisson_square(n: int, lam: float, seed: int) -> Csr:
    """n x n; row sizes Poisson(lam) (capped at n), distinct uniform columns, N(0,1)."""
    rng = np.random.default_rng(seed)
    counts = rng.poisson(lam, size=n)
    rp, ci = _distinct_columns(rng, counts, n)
    return Csr(n, n, rp, ci, rng.standard_normal(ci.shape[0]))


@dataclass
class BatchSpec:
    n: int
    lam: float
    seed_a: int
    seed_b: int


def batch_specs(count: int, seed: int, n_lo: int = 1000, n_hi: int = 65536,
                lam_lo: float = 4.0, lam_hi: float = 32.0) -> list[BatchSpec]:
    """Shapes of a batch of independent products C_i = A_i * B_i.

    n_i ~ U[n_lo, n_hi] (integers), one lambda_i ~ U[lam_lo, lam_hi] shared by
    A_i and B_i.
    """
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_lo, n_hi + 1, size=count)
    lams = rng.uniform(lam_lo, lam_hi, size=count)
    return [BatchSpec(int(ns[i]), float(lams[i]), seed * 100003 + 2 * i + 1,
                      seed * 100003 + 2 * i + 2) for i in range(count)]


def _batch_pair(s: BatchSpec) -> tuple[Csr, Csr]:
    return poisson_square(s.n, s.lam, s.seed_a), poisson_square(s.n, s.lam, s.seed_b)


def batch_matrices(specs: list[BatchSpec], workers: int = 0) -> list[tuple[Csr, Csr]]:
    """The batch's operands.  Each pair depends only on its own seeds, so with
    workers > 1 they are generated in that many spawned processes (same result)."""
    if workers <= 1 or len(specs) < 2 * workers:
        return [_batch_pair(s) for s in specs]
    import multiprocessing as mp

    with mp.get_context("spawn").Pool(workers) as pool:
        return pool.map(_batch_pair, specs, chunksize=max(1, len(specs) // (4 * workers)))


def batch_revalue(pairs, recompute: int, base_seed: int):
    """Fresh N(0,1) values for recomputation r (seed = base + 1000*r + i)."""
    out = []
    for i, (A, B) in enumerate(pairs):
        s = base_seed + 1000 * recompute + i
        out.append((revalue(A, 2 * s + 1), revalue(B, 2 * s + 2)))
    return out


def shuffle_columns(A: Csr, seed: int) -> Csr:
    """Same matrix with the entries of every row in a random order."""
    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(A.nrows, dtype=np.int64), A.row_lengths())
    order = np.lexsort((rng.random(A.nnz), rows))
    return Csr(A.nrows, A.ncols, A.row_ptr, A.col_idx[order], A.values[order])


def to_dense(A: Csr) -> np.ndarray:
    D = np.zeros((A.nrows, A.ncols), dtype=np.float64)
    rows = np.repeat(np.arange(A.nrows), A.row_lengths())
    np.add.at(D, (rows, A.col_idx.astype(np.int64)), A.values.astype(np.float64))
    return D


def pattern_dense(A: Csr) -> np.ndarray:
    D = np.zeros((A.nrows, A.ncols), dtype=np.int64)
    rows = np.repeat(np.arange(A.nrows), A.row_lengths())
    D[rows, A.col_idx.astype(np.int64)] = 1
    return D


def tiny_random(m: int, n: int, density: float, seed: int, dist: str = "int",
                zero_frac: float = 0.0) -> Csr:
    """Small random matrix by Bernoulli(density) per entry; optional explicit zeros."""
    rng = np.random.default_rng(seed)
    mask = rng.random((m, n)) < density
    counts = mask.sum(axis=1)
    rp = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    ci = np.nonzero(mask)[1].astype(np.int32)
    vals = draw_values(rng, ci.shape[0], dist)
    if zero_frac > 0:
        vals[rng.random(ci.shape[0]) < zero_frac] = 0.0
    return Csr(m, n, rp, ci, vals)
