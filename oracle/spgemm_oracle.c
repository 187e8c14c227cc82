/*
 * Plain sequential CPU oracle for two-phase sparse matrix-matrix multiply
 * C = A * B on CSR.  TEST INFRASTRUCTURE ONLY: tests, the smoke check and the
 * benchmark's CPU-baseline leg call it; the GPU library never does and shares
 * no code, header or table with it.
 *
 * What it computes is the plain definition of the product (Gustavson's
 * row-by-row formulation, Background section, Algorithm 1):
 *   pattern(C) = { (i,j) : some k has A(i,k) and B(k,j) stored }   (structural:
 *                entries that cancel to 0.0 stay, because the symbolic phase
 *                never looks at values, Algorithms section, Algorithm 2)
 *   C(i,j)     = sum over stored A(i,k) of A(i,k) * B(k,j)
 * computed in IEEE double with each product rounded before the add (build with
 * -ffp-contract=off), with a dense sparse-accumulator ("dense accumulator",
 * Accumulators subsection: a value array of size k plus a marker array, the
 * touched columns kept in a list) and the touched columns of each row sorted
 * ascending on output.
 *
 * All index arithmetic is int64.  Inputs: row_ptr int64, col_idx int32,
 * values double (callers widen float exactly).  Return codes: 0 ok,
 * -1 bad argument or index out of range, -2 row_ptr mismatch, -3 out of memory.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static int check_csr(int64_t m, int64_t ncols, const int64_t *rp, const int32_t *ci) {
    if (m < 0 || ncols < 0) return -1;
    if (m > 0 && rp[0] != 0) return -1;
    for (int64_t i = 0; i < m; ++i) {
        if (rp[i + 1] < rp[i]) return -1;
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e)
            if (ci[e] < 0 || (int64_t)ci[e] >= ncols) return -1;
    }
    return 0;
}

/* f_m: number of multiplications, i.e. sum over stored A(i,k) of |B(k,:)|
 * (Background section).  row_flops (nullable) gets the per-row counts;
 * *max_row_flops the largest one.  Returns f_m, or -1 on bad input. */
int64_t spo_flops(int64_t m, int64_t n, const int64_t *arp, const int32_t *aci,
                  const int64_t *brp, int64_t *row_flops, int64_t *max_row_flops) {
    if (check_csr(m, n, arp, aci)) return -1;
    int64_t total = 0, mx = 0;
    for (int64_t i = 0; i < m; ++i) {
        int64_t f = 0;
        for (int64_t e = arp[i]; e < arp[i + 1]; ++e) {
            int64_t r = aci[e];
            f += brp[r + 1] - brp[r];
        }
        if (row_flops) row_flops[i] = f;
        if (f > mx) mx = f;
        total += f;
    }
    if (max_row_flops) *max_row_flops = mx;
    return total;
}

/* Number of distinct column blocks col / width in each row of B: the row
 * lengths of B after packing `width` columns into one bit-set word
 * (Compression subsection).  Returns 0, or -1 / -3. */
int spo_block_counts(int64_t n, int64_t k, const int64_t *brp, const int32_t *bci,
                     int32_t width, int64_t *counts) {
    if (width <= 0 || check_csr(n, k, brp, bci)) return -1;
    int64_t nblk = (k + width - 1) / width;
    int64_t *mark = (int64_t *)malloc((size_t)(nblk > 0 ? nblk : 1) * sizeof(int64_t));
    if (!mark) return -3;
    for (int64_t b = 0; b < nblk; ++b) mark[b] = -1;
    for (int64_t r = 0; r < n; ++r) {
        int64_t c = 0;
        for (int64_t e = brp[r]; e < brp[r + 1]; ++e) {
            int64_t blk = bci[e] / width;
            if (mark[blk] != r) { mark[blk] = r; ++c; }
        }
        counts[r] = c;
    }
    free(mark);
    return 0;
}

/* Symbolic phase by definition: crp[i+1]-crp[i] = |pattern(C(i,:))|,
 * crp[0] = 0 (exclusive scan of the row sizes). */
int spo_symbolic(int64_t m, int64_t n, int64_t k,
                 const int64_t *arp, const int32_t *aci,
                 const int64_t *brp, const int32_t *bci, int64_t *crp) {
    if (check_csr(m, n, arp, aci) || check_csr(n, k, brp, bci)) return -1;
    int64_t *mark = (int64_t *)malloc((size_t)(k > 0 ? k : 1) * sizeof(int64_t));
    if (!mark) return -3;
    for (int64_t j = 0; j < k; ++j) mark[j] = -1;
    crp[0] = 0;
    for (int64_t i = 0; i < m; ++i) {
        int64_t cnt = 0;
        for (int64_t e = arp[i]; e < arp[i + 1]; ++e) {
            int64_t r = aci[e];
            for (int64_t f = brp[r]; f < brp[r + 1]; ++f) {
                int64_t j = bci[f];
                if (mark[j] != i) { mark[j] = i; ++cnt; }
            }
        }
        crp[i + 1] = crp[i] + cnt;
    }
    free(mark);
    return 0;
}

static int cmp_i32(const void *x, const void *y) {
    int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    return (a > b) - (a < b);
}

/* Numeric phase by definition.  crp must be the symbolic result.  Writes
 * sorted columns cci and values cval; cabs (nullable) gets, per entry,
 * sum over k of |A(i,k) * B(k,j)| (the scale the floating-point tolerances
 * are stated against). */
int spo_numeric(int64_t m, int64_t n, int64_t k,
                const int64_t *arp, const int32_t *aci, const double *aval,
                const int64_t *brp, const int32_t *bci, const double *bval,
                const int64_t *crp, int32_t *cci, double *cval, double *cabs) {
    if (check_csr(m, n, arp, aci) || check_csr(n, k, brp, bci)) return -1;
    size_t kk = (size_t)(k > 0 ? k : 1);
    int64_t *mark = (int64_t *)malloc(kk * sizeof(int64_t));
    double *acc = (double *)malloc(kk * sizeof(double));
    double *aab = (double *)malloc(kk * sizeof(double));
    int32_t *touched = (int32_t *)malloc(kk * sizeof(int32_t));
    if (!mark || !acc || !aab || !touched) {
        free(mark); free(acc); free(aab); free(touched);
        return -3;
    }
    for (int64_t j = 0; j < k; ++j) mark[j] = -1;
    int rc = 0;
    for (int64_t i = 0; i < m && rc == 0; ++i) {
        int64_t nt = 0;
        for (int64_t e = arp[i]; e < arp[i + 1]; ++e) {
            int64_t r = aci[e];
            double a = aval[e];
            for (int64_t f = brp[r]; f < brp[r + 1]; ++f) {
                int32_t j = bci[f];
                double p = a * bval[f];
                if (mark[j] != i) {
                    mark[j] = i;
                    acc[j] = 0.0;
                    aab[j] = 0.0;
                    touched[nt++] = j;
                }
                acc[j] = acc[j] + p;
                aab[j] = aab[j] + (p < 0 ? -p : p);
            }
        }
        if (crp[i + 1] - crp[i] != nt) { rc = -2; break; }
        qsort(touched, (size_t)nt, sizeof(int32_t), cmp_i32);
        int64_t base = crp[i];
        for (int64_t t = 0; t < nt; ++t) {
            int32_t j = touched[t];
            cci[base + t] = j;
            cval[base + t] = acc[j];
            if (cabs) cabs[base + t] = aab[j];
        }
    }
    free(mark); free(acc); free(aab); free(touched);
    return rc;
}

/* Gradient of L = sum over pattern(C) of G(i,j) * C(i,j) with C = A * B,
 * restricted to the stored entries of A and B:
 *   dA(i,k) = sum over stored B(k,j) of G(i,j) * B(k,j)
 *   dB(k,j) = sum over stored A(i,k) of A(i,k) * G(i,j)
 * G is given on pattern(C) with sorted columns (crp, cci, gval).  Each C entry
 * is located by binary search in its sorted row.  dA, dB are nnz(A), nnz(B). */
static int64_t find_col(const int32_t *cci, int64_t lo, int64_t hi, int32_t j) {
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (cci[mid] < j) lo = mid + 1; else hi = mid;
    }
    return lo;
}

int spo_grad(int64_t m, int64_t n, int64_t k,
             const int64_t *arp, const int32_t *aci, const double *aval,
             const int64_t *brp, const int32_t *bci, const double *bval,
             const int64_t *crp, const int32_t *cci, const double *gval,
             double *dA, double *dB) {
    if (check_csr(m, n, arp, aci) || check_csr(n, k, brp, bci)) return -1;
    int64_t nnzb = n > 0 ? brp[n] : 0;
    for (int64_t f = 0; f < nnzb; ++f) dB[f] = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t e = arp[i]; e < arp[i + 1]; ++e) {
            int64_t r = aci[e];
            double a = aval[e], s = 0.0;
            for (int64_t f = brp[r]; f < brp[r + 1]; ++f) {
                int64_t p = find_col(cci, crp[i], crp[i + 1], bci[f]);
                if (p >= crp[i + 1] || cci[p] != bci[f]) return -2;
                s = s + gval[p] * bval[f];
                dB[f] = dB[f] + a * gval[p];
            }
            dA[e] = s;
        }
    }
    return 0;
}

/* Selected rows of C = A * B by the same definition (for products too large
 * to form whole): rows[0..nsel) are row indices of A; out_rp (nsel+1) gets
 * the offsets of the selected rows in the compact output.  Call with
 * out_ci == NULL to get the sizes only (out_rp filled), then again with the
 * arrays of out_rp[nsel] entries.  Columns sorted per row. */
int spo_rows(int64_t m, int64_t n, int64_t k,
             const int64_t *arp, const int32_t *aci, const double *aval,
             const int64_t *brp, const int32_t *bci, const double *bval,
             int64_t nsel, const int64_t *rows,
             int64_t *out_rp, int32_t *out_ci, double *out_val, double *out_abs) {
    if (check_csr(m, n, arp, aci) || check_csr(n, k, brp, bci)) return -1;
    size_t kk = (size_t)(k > 0 ? k : 1);
    int64_t *mark = (int64_t *)malloc(kk * sizeof(int64_t));
    double *acc = (double *)malloc(kk * sizeof(double));
    double *aab = (double *)malloc(kk * sizeof(double));
    int32_t *touched = (int32_t *)malloc(kk * sizeof(int32_t));
    if (!mark || !acc || !aab || !touched) {
        free(mark); free(acc); free(aab); free(touched);
        return -3;
    }
    for (int64_t j = 0; j < k; ++j) mark[j] = -1;
    if (!out_ci) out_rp[0] = 0;
    for (int64_t s = 0; s < nsel; ++s) {
        int64_t i = rows[s];
        if (i < 0 || i >= m) { free(mark); free(acc); free(aab); free(touched); return -1; }
        int64_t nt = 0;
        for (int64_t e = arp[i]; e < arp[i + 1]; ++e) {
            int64_t r = aci[e];
            double a = aval ? aval[e] : 0.0;
            for (int64_t f = brp[r]; f < brp[r + 1]; ++f) {
                int32_t j = bci[f];
                if (mark[j] != s) {
                    mark[j] = s;
                    acc[j] = 0.0;
                    aab[j] = 0.0;
                    touched[nt++] = j;
                }
                if (out_ci) {
                    double p = a * bval[f];
                    acc[j] = acc[j] + p;
                    aab[j] = aab[j] + (p < 0 ? -p : p);
                }
            }
        }
        if (!out_ci) { out_rp[s + 1] = out_rp[s] + nt; continue; }
        if (out_rp[s + 1] - out_rp[s] != nt) { free(mark); free(acc); free(aab); free(touched); return -2; }
        qsort(touched, (size_t)nt, sizeof(int32_t), cmp_i32);
        for (int64_t t = 0; t < nt; ++t) {
            int32_t j = touched[t];
            out_ci[out_rp[s] + t] = j;
            out_val[out_rp[s] + t] = acc[j];
            if (out_abs) out_abs[out_rp[s] + t] = aab[j];
        }
    }
    free(mark); free(acc); free(aab); free(touched);
    return 0;
}

/* Masked product by definition (graph-analytics use of the symbolic
 * structure, Background section; triangle counting over the compressed
 * structure, Compression subsection): for every stored entry (i, j) of the
 * mask M (m x k, values ignored),
 *   out[e] = sum over stored A(i,k) with B(k,j) stored of A(i,k) * B(k,j)
 * (0.0 when there is no such k), or, with structural != 0, the number of such
 * k (values ignored; the count of paths i -> k -> j).  Row i of A*B is formed
 * with the dense accumulator of spo_numeric, then read at M's columns.
 * out_abs (nullable): sum of |A(i,k) * B(k,j)| per entry.  Returns 0 / -1 / -3. */
int spo_masked(int64_t m, int64_t n, int64_t k,
               const int64_t *arp, const int32_t *aci, const double *aval,
               const int64_t *brp, const int32_t *bci, const double *bval,
               const int64_t *mrp, const int32_t *mci, int structural,
               double *out, double *out_abs) {
    if (check_csr(m, n, arp, aci) || check_csr(n, k, brp, bci) || check_csr(m, k, mrp, mci)) return -1;
    size_t kk = (size_t)(k > 0 ? k : 1);
    int64_t *mark = (int64_t *)malloc(kk * sizeof(int64_t));
    double *acc = (double *)malloc(kk * sizeof(double));
    double *aab = (double *)malloc(kk * sizeof(double));
    if (!mark || !acc || !aab) {
        free(mark); free(acc); free(aab);
        return -3;
    }
    for (int64_t j = 0; j < k; ++j) mark[j] = -1;
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t e = arp[i]; e < arp[i + 1]; ++e) {
            int64_t r = aci[e];
            for (int64_t f = brp[r]; f < brp[r + 1]; ++f) {
                int32_t j = bci[f];
                double p = structural ? 1.0 : aval[e] * bval[f];
                if (mark[j] != i) {
                    mark[j] = i;
                    acc[j] = 0.0;
                    aab[j] = 0.0;
                }
                acc[j] = acc[j] + p;
                aab[j] = aab[j] + (p < 0 ? -p : p);
            }
        }
        for (int64_t e = mrp[i]; e < mrp[i + 1]; ++e) {
            int32_t j = mci[e];
            out[e] = mark[j] == i ? acc[j] : 0.0;
            if (out_abs) out_abs[e] = mark[j] == i ? aab[j] : 0.0;
        }
    }
    free(mark); free(acc); free(aab);
    return 0;
}

/* Comparison helper for large products (test infrastructure, not part of
 * the definition): for each selected row rows[s] of C = A * B, form the row
 * by the definition above (dense accumulator, sorted columns) and compare it
 * with a candidate row given as (gci, gval) at offsets grp[s] .. grp[s+1]:
 * columns must be identical; each value must satisfy
 *   |g - c| <= tol * max(|c|, S)   (rel_mode 0)   or   |g - c| <= tol * S  (rel_mode 1)
 * with S = sum |A(i,k) * B(k,j)|.  stats[0] = max |g - c| / S over entries
 * (S > 0), stats[1] = entries over the bound, stats[2] = entries compared,
 * stats[3] = rows whose columns differ.  Every `stride`-th entry's |g - c| / S
 * goes to sub[] (capacity sub_cap; *nsub counts them) for a median.
 * Returns 0, or -1 / -3. */
int spo_rows_check(int64_t m, int64_t n, int64_t k,
                   const int64_t *arp, const int32_t *aci, const double *aval,
                   const int64_t *brp, const int32_t *bci, const double *bval,
                   int64_t nsel, const int64_t *rows,
                   const int64_t *grp, const int32_t *gci, const double *gval,
                   double tol, int rel_mode, double *stats,
                   int64_t stride, float *sub, int64_t sub_cap, int64_t *nsub) {
    if (check_csr(m, n, arp, aci) || check_csr(n, k, brp, bci)) return -1;
    size_t kk = (size_t)(k > 0 ? k : 1);
    int64_t *mark = (int64_t *)malloc(kk * sizeof(int64_t));
    double *acc = (double *)malloc(kk * sizeof(double));
    double *aab = (double *)malloc(kk * sizeof(double));
    int32_t *touched = (int32_t *)malloc(kk * sizeof(int32_t));
    if (!mark || !acc || !aab || !touched) {
        free(mark); free(acc); free(aab); free(touched);
        return -3;
    }
    for (int64_t j = 0; j < k; ++j) mark[j] = -1;
    double mx = 0.0, bad = 0.0, cnt = 0.0, badrows = 0.0;
    int64_t ns = 0, seen = 0;
    for (int64_t s = 0; s < nsel; ++s) {
        int64_t i = rows[s];
        if (i < 0 || i >= m) { free(mark); free(acc); free(aab); free(touched); return -1; }
        int64_t nt = 0;
        for (int64_t e = arp[i]; e < arp[i + 1]; ++e) {
            int64_t r = aci[e];
            double a = aval[e];
            for (int64_t f = brp[r]; f < brp[r + 1]; ++f) {
                int32_t j = bci[f];
                double p = a * bval[f];
                if (mark[j] != s) {
                    mark[j] = s;
                    acc[j] = 0.0;
                    aab[j] = 0.0;
                    touched[nt++] = j;
                }
                acc[j] = acc[j] + p;
                aab[j] = aab[j] + (p < 0 ? -p : p);
            }
        }
        qsort(touched, (size_t)nt, sizeof(int32_t), cmp_i32);
        int64_t g0 = grp[s], gn = grp[s + 1] - grp[s];
        int same = gn == nt;
        for (int64_t t = 0; same && t < nt; ++t) same = gci[g0 + t] == touched[t];
        if (!same) { badrows += 1.0; continue; }
        for (int64_t t = 0; t < nt; ++t) {
            int32_t j = touched[t];
            double c = acc[j], S = aab[j], g = gval[g0 + t];
            double d = g - c;
            if (d < 0) d = -d;
            double ac = c < 0 ? -c : c;
            double bound = tol * (rel_mode == 0 ? (ac > S ? ac : S) : S);
            if (d > bound) bad += 1.0;
            double rel = S > 0 ? d / S : 0.0;
            if (rel > mx) mx = rel;
            cnt += 1.0;
            if (stride > 0 && (seen % stride) == 0 && ns < sub_cap) sub[ns++] = (float)rel;
            ++seen;
        }
    }
    stats[0] = mx;
    stats[1] = bad;
    stats[2] = cnt;
    stats[3] = badrows;
    *nsub = ns;
    free(mark); free(acc); free(aab); free(touched);
    return 0;
}
