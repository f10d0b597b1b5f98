/*
 * oracle.c -- plain sequential FP64 solvers for the structured systems A x = f
 * treated by the partition method of Amodio & Brugnano, "Parallel
 * factorizations in numerical analysis" (Sec. 2, eq. (syst)).
 *
 * TEST INFRASTRUCTURE ONLY.  The product library never links, loads or calls
 * this file.  It is used by the test-suite (parity reference), by the smoke
 * check and by the CPU-baseline leg of the benchmark, nothing else.
 *
 * The partition method computes the unique solution x = A^{-1} f of eq. (syst)
 * up to rounding, so every routine below is the plain definition of that
 * result written out: Gaussian elimination with row partial pivoting over the
 * whole matrix in its natural ordering (ties broken by the first index of the
 * largest magnitude), followed by forward and back substitution.  There is no
 * partitioning, blocking, reordering or fusion here.
 *
 * Conventions shared with the test-suite (not with the GPU code):
 *   - an m x m block is stored column-major: entry (i,j) at blk[i + j*m];
 *   - a block array holds consecutive blocks: block k starts at k*m*m;
 *   - block tridiagonal (BTRI) with nb block rows: D[k] = A(k,k) (k < nb),
 *     Lo[j] = A(j+1,j), Up[j] = A(j,j+1) (j < nb-1);
 *   - BABD (lower block bidiagonal plus top-right corner, Sec. 2, the
 *     bidiagonal form of eq. (parpart1)): D[0] = A(0,0), D[k] = A(k,k),
 *     Lo[j] = A(j+1,j), C = A(0,nb-1);
 *   - right-hand sides and solutions are n x nrhs column-major with leading
 *     dimension ld >= n = m*nb.
 * Every solver returns 0 on success, k+1 when the k-th pivot is exactly zero,
 * and -1 on allocation failure.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define BLK(arr, k, m) ((arr) + (size_t)(k) * (size_t)(m) * (size_t)(m))

/* ------------------------------------------------------------------------ */
/* Scalar tridiagonal: the Thomas algorithm (plain Gaussian elimination
 * without pivoting of a tridiagonal matrix).  lo[i] = A(i+1,i),
 * d[i] = A(i,i), up[i] = A(i,i+1).  Valid without pivoting for the strictly
 * diagonally dominant matrices it is used on. */
int orc_thomas(int64_t n, const double *lo, const double *d, const double *up,
               int64_t nrhs, const double *f, int64_t ldf, double *x,
               int64_t ldx)
{
    double *c = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!c) return -1;
    /* Forward elimination on the matrix: pivots piv_i = d_i - lo_{i-1} c_{i-1},
     * c_i = up_i / piv_i. */
    double *piv = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!piv) { free(c); return -1; }
    for (int64_t i = 0; i < n; ++i) {
        double p = d[i] - (i > 0 ? lo[i - 1] * c[i - 1] : 0.0);
        if (p == 0.0) { free(c); free(piv); return (int)(i + 1); }
        piv[i] = p;
        c[i] = (i < n - 1) ? up[i] / p : 0.0;
    }
    for (int64_t r = 0; r < nrhs; ++r) {
        const double *fr = f + r * ldf;
        double *xr = x + r * ldx;
        for (int64_t i = 0; i < n; ++i)
            xr[i] = (fr[i] - (i > 0 ? lo[i - 1] * xr[i - 1] : 0.0)) / piv[i];
        for (int64_t i = n - 2; i >= 0; --i) xr[i] -= c[i] * xr[i + 1];
    }
    free(c);
    free(piv);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Dense LU with row partial pivoting: a is n x n column-major with leading
 * dimension n, overwritten by the multipliers (below the diagonal, each
 * column as it was when it was eliminated) and U; ipiv[k] is the row swapped
 * with row k at step k.  So U = M_{n-1} S_{n-1} ... M_0 S_0 A, with S_k the
 * swap and M_k the elimination of step k. */
int orc_dense_getrf(int64_t n, double *a, int64_t *ipiv)
{
    int info = 0;
    for (int64_t k = 0; k < n; ++k) {
        int64_t p = k;
        double best = fabs(a[k + k * n]);
        for (int64_t i = k + 1; i < n; ++i) {
            double v = fabs(a[i + k * n]);
            if (v > best) { best = v; p = i; }
        }
        ipiv[k] = p;
        if (a[p + k * n] == 0.0) { if (!info) info = (int)(k + 1); continue; }
        /* swap only the trailing columns: the multipliers of earlier steps
         * stay as computed, which is what the interleaved solves expect */
        if (p != k)
            for (int64_t j = k; j < n; ++j) {
                double t = a[k + j * n]; a[k + j * n] = a[p + j * n]; a[p + j * n] = t;
            }
        double inv = 1.0 / a[k + k * n];
        for (int64_t i = k + 1; i < n; ++i) a[i + k * n] *= inv;
        for (int64_t j = k + 1; j < n; ++j) {
            double ukj = a[k + j * n];
            if (ukj == 0.0) continue;
            for (int64_t i = k + 1; i < n; ++i) a[i + j * n] -= a[i + k * n] * ukj;
        }
    }
    return info;
}

/* Solve with the dense factors: trans = 0 solves A x = b, trans = 1 solves
 * A^T x = b.  b is n x nrhs column-major (leading dimension ldb), in place. */
void orc_dense_getrs(int trans, int64_t n, const double *a, const int64_t *ipiv,
                     int64_t nrhs, double *b, int64_t ldb)
{
    for (int64_t r = 0; r < nrhs; ++r) {
        double *x = b + r * ldb;
        if (!trans) {
            for (int64_t k = 0; k < n; ++k) {           /* P, then L^{-1} */
                int64_t p = ipiv[k];
                if (p != k) { double t = x[k]; x[k] = x[p]; x[p] = t; }
                for (int64_t i = k + 1; i < n; ++i) x[i] -= a[i + k * n] * x[k];
            }
            for (int64_t k = n - 1; k >= 0; --k) {      /* U^{-1} */
                x[k] /= a[k + k * n];
                for (int64_t i = 0; i < k; ++i) x[i] -= a[i + k * n] * x[k];
            }
        } else {
            for (int64_t k = 0; k < n; ++k) {           /* U^{-T} */
                double s = x[k];
                for (int64_t i = 0; i < k; ++i) s -= a[i + k * n] * x[i];
                x[k] = s / a[k + k * n];
            }
            for (int64_t k = n - 1; k >= 0; --k) {      /* L^{-T}, then P^T */
                double s = x[k];
                for (int64_t i = k + 1; i < n; ++i) s -= a[i + k * n] * x[i];
                x[k] = s;
                int64_t p = ipiv[k];
                if (p != k) { double t = x[k]; x[k] = x[p]; x[p] = t; }
            }
        }
    }
}

int orc_dense_solve(int64_t n, const double *a_in, int64_t nrhs,
                    const double *f, int64_t ldf, double *x, int64_t ldx)
{
    double *a = (double *)malloc(sizeof(double) * (size_t)(n * n > 0 ? n * n : 1));
    int64_t *ipiv = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!a || !ipiv) { free(a); free(ipiv); return -1; }
    memcpy(a, a_in, sizeof(double) * (size_t)(n * n));
    int info = orc_dense_getrf(n, a, ipiv);
    if (!info) {
        for (int64_t r = 0; r < nrhs; ++r)
            memcpy(x + r * ldx, f + r * ldf, sizeof(double) * (size_t)n);
        orc_dense_getrs(0, n, a, ipiv, nrhs, x, ldx);
    }
    free(a);
    free(ipiv);
    return info;
}

/* ------------------------------------------------------------------------ */
/* Banded LU with row partial pivoting (gbtrf semantics, unblocked).
 * The band is held in an array ab of ldab = 2*kl + ku + 1 rows and n columns
 * (column-major); entry A(i,j) lives at ab[(kl + ku + i - j) + j*ldab].  The
 * top kl rows are room for the fill-in that row interchanges create in U,
 * whose upper bandwidth grows to kl + ku. */
#define AB(i, j) ab[(size_t)(kv + (i) - (j)) + (size_t)(j) * (size_t)ldab]

int orc_band_getrf(int64_t n, int64_t kl, int64_t ku, double *ab, int64_t ldab,
                   int64_t *ipiv)
{
    const int64_t kv = kl + ku;
    int info = 0;
    int64_t ju = 0; /* last column touched by U so far */
    for (int64_t j = 0; j < n; ++j) {
        int64_t km = kl < n - 1 - j ? kl : n - 1 - j;
        int64_t jp = 0;
        double best = fabs(AB(j, j));
        for (int64_t i = 1; i <= km; ++i) {
            double v = fabs(AB(j + i, j));
            if (v > best) { best = v; jp = i; }
        }
        ipiv[j] = j + jp;
        if (AB(j + jp, j) == 0.0) { if (!info) info = (int)(j + 1); continue; }
        int64_t lim = j + ku + jp < n - 1 ? j + ku + jp : n - 1;
        if (lim > ju) ju = lim;
        if (jp != 0)
            for (int64_t c = j; c <= ju; ++c) {
                double t = AB(j, c); AB(j, c) = AB(j + jp, c); AB(j + jp, c) = t;
            }
        double inv = 1.0 / AB(j, j);
        for (int64_t i = 1; i <= km; ++i) AB(j + i, j) *= inv;
        for (int64_t c = j + 1; c <= ju; ++c) {
            double ujc = AB(j, c);
            if (ujc == 0.0) continue;
            for (int64_t i = 1; i <= km; ++i) AB(j + i, c) -= AB(j + i, j) * ujc;
        }
    }
    return info;
}

/* Solve with the band factors (gbtrs semantics): trans = 0 solves A x = b,
 * trans = 1 solves A^T x = b; b is n x nrhs column-major, in place. */
void orc_band_getrs(int trans, int64_t n, int64_t kl, int64_t ku,
                    const double *ab, int64_t ldab, const int64_t *ipiv,
                    int64_t nrhs, double *b, int64_t ldb)
{
    const int64_t kv = kl + ku;
    for (int64_t r = 0; r < nrhs; ++r) {
        double *x = b + r * ldb;
        if (!trans) {
            for (int64_t j = 0; j < n; ++j) {            /* L^{-1} P */
                int64_t km = kl < n - 1 - j ? kl : n - 1 - j;
                int64_t p = ipiv[j];
                if (p != j) { double t = x[j]; x[j] = x[p]; x[p] = t; }
                for (int64_t i = 1; i <= km; ++i) x[j + i] -= AB(j + i, j) * x[j];
            }
            for (int64_t j = n - 1; j >= 0; --j) {       /* U^{-1}, bandwidth kv */
                x[j] /= AB(j, j);
                int64_t i0 = j - kv > 0 ? j - kv : 0;
                for (int64_t i = i0; i < j; ++i) x[i] -= AB(i, j) * x[j];
            }
        } else {
            for (int64_t j = 0; j < n; ++j) {            /* U^{-T} */
                double s = x[j];
                int64_t i0 = j - kv > 0 ? j - kv : 0;
                for (int64_t i = i0; i < j; ++i) s -= AB(i, j) * x[i];
                x[j] = s / AB(j, j);
            }
            for (int64_t j = n - 1; j >= 0; --j) {       /* L^{-T}, then P^T */
                int64_t km = kl < n - 1 - j ? kl : n - 1 - j;
                double s = x[j];
                for (int64_t i = 1; i <= km; ++i) s -= AB(j + i, j) * x[j + i];
                x[j] = s;
                int64_t p = ipiv[j];
                if (p != j) { double t = x[j]; x[j] = x[p]; x[p] = t; }
            }
        }
    }
}
#undef AB

/* Scatter a BTRI matrix into band storage with kl = ku = 2m-1 (the
 * element-level bandwidth of a block tridiagonal matrix). */
static void btri_to_band(int64_t m, int64_t nb, const double *D, const double *Lo,
                         const double *Up, double *ab, int64_t ldab)
{
    const int64_t kl = 2 * m - 1, ku = 2 * m - 1, kv = kl + ku;
    const int64_t n = m * nb;
    memset(ab, 0, sizeof(double) * (size_t)ldab * (size_t)n);
    for (int64_t k = 0; k < nb; ++k)
        for (int64_t j = 0; j < m; ++j)
            for (int64_t i = 0; i < m; ++i) {
                int64_t r = k * m + i, c = k * m + j;
                ab[(size_t)(kv + r - c) + (size_t)c * ldab] = BLK(D, k, m)[i + j * m];
                if (k + 1 < nb) {
                    /* Lo[k] = A(k+1,k), Up[k] = A(k,k+1) */
                    int64_t rl = (k + 1) * m + i, cl = k * m + j;
                    ab[(size_t)(kv + rl - cl) + (size_t)cl * ldab] = BLK(Lo, k, m)[i + j * m];
                    int64_t ru = k * m + i, cu = (k + 1) * m + j;
                    ab[(size_t)(kv + ru - cu) + (size_t)cu * ldab] = BLK(Up, k, m)[i + j * m];
                }
            }
}

/* Factor a BTRI matrix as a band matrix.  On success *ab_out / *ipiv_out
 * hold malloc'ed factors (free with orc_free). */
int orc_btri_band_factor(int64_t m, int64_t nb, const double *D, const double *Lo,
                         const double *Up, double **ab_out, int64_t **ipiv_out)
{
    const int64_t kl = 2 * m - 1, ku = 2 * m - 1, ldab = 2 * kl + ku + 1;
    const int64_t n = m * nb;
    double *ab = (double *)malloc(sizeof(double) * (size_t)ldab * (size_t)n);
    int64_t *ipiv = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!ab || !ipiv) { free(ab); free(ipiv); return -1; }
    btri_to_band(m, nb, D, Lo, Up, ab, ldab);
    int info = orc_band_getrf(n, kl, ku, ab, ldab, ipiv);
    *ab_out = ab;
    *ipiv_out = ipiv;
    return info;
}

void orc_btri_band_solve(int trans, int64_t m, int64_t nb, const double *ab,
                         const int64_t *ipiv, int64_t nrhs, double *b, int64_t ldb)
{
    const int64_t kl = 2 * m - 1, ku = 2 * m - 1, ldab = 2 * kl + ku + 1;
    orc_band_getrs(trans, m * nb, kl, ku, ab, ldab, ipiv, nrhs, b, ldb);
}

void orc_free(void *p) { free(p); }

/* Plain solve of a BTRI system through the band LU with partial pivoting. */
int orc_btri_solve(int64_t m, int64_t nb, const double *D, const double *Lo,
                   const double *Up, int64_t nrhs, const double *f, int64_t ldf,
                   double *x, int64_t ldx)
{
    double *ab; int64_t *ipiv;
    int info = orc_btri_band_factor(m, nb, D, Lo, Up, &ab, &ipiv);
    if (info < 0) return info;
    if (!info) {
        const int64_t n = m * nb;
        for (int64_t r = 0; r < nrhs; ++r)
            memcpy(x + r * ldx, f + r * ldf, sizeof(double) * (size_t)n);
        orc_btri_band_solve(0, m, nb, ab, ipiv, nrhs, x, ldx);
    }
    free(ab);
    free(ipiv);
    return info;
}

/* ------------------------------------------------------------------------ */
/* BABD: Gaussian elimination with row partial pivoting in the natural block
 * ordering (boundary-condition block row first).  Eliminating block column k
 * only involves the m "pending" rows (which carry the current diagonal block
 * T in column k and a fill-in block W in the last column -- the fill-in block
 * vector that the corner creates, Sec. 2 after eq. (redmatr1)) and block row
 * k+1 (Lo[k] in column k, D[k+1] in column k+1).  So each step is the LU with
 * partial pivoting of the 2m x m panel [T; Lo[k]], applied to the columns
 * k+1 and nb-1; the top m rows become final, the bottom m rows become the new
 * pending rows.  When k+1 == nb-1 the two companion columns coincide.
 * This is exactly dense GEPP on the matrix (no other row has a nonzero in
 * column k below the diagonal).
 *
 * Factor storage (per step k = 0..nb-2, m = block size, q = 2m):
 *   piv[k*m + c]       panel row swapped with panel row c at column c
 *   L[k]   (q x m)     the factored panel: U11 on and above the diagonal,
 *                      the multipliers of each column (as computed) below
 *   U1[k]  (m x m)     final rows k, column k+1   (zero when k+1 == nb-1)
 *   Uc[k]  (m x m)     final rows k, column nb-1
 * plus the last pending block T (m x m) factored with its own pivots.       */
typedef struct {
    int64_t m, nb;
    int64_t *piv;   /* (nb-1)*m + m */
    double *L;      /* (nb-1) * 2m*m */
    double *U1;     /* (nb-1) * m*m */
    double *Uc;     /* (nb-1) * m*m */
    double *T;      /* m*m, LU of the last pending block */
} babd_lu;

void orc_babd_free(void *h)
{
    babd_lu *f = (babd_lu *)h;
    if (!f) return;
    free(f->piv); free(f->L); free(f->U1); free(f->Uc); free(f->T); free(f);
}

int orc_babd_factor(int64_t m, int64_t nb, const double *D, const double *Lo,
                    const double *C, void **out)
{
    const int64_t q = 2 * m, steps = nb - 1;
    babd_lu *f = (babd_lu *)calloc(1, sizeof(babd_lu));
    if (!f) return -1;
    f->m = m; f->nb = nb;
    f->piv = (int64_t *)malloc(sizeof(int64_t) * (size_t)(steps * m + m));
    f->L = (double *)malloc(sizeof(double) * (size_t)(steps * q * m + 1));
    f->U1 = (double *)malloc(sizeof(double) * (size_t)(steps * m * m + 1));
    f->Uc = (double *)malloc(sizeof(double) * (size_t)(steps * m * m + 1));
    f->T = (double *)malloc(sizeof(double) * (size_t)(m * m));
    double *T = (double *)malloc(sizeof(double) * (size_t)(m * m));
    double *W = (double *)malloc(sizeof(double) * (size_t)(m * m));
    double *cmp = (double *)malloc(sizeof(double) * (size_t)(q * 2 * m)); /* q x 2m */
    if (!f->piv || !f->L || !f->U1 || !f->Uc || !f->T || !T || !W || !cmp) {
        free(T); free(W); free(cmp); orc_babd_free(f); return -1;
    }
    int info = 0;
    memcpy(T, D, sizeof(double) * (size_t)(m * m));   /* A(0,0) */
    memcpy(W, C, sizeof(double) * (size_t)(m * m));   /* A(0,nb-1) */
    for (int64_t k = 0; k < steps; ++k) {
        double *P = f->L + (size_t)k * q * m;          /* panel q x m */
        int64_t *pv = f->piv + k * m;
        const int last = (k + 1 == nb - 1);
        /* panel = [T; Lo[k]] */
        for (int64_t j = 0; j < m; ++j)
            for (int64_t i = 0; i < m; ++i) {
                P[i + j * q] = T[i + j * m];
                P[m + i + j * q] = BLK(Lo, k, m)[i + j * m];
            }
        /* companion columns: cols 0..m-1 = block column k+1, cols m..2m-1 =
         * block column nb-1; rows 0..m-1 pending rows, rows m..2m-1 row k+1 */
        for (int64_t j = 0; j < m; ++j)
            for (int64_t i = 0; i < m; ++i) {
                cmp[i + j * q] = 0.0;
                cmp[m + i + j * q] = BLK(D, k + 1, m)[i + j * m];
                cmp[i + (m + j) * q] = W[i + j * m];
                cmp[m + i + (m + j) * q] = 0.0;
            }
        if (last) /* column k+1 is column nb-1: merge into the first half */
            for (int64_t j = 0; j < m; ++j)
                for (int64_t i = 0; i < q; ++i) {
                    cmp[i + j * q] += cmp[i + (m + j) * q];
                    cmp[i + (m + j) * q] = 0.0;
                }
        for (int64_t c = 0; c < m; ++c) {
            int64_t p = c;
            double best = fabs(P[c + c * q]);
            for (int64_t i = c + 1; i < q; ++i) {
                double v = fabs(P[i + c * q]);
                if (v > best) { best = v; p = i; }
            }
            pv[c] = p;
            if (P[p + c * q] == 0.0) { if (!info) info = (int)(k * m + c + 1); continue; }
            if (p != c) {
                for (int64_t j = c; j < m; ++j) {
                    double t = P[c + j * q]; P[c + j * q] = P[p + j * q]; P[p + j * q] = t;
                }
                for (int64_t j = 0; j < 2 * m; ++j) {
                    double t = cmp[c + j * q]; cmp[c + j * q] = cmp[p + j * q]; cmp[p + j * q] = t;
                }
            }
            double inv = 1.0 / P[c + c * q];
            for (int64_t i = c + 1; i < q; ++i) P[i + c * q] *= inv;
            for (int64_t j = c + 1; j < m; ++j) {
                double u = P[c + j * q];
                for (int64_t i = c + 1; i < q; ++i) P[i + j * q] -= P[i + c * q] * u;
            }
            for (int64_t j = 0; j < 2 * m; ++j) {
                double u = cmp[c + j * q];
                for (int64_t i = c + 1; i < q; ++i) cmp[i + j * q] -= P[i + c * q] * u;
            }
        }
        /* top rows final; bottom rows become the new pending block */
        for (int64_t j = 0; j < m; ++j)
            for (int64_t i = 0; i < m; ++i) {
                BLK(f->U1, k, m)[i + j * m] = last ? 0.0 : cmp[i + j * q];
                BLK(f->Uc, k, m)[i + j * m] = last ? cmp[i + j * q] : cmp[i + (m + j) * q];
                T[i + j * m] = cmp[m + i + j * q];
                W[i + j * m] = cmp[m + i + (m + j) * q];
            }
        if (last) memset(W, 0, sizeof(double) * (size_t)(m * m));
    }
    if (nb == 1) { /* a single block: A = D[0] + C (both sit at (0,0)) */
        for (int64_t i = 0; i < m * m; ++i) T[i] += W[i];
    }
    memcpy(f->T, T, sizeof(double) * (size_t)(m * m));
    int i2 = orc_dense_getrf(m, f->T, f->piv + steps * m);
    if (i2 && !info) info = (int)(steps * m + i2);
    free(T); free(W); free(cmp);
    *out = f;
    return info;
}

/* trans = 0: A x = b; trans = 1: A^T x = b.  b is n x nrhs, in place. */
void orc_babd_solve_factored(int trans, const void *h, int64_t nrhs, double *b,
                             int64_t ldb)
{
    const babd_lu *f = (const babd_lu *)h;
    const int64_t m = f->m, nb = f->nb, q = 2 * m, steps = nb - 1;
    double *tmp = (double *)malloc(sizeof(double) * (size_t)q);
    for (int64_t r = 0; r < nrhs; ++r) {
        double *x = b + r * ldb;
        if (!trans) {
            /* forward: the row operations of each step act on positions
             * [k*m, (k+2)*m), i.e. the pending rows and block row k+1 */
            for (int64_t k = 0; k < steps; ++k) {
                const double *P = f->L + (size_t)k * q * m;
                const int64_t *pv = f->piv + k * m;
                double *y = x + k * m;
                for (int64_t c = 0; c < m; ++c) {
                    int64_t p = pv[c];
                    if (p != c) { double t = y[c]; y[c] = y[p]; y[p] = t; }
                    for (int64_t i = c + 1; i < q; ++i) y[i] -= P[i + c * q] * y[c];
                }
            }
            double *yl = x + steps * m;   /* last pending block */
            orc_dense_getrs(0, m, f->T, f->piv + steps * m, 1, yl, m);
            const double *xl = yl;
            for (int64_t k = steps - 1; k >= 0; --k) {
                const double *P = f->L + (size_t)k * q * m;
                double *y = x + k * m;
                const double *xn = x + (k + 1) * m;
                for (int64_t i = 0; i < m; ++i) {
                    double s = y[i];
                    for (int64_t j = 0; j < m; ++j)
                        s -= BLK(f->U1, k, m)[i + j * m] * xn[j] +
                             BLK(f->Uc, k, m)[i + j * m] * xl[j];
                    y[i] = s;
                }
                for (int64_t i = m - 1; i >= 0; --i) {   /* U11^{-1} */
                    for (int64_t j = i + 1; j < m; ++j) y[i] -= P[i + j * q] * y[j];
                    y[i] /= P[i + i * q];
                }
            }
        } else {
            /* U^T w = b (U^T is block lower triangular), then the transposed
             * row operations in reverse order. */
            double *acc = x + steps * m;   /* rhs of the last block column */
            for (int64_t k = 0; k < steps; ++k) {
                const double *P = f->L + (size_t)k * q * m;
                double *y = x + k * m;
                for (int64_t i = 0; i < m; ++i) {     /* U11^{-T} */
                    for (int64_t j = 0; j < i; ++j) y[i] -= P[j + i * q] * y[j];
                    y[i] /= P[i + i * q];
                }
                double *yn = x + (k + 1) * m;   /* U1 is zero at the last step */
                for (int64_t j = 0; j < m; ++j)
                    for (int64_t i = 0; i < m; ++i)
                        yn[j] -= BLK(f->U1, k, m)[i + j * m] * y[i];
                for (int64_t j = 0; j < m; ++j)
                    for (int64_t i = 0; i < m; ++i)
                        acc[j] -= BLK(f->Uc, k, m)[i + j * m] * y[i];
            }
            orc_dense_getrs(1, m, f->T, f->piv + steps * m, 1, acc, m);
            for (int64_t k = steps - 1; k >= 0; --k) {
                const double *P = f->L + (size_t)k * q * m;
                const int64_t *pv = f->piv + k * m;
                double *y = x + k * m;
                for (int64_t i = 0; i < q; ++i) tmp[i] = y[i];
                for (int64_t c = m - 1; c >= 0; --c) {
                    double s = tmp[c];
                    for (int64_t i = c + 1; i < q; ++i) s -= P[i + c * q] * tmp[i];
                    tmp[c] = s;
                    int64_t p = pv[c];
                    if (p != c) { double t = tmp[c]; tmp[c] = tmp[p]; tmp[p] = t; }
                }
                for (int64_t i = 0; i < q; ++i) y[i] = tmp[i];
            }
        }
    }
    free(tmp);
}

int orc_babd_solve(int64_t m, int64_t nb, const double *D, const double *Lo,
                   const double *C, int64_t nrhs, const double *f, int64_t ldf,
                   double *x, int64_t ldx)
{
    void *h = NULL;
    int info = orc_babd_factor(m, nb, D, Lo, C, &h);
    if (info < 0) return info;
    if (!info) {
        for (int64_t r = 0; r < nrhs; ++r)
            memcpy(x + r * ldx, f + r * ldf, sizeof(double) * (size_t)(m * nb));
        orc_babd_solve_factored(0, h, nrhs, x, ldx);
    }
    orc_babd_free(h);
    return info;
}

/* ------------------------------------------------------------------------ */
/* Residuals r = f - A x and infinity norms, all in FP64. */
void orc_btri_residual(int64_t m, int64_t nb, const double *D, const double *Lo,
                       const double *Up, int64_t nrhs, const double *f, int64_t ldf,
                       const double *x, int64_t ldx, double *r, int64_t ldr)
{
    for (int64_t c = 0; c < nrhs; ++c)
        for (int64_t k = 0; k < nb; ++k)
            for (int64_t i = 0; i < m; ++i) {
                double s = f[k * m + i + c * ldf];
                for (int64_t j = 0; j < m; ++j) {
                    s -= BLK(D, k, m)[i + j * m] * x[k * m + j + c * ldx];
                    if (k > 0) s -= BLK(Lo, k - 1, m)[i + j * m] * x[(k - 1) * m + j + c * ldx];
                    if (k + 1 < nb) s -= BLK(Up, k, m)[i + j * m] * x[(k + 1) * m + j + c * ldx];
                }
                r[k * m + i + c * ldr] = s;
            }
}

void orc_babd_residual(int64_t m, int64_t nb, const double *D, const double *Lo,
                       const double *C, int64_t nrhs, const double *f, int64_t ldf,
                       const double *x, int64_t ldx, double *r, int64_t ldr)
{
    for (int64_t c = 0; c < nrhs; ++c)
        for (int64_t k = 0; k < nb; ++k)
            for (int64_t i = 0; i < m; ++i) {
                double s = f[k * m + i + c * ldf];
                for (int64_t j = 0; j < m; ++j) {
                    s -= BLK(D, k, m)[i + j * m] * x[k * m + j + c * ldx];
                    if (k > 0) s -= BLK(Lo, k - 1, m)[i + j * m] * x[(k - 1) * m + j + c * ldx];
                    if (k == 0) s -= C[i + j * m] * x[(nb - 1) * m + j + c * ldx];
                }
                r[k * m + i + c * ldr] = s;
            }
}

/* ||A||_inf = largest absolute row sum. */
double orc_btri_norminf(int64_t m, int64_t nb, const double *D, const double *Lo,
                        const double *Up)
{
    double best = 0.0;
    for (int64_t k = 0; k < nb; ++k)
        for (int64_t i = 0; i < m; ++i) {
            double s = 0.0;
            for (int64_t j = 0; j < m; ++j) {
                s += fabs(BLK(D, k, m)[i + j * m]);
                if (k > 0) s += fabs(BLK(Lo, k - 1, m)[i + j * m]);
                if (k + 1 < nb) s += fabs(BLK(Up, k, m)[i + j * m]);
            }
            if (s > best) best = s;
        }
    return best;
}

double orc_babd_norminf(int64_t m, int64_t nb, const double *D, const double *Lo,
                        const double *C)
{
    double best = 0.0;
    for (int64_t k = 0; k < nb; ++k)
        for (int64_t i = 0; i < m; ++i) {
            double s = 0.0;
            for (int64_t j = 0; j < m; ++j) {
                s += fabs(BLK(D, k, m)[i + j * m]);
                if (k > 0) s += fabs(BLK(Lo, k - 1, m)[i + j * m]);
                if (k == 0 && nb > 1) s += fabs(C[i + j * m]);
            }
            if (s > best) best = s;
        }
    return best;
}

/* ------------------------------------------------------------------------ */
/* Hager's estimate of ||A^{-1}||_1 (Hager 1984, Higham's refinement of the
 * stopping rule), applied to A^T so that it returns ||A^{-1}||_inf.
 * solve(trans, v) must overwrite v with A^{-1} v (trans = 0) or A^{-T} v. */
typedef void (*solve_fn)(int trans, void *ctx, double *v);

static double hager_inv_norminf(int64_t n, solve_fn solve, void *ctx)
{
    /* ||A^{-1}||_inf = ||B||_1 with B = A^{-T}; B v = A^{-T} v and
     * B^T v = A^{-1} v. */
    double *x = (double *)malloc(sizeof(double) * (size_t)n);
    double *xi = (double *)malloc(sizeof(double) * (size_t)n);
    if (!x || !xi) { free(x); free(xi); return NAN; }
    for (int64_t i = 0; i < n; ++i) x[i] = 1.0 / (double)n;
    double est = 0.0;
    int64_t jlast = -1;
    for (int it = 0; it < 5; ++it) {
        solve(1, ctx, x);                     /* y = B x */
        double ny = 0.0;
        for (int64_t i = 0; i < n; ++i) ny += fabs(x[i]);
        if (it > 0 && ny <= est) break;
        est = ny;
        for (int64_t i = 0; i < n; ++i) xi[i] = x[i] >= 0.0 ? 1.0 : -1.0;
        solve(0, ctx, xi);                    /* z = B^T sign(y) */
        int64_t j = 0;
        double zmax = fabs(xi[0]);
        for (int64_t i = 1; i < n; ++i)
            if (fabs(xi[i]) > zmax) { zmax = fabs(xi[i]); j = i; }
        if (it > 0 && j == jlast) break;
        jlast = j;
        memset(x, 0, sizeof(double) * (size_t)n);
        x[j] = 1.0;
    }
    /* Higham's alternating-sign test vector guards against bad cases. */
    for (int64_t i = 0; i < n; ++i)
        x[i] = (i % 2 ? -1.0 : 1.0) * (1.0 + (double)i / (double)(n > 1 ? n - 1 : 1));
    solve(1, ctx, x);
    double alt = 0.0;
    for (int64_t i = 0; i < n; ++i) alt += fabs(x[i]);
    alt = 2.0 * alt / (3.0 * (double)n);
    free(x);
    free(xi);
    return alt > est ? alt : est;
}

typedef struct { int64_t m, nb; const double *ab; const int64_t *ipiv; } band_ctx;

static void band_solve_cb(int trans, void *ctx, double *v)
{
    band_ctx *c = (band_ctx *)ctx;
    orc_btri_band_solve(trans, c->m, c->nb, c->ab, c->ipiv, 1, v, c->m * c->nb);
}

/* kappa_inf(A) estimate for a BTRI matrix; returns a negative value if the
 * matrix is singular. */
double orc_btri_condest(int64_t m, int64_t nb, const double *D, const double *Lo,
                        const double *Up)
{
    double *ab; int64_t *ipiv;
    int info = orc_btri_band_factor(m, nb, D, Lo, Up, &ab, &ipiv);
    if (info) { if (info > 0) { free(ab); free(ipiv); } return -1.0; }
    band_ctx c = {m, nb, ab, ipiv};
    double inv = hager_inv_norminf(m * nb, band_solve_cb, &c);
    free(ab);
    free(ipiv);
    return inv * orc_btri_norminf(m, nb, D, Lo, Up);
}

typedef struct { int64_t n; const void *h; } babd_ctx;

static void babd_solve_cb(int trans, void *ctx, double *v)
{
    babd_ctx *c = (babd_ctx *)ctx;
    orc_babd_solve_factored(trans, c->h, 1, v, c->n);
}

double orc_babd_condest(int64_t m, int64_t nb, const double *D, const double *Lo,
                        const double *C)
{
    void *h = NULL;
    int info = orc_babd_factor(m, nb, D, Lo, C, &h);
    if (info) { if (info > 0) orc_babd_free(h); return -1.0; }
    babd_ctx c = {m * nb, h};
    double inv = hager_inv_norminf(m * nb, babd_solve_cb, &c);
    orc_babd_free(h);
    return inv * orc_babd_norminf(m, nb, D, Lo, C);
}

/* ------------------------------------------------------------------------ */
/* Transposed solves A^T x = f (used to pin the factor storage that the
 * condition estimators rely on). */
int orc_btri_solve_trans(int64_t m, int64_t nb, const double *D, const double *Lo,
                         const double *Up, int64_t nrhs, const double *f, int64_t ldf,
                         double *x, int64_t ldx)
{
    double *ab; int64_t *ipiv;
    int info = orc_btri_band_factor(m, nb, D, Lo, Up, &ab, &ipiv);
    if (info < 0) return info;
    if (!info) {
        for (int64_t r = 0; r < nrhs; ++r)
            memcpy(x + r * ldx, f + r * ldf, sizeof(double) * (size_t)(m * nb));
        orc_btri_band_solve(1, m, nb, ab, ipiv, nrhs, x, ldx);
    }
    free(ab);
    free(ipiv);
    return info;
}

int orc_babd_solve_trans(int64_t m, int64_t nb, const double *D, const double *Lo,
                         const double *C, int64_t nrhs, const double *f, int64_t ldf,
                         double *x, int64_t ldx)
{
    void *h = NULL;
    int info = orc_babd_factor(m, nb, D, Lo, C, &h);
    if (info < 0) return info;
    if (!info) {
        for (int64_t r = 0; r < nrhs; ++r)
            memcpy(x + r * ldx, f + r * ldf, sizeof(double) * (size_t)(m * nb));
        orc_babd_solve_factored(1, h, nrhs, x, ldx);
    }
    orc_babd_free(h);
    return info;
}
