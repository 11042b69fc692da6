/*
 * FP64 CPU oracle for the adaptive-VQE hot path.  TEST INFRASTRUCTURE ONLY:
 * the parity tests, the smoke check and the CPU-baseline leg of the benchmark
 * call it; the product path never does.  It shares no code with the HIP path.
 *
 * Plain, slow, obviously correct C.  Complex numbers are interleaved
 * (re, im) doubles.  Build with -O2 -ffp-contract=off (no fused multiply-add,
 * no reassociation) so every sum is taken in the order written here.
 *
 * Functions and the passages they follow:
 *   orc_csr_build   Pauli sum (Eq. 3) -> CSR, the on-the-fly sparse
 *                   compilation of Sec. III-E.
 *   orc_csr_rows    selected rows of that CSR (for sampled checks of very
 *                   large operators).
 *   orc_spmv        y = M x, the sparse product each Taylor step and the
 *                   energy are made of (Sec. III-C, Eq. 7).
 *   orc_taylor5     the fifth-order update of Eq. 6, evaluated as the five
 *                   chained products of Eq. 7 and the accumulation of Eq. 8.
 *   orc_normalize   rescale to unit norm (the paper is silent; the update of
 *                   Eq. 8 is not norm-preserving).
 *   orc_energy      Rayleigh quotient <psi|H|psi>/<psi|psi> (Eq. 1).
 *   orc_gradients   g_j = <psi|[H, A_j]|psi> (Eq. 5), which for Hermitian H
 *                   and anti-Hermitian A_j equals 2 Re <H psi | A_j psi>.
 *   orc_select      index of the largest |g_j| (Sec. III-D, step 3).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads used by the parallel loops from now on (for timing the oracle at a
 * given core count; results do not depend on it, since every row is computed
 * by one thread in the order written). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}

static int popcount64(uint64_t v)
{
    int n = 0;
    while (v) {
        v &= v - 1;
        n++;
    }
    return n;
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/*
 * Contribution of Pauli term t to matrix entry (row, col), col = row ^ x:
 *   P(x,z)|col> = i^{popcount(x&z)} (-1)^{popcount(z&col)} |col ^ x>,
 * so the entry is coeff * i^k * s with k = popcount(x&z) mod 4 and
 * s = (-1)^{popcount(z&col)}.  Multiplying by i^k and by s only swaps and
 * negates parts, which is exact.
 */
static void term_value(double cre, double cim, uint64_t x, uint64_t z, uint64_t col,
                       double *vre, double *vim)
{
    int k = popcount64(x & z) & 3;
    double re, im;
    switch (k) {
    case 0: re = cre;  im = cim;  break;
    case 1: re = -cim; im = cre;  break;
    case 2: re = -cre; im = -cim; break;
    default: re = cim; im = -cre; break;
    }
    if (popcount64(z & col) & 1) {
        re = -re;
        im = -im;
    }
    *vre = re;
    *vim = im;
}

/*
 * Row r of the CSR matrix of sum_t c_t P_t.  Every term contributes to column
 * r ^ x_t; contributions to one column are summed in ascending term index
 * starting from +0.0.  An entry is kept unless |re| <= tol and |im| <= tol.
 * Kept entries are written in ascending column order.  Returns the number
 * kept; writes entries only when col_out != NULL.
 */
static int64_t build_row(int n_qubits, int64_t n_terms, const uint64_t *x, const uint64_t *z,
                         const double *coeff, double tol, uint64_t r,
                         double *acc, unsigned char *seen, int32_t *cols,
                         int32_t *col_out, double *val_out)
{
    int64_t n_touched = 0, kept = 0;
    (void)n_qubits;
    for (int64_t t = 0; t < n_terms; t++) {
        uint64_t c = r ^ x[t];
        double vre, vim;
        term_value(coeff[2 * t], coeff[2 * t + 1], x[t], z[t], c, &vre, &vim);
        if (!seen[c]) {
            seen[c] = 1;
            acc[2 * c] = 0.0;
            acc[2 * c + 1] = 0.0;
            cols[n_touched++] = (int32_t)c;
        }
        acc[2 * c] = acc[2 * c] + vre;
        acc[2 * c + 1] = acc[2 * c + 1] + vim;
    }
    qsort(cols, (size_t)n_touched, sizeof(int32_t), cmp_i32);
    for (int64_t i = 0; i < n_touched; i++) {
        int32_t c = cols[i];
        double re = acc[2 * c], im = acc[2 * c + 1];
        seen[c] = 0;
        if (fabs(re) <= tol && fabs(im) <= tol)
            continue;
        if (col_out) {
            col_out[kept] = c;
            val_out[2 * kept] = re;
            val_out[2 * kept + 1] = im;
        }
        kept++;
    }
    return kept;
}

/*
 * CSR of a Pauli sum.  Phase 1 (col == NULL): fills rowptr[0..dim].  Phase 2:
 * fills col[nnz] and val[2*nnz] (rowptr must hold the phase-1 result).
 * Returns nnz, or -1 on a bad argument or allocation failure.
 */
int64_t orc_csr_build(int n_qubits, int64_t n_terms, const uint64_t *x, const uint64_t *z,
                      const double *coeff, double tol, int64_t *rowptr,
                      int32_t *col, double *val)
{
    if (n_qubits < 1 || n_qubits > 26 || n_terms < 0)
        return -1;
    uint64_t dim = (uint64_t)1 << n_qubits;
    for (int64_t t = 0; t < n_terms; t++)
        if ((x[t] | z[t]) >> n_qubits)
            return -1;
    int failed = 0;
#pragma omp parallel
    {
        double *acc = (double *)malloc(2 * dim * sizeof(double));
        unsigned char *seen = (unsigned char *)calloc(dim, 1);
        int32_t *cols = (int32_t *)malloc((size_t)(n_terms > 0 ? n_terms : 1) * sizeof(int32_t));
        if (!acc || !seen || !cols) {
#pragma omp atomic write
            failed = 1;
        } else {
#pragma omp for schedule(static)
            for (int64_t r = 0; r < (int64_t)dim; r++) {
                if (col == NULL)
                    rowptr[r + 1] = build_row(n_qubits, n_terms, x, z, coeff, tol, (uint64_t)r,
                                              acc, seen, cols, NULL, NULL);
                else
                    build_row(n_qubits, n_terms, x, z, coeff, tol, (uint64_t)r, acc, seen, cols,
                              col + rowptr[r], val + 2 * rowptr[r]);
            }
        }
        free(acc);
        free(seen);
        free(cols);
    }
    if (failed)
        return -1;
    if (col == NULL) {
        rowptr[0] = 0;
        for (uint64_t r = 0; r < dim; r++)
            rowptr[r + 1] += rowptr[r];
    }
    return rowptr[dim];
}

/*
 * Selected rows of the CSR matrix of a Pauli sum (Eq. 3), for checking a
 * product at sampled rows when the whole matrix is too large to build: row j
 * of the result is row rows[j] of orc_csr_build's matrix (same entries, same
 * ordered sums, same drop rule), columns global.  Phase 1 (col == NULL) fills
 * rowptr[0..n_rows] with the prefix sums of the rows' lengths; phase 2 fills
 * col and val.  Returns the number of entries, or -1 on a bad argument or an
 * allocation failure.
 */
int64_t orc_csr_rows(int n_qubits, int64_t n_terms, const uint64_t *x, const uint64_t *z,
                     const double *coeff, double tol, const int64_t *rows, int64_t n_rows,
                     int64_t *rowptr, int32_t *col, double *val)
{
    if (n_qubits < 1 || n_qubits > 26 || n_terms < 0 || n_rows < 0)
        return -1;
    uint64_t dim = (uint64_t)1 << n_qubits;
    for (int64_t t = 0; t < n_terms; t++)
        if ((x[t] | z[t]) >> n_qubits)
            return -1;
    for (int64_t j = 0; j < n_rows; j++)
        if (rows[j] < 0 || (uint64_t)rows[j] >= dim)
            return -1;
    int failed = 0;
#pragma omp parallel
    {
        double *acc = (double *)malloc(2 * dim * sizeof(double));
        unsigned char *seen = (unsigned char *)calloc(dim, 1);
        int32_t *cols = (int32_t *)malloc((size_t)(n_terms > 0 ? n_terms : 1) * sizeof(int32_t));
        if (!acc || !seen || !cols) {
#pragma omp atomic write
            failed = 1;
        } else {
#pragma omp for schedule(static)
            for (int64_t j = 0; j < n_rows; j++) {
                if (col == NULL)
                    rowptr[j + 1] = build_row(n_qubits, n_terms, x, z, coeff, tol,
                                              (uint64_t)rows[j], acc, seen, cols, NULL, NULL);
                else
                    build_row(n_qubits, n_terms, x, z, coeff, tol, (uint64_t)rows[j], acc, seen,
                              cols, col + rowptr[j], val + 2 * rowptr[j]);
            }
        }
        free(acc);
        free(seen);
        free(cols);
    }
    if (failed)
        return -1;
    if (col == NULL) {
        rowptr[0] = 0;
        for (int64_t j = 0; j < n_rows; j++)
            rowptr[j + 1] += rowptr[j];
    }
    return rowptr[n_rows];
}

/* y_r = sum_{k in row r} val_k * x[col_k], complex, ascending k. */
void orc_spmv(int64_t dim, const int64_t *rowptr, const int32_t *col, const double *val,
              const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < dim; r++) {
        double re = 0.0, im = 0.0;
        for (int64_t k = rowptr[r]; k < rowptr[r + 1]; k++) {
            double a = val[2 * k], b = val[2 * k + 1];
            double c = x[2 * col[k]], d = x[2 * col[k] + 1];
            re = re + (a * c - b * d);
            im = im + (a * d + b * c);
        }
        y[2 * r] = re;
        y[2 * r + 1] = im;
    }
}

/*
 * Fifth-order Taylor update (Eq. 6-8):
 *   v_0 = psi, v_n = A v_{n-1} (n = 1..5),
 *   c_0 = 1, c_n = c_{n-1} * theta / n,
 *   out = psi + c_1 v_1 + c_2 v_2 + ... + c_5 v_5, summed in increasing n.
 * out may alias psi.  work holds 2 vectors of 2*dim doubles.
 */
void orc_taylor5(int64_t dim, const int64_t *rowptr, const int32_t *col, const double *val,
                 double theta, const double *psi, double *out, double *work)
{
    double *prev = work, *next = work + 2 * dim;
    double *acc = (double *)malloc(2 * (size_t)dim * sizeof(double));
    memcpy(acc, psi, 2 * (size_t)dim * sizeof(double));
    memcpy(prev, psi, 2 * (size_t)dim * sizeof(double));
    double c = 1.0;
    for (int n = 1; n <= 5; n++) {
        orc_spmv(dim, rowptr, col, val, prev, next);
        c = c * theta / (double)n;
        for (int64_t r = 0; r < dim; r++) {
            acc[2 * r] = acc[2 * r] + c * next[2 * r];
            acc[2 * r + 1] = acc[2 * r + 1] + c * next[2 * r + 1];
        }
        double *t = prev;
        prev = next;
        next = t;
    }
    memcpy(out, acc, 2 * (size_t)dim * sizeof(double));
    free(acc);
}

/* psi <- psi / sqrt(sum |psi_r|^2); returns the squared norm before scaling. */
double orc_normalize(int64_t dim, double *psi)
{
    double s = 0.0;
    for (int64_t r = 0; r < dim; r++)
        s = s + (psi[2 * r] * psi[2 * r] + psi[2 * r + 1] * psi[2 * r + 1]);
    double inv = 1.0 / sqrt(s);
    for (int64_t r = 0; r < dim; r++) {
        psi[2 * r] = psi[2 * r] * inv;
        psi[2 * r + 1] = psi[2 * r + 1] * inv;
    }
    return s;
}

/*
 * Energy (Eq. 1): sigma = H psi, out[0] = Re<psi|sigma>/<psi|psi>,
 * out[1] = <psi|psi>, out[2] = Im<psi|sigma> (zero for Hermitian H).
 * sigma_out (2*dim doubles) receives H psi.
 */
void orc_energy(int64_t dim, const int64_t *rowptr, const int32_t *col, const double *val,
                const double *psi, double *sigma_out, double *out)
{
    orc_spmv(dim, rowptr, col, val, psi, sigma_out);
    double nre = 0.0, nim = 0.0, den = 0.0;
    for (int64_t r = 0; r < dim; r++) {
        double a = psi[2 * r], b = psi[2 * r + 1];
        double c = sigma_out[2 * r], d = sigma_out[2 * r + 1];
        /* conj(a + ib) (c + id) = (ac + bd) + i(ad - bc) */
        nre = nre + (a * c + b * d);
        nim = nim + (a * d - b * c);
        den = den + (a * a + b * b);
    }
    out[0] = nre / den;
    out[1] = den;
    out[2] = nim;
}

/*
 * g_j = 2 Re sum_r conj(sigma_r) (A_j psi)_r for j = 0..M-1, sigma = H psi.
 * Operator j is the CSR (rowptrs[j], cols[j], vals[j]).  work: 2*dim doubles.
 */
void orc_gradients(int64_t dim, int32_t M, const int64_t *const *rowptrs,
                   const int32_t *const *cols, const double *const *vals,
                   const double *psi, const double *sigma, double *g, double *work)
{
    for (int32_t j = 0; j < M; j++) {
        orc_spmv(dim, rowptrs[j], cols[j], vals[j], psi, work);
        double s = 0.0;
        for (int64_t r = 0; r < dim; r++) {
            /* Re(conj(s) w) = s_re w_re + s_im w_im */
            s = s + (sigma[2 * r] * work[2 * r] + sigma[2 * r + 1] * work[2 * r + 1]);
        }
        g[j] = 2.0 * s;
    }
}

/*
 * Largest |g_j| with the tie rule: the candidates are all j with
 * |g_j| >= gmax * (1 - rel_tie); the lowest such index wins.
 * Writes gmax; returns the index (or -1 if M == 0).
 */
int32_t orc_select(int32_t M, const double *g, double rel_tie, double *gmax_out)
{
    double gmax = 0.0;
    for (int32_t j = 0; j < M; j++)
        if (fabs(g[j]) > gmax)
            gmax = fabs(g[j]);
    *gmax_out = gmax;
    for (int32_t j = 0; j < M; j++)
        if (fabs(g[j]) >= gmax * (1.0 - rel_tie))
            return j;
    return M > 0 ? 0 : -1;
}
