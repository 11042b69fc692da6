/*
 * Driver for the host-sanitizer build of the FP64 oracle (oracle.c compiled
 * with AddressSanitizer and UndefinedBehaviorSanitizer).  Reads a workload on
 * stdin -- a Hamiltonian Pauli pack, the pool's packs, a state and an angle --
 * and runs every oracle function on it: the CSR build (two phases), the
 * energy, the pool gradients, the selection, the fifth-order update of the
 * selected generator and the renormalisation, then prints every result with
 * 17 significant digits for comparison with the regular build.
 *
 * Input (text): n_qubits; the Hamiltonian as "n_terms drop_tol" and n_terms
 * lines "x z re im"; M; per generator the same; dim lines "re im" (the
 * state); theta.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int64_t orc_csr_build(int n_qubits, int64_t n_terms, const uint64_t *x, const uint64_t *z,
                      const double *coeff, double tol, int64_t *rowptr, int32_t *col, double *val);
void orc_spmv(int64_t dim, const int64_t *rowptr, const int32_t *col, const double *val,
              const double *x, double *y);
void orc_taylor5(int64_t dim, const int64_t *rowptr, const int32_t *col, const double *val,
                 double theta, const double *psi, double *out, double *work);
double orc_normalize(int64_t dim, double *psi);
void orc_energy(int64_t dim, const int64_t *rowptr, const int32_t *col, const double *val,
                const double *psi, double *sigma_out, double *out);
void orc_gradients(int64_t dim, int32_t M, const int64_t *const *rowptrs,
                   const int32_t *const *cols, const double *const *vals, const double *psi,
                   const double *sigma, double *g, double *work);
int32_t orc_select(int32_t M, const double *g, double rel_tie, double *gmax_out);

typedef struct {
    int64_t *rowptr;
    int32_t *col;
    double *val;
    int64_t nnz;
} Csr;

static void *xmalloc(size_t n)
{
    void *p = malloc(n ? n : 1);
    if (!p) {
        fprintf(stderr, "out of memory\n");
        exit(2);
    }
    return p;
}

static void need(int ok)
{
    if (!ok) {
        fprintf(stderr, "malformed input\n");
        exit(2);
    }
}

/* Read one pack ("n_terms drop_tol" and its terms) and compile it. */
static Csr read_and_build(int nq)
{
    long long n;
    double tol;
    need(scanf("%lld %lf", &n, &tol) == 2 && n >= 0);
    const int64_t nt = n;
    uint64_t *x = xmalloc(nt * sizeof *x), *z = xmalloc(nt * sizeof *z);
    double *c = xmalloc(2 * nt * sizeof *c);
    for (int64_t t = 0; t < nt; t++) {
        unsigned long long a, b;
        need(scanf("%llu %llu %lf %lf", &a, &b, &c[2 * t], &c[2 * t + 1]) == 4);
        x[t] = a;
        z[t] = b;
    }
    Csr m;
    const int64_t dim = (int64_t)1 << nq;
    m.rowptr = xmalloc((dim + 1) * sizeof(int64_t));
    m.nnz = orc_csr_build(nq, nt, x, z, c, tol, m.rowptr, NULL, NULL);
    need(m.nnz >= 0);
    m.col = xmalloc(m.nnz * sizeof(int32_t));
    m.val = xmalloc(2 * m.nnz * sizeof(double));
    need(orc_csr_build(nq, nt, x, z, c, tol, m.rowptr, m.col, m.val) == m.nnz);
    /* a bad argument is refused, not read out of bounds */
    uint64_t bad = (uint64_t)1 << nq;
    need(orc_csr_build(nq, 1, &bad, z, c, tol, m.rowptr, NULL, NULL) == -1);
    free(x);
    free(z);
    free(c);
    return m;
}

int main(void)
{
    int nq;
    need(scanf("%d", &nq) == 1 && nq >= 1 && nq <= 20);
    const int64_t dim = (int64_t)1 << nq;
    Csr H = read_and_build(nq);
    int M;
    need(scanf("%d", &M) == 1 && M > 0);
    Csr *pool = xmalloc(M * sizeof(Csr));
    const int64_t **rp = xmalloc(M * sizeof *rp);
    const int32_t **cp = xmalloc(M * sizeof *cp);
    const double **vp = xmalloc(M * sizeof *vp);
    for (int j = 0; j < M; j++) {
        pool[j] = read_and_build(nq);
        rp[j] = pool[j].rowptr;
        cp[j] = pool[j].col;
        vp[j] = pool[j].val;
    }
    double *psi = xmalloc(2 * dim * sizeof(double));
    for (int64_t r = 0; r < dim; r++)
        need(scanf("%lf %lf", &psi[2 * r], &psi[2 * r + 1]) == 2);
    double theta;
    need(scanf("%lf", &theta) == 1);

    double *sigma = xmalloc(2 * dim * sizeof(double)), out[3];
    orc_energy(dim, H.rowptr, H.col, H.val, psi, sigma, out);
    double *g = xmalloc(M * sizeof(double)), *work = xmalloc(4 * dim * sizeof(double));
    orc_gradients(dim, M, rp, cp, vp, psi, sigma, g, work);
    double gmax;
    const int32_t k = orc_select(M, g, 1e-6, &gmax);
    double *next = xmalloc(2 * dim * sizeof(double));
    orc_taylor5(dim, pool[k].rowptr, pool[k].col, pool[k].val, theta, psi, next, work);
    const double n2 = orc_normalize(dim, next);
    double *y = xmalloc(2 * dim * sizeof(double));
    orc_spmv(dim, H.rowptr, H.col, H.val, next, y);

    printf("nnz %lld\n", (long long)H.nnz);
    printf("energy %.17g %.17g %.17g\n", out[0], out[1], out[2]);
    for (int j = 0; j < M; j++)
        printf("g %d %.17g\n", j, g[j]);
    printf("select %d %.17g\n", k, gmax);
    printf("norm2 %.17g\n", n2);
    for (int64_t r = 0; r < dim; r++)
        printf("psi %.17g %.17g\n", next[2 * r], next[2 * r + 1]);
    for (int64_t r = 0; r < dim; r++)
        printf("hpsi %.17g %.17g\n", y[2 * r], y[2 * r + 1]);

    for (int j = 0; j < M; j++) {
        free(pool[j].rowptr);
        free(pool[j].col);
        free(pool[j].val);
    }
    free(pool);
    free(rp);
    free(cp);
    free(vp);
    free(H.rowptr);
    free(H.col);
    free(H.val);
    free(psi);
    free(sigma);
    free(g);
    free(work);
    free(next);
    free(y);
    return 0;
}
