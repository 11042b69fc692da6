/*
 * The C ABI used from plain C (no Python): compile a 4-qubit Hamiltonian and a
 * generator from Pauli terms (Eq. 3), take the energy (Eq. 1), apply the
 * fifth-order update (Eq. 6-8) with renormalisation and take the energy again.
 * Prints "E0 <value>" and "E1 <value>" (17 significant digits) for the tests to
 * compare with the oracle; exits non-zero on any error.
 *
 *   gcc -std=c11 -I include -I /opt/rocm/include -D__HIP_PLATFORM_AMD__ \
 *       tests/c_api_demo.c -L paper_2606_29692_amd -ladaptvqe \
 *       -L /opt/rocm/lib -lamdhip64 -o c_api_demo
 */
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "adaptvqe.h"

#define NQ 4
#define DIM (1 << NQ)

static int check_hip(hipError_t e, const char *what)
{
    if (e != hipSuccess) {
        fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
        return 1;
    }
    return 0;
}

static int check(vqe_ctx *ctx, int rc, const char *what)
{
    if (rc != VQE_OK) {
        fprintf(stderr, "%s: %s (%s)\n", what, vqe_strerror(rc), vqe_last_error(ctx));
        return 1;
    }
    return 0;
}

/* Two-phase build of a CSR operator in device memory. */
static int build(vqe_ctx *ctx, int64_t n, const uint64_t *x, const uint64_t *z, const double *c,
                 vqe_csr *out)
{
    int64_t nnz = 0;
    out->col = NULL;
    out->val = NULL;
    if (check_hip(hipMalloc((void **)&out->rowptr, (DIM + 1) * sizeof(int32_t)), "hipMalloc rowptr"))
        return 1;
    if (check(ctx, csr_build_from_pauli(ctx, NQ, n, x, z, c, 1e-12, VQE_C128, 0.0, out, &nnz),
              "csr_build_from_pauli (sizing)"))
        return 1;
    const int64_t m = nnz > 0 ? nnz : 1;
    if (check_hip(hipMalloc((void **)&out->col, m * sizeof(int32_t)), "hipMalloc col") ||
        check_hip(hipMalloc(&out->val, m * 2 * sizeof(double)), "hipMalloc val"))
        return 1;
    return check(ctx, csr_build_from_pauli(ctx, NQ, n, x, z, c, 1e-12, VQE_C128, 0.0, out, &nnz),
                 "csr_build_from_pauli (fill)");
}

int main(void)
{
    /* H = 0.5 Z0 + 0.3 Z1 - 0.2 Z2 + 0.1 Z3 + 0.25 X0X1 + 0.25 Y0Y1 + 0.15 Z0Z1 + 0.05 X2X3
     * as (x, z) masks, P(x, z)|c> = i^{|x & z|} (-1)^{|z & c|} |c ^ x> */
    const uint64_t hx[8] = {0, 0, 0, 0, 3, 3, 0, 12};
    const uint64_t hz[8] = {1, 2, 4, 8, 0, 3, 3, 0};
    const double hc[16] = {0.5, 0, 0.3, 0, -0.2, 0, 0.1, 0, 0.25, 0, 0.25, 0, 0.15, 0, 0.05, 0};
    /* A = i X0 Y1: anti-Hermitian, one entry per row, A^3 = -A */
    const uint64_t ax[1] = {3};
    const uint64_t az[1] = {2};
    const double ac[2] = {0.0, 1.0};
    const double theta = 0.3;

    vqe_ctx *ctx = NULL;
    int rc = vqe_create(0, NULL, &ctx);
    if (rc != VQE_OK) {
        fprintf(stderr, "vqe_create: %s\n", vqe_strerror(rc));
        return 1;
    }
    vqe_csr H, A;
    if (build(ctx, 8, hx, hz, hc, &H) || build(ctx, 1, ax, az, ac, &A))
        return 1;

    double psi_h[2 * DIM] = {0};
    psi_h[2 * 1] = 1.0;                               /* |0001> */
    void *psi = NULL, *sigma = NULL;
    double *out = NULL;
    if (check_hip(hipMalloc(&psi, sizeof(psi_h)), "hipMalloc psi") ||
        check_hip(hipMalloc(&sigma, sizeof(psi_h)), "hipMalloc sigma") ||
        check_hip(hipMalloc((void **)&out, 3 * sizeof(double)), "hipMalloc out") ||
        check_hip(hipMemcpy(psi, psi_h, sizeof(psi_h), hipMemcpyHostToDevice), "copy psi"))
        return 1;

    double e[3];
    if (check(ctx, energy(ctx, &H, psi, sigma, out), "energy") ||
        check_hip(hipDeviceSynchronize(), "sync") ||
        check_hip(hipMemcpy(e, out, sizeof(e), hipMemcpyDeviceToHost), "copy energy"))
        return 1;
    printf("E0 %.17g\n", e[0]);
    if (check(ctx, taylor5_apply(ctx, &A, theta, psi, 1, NULL), "taylor5_apply") ||
        check(ctx, energy(ctx, &H, psi, sigma, out), "energy") ||
        check_hip(hipDeviceSynchronize(), "sync") ||
        check_hip(hipMemcpy(e, out, sizeof(e), hipMemcpyDeviceToHost), "copy energy"))
        return 1;
    printf("E1 %.17g\n", e[0]);

    hipFree(out);
    hipFree(sigma);
    hipFree(psi);
    hipFree(H.rowptr);
    hipFree(H.col);
    hipFree(H.val);
    hipFree(A.rowptr);
    hipFree(A.col);
    hipFree(A.val);
    vqe_destroy(ctx);
    return 0;
}
