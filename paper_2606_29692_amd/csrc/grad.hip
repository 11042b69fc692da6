// Pool-gradient screen (Eq. 5) and the selection of Sec. III-D.
//
// g_j = <psi|[H, A_j]|psi> = 2 Re sum_r conj(sigma_r) (A_j psi)_r for
// anti-Hermitian A_j and Hermitian H, with sigma = H psi computed once by the
// energy kernel and shared by every generator.  A workgroup takes one
// generator and one chunk of its rows and applies it to every state of its
// group (states that share the pool), so each pool CSR chunk is read once per
// group; psi and sigma are gathered from L2.  Partial sums are FP64 and are
// reduced in a fixed order (workgroup tree, then chunks in ascending order).
#include "kernels.hpp"

namespace {

template <int DT, bool BATCH>
__global__ void __launch_bounds__(256)
k_pool_grad(GradGroup single, const GradGroup *__restrict__ groups, const int4 *__restrict__ tasks)
{
    int gi, j, chunk;
    if (BATCH) {
        const int4 t = tasks[blockIdx.x];
        if (t.x < 0)
            return;
        gi = t.x;
        j = t.y;
        chunk = t.z;
    } else {
        gi = 0;
        j = blockIdx.x / single.nchunks;
        chunk = blockIdx.x % single.nchunks;
    }
    const GradGroup &G = BATCH ? groups[gi] : single;
    const int ns = G.n_states;
    const int64_t dim = G.dim;
    const vqe_csr op = G.ops[j];
    const int32_t *__restrict__ rowptr = op.rowptr;
    const int32_t *__restrict__ col = op.col;
    const int64_t r0 = (int64_t)chunk * G.chunk_rows;
    const int64_t r1 = r0 + G.chunk_rows < dim ? r0 + G.chunk_rows : dim;
    const void *psi[GRAD_MAX_GROUP];
    const void *sig[GRAD_MAX_GROUP];
    double shift[GRAD_MAX_GROUP];
    double acc[GRAD_MAX_GROUP];
#pragma unroll
    for (int s = 0; s < GRAD_MAX_GROUP; s++) {
        psi[s] = s < ns ? G.psi[s] : nullptr;
        sig[s] = s < ns ? G.sigma[s] : nullptr;
        shift[s] = s < ns ? G.shift[s] : 0.0;
        acc[s] = 0.0;
    }
    const bool pairing = (op.flags & VQE_PAIRING) != 0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) {
        const int k0 = rowptr[r], k1 = rowptr[r + 1];
        if (k0 == k1)
            continue;
        if (pairing) {
            // pair {r, c} with A[r,c] = a, A[c,r] = b, handled by its lower row:
            // conj(sigma_r) a psi_c + conj(sigma_c) b psi_r
            const int64_t c = col[k0];
            if (c < r)
                continue;
            const double2 a = Elem<DT>::ld(op.val, k0);
            const double2 b = c == r ? make_double2(0.0, 0.0) : Elem<DT>::ld(op.val, rowptr[c]);
#pragma unroll
            for (int s = 0; s < GRAD_MAX_GROUP; s++) {
                if (s < ns) {
                    const double2 pr = Elem<DT>::ld(psi[s], r);
                    const double2 pc = Elem<DT>::ld(psi[s], c);
                    const double2 qr = Elem<DT>::ld(sig[s], r);
                    const double2 qc = Elem<DT>::ld(sig[s], c);
                    const double sr_x = qr.x + shift[s] * pr.x, sr_y = qr.y + shift[s] * pr.y;
                    const double sc_x = qc.x + shift[s] * pc.x, sc_y = qc.y + shift[s] * pc.y;
                    const double wr = a.x * pc.x - a.y * pc.y, wi = a.x * pc.y + a.y * pc.x;
                    const double ur = b.x * pr.x - b.y * pr.y, ui = b.x * pr.y + b.y * pr.x;
                    acc[s] += (sr_x * wr + sr_y * wi) + (sc_x * ur + sc_y * ui);
                }
            }
            continue;
        }
        double2 sg[GRAD_MAX_GROUP];
#pragma unroll
        for (int s = 0; s < GRAD_MAX_GROUP; s++) {
            if (s < ns) {
                const double2 a = Elem<DT>::ld(sig[s], r);
                const double2 p = Elem<DT>::ld(psi[s], r);
                sg[s] = make_double2(a.x + shift[s] * p.x, a.y + shift[s] * p.y);
            }
        }
        for (int k = k0; k < k1; k++) {
            const int c = col[k];
            const double2 a = Elem<DT>::ld(op.val, k);
#pragma unroll
            for (int s = 0; s < GRAD_MAX_GROUP; s++) {
                if (s < ns) {
                    const double2 x = Elem<DT>::ld(psi[s], c);
                    const double wr = a.x * x.x - a.y * x.y;
                    const double wi = a.x * x.y + a.y * x.x;
                    acc[s] += sg[s].x * wr + sg[s].y * wi;
                }
            }
        }
    }
    __shared__ double s_red[4][GRAD_MAX_GROUP];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int s = 0; s < GRAD_MAX_GROUP; s++) {
        if (s < ns) {
            const double v = wave_sum(acc[s]);
            if (lane == 0)
                s_red[wid][s] = v;
        }
    }
    __syncthreads();
    if (threadIdx.x < ns) {
        const int s = threadIdx.x;
        const double v = ((s_red[0][s] + s_red[1][s]) + s_red[2][s]) + s_red[3][s];
        G.partials[s][(int64_t)j * G.nchunks + chunk] = v;
    }
}

template <bool BATCH>
__global__ void __launch_bounds__(256)
k_grad_fin(GradGroup single, const GradGroup *__restrict__ groups, const int2 *__restrict__ items)
{
    int gi = 0, slot = 0;
    if (BATCH) {
        const int2 it = items[blockIdx.x];
        gi = it.x;
        slot = it.y;
    }
    const GradGroup &G = BATCH ? groups[gi] : single;
    const double *p = G.partials[slot];
    double *g = G.g_out[slot];
    for (int j = threadIdx.x; j < G.M; j += 256) {
        double s = 0.0;
        for (int c = 0; c < G.nchunks; c++)
            s += p[(int64_t)j * G.nchunks + c];
        g[j] = 2.0 * s;
    }
}

template <bool BATCH>
__global__ void __launch_bounds__(64)
k_select_t(SelectState single, const SelectState *__restrict__ states, double rel_tie)
{
    const SelectState st = BATCH ? states[blockIdx.x] : single;
    if (VQE_SKIP(st))
        return;
    const int lane = threadIdx.x;
    double gmax = 0.0;
    for (int j = lane; j < st.M; j += 64)
        gmax = fmax(gmax, fabs(st.g[j]));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        gmax = fmax(gmax, __shfl_xor(gmax, o, 64));
    const double thr = gmax * (1.0 - rel_tie);
    int best = 0x7fffffff;
    for (int j = lane; j < st.M; j += 64)
        if (fabs(st.g[j]) >= thr && j < best)
            best = j;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        best = min(best, __shfl_xor(best, o, 64));
    if (lane == 0) {
        st.k_out[0] = best == 0x7fffffff ? 0 : best;
        st.gmax_out[0] = gmax;
    }
}

}  // namespace

void launch_pool_grad(int dtype, const GradGroup *groups, const int4 *tasks, unsigned grid,
                      hipStream_t s)
{
    GradGroup dummy{};
    if (dtype == VQE_C128)
        k_pool_grad<VQE_C128, true><<<grid, 256, 0, s>>>(dummy, groups, tasks);
    else
        k_pool_grad<VQE_C64, true><<<grid, 256, 0, s>>>(dummy, groups, tasks);
}

void launch_grad_finalize(const GradGroup *groups, const int2 *items, unsigned n_items,
                          hipStream_t s)
{
    GradGroup dummy{};
    k_grad_fin<true><<<n_items, 256, 0, s>>>(dummy, groups, items);
}

static int check_pool(vqe_ctx *ctx, const vqe_pool *pool, const vqe_csr *H)
{
    if (!pool || pool->M < 0 || (pool->M > 0 && (!pool->ops || !pool->ops_host)))
        return vqe_fail(ctx, VQE_EINVAL, "pool_gradients: bad pool");
    if (pool->n_qubits != H->n_qubits || pool->dtype != H->dtype)
        return vqe_fail(ctx, VQE_EINVAL, "pool_gradients: pool and H differ in size or dtype");
    for (int j = 0; j < pool->M; j++) {
        const vqe_csr &o = pool->ops_host[j];
        if (o.dim != H->dim || o.dtype != H->dtype || !o.rowptr || (o.nnz > 0 && (!o.col || !o.val)))
            return vqe_fail(ctx, VQE_EINVAL, "pool_gradients: generator %d does not match H", j);
    }
    return VQE_OK;
}

int vqe_pool_grad_launch(vqe_ctx *ctx, const vqe_csr *H, const vqe_pool *pool, const void *psi,
                         const void *sigma, double *g_out)
{
    const int64_t dim = H->dim;
    const int chunk_rows = (int)(dim < GRAD_CHUNK_ROWS ? dim : GRAD_CHUNK_ROWS);
    const int nchunks = (int)((dim + chunk_rows - 1) / chunk_rows);
    const int M = pool->M;
    if (M == 0)
        return VQE_OK;
    // workspace: [gradient partials][product partials][sigma][energy]
    const int lanes = vqe_effective_schedule(H, vqe_default_schedule(H));
    const size_t o_sp = vqe_align((size_t)M * nchunks * sizeof(double));
    const size_t o_sigma = o_sp + vqe_spmv_partials_bytes(dim, lanes);
    const size_t o_e = o_sigma + vqe_align(dim * vqe_elem_bytes(H->dtype));
    int rc = vqe_ws_reserve(ctx, sigma ? o_sp : o_e + 256);
    if (rc)
        return rc;
    char *ws = (char *)ctx->ws;
    if (!sigma) {
        rc = vqe_spmv_energy_core(ctx, H, psi, ws + o_sigma, (double *)(ws + o_e), lanes,
                                  (double *)(ws + o_sp));
        if (rc)
            return rc;
        sigma = ws + o_sigma;
    }
    GradGroup G{};
    G.ops = pool->ops;
    G.M = M;
    G.n_states = 1;
    G.nchunks = nchunks;
    G.chunk_rows = chunk_rows;
    G.dim = dim;
    G.psi[0] = psi;
    G.sigma[0] = sigma;
    G.shift[0] = H->diag_shift;
    G.partials[0] = (double *)ws;
    G.g_out[0] = g_out;
    const unsigned grid = (unsigned)M * (unsigned)nchunks;
    if (H->dtype == VQE_C128)
        k_pool_grad<VQE_C128, false><<<grid, 256, 0, ctx->stream>>>(G, nullptr, nullptr);
    else
        k_pool_grad<VQE_C64, false><<<grid, 256, 0, ctx->stream>>>(G, nullptr, nullptr);
    k_grad_fin<false><<<1, 256, 0, ctx->stream>>>(G, nullptr, nullptr);
    VQE_LAUNCH_CHECK(ctx);
    return VQE_OK;
}

extern "C" int pool_gradients(vqe_ctx *ctx, const vqe_csr *H, const vqe_pool *pool,
                              const void *psi, const void *sigma, double *g_out)
{
    if (!ctx)
        return VQE_EINVAL;
    int rc = check_csr(ctx, H, "pool_gradients");
    if (rc)
        return rc;
    rc = check_pool(ctx, pool, H);
    if (rc)
        return rc;
    if (!psi || (!g_out && pool->M > 0))
        return vqe_fail(ctx, VQE_EINVAL, "pool_gradients: null psi or g_out");
    return vqe_pool_grad_launch(ctx, H, pool, psi, sigma, g_out);
}

int vqe_select_launch(vqe_ctx *ctx, int32_t M, const double *g, double rel_tie, int32_t *k_out,
                      double *gmax_out)
{
    SelectState st{g, M, k_out, gmax_out};
    k_select_t<false><<<1, 64, 0, ctx->stream>>>(st, nullptr, rel_tie);
    VQE_LAUNCH_CHECK(ctx);
    return VQE_OK;
}

extern "C" int vqe_select(vqe_ctx *ctx, int32_t M, const double *g, double rel_tie,
                          int32_t *k_out, double *gmax_out)
{
    if (!ctx)
        return VQE_EINVAL;
    if (M < 1 || !g || !k_out || !gmax_out || !(rel_tie >= 0.0 && rel_tie < 1.0))
        return vqe_fail(ctx, VQE_EINVAL, "vqe_select: bad arguments");
    return vqe_select_launch(ctx, M, g, rel_tie, k_out, gmax_out);
}
