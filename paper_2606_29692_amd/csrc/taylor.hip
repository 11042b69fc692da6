// Fifth-order Taylor state update (Eq. 6): v_n = A v_{n-1} for n = 1..5
// (Eq. 7) and psi' = psi + sum_n c_n v_n with c_n = c_{n-1} theta / n (Eq. 8).
//
// Pairing generators (every fermionic single or double excitation under JW
// or BK) hold at most one entry per row and pair row r with column c = col(r)
// and col(c) = r.  On such a pair {r, c} the operator is the 2x2 block
// [[0, a], [b, 0]], so one thread owns the pair and runs all five products
// and the accumulation in FP64 registers: one fused kernel, no barriers, no
// intermediate vectors.  Rows without an entry keep their amplitude.
//
// Other operators use either one persistent workgroup per state (five passes
// separated by workgroup barriers, vectors in L2-resident scratch) or, when
// large, five chained grid-wide launches.
//
// In a batch plan whose pools have compact pair tables, the update walks the
// selected generator's pairs instead of its CSR rows.
//
// Renormalisation: an FP64 fixed-order norm (per-block partials, then every
// block re-sums the partials of its state) followed by the rescale.
#include "kernels.hpp"

namespace {

__device__ __forceinline__ void taylor_coeffs(double theta, double c[6])
{
    c[0] = 1.0;
#pragma unroll
    for (int n = 1; n <= 5; n++)
        c[n] = c[n - 1] * theta / (double)n;
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

template <int DT, bool BATCH>
__global__ void __launch_bounds__(TAYLOR_ROWS_PER_BLOCK)
k_taylor_pair(TaylorState single, const TaylorState *__restrict__ states,
              const int2 *__restrict__ tasks)
{
    int blk;
    const TaylorState *stp;
    if (BATCH) {
        const int2 t = tasks[blockIdx.x];
        if (t.x < 0)
            return;
        stp = states + t.x;
        blk = t.y;
        if (VQE_SKIP(*stp))
            return;
    } else {
        stp = &single;
        blk = blockIdx.x;
    }
    const int64_t r = (int64_t)blk * TAYLOR_ROWS_PER_BLOCK + threadIdx.x;
    const int64_t dim = stp->dim;
    if (r >= dim)
        return;
    const int32_t *rowptr;
    const int32_t *col;
    const void *val;
    if (stp->k) {
        const int32_t kk = *stp->k;
        if (kk < 0 || kk >= stp->M)
            return;
        const vqe_csr *op = stp->ops + kk;
        rowptr = op->rowptr;
        col = op->col;
        val = op->val;
    } else {
        rowptr = stp->op.rowptr;
        col = stp->op.col;
        val = stp->op.val;
    }
    const int k0 = gmem(rowptr)[r];
    if (gmem(rowptr)[r + 1] - k0 != 1)
        return;
    const int64_t c = gmem(col)[k0];
    if (c < r)
        return;   // the partner row owns the pair
    const double theta = stp->theta ? *stp->theta : stp->theta_value;
    double cf[6];
    taylor_coeffs(theta, cf);
    void *psi = stp->psi;
    const double2 a = Elem<DT>::ld(val, k0);
    if (c == r) {
        // 1x1 block: v_n = a^n psi_r
        double2 v = Elem<DT>::ld(psi, r);
        double2 acc = v;
#pragma unroll
        for (int n = 1; n <= 5; n++) {
            v = cmul(a, v);
            acc.x += cf[n] * v.x;
            acc.y += cf[n] * v.y;
        }
        Elem<DT>::st(psi, r, acc);
        return;
    }
    const double2 b = Elem<DT>::ld(val, gmem(rowptr)[c]);
    double2 vr = Elem<DT>::ld(psi, r), vc = Elem<DT>::ld(psi, c);
    double2 ar = vr, ac = vc;
#pragma unroll
    for (int n = 1; n <= 5; n++) {
        const double2 nr = cmul(a, vc);   // (A v)_r = A[r,c] v_c
        const double2 nc = cmul(b, vr);   // (A v)_c = A[c,r] v_r
        vr = nr;
        vc = nc;
        ar.x += cf[n] * vr.x;
        ar.y += cf[n] * vr.y;
        ac.x += cf[n] * vc.x;
        ac.y += cf[n] * vc.y;
    }
    Elem<DT>::st(psi, r, ar);
    Elem<DT>::st(psi, c, ac);
}

// Batched update through the compact pair table of the state's pool: one
// thread per pair {r, c = r ^ x_k} of the selected generator k, entries +-1.
template <int DT>
__global__ void __launch_bounds__(TAYLOR_ROWS_PER_BLOCK)
k_taylor_compact(const TaylorState *__restrict__ states, const int2 *__restrict__ tasks)
{
    const int2 task = tasks[blockIdx.x];
    if (task.x < 0)
        return;
    const TaylorState *stp = states + task.x;
    if (VQE_SKIP(*stp))
        return;
    const int32_t k = *stp->k;
    if (k < 0 || k >= stp->M)
        return;
    const PairTable *tb = stp->table;
    const int p0 = gmem(tb->pts)[k * tb->nt], p1 = gmem(tb->pts)[(k + 1) * tb->nt];
    const int p = p0 + task.y * TAYLOR_ROWS_PER_BLOCK + threadIdx.x;
    if (p >= p1)
        return;
    const uint32_t w = gmem(tb->words)[p];
    const int64_t r = w & 0x3fffffffu;
    const int64_t c = r ^ (int64_t)gmem(tb->xmask)[k];
    const double sa = (w >> 30) & 1u ? -1.0 : 1.0;   // A[r,c]
    const double sb = (w >> 31) ? -1.0 : 1.0;         // A[c,r]
    const double theta = *stp->theta;
    double cf[6];
    taylor_coeffs(theta, cf);
    void *psi = stp->psi;
    double2 vr = Elem<DT>::ld(psi, r), vc = Elem<DT>::ld(psi, c);
    double2 ar = vr, ac = vc;
#pragma unroll
    for (int n = 1; n <= 5; n++) {
        const double2 nr = make_double2(sa * vc.x, sa * vc.y);
        const double2 nc = make_double2(sb * vr.x, sb * vr.y);
        vr = nr;
        vc = nc;
        ar.x += cf[n] * vr.x;
        ar.y += cf[n] * vr.y;
        ac.x += cf[n] * vc.x;
        ac.y += cf[n] * vc.y;
    }
    Elem<DT>::st(psi, r, ar);
    Elem<DT>::st(psi, c, ac);
}

template <int DT, bool BATCH>
__global__ void __launch_bounds__(256)
k_norm_partials(TaylorState single, const TaylorState *__restrict__ states,
                const int2 *__restrict__ tasks)
{
    int blk;
    const TaylorState *stp;
    if (BATCH) {
        const int2 t = tasks[blockIdx.x];
        if (t.x < 0)
            return;
        stp = states + t.x;
        blk = t.y;
        if (VQE_SKIP(*stp))
            return;
    } else {
        stp = &single;
        blk = blockIdx.x;
    }
    const int64_t r0 = (int64_t)blk * NORM_ROWS_PER_BLOCK;
    const int64_t r1 = r0 + NORM_ROWS_PER_BLOCK < stp->dim ? r0 + NORM_ROWS_PER_BLOCK : stp->dim;
    double s = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) {
        const double2 p = Elem<DT>::ld(stp->psi, r);
        s += p.x * p.x + p.y * p.y;
    }
    __shared__ double red[4];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0)
        gmem(stp->norm_partials)[blk] = ((red[0] + red[1]) + red[2]) + red[3];
}

template <int DT, bool BATCH>
__global__ void __launch_bounds__(256)
k_norm_scale(TaylorState single, const TaylorState *__restrict__ states,
             const int2 *__restrict__ tasks)
{
    int blk;
    const TaylorState *stp;
    if (BATCH) {
        const int2 t = tasks[blockIdx.x];
        if (t.x < 0)
            return;
        stp = states + t.x;
        blk = t.y;
        if (VQE_SKIP(*stp))
            return;
    } else {
        stp = &single;
        blk = blockIdx.x;
    }
    __shared__ double s_n2;
    if (threadIdx.x < 64) {
        double s = 0.0;
        for (int b = threadIdx.x; b < stp->nblocks; b += 64)
            s += gmem(stp->norm_partials)[b];
        s = wave_sum(s);
        if (threadIdx.x == 0)
            s_n2 = s;
    }
    __syncthreads();
    const double n2 = s_n2;
    if (blk == 0 && threadIdx.x == 0 && stp->norm2_out)
        stp->norm2_out[0] = n2;
    if (!stp->renorm)
        return;
    const double inv = 1.0 / sqrt(n2);
    const int64_t r0 = (int64_t)blk * NORM_ROWS_PER_BLOCK;
    const int64_t r1 = r0 + NORM_ROWS_PER_BLOCK < stp->dim ? r0 + NORM_ROWS_PER_BLOCK : stp->dim;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) {
        const double2 p = Elem<DT>::ld(stp->psi, r);
        Elem<DT>::st(stp->psi, r, make_double2(p.x * inv, p.y * inv));
    }
}

// Generic operator, one persistent workgroup: five passes with barriers.
// v0/v1 and acc are FP64 scratch of dim elements each.
template <int DT>
__global__ void __launch_bounds__(1024)
k_taylor_generic_wg(vqe_csr A, double theta, void *psi, double2 *v0, double2 *v1, double2 *acc)
{
    const int64_t dim = A.dim;
    for (int64_t r = threadIdx.x; r < dim; r += 1024) {
        const double2 p = Elem<DT>::ld(psi, r);
        v0[r] = p;
        acc[r] = p;
    }
    __syncthreads();
    double cf[6];
    taylor_coeffs(theta, cf);
    double2 *prev = v0, *next = v1;
    for (int n = 1; n <= 5; n++) {
        for (int64_t r = threadIdx.x; r < dim; r += 1024) {
            double re = 0.0, im = 0.0;
            for (int k = A.rowptr[r]; k < A.rowptr[r + 1]; k++) {
                const double2 a = Elem<DT>::ld(A.val, k);
                const double2 x = prev[A.col[k]];
                re += a.x * x.x - a.y * x.y;
                im += a.x * x.y + a.y * x.x;
            }
            next[r] = make_double2(re, im);
            double2 s = acc[r];
            s.x += cf[n] * re;
            s.y += cf[n] * im;
            acc[r] = s;
        }
        __syncthreads();
        double2 *t = prev;
        prev = next;
        next = t;
    }
    for (int64_t r = threadIdx.x; r < dim; r += 1024)
        Elem<DT>::st(psi, r, acc[r]);
}

// Generic operator, grid-wide: one launch per product.
template <int DT>
__global__ void __launch_bounds__(256)
k_taylor_generic_step(vqe_csr A, double cn, const double2 *prev, double2 *next, double2 *acc)
{
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= A.dim)
        return;
    double re = 0.0, im = 0.0;
    for (int k = A.rowptr[r]; k < A.rowptr[r + 1]; k++) {
        const double2 a = Elem<DT>::ld(A.val, k);
        const double2 x = prev[A.col[k]];
        re += a.x * x.x - a.y * x.y;
        im += a.x * x.y + a.y * x.x;
    }
    next[r] = make_double2(re, im);
    double2 s = acc[r];
    s.x += cn * re;
    s.y += cn * im;
    acc[r] = s;
}

template <int DT>
__global__ void k_load_state(int64_t dim, const void *psi, double2 *v0, double2 *acc)
{
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r < dim) {
        const double2 p = Elem<DT>::ld(psi, r);
        v0[r] = p;
        acc[r] = p;
    }
}

template <int DT>
__global__ void k_store_state(int64_t dim, const double2 *acc, void *psi)
{
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r < dim)
        Elem<DT>::st(psi, r, acc[r]);
}

constexpr int64_t kGenericWgMaxNnz = 1 << 18;

__global__ void __launch_bounds__(256)
k_theta_row(const double *__restrict__ src, double *__restrict__ dst, int n)
{
    const int i = (int)blockIdx.x * 256 + (int)threadIdx.x;
    if (i < n)
        dst[i] = src[i];
}

}  // namespace

void launch_theta_row(const double *src, double *dst, int n, hipStream_t s)
{
    if (n > 0)
        k_theta_row<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(src, dst, n);
}

void launch_taylor_pair(int dtype, const TaylorState *states, const int2 *tasks, unsigned grid,
                        hipStream_t s)
{
    TaylorState dummy{};
    if (dtype == VQE_C128)
        k_taylor_pair<VQE_C128, true><<<grid, TAYLOR_ROWS_PER_BLOCK, 0, s>>>(dummy, states, tasks);
    else
        k_taylor_pair<VQE_C64, true><<<grid, TAYLOR_ROWS_PER_BLOCK, 0, s>>>(dummy, states, tasks);
}

void launch_taylor_compact(int dtype, const TaylorState *states, const int2 *tasks,
                           unsigned grid, hipStream_t s)
{
    if (dtype == VQE_C128)
        k_taylor_compact<VQE_C128><<<grid, TAYLOR_ROWS_PER_BLOCK, 0, s>>>(states, tasks);
    else
        k_taylor_compact<VQE_C64><<<grid, TAYLOR_ROWS_PER_BLOCK, 0, s>>>(states, tasks);
}

void launch_norm(int dtype, const TaylorState *states, const int2 *tasks, unsigned grid,
                 hipStream_t s)
{
    TaylorState dummy{};
    if (dtype == VQE_C128) {
        k_norm_partials<VQE_C128, true><<<grid, 256, 0, s>>>(dummy, states, tasks);
        k_norm_scale<VQE_C128, true><<<grid, 256, 0, s>>>(dummy, states, tasks);
    } else {
        k_norm_partials<VQE_C64, true><<<grid, 256, 0, s>>>(dummy, states, tasks);
        k_norm_scale<VQE_C64, true><<<grid, 256, 0, s>>>(dummy, states, tasks);
    }
}

template <int DT>
static int taylor_single(vqe_ctx *ctx, const vqe_csr *A, double theta, void *psi, int renorm,
                         double *norm2_out)
{
    hipStream_t s = ctx->stream;
    const int64_t dim = A->dim;
    const int64_t nnorm = (dim + NORM_ROWS_PER_BLOCK - 1) / NORM_ROWS_PER_BLOCK;
    const bool pairing = (A->flags & VQE_PAIRING) != 0;
    size_t need = vqe_align(nnorm * sizeof(double));
    const size_t o_vec = need;
    if (!pairing)
        need += 3 * vqe_align(dim * sizeof(double2));
    int rc = vqe_ws_reserve(ctx, need);
    if (rc)
        return rc;
    char *ws = (char *)ctx->ws;
    TaylorState st{};
    st.op = *A;
    st.theta_value = theta;
    st.psi = psi;
    st.dim = dim;
    st.norm_partials = (double *)ws;
    st.norm2_out = norm2_out;
    st.nblocks = (int32_t)nnorm;
    st.renorm = renorm;
    if (pairing) {
        const unsigned grid = (unsigned)((dim + TAYLOR_ROWS_PER_BLOCK - 1) / TAYLOR_ROWS_PER_BLOCK);
        k_taylor_pair<DT, false><<<grid, TAYLOR_ROWS_PER_BLOCK, 0, s>>>(st, nullptr, nullptr);
    } else {
        double2 *v0 = (double2 *)(ws + o_vec);
        double2 *v1 = (double2 *)(ws + o_vec + vqe_align(dim * sizeof(double2)));
        double2 *acc = (double2 *)(ws + o_vec + 2 * vqe_align(dim * sizeof(double2)));
        if (A->nnz <= kGenericWgMaxNnz) {
            k_taylor_generic_wg<DT><<<1, 1024, 0, s>>>(*A, theta, psi, v0, v1, acc);
        } else {
            const unsigned grid = (unsigned)((dim + 255) / 256);
            k_load_state<DT><<<grid, 256, 0, s>>>(dim, psi, v0, acc);
            double c = 1.0;
            double2 *prev = v0, *next = v1;
            for (int n = 1; n <= 5; n++) {
                c = c * theta / (double)n;
                k_taylor_generic_step<DT><<<grid, 256, 0, s>>>(*A, c, prev, next, acc);
                double2 *t = prev;
                prev = next;
                next = t;
            }
            k_store_state<DT><<<grid, 256, 0, s>>>(dim, acc, psi);
        }
    }
    if (renorm || norm2_out) {
        k_norm_partials<DT, false><<<(unsigned)nnorm, 256, 0, s>>>(st, nullptr, nullptr);
        k_norm_scale<DT, false><<<(unsigned)nnorm, 256, 0, s>>>(st, nullptr, nullptr);
    }
    VQE_LAUNCH_CHECK(ctx);
    return VQE_OK;
}

int vqe_taylor_launch(vqe_ctx *ctx, const vqe_csr *A, double theta, void *psi, int renorm,
                      double *norm2_out)
{
    return A->dtype == VQE_C128 ? taylor_single<VQE_C128>(ctx, A, theta, psi, renorm, norm2_out)
                                : taylor_single<VQE_C64>(ctx, A, theta, psi, renorm, norm2_out);
}

extern "C" int taylor5_apply(vqe_ctx *ctx, const vqe_csr *A, double theta, void *psi,
                             int32_t renormalize, double *norm2_out)
{
    if (!ctx)
        return VQE_EINVAL;
    int rc = check_csr(ctx, A, "taylor5_apply");
    if (rc)
        return rc;
    if (!psi)
        return vqe_fail(ctx, VQE_EINVAL, "taylor5_apply: null psi");
    if (!std::isfinite(theta))
        return vqe_fail(ctx, VQE_EINVAL, "taylor5_apply: theta is not finite");
    if (A->diag_shift != 0.0)
        return vqe_fail(ctx, VQE_EINVAL, "taylor5_apply: generator has a diagonal shift");
    return vqe_taylor_launch(ctx, A, theta, psi, renormalize, norm2_out);
}
