// sigma = S psi with the FP64 energy reduction (Eq. 1) fused into the epilogue.
//
// Row-bucketed CSR-vector product: a sub-group of L lanes (L = 8..64, fixed
// per operator) owns one row, streams its column indices and values with
// coalesced loads (four strided loads in flight per lane), gathers psi from
// L2, multiplies in FP64 and reduces with a butterfly.  The sub-group leader
// writes sigma_r and accumulates conj(psi_r) sigma_r and |psi_r|^2; each
// workgroup writes one FP64 partial triple, and a one-wave-per-state kernel
// sums the partials in a fixed order.  The grid is either one state (block b
// -> rows of b) or a batch task table built so that all blocks of a state run
// on the same XCD (workgroup IDs are dealt round-robin over the 8 XCDs).
#include "kernels.hpp"

namespace {

template <int DT, int L, bool BATCH>
__global__ void __launch_bounds__(256)
k_spmv_energy(SpmvState single, const SpmvState *__restrict__ states,
              const int2 *__restrict__ tasks)
{
    SpmvState st;
    int blk;
    if (BATCH) {
        int2 t = tasks[blockIdx.x];
        if (t.x < 0)
            return;
        st = states[t.x];
        blk = t.y;
    } else {
        st = single;
        blk = blockIdx.x;
    }
    constexpr int G = VQE_WAVE / L;
    constexpr int RPB = spmv_rows_per_block(L);
    constexpr int U = 4;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int sub = lane / L, sl = lane % L;
    const int32_t *__restrict__ rowptr = st.rowptr;
    const int32_t *__restrict__ col = st.col;
    using V = typename Elem<DT>::T;
    const V *__restrict__ val = reinterpret_cast<const V *>(st.val);
    double e_re = 0.0, e_im = 0.0, e_n2 = 0.0;
#pragma unroll
    for (int it = 0; it < SPMV_RPT; it++) {
        const int64_t r = (int64_t)blk * RPB + (it * 4 + wid) * G + sub;
        double are = 0.0, aim = 0.0;
        if (r < st.dim) {
            const int k1 = rowptr[r + 1];
            for (int k = rowptr[r] + sl; k < k1; k += U * L) {
                int c[U];
                V v[U];
#pragma unroll
                for (int u = 0; u < U; u++) {
                    const int kk = k + u * L;
                    if (kk < k1) {
                        c[u] = __builtin_nontemporal_load(col + kk);
                        v[u] = val[kk];
                    } else {
                        c[u] = -1;
                    }
                }
#pragma unroll
                for (int u = 0; u < U; u++) {
                    if (c[u] >= 0) {
                        const double2 x = Elem<DT>::ld(st.psi, c[u]);
                        const double ar = (double)v[u].x, ai = (double)v[u].y;
                        are += ar * x.x - ai * x.y;
                        aim += ar * x.y + ai * x.x;
                    }
                }
            }
        }
        are = group_sum<L>(are);
        aim = group_sum<L>(aim);
        if (sl == 0 && r < st.dim) {
            Elem<DT>::st(st.sigma, r, make_double2(are, aim));
            const double2 p = Elem<DT>::ld(st.psi, r);
            e_re += p.x * are + p.y * aim;
            e_im += p.x * aim - p.y * are;
            e_n2 += p.x * p.x + p.y * p.y;
        }
    }
    __shared__ double s_part[4][3];
    e_re = wave_sum(e_re);
    e_im = wave_sum(e_im);
    e_n2 = wave_sum(e_n2);
    if (lane == 0) {
        s_part[wid][0] = e_re;
        s_part[wid][1] = e_im;
        s_part[wid][2] = e_n2;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const int q = threadIdx.x;
        const double v = ((s_part[0][q] + s_part[1][q]) + s_part[2][q]) + s_part[3][q];
        st.partials[(int64_t)blk * 3 + q] = v;
    }
}

}  // namespace

// One wave per state: fixed-order sum of the block partials, then
// out = {shift + re/n2, n2, im}.
__global__ void __launch_bounds__(64)
k_energy_finalize(SpmvState single, const SpmvState *__restrict__ states, int n_states)
{
    const int s = blockIdx.x;
    if (s >= n_states)
        return;
    const SpmvState st = states ? states[s] : single;
    const int lane = threadIdx.x;
    double re = 0.0, im = 0.0, n2 = 0.0;
    for (int b = lane; b < st.nblocks; b += 64) {
        re += st.partials[(int64_t)b * 3 + 0];
        im += st.partials[(int64_t)b * 3 + 1];
        n2 += st.partials[(int64_t)b * 3 + 2];
    }
    re = wave_sum(re);
    im = wave_sum(im);
    n2 = wave_sum(n2);
    if (lane == 0 && st.energy_out) {
        st.energy_out[0] = st.shift + re / n2;
        st.energy_out[1] = n2;
        st.energy_out[2] = im;
    }
}

template <int DT, int L>
static void launch_spmv_t(const SpmvState &single, const SpmvState *states, const int2 *tasks,
                          unsigned grid, hipStream_t s)
{
    if (tasks)
        k_spmv_energy<DT, L, true><<<grid, 256, 0, s>>>(single, states, tasks);
    else
        k_spmv_energy<DT, L, false><<<grid, 256, 0, s>>>(single, states, tasks);
}

void launch_spmv(int dtype, int lanes, const SpmvState &single, const SpmvState *states,
                 const int2 *tasks, unsigned grid, hipStream_t s)
{
    if (dtype == VQE_C128) {
        switch (lanes) {
        case 8: launch_spmv_t<VQE_C128, 8>(single, states, tasks, grid, s); break;
        case 16: launch_spmv_t<VQE_C128, 16>(single, states, tasks, grid, s); break;
        case 32: launch_spmv_t<VQE_C128, 32>(single, states, tasks, grid, s); break;
        default: launch_spmv_t<VQE_C128, 64>(single, states, tasks, grid, s); break;
        }
    } else {
        switch (lanes) {
        case 8: launch_spmv_t<VQE_C64, 8>(single, states, tasks, grid, s); break;
        case 16: launch_spmv_t<VQE_C64, 16>(single, states, tasks, grid, s); break;
        case 32: launch_spmv_t<VQE_C64, 32>(single, states, tasks, grid, s); break;
        default: launch_spmv_t<VQE_C64, 64>(single, states, tasks, grid, s); break;
        }
    }
}

extern "C" int32_t vqe_default_lanes(const vqe_csr *H)
{
    if (!H || H->dim <= 0)
        return 32;
    const double avg = (double)H->nnz / (double)H->dim;
    if (avg >= 96.0)
        return 64;
    if (avg >= 40.0)
        return 32;
    if (avg >= 12.0)
        return 16;
    return 8;
}

int check_csr(vqe_ctx *ctx, const vqe_csr *M, const char *what)
{
    if (!M)
        return vqe_fail(ctx, VQE_EINVAL, "%s: null operator", what);
    if (M->n_qubits < 1 || M->n_qubits > 30 || M->dim != ((int64_t)1 << M->n_qubits))
        return vqe_fail(ctx, VQE_EINVAL, "%s: bad operator size", what);
    if (M->dtype != VQE_C128 && M->dtype != VQE_C64)
        return vqe_fail(ctx, VQE_EINVAL, "%s: bad operator dtype", what);
    if (!M->rowptr || (M->nnz > 0 && (!M->col || !M->val)))
        return vqe_fail(ctx, VQE_EINVAL, "%s: operator arrays not set", what);
    if (M->nnz < 0 || M->nnz > 0x7fffffff)
        return vqe_fail(ctx, VQE_ESIZE, "%s: bad nnz", what);
    return VQE_OK;
}

int vqe_spmv_energy_core(vqe_ctx *ctx, const vqe_csr *H, const void *psi, void *sigma,
                         double *out, int lanes, double *partials)
{
    const int64_t dim = H->dim;
    const int rpb = spmv_rows_per_block(lanes);
    const int64_t nblk = (dim + rpb - 1) / rpb;
    SpmvState st{};
    st.rowptr = H->rowptr;
    st.col = H->col;
    st.val = H->val;
    st.psi = psi;
    st.sigma = sigma;
    st.partials = partials;
    st.energy_out = out;
    st.dim = dim;
    st.shift = H->diag_shift;
    st.nblocks = (int32_t)nblk;
    st.lanes = lanes;
    launch_spmv(H->dtype, lanes, st, nullptr, nullptr, (unsigned)nblk, ctx->stream);
    k_energy_finalize<<<1, 64, 0, ctx->stream>>>(st, nullptr, 1);
    VQE_LAUNCH_CHECK(ctx);
    return VQE_OK;
}

size_t vqe_spmv_partials_bytes(int64_t dim, int lanes)
{
    const int rpb = spmv_rows_per_block(lanes);
    return vqe_align((size_t)((dim + rpb - 1) / rpb) * 3 * sizeof(double));
}

int vqe_spmv_energy_launch(vqe_ctx *ctx, const vqe_csr *H, const void *psi, void *sigma,
                           double *out, int lanes)
{
    const size_t o_sigma = vqe_spmv_partials_bytes(H->dim, lanes);
    size_t need = o_sigma;
    if (!sigma)
        need += vqe_align(H->dim * vqe_elem_bytes(H->dtype));
    int rc = vqe_ws_reserve(ctx, need);
    if (rc)
        return rc;
    void *sg = sigma ? sigma : (char *)ctx->ws + o_sigma;
    return vqe_spmv_energy_core(ctx, H, psi, sg, out, lanes, (double *)ctx->ws);
}

extern "C" int energy(vqe_ctx *ctx, const vqe_csr *H, const void *psi, void *sigma_out,
                      double *out)
{
    if (!ctx)
        return VQE_EINVAL;
    int rc = check_csr(ctx, H, "energy");
    if (rc)
        return rc;
    if (!psi || !out)
        return vqe_fail(ctx, VQE_EINVAL, "energy: null psi or out");
    return vqe_spmv_energy_launch(ctx, H, psi, sigma_out, out, vqe_default_lanes(H));
}

extern "C" int vqe_time_spmv(vqe_ctx *ctx, const vqe_csr *H, const void *psi, void *sigma,
                             int32_t lanes, int32_t reps, float *ms_out)
{
    if (!ctx)
        return VQE_EINVAL;
    int rc = check_csr(ctx, H, "vqe_time_spmv");
    if (rc)
        return rc;
    if (!psi || !sigma || !ms_out || reps < 1)
        return vqe_fail(ctx, VQE_EINVAL, "vqe_time_spmv: bad arguments");
    if (lanes != 8 && lanes != 16 && lanes != 32 && lanes != 64)
        return vqe_fail(ctx, VQE_EINVAL, "vqe_time_spmv: lanes must be 8, 16, 32 or 64");
    // energy result goes after the partials in the workspace
    const size_t o_out = vqe_spmv_partials_bytes(H->dim, lanes);
    rc = vqe_ws_reserve(ctx, o_out + 256);
    if (rc)
        return rc;
    double *out = (double *)((char *)ctx->ws + o_out);
    hipEvent_t e0, e1;
    VQE_HIP(ctx, hipEventCreate(&e0));
    VQE_HIP(ctx, hipEventCreate(&e1));
    double *part = (double *)ctx->ws;
    rc = vqe_spmv_energy_core(ctx, H, psi, sigma, out, lanes, part);   // warm-up
    if (rc)
        return rc;
    VQE_HIP(ctx, hipEventRecord(e0, ctx->stream));
    for (int i = 0; i < reps && rc == VQE_OK; i++)
        rc = vqe_spmv_energy_core(ctx, H, psi, sigma, out, lanes, part);
    VQE_HIP(ctx, hipEventRecord(e1, ctx->stream));
    VQE_HIP(ctx, hipEventSynchronize(e1));
    float ms = 0.f;
    VQE_HIP(ctx, hipEventElapsedTime(&ms, e0, e1));
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    *ms_out = ms / (float)reps;
    return rc;
}
