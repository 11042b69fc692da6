// Commuting-family partition of a matrix-free pool (Sec. III-F, Alg. 1).
//
// Graph (device).  For generators in matrix-free form, A|c> = f(c)|c ^ x>
// with f(c) = v (-1)^{|zsign & c|} on the support coset and 0 elsewhere, so
//     A_i A_j |c> = f_j(c) f_i(c ^ x_j) |c ^ x_i ^ x_j>,
//     A_j A_i |c> = f_i(c) f_j(c ^ x_i) |c ^ x_i ^ x_j>.
// Both products carry the factor v_i v_j; [A_i, A_j] = 0 exactly when, for
// every column c, the two terms are either both absent or both present with
// the same sign.  That is integer work only: one wave per pair of
// generators scans the columns (stopping at the first difference).
//
// Colouring (host).  Alg. 1: vertices by descending degree in the
// non-commutation graph (ties by index), each placed in the lowest-indexed
// family that holds none of its neighbours, or in a new family.
#include "kernels.hpp"

#include <algorithm>
#include <numeric>
#include <vector>

namespace {

__device__ __forceinline__ bool in_support(const vqe_mf_desc &d, uint64_t c)
{
    bool on = true;
    for (int i = 0; i < d.n_con; i++)
        on = on && (uint64_t)(__popcll(d.beta[i] & c) & 1) == (uint64_t)((d.kbits >> i) & 1u);
    return on;
}

__global__ void __launch_bounds__(256)
k_noncommute(const vqe_mf_desc *__restrict__ desc, int32_t M, int64_t dim, uint8_t *__restrict__ adj)
{
    const int i = blockIdx.y;
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (j >= M || j <= i)
        return;
    const vqe_mf_desc &a = desc[i], &b = desc[j];
    bool differ = false;
    for (int64_t c0 = 0; c0 < dim && !differ; c0 += 64) {
        const uint64_t c = (uint64_t)(c0 + lane);
        bool d = false;
        if ((int64_t)c < dim) {
            // A_i A_j |c>: f_j(c) f_i(c ^ x_j);  A_j A_i |c>: f_i(c) f_j(c ^ x_i)
            const bool u_on = in_support(b, c) && in_support(a, c ^ b.x);
            const bool w_on = in_support(a, c) && in_support(b, c ^ a.x);
            const int su = (__popcll(b.zsign & c) + __popcll(a.zsign & (c ^ b.x))) & 1;
            const int sw = (__popcll(a.zsign & c) + __popcll(b.zsign & (c ^ a.x))) & 1;
            d = (u_on != w_on) || (u_on && su != sw);
        }
        differ = __ballot(d) != 0;   // uniform across the wave
    }
    if (lane == 0) {
        adj[(int64_t)i * M + j] = differ ? 1 : 0;
        adj[(int64_t)j * M + i] = differ ? 1 : 0;
    }
}

__global__ void k_zero_diag(int32_t M, uint8_t *adj)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < M)
        adj[(int64_t)i * M + i] = 0;
}

}  // namespace

extern "C" int vqe_mf_noncommutation(vqe_ctx *ctx, const vqe_mf_pool *pool, uint8_t *adj)
{
    if (!ctx)
        return VQE_EINVAL;
    if (!pool || !adj)
        return vqe_fail(ctx, VQE_EINVAL, "vqe_mf_noncommutation: null pool or output");
    const int M = vqe_mf_pool_size(pool);
    const int n = vqe_mf_pool_qubits(pool);
    std::vector<vqe_mf_desc> d(M);
    for (int j = 0; j < M; j++)
        (void)vqe_mf_pool_get(pool, j, &d[j]);
    int rc = vqe_ws_reserve(ctx, (size_t)M * sizeof(vqe_mf_desc));
    if (rc)
        return rc;
    VQE_HIP(ctx, hipMemcpyAsync(ctx->ws, d.data(), d.size() * sizeof(vqe_mf_desc),
                                hipMemcpyHostToDevice, ctx->stream));
    const dim3 grid((unsigned)((M + 3) / 4), (unsigned)M);
    k_noncommute<<<grid, 256, 0, ctx->stream>>>((const vqe_mf_desc *)ctx->ws, M, (int64_t)1 << n, adj);
    k_zero_diag<<<(unsigned)((M + 255) / 256), 256, 0, ctx->stream>>>(M, adj);
    VQE_LAUNCH_CHECK(ctx);
    // the host descriptors are a local copy: finish before returning
    VQE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return VQE_OK;
}

extern "C" int vqe_partition_greedy(int32_t M, const uint8_t *adj, int32_t *family,
                                    int32_t *n_families)
{
    if (M < 0 || (M > 0 && (!adj || !family)) || !n_families)
        return VQE_EINVAL;
    std::vector<int64_t> degree(M, 0);
    for (int i = 0; i < M; i++)
        for (int j = 0; j < M; j++)
            degree[i] += (i != j && adj[(int64_t)i * M + j]) ? 1 : 0;
    std::vector<int> order(M);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return degree[a] > degree[b]; });
    std::vector<std::vector<int>> fam;
    for (int v : order) {
        int placed = -1;
        for (size_t k = 0; k < fam.size() && placed < 0; k++) {
            bool free = true;
            for (int u : fam[k])
                if (adj[(int64_t)v * M + u]) {
                    free = false;
                    break;
                }
            if (free)
                placed = (int)k;
        }
        if (placed < 0) {
            placed = (int)fam.size();
            fam.emplace_back();
        }
        fam[placed].push_back(v);
        family[v] = placed;
    }
    *n_families = (int32_t)fam.size();
    return VQE_OK;
}
