// Pauli sum -> CSR on the GPU (Eq. 3 compiled as in Sec. III-E).
//
// Term t adds to entry (r, r ^ x_t) the value c_t * i^{|x_t & z_t|} *
// (-1)^{|z_t & (r ^ x_t)|}.  Terms with the same x land in the same column of
// every row, so the terms are first grouped by x (a device sort of the keys
// (x << 32 | t), which keeps ascending t inside a group).  Each row is then
// handled by one wave whose lanes walk the groups: a lane sums its group's
// terms in ascending t from +0.0 with plain additions (multiplying by i^k and
// +-1 only permutes and negates parts, so every contribution is exact and the
// sum is bit-identical to any sequential evaluation in that order).  Kept
// entries are compacted into LDS and sorted by column with a bitonic network.
//
// This file is built with -ffp-contract=off.
#include "common.hpp"

#include <algorithm>
#include <vector>

namespace {

constexpr int kMaxRow = 2048;   // longest supported row (entries kept per row)

__global__ void k_make_keys(const uint64_t *__restrict__ x, int64_t T, int64_t P,
                            uint64_t *__restrict__ keys)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P)
        return;
    keys[i] = i < T ? ((x[i] << 32) | (uint64_t)i) : ~(uint64_t)0;
}

// One compare-exchange stage of a bitonic sort over P (a power of two) keys.
__global__ void k_bitonic_step(uint64_t *__restrict__ a, int64_t j, int64_t k, int64_t P)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P)
        return;
    int64_t l = i ^ j;
    if (l > i) {
        uint64_t ai = a[i], al = a[l];
        bool ascending = (i & k) == 0;
        if ((ai > al) == ascending) {
            a[i] = al;
            a[l] = ai;
        }
    }
}

// Single-workgroup grouping of the sorted keys: group heads, group x values,
// group starts, and the terms' z and coefficients in sorted order.
__global__ void __launch_bounds__(1024)
k_group(const uint64_t *__restrict__ keys, int64_t T, const uint64_t *__restrict__ z,
        const double2 *__restrict__ coeff, uint64_t *__restrict__ gx,
        int64_t *__restrict__ gstart, int64_t *__restrict__ n_groups,
        uint64_t *__restrict__ tz, double2 *__restrict__ tc)
{
    __shared__ int64_t s_wave[16];
    __shared__ int64_t s_carry;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    if (tid == 0)
        s_carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < T; base += 1024) {
        int64_t i = base + tid;
        int head = 0;
        if (i < T) {
            uint64_t key = keys[i];
            uint64_t t = key & 0xffffffffull;
            tz[i] = z[t];
            tc[i] = coeff[t];
            head = (i == 0) || ((keys[i - 1] >> 32) != (key >> 32));
        }
        uint64_t m = __ballot(head);
        int64_t before = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0)
            s_wave[wid] = __popcll(m);
        __syncthreads();
        int64_t off = s_carry;
        for (int w = 0; w < wid; w++)
            off += s_wave[w];
        if (head) {
            int64_t g = off + before;
            gx[g] = keys[i] >> 32;
            gstart[g] = i;
        }
        __syncthreads();
        if (tid == 0) {
            int64_t tot = 0;
            for (int w = 0; w < 16; w++)
                tot += s_wave[w];
            s_carry += tot;
        }
        __syncthreads();
    }
    if (tid == 0) {
        *n_groups = s_carry;
        gstart[s_carry] = T;
    }
}

__device__ __forceinline__ double2 term_value(double2 c, uint64_t x, uint64_t z, uint64_t col)
{
    int k = __popcll(x & z) & 3;
    double re, im;
    switch (k) {
    case 0: re = c.x; im = c.y; break;
    case 1: re = -c.y; im = c.x; break;
    case 2: re = -c.x; im = -c.y; break;
    default: re = c.y; im = -c.x; break;
    }
    if (__popcll(z & col) & 1) {
        re = -re;
        im = -im;
    }
    return make_double2(re, im);
}

// Entry of row r contributed by group g, summed in ascending term order.
__device__ __forceinline__ double2 group_entry(int64_t g, uint64_t r, const uint64_t *gx,
                                               const int64_t *gstart, const uint64_t *tz,
                                               const double2 *tc)
{
    uint64_t x = gx[g];
    uint64_t col = r ^ x;
    double re = 0.0, im = 0.0;
    for (int64_t i = gstart[g]; i < gstart[g + 1]; i++) {
        double2 v = term_value(tc[i], x, tz[i], col);
        re = re + v.x;
        im = im + v.y;
    }
    return make_double2(re, im);
}

__device__ __forceinline__ bool keep_entry(double2 v, double tol, bool force)
{
    return force || !(fabs(v.x) <= tol && fabs(v.y) <= tol);
}

// Phase 1: kept entries per row; for rows with exactly one entry, its column.
__global__ void __launch_bounds__(64)
k_row_count(int64_t dim, const uint64_t *__restrict__ gx, const int64_t *__restrict__ gstart,
            const int64_t *__restrict__ n_groups, const uint64_t *__restrict__ tz,
            const double2 *__restrict__ tc, double tol, int force_diag,
            int32_t *__restrict__ counts, int32_t *__restrict__ onecol)
{
    const int64_t r = blockIdx.x;
    const int lane = threadIdx.x;
    if (r >= dim)
        return;
    const int64_t G = *n_groups;
    int64_t cnt = 0;
    int64_t last_col = -1;
    for (int64_t g0 = 0; g0 < G; g0 += 64) {
        int64_t g = g0 + lane;
        bool keep = false;
        int64_t col = -1;
        if (g < G) {
            double2 v = group_entry(g, (uint64_t)r, gx, gstart, tz, tc);
            col = (int64_t)((uint64_t)r ^ gx[g]);
            keep = keep_entry(v, tol, force_diag && col == r);
        }
        uint64_t m = __ballot(keep);
        if (m) {
            // column of the highest kept lane (used only when the row has one entry)
            int hi = 63 - __clzll(m);
            int64_t c = __shfl(col, hi, 64);
            last_col = c;
        }
        cnt += __popcll(m);
    }
    if (lane == 0) {
        counts[r] = (int32_t)(cnt > 0x7fffffff ? 0x7fffffff : cnt);
        onecol[r] = cnt == 1 ? (int32_t)last_col : -1;
    }
}

// Multi-block exclusive scan of int32 counts into int64 (3 kernels).
__global__ void __launch_bounds__(1024)
k_scan_block(const int32_t *__restrict__ in, int64_t n, int64_t *__restrict__ out,
             int64_t *__restrict__ block_sums)
{
    __shared__ int64_t s[1024];
    const int tid = threadIdx.x;
    int64_t i = (int64_t)blockIdx.x * 1024 + tid;
    int64_t v = i < n ? (int64_t)in[i] : 0;
    s[tid] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        int64_t t = tid >= o ? s[tid - o] : 0;
        __syncthreads();
        s[tid] += t;
        __syncthreads();
    }
    if (i < n)
        out[i] = s[tid] - v;   // exclusive within block
    if (tid == 1023)
        block_sums[blockIdx.x] = s[1023];
}

__global__ void __launch_bounds__(1024)
k_scan_sums(int64_t *__restrict__ sums, int64_t nb, int64_t *__restrict__ total)
{
    __shared__ int64_t s[1024];
    __shared__ int64_t carry;
    const int tid = threadIdx.x;
    if (tid == 0)
        carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nb; base += 1024) {
        int64_t i = base + tid;
        int64_t v = i < nb ? sums[i] : 0;
        s[tid] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            int64_t t = tid >= o ? s[tid - o] : 0;
            __syncthreads();
            s[tid] += t;
            __syncthreads();
        }
        if (i < nb)
            sums[i] = carry + s[tid] - v;
        __syncthreads();
        if (tid == 1023)
            carry += s[1023];
        __syncthreads();
    }
    if (tid == 0)
        *total = carry;
}

// rowptr[i] = exclusive prefix (int32, valid when the total fits), rowptr[n] = total.
__global__ void k_scan_finish(const int64_t *__restrict__ part, const int64_t *__restrict__ sums,
                              int64_t n, const int64_t *__restrict__ total,
                              int32_t *__restrict__ rowptr)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        int64_t v = part[i] + sums[i / 1024];
        rowptr[i] = (int32_t)(v > 0x7fffffff ? 0x7fffffff : v);
    } else if (i == n) {
        int64_t t = *total;
        rowptr[n] = (int32_t)(t > 0x7fffffff ? 0x7fffffff : t);
    }
}

// Pairing check: every row has <= 1 entry and col(col(r)) == r.  Also the
// longest row.  stats[0] += violations, stats[1] = max row length.
__global__ void k_pairing(int64_t dim, const int32_t *__restrict__ counts,
                          const int32_t *__restrict__ onecol, unsigned long long *__restrict__ stats)
{
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false;
    int32_t len = 0;
    if (r < dim) {
        len = counts[r];
        if (len > 1)
            bad = true;
        else if (len == 1) {
            int32_t c = onecol[r];
            bad = (c < 0 || c >= dim || onecol[c] != (int32_t)r);
        }
    }
    uint64_t m = __ballot(bad);
    // wave-level max of the row length
    int32_t mx = len;
    for (int o = 32; o > 0; o >>= 1)
        mx = max(mx, __shfl_xor(mx, o, 64));
    if ((threadIdx.x & 63) == 0) {
        if (m)
            atomicAdd(&stats[0], (unsigned long long)__popcll(m));
        atomicMax(&stats[1], (unsigned long long)mx);
    }
}

// Phase 2: recompute each row's kept entries, sort by column in LDS, write.
template <int DT>
__global__ void __launch_bounds__(64)
k_row_fill(int64_t dim, const uint64_t *__restrict__ gx, const int64_t *__restrict__ gstart,
           const int64_t *__restrict__ n_groups, const uint64_t *__restrict__ tz,
           const double2 *__restrict__ tc, double tol, double shift, int force_diag, int pad,
           const int32_t *__restrict__ rowptr, int32_t *__restrict__ col_out,
           void *__restrict__ val_out)
{
    extern __shared__ unsigned char smem[];
    int32_t *s_col = reinterpret_cast<int32_t *>(smem);
    double2 *s_val = reinterpret_cast<double2 *>(smem + vqe_align((size_t)pad * 4));
    const int64_t r = blockIdx.x;
    const int lane = threadIdx.x;
    if (r >= dim)
        return;
    const int64_t G = *n_groups;
    int base = 0;
    for (int64_t g0 = 0; g0 < G; g0 += 64) {
        int64_t g = g0 + lane;
        bool keep = false;
        double2 v = make_double2(0.0, 0.0);
        int32_t col = 0;
        if (g < G) {
            v = group_entry(g, (uint64_t)r, gx, gstart, tz, tc);
            col = (int32_t)((uint64_t)r ^ gx[g]);
            keep = keep_entry(v, tol, force_diag && col == r);
        }
        uint64_t m = __ballot(keep);
        if (keep) {
            int pos = base + __popcll(m & ((1ull << lane) - 1ull));
            if (pos < pad) {
                s_col[pos] = col;
                s_val[pos] = v;
            }
        }
        base += __popcll(m);
    }
    // the kept count equals the sizing pass (same ordered sums); clamp anyway
    // so a row can never write past its own slot range
    const int64_t o = rowptr[r];
    const int64_t room = (int64_t)rowptr[r + 1] - o;
    int n = base < pad ? base : pad;
    if (n > room)
        n = (int)(room > 0 ? room : 0);
    for (int i = n + lane; i < pad; i += 64) {
        s_col[i] = 0x7fffffff;
        s_val[i] = make_double2(0.0, 0.0);
    }
    __syncthreads();
    for (int k = 2; k <= pad; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = lane; i < pad; i += 64) {
                int l = i ^ j;
                if (l > i) {
                    int32_t ci = s_col[i], cl = s_col[l];
                    bool ascending = (i & k) == 0;
                    if ((ci > cl) == ascending) {
                        double2 vi = s_val[i];
                        s_col[i] = cl;
                        s_col[l] = ci;
                        s_val[i] = s_val[l];
                        s_val[l] = vi;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = lane; i < n; i += 64) {
        double2 v = s_val[i];
        int32_t c = s_col[i];
        if (c == (int32_t)r)
            v.x = v.x - shift;
        col_out[o + i] = c;
        Elem<DT>::st(val_out, o + i, v);
    }
}

__global__ void k_row_max(int64_t dim, const int32_t *__restrict__ rowptr,
                          unsigned long long *__restrict__ mx)
{
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t len = r < dim ? rowptr[r + 1] - rowptr[r] : 0;
    for (int o = 32; o > 0; o >>= 1)
        len = max(len, __shfl_xor(len, o, 64));
    if ((threadIdx.x & 63) == 0)
        atomicMax(mx, (unsigned long long)len);
}

inline int64_t next_pow2(int64_t v)
{
    int64_t p = 1;
    while (p < v)
        p <<= 1;
    return p;
}

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

}  // namespace

// ------------------------------------------------------------------ host side
extern "C" int csr_build_from_pauli(vqe_ctx *ctx, int32_t n_qubits, int64_t n_terms,
                                    const uint64_t *xmask, const uint64_t *zmask,
                                    const double *coeff, double drop_tol, int32_t dtype,
                                    double diag_shift, vqe_csr *inout, int64_t *nnz_out)
{
    if (!ctx || !inout)
        return vqe_fail(ctx, VQE_EINVAL, "csr_build_from_pauli: null context or descriptor");
    if (n_qubits < 1 || n_qubits > 30)
        return vqe_fail(ctx, VQE_EINVAL, "csr_build_from_pauli: n_qubits %d outside [1, 30]",
                        n_qubits);
    if (n_terms < 0 || (n_terms > 0 && (!xmask || !zmask || !coeff)))
        return vqe_fail(ctx, VQE_EINVAL, "csr_build_from_pauli: bad term arrays");
    if (n_terms >= ((int64_t)1 << 31))
        return vqe_fail(ctx, VQE_ESIZE, "csr_build_from_pauli: too many terms");
    if (dtype != VQE_C128 && dtype != VQE_C64)
        return vqe_fail(ctx, VQE_EINVAL, "csr_build_from_pauli: unknown dtype %d", dtype);
    if (!std::isfinite(drop_tol) || drop_tol < 0 || !std::isfinite(diag_shift))
        return vqe_fail(ctx, VQE_EINVAL, "csr_build_from_pauli: bad drop_tol or diag_shift");
    if (dtype == VQE_C128 && diag_shift != 0.0)
        return vqe_fail(ctx, VQE_EINVAL, "csr_build_from_pauli: diag_shift needs VQE_C64");
    if (!inout->rowptr)
        return vqe_fail(ctx, VQE_EINVAL, "csr_build_from_pauli: rowptr is null");
    const bool fill = inout->col != nullptr || inout->val != nullptr;
    if (fill && (!inout->col || !inout->val))
        return vqe_fail(ctx, VQE_EINVAL, "csr_build_from_pauli: col and val must both be set");
    const uint64_t lim = ~(uint64_t)0 << n_qubits;
    for (int64_t t = 0; t < n_terms; t++)
        if ((xmask[t] | zmask[t]) & lim)
            return vqe_fail(ctx, VQE_EINVAL,
                            "csr_build_from_pauli: term %lld has a mask bit >= n_qubits",
                            (long long)t);
    for (int64_t t = 0; t < 2 * n_terms; t++)
        if (!std::isfinite(coeff[t]))
            return vqe_fail(ctx, VQE_EINVAL, "csr_build_from_pauli: non-finite coefficient");

    const int64_t dim = (int64_t)1 << n_qubits;
    const bool force_diag = diag_shift != 0.0;
    // With a shift every row needs its diagonal entry: an extra zero identity
    // term (last, so the order of the given terms is unchanged) makes sure the
    // x = 0 group exists.
    std::vector<uint64_t> hx(xmask, xmask + n_terms), hz(zmask, zmask + n_terms);
    std::vector<double> hc(coeff, coeff + 2 * n_terms);
    if (force_diag) {
        hx.push_back(0);
        hz.push_back(0);
        hc.push_back(0.0);
        hc.push_back(0.0);
    }
    const int64_t T = (int64_t)hx.size();
    const int64_t P = next_pow2(std::max<int64_t>(T, 1));
    const int64_t nb = (dim + 1023) / 1024;

    // workspace layout
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += vqe_align(bytes); return o; };
    const size_t o_x = take(T * 8 + 8), o_z = take(T * 8 + 8), o_c = take(T * 16 + 16);
    const size_t o_keys = take(P * 8), o_gx = take(T * 8 + 8), o_gs = take((T + 1) * 8);
    const size_t o_tz = take(T * 8 + 8), o_tc = take(T * 16 + 16), o_ng = take(8);
    const size_t o_cnt = take(dim * 4), o_one = take(dim * 4), o_part = take(dim * 8);
    const size_t o_bs = take(nb * 8 + 8), o_tot = take(8), o_stats = take(16);
    int rc = vqe_ws_reserve(ctx, off);
    if (rc)
        return rc;
    char *ws = (char *)ctx->ws;
    uint64_t *d_x = (uint64_t *)(ws + o_x), *d_z = (uint64_t *)(ws + o_z);
    double2 *d_c = (double2 *)(ws + o_c);
    uint64_t *d_keys = (uint64_t *)(ws + o_keys), *d_gx = (uint64_t *)(ws + o_gx);
    int64_t *d_gs = (int64_t *)(ws + o_gs), *d_ng = (int64_t *)(ws + o_ng);
    uint64_t *d_tz = (uint64_t *)(ws + o_tz);
    double2 *d_tc = (double2 *)(ws + o_tc);
    int32_t *d_cnt = (int32_t *)(ws + o_cnt), *d_one = (int32_t *)(ws + o_one);
    int64_t *d_part = (int64_t *)(ws + o_part), *d_bs = (int64_t *)(ws + o_bs);
    int64_t *d_tot = (int64_t *)(ws + o_tot);
    unsigned long long *d_stats = (unsigned long long *)(ws + o_stats);
    hipStream_t s = ctx->stream;

    if (T > 0) {
        VQE_HIP(ctx, hipMemcpyAsync(d_x, hx.data(), T * 8, hipMemcpyHostToDevice, s));
        VQE_HIP(ctx, hipMemcpyAsync(d_z, hz.data(), T * 8, hipMemcpyHostToDevice, s));
        VQE_HIP(ctx, hipMemcpyAsync(d_c, hc.data(), T * 16, hipMemcpyHostToDevice, s));
    }
    k_make_keys<<<grid_for(P, 256), 256, 0, s>>>(d_x, T, P, d_keys);
    for (int64_t k = 2; k <= P; k <<= 1)
        for (int64_t j = k >> 1; j > 0; j >>= 1)
            k_bitonic_step<<<grid_for(P, 256), 256, 0, s>>>(d_keys, j, k, P);
    k_group<<<1, 1024, 0, s>>>(d_keys, T, d_z, d_c, d_gx, d_gs, d_ng, d_tz, d_tc);
    VQE_LAUNCH_CHECK(ctx);

    if (!fill) {
        k_row_count<<<(unsigned)dim, 64, 0, s>>>(dim, d_gx, d_gs, d_ng, d_tz, d_tc, drop_tol,
                                                 force_diag ? 1 : 0, d_cnt, d_one);
        k_scan_block<<<(unsigned)nb, 1024, 0, s>>>(d_cnt, dim, d_part, d_bs);
        k_scan_sums<<<1, 1024, 0, s>>>(d_bs, nb, d_tot);
        k_scan_finish<<<grid_for(dim + 1, 256), 256, 0, s>>>(d_part, d_bs, dim, d_tot,
                                                               inout->rowptr);
        VQE_HIP(ctx, hipMemsetAsync(d_stats, 0, 16, s));
        k_pairing<<<grid_for(dim, 256), 256, 0, s>>>(dim, d_cnt, d_one, d_stats);
        VQE_LAUNCH_CHECK(ctx);
        int64_t *h = ctx->host_scalars;
        VQE_HIP(ctx, hipMemcpyAsync(h, d_tot, 8, hipMemcpyDeviceToHost, s));
        VQE_HIP(ctx, hipMemcpyAsync(h + 1, d_stats, 16, hipMemcpyDeviceToHost, s));
        VQE_HIP(ctx, hipStreamSynchronize(s));
        const int64_t nnz = h[0];
        const int64_t violations = h[1], maxrow = h[2];
        if (nnz > 0x7fffffff)
            return vqe_fail(ctx, VQE_ESIZE, "csr_build_from_pauli: nnz %lld exceeds INT32_MAX",
                            (long long)nnz);
        if (maxrow > kMaxRow)
            return vqe_fail(ctx, VQE_ESIZE,
                            "csr_build_from_pauli: a row holds %lld entries (max %d)",
                            (long long)maxrow, kMaxRow);
        inout->n_qubits = n_qubits;
        inout->dtype = dtype;
        inout->dim = dim;
        inout->nnz = nnz;
        inout->diag_shift = diag_shift;
        // every entry is real when every term's c_t i^{|x_t & z_t|} is real
        bool real = true;
        for (int64_t t = 0; t < T && real; t++) {
            const int k = __builtin_popcountll(hx[t] & hz[t]) & 3;
            real = (k & 1) ? hc[2 * t] == 0.0 : hc[2 * t + 1] == 0.0;
        }
        inout->flags = (violations == 0 ? VQE_PAIRING : 0u) | (real ? VQE_REAL : 0u);
        if (nnz_out)
            *nnz_out = nnz;
        return VQE_OK;
    }

    // phase 2
    if (inout->dim != dim || inout->dtype != dtype || inout->n_qubits != n_qubits)
        return vqe_fail(ctx, VQE_EINVAL,
                        "csr_build_from_pauli: descriptor does not match the sizing call");
    VQE_HIP(ctx, hipMemsetAsync(d_stats, 0, 16, s));
    k_row_max<<<grid_for(dim, 256), 256, 0, s>>>(dim, inout->rowptr, d_stats);
    VQE_LAUNCH_CHECK(ctx);
    int64_t *h = ctx->host_scalars;
    VQE_HIP(ctx, hipMemcpyAsync(h, d_stats, 8, hipMemcpyDeviceToHost, s));
    VQE_HIP(ctx, hipStreamSynchronize(s));
    const int64_t maxrow = h[0];
    if (maxrow > kMaxRow)
        return vqe_fail(ctx, VQE_ESIZE, "csr_build_from_pauli: row too long");
    const int pad = (int)std::max<int64_t>(next_pow2(std::max<int64_t>(maxrow, 1)), 64);
    const size_t lds = vqe_align((size_t)pad * 4) + (size_t)pad * 16;
    if (dtype == VQE_C128)
        k_row_fill<VQE_C128><<<(unsigned)dim, 64, lds, s>>>(
            dim, d_gx, d_gs, d_ng, d_tz, d_tc, drop_tol, diag_shift, force_diag ? 1 : 0, pad,
            inout->rowptr, inout->col, inout->val);
    else
        k_row_fill<VQE_C64><<<(unsigned)dim, 64, lds, s>>>(
            dim, d_gx, d_gs, d_ng, d_tz, d_tc, drop_tol, diag_shift, force_diag ? 1 : 0, pad,
            inout->rowptr, inout->col, inout->val);
    VQE_LAUNCH_CHECK(ctx);
    if (nnz_out)
        *nnz_out = inout->nnz;
    return VQE_OK;
}
