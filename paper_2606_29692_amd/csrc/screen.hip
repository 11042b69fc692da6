// Batched pool-gradient screen (Eq. 5) over a pair table staged per state in LDS.
//
// A pairing generator couples row r with c = col(r) (col(c) = r), so
//   g_j = 2 Re sum over pairs {r <= c} [conj(sigma_r) A[r,c] psi_c + conj(sigma_c) A[c,r] psi_r]
// with sigma = H psi (the stored product plus the diagonal shift times psi,
// added back in FP64).  At plan creation the pool's CSR is re-laid out once
// into a pair table: per generator, its pairs {r, c, A[r,c], A[c,r]} sorted by
// the lower row r and split by row tile.  A row tile is the largest power of
// two of rows whose psi and sigma fit in 128 KiB of LDS (8192 rows for FP32
// storage).  A workgroup takes one state, one tile and a range of generators:
// it stages psi and sigma of its tile in LDS and walks the pairs of its
// generators whose lower row lies in the tile; partner rows in the same tile
// come from LDS, others from global memory.  Every state reads each pair once
// and psi/sigma once per workgroup instead of once per generator.
// Sums are FP64: per generator and tile, one wave (lane-strided partial sums,
// then a butterfly), then tiles in ascending order.
#include "kernels.hpp"
#include "step_fin.hpp"

#include <algorithm>
#include <vector>

namespace {

// Owner rows (rows r with one entry and col(r) >= r) per (generator, tile).
__global__ void __launch_bounds__(256)
k_pair_count(const vqe_csr *__restrict__ ops, int32_t nt, int32_t tile_rows,
             int32_t *__restrict__ counts)
{
    const int j = blockIdx.x / nt, t = blockIdx.x % nt;
    const vqe_csr op = ops[j];
    const int64_t r0 = (int64_t)t * tile_rows;
    int n = 0;
    for (int64_t r = r0 + threadIdx.x; r < r0 + tile_rows; r += 256) {
        const int k0 = op.rowptr[r];
        if (op.rowptr[r + 1] - k0 == 1 && (int64_t)op.col[k0] >= r)
            n++;
    }
    __shared__ int s[4];
    for (int o = 32; o > 0; o >>= 1)
        n += __shfl_xor(n, o, 64);
    if ((threadIdx.x & 63) == 0)
        s[threadIdx.x >> 6] = n;
    __syncthreads();
    if (threadIdx.x == 0)
        counts[blockIdx.x] = s[0] + s[1] + s[2] + s[3];
}

// Ordered compaction of the owner rows of (generator, tile) into the table.
template <int DT>
__global__ void __launch_bounds__(256)
k_pair_fill(const vqe_csr *__restrict__ ops, int32_t nt, int32_t tile_rows,
            const int32_t *__restrict__ pts, int32_t *__restrict__ pr, int32_t *__restrict__ pc,
            void *__restrict__ pa, void *__restrict__ pb)
{
    const int j = blockIdx.x / nt, t = blockIdx.x % nt;
    const vqe_csr op = ops[j];
    const int64_t r0 = (int64_t)t * tile_rows;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __shared__ int s_w[4];
    int carry = pts[blockIdx.x];
    for (int64_t base = r0; base < r0 + tile_rows; base += 256) {
        const int64_t r = base + threadIdx.x;
        bool own = false;
        int k0 = 0;
        if (r < r0 + tile_rows) {
            k0 = op.rowptr[r];
            own = op.rowptr[r + 1] - k0 == 1 && (int64_t)op.col[k0] >= r;
        }
        const uint64_t m = __ballot(own);
        if (lane == 0)
            s_w[wid] = __popcll(m);
        __syncthreads();
        int off = carry;
        for (int w = 0; w < wid; w++)
            off += s_w[w];
        if (own) {
            const int i = off + __popcll(m & ((1ull << lane) - 1ull));
            const int32_t c = op.col[k0];
            pr[i] = (int32_t)r;
            pc[i] = c;
            Elem<DT>::st(pa, i, Elem<DT>::ld(op.val, k0));
            Elem<DT>::st(pb, i, c == (int32_t)r ? make_double2(0.0, 0.0)
                                                : Elem<DT>::ld(op.val, op.rowptr[c]));
        }
        carry += s_w[0] + s_w[1] + s_w[2] + s_w[3];
        __syncthreads();
    }
}

// A generator qualifies for the compact table when every pair has the same
// flip mask x = r ^ c (x != 0) and real entries of exactly +1 or -1 (true of
// every fermionic excitation under JW and BK).  bad[j] counts violations.
template <int DT>
__global__ void __launch_bounds__(256)
k_pair_check(int32_t nt, const int32_t *__restrict__ pts, const int32_t *__restrict__ pr,
             const int32_t *__restrict__ pc, const void *__restrict__ pa,
             const void *__restrict__ pb, int32_t *__restrict__ xmask, int32_t *__restrict__ bad)
{
    const int j = blockIdx.x;
    const int p0 = pts[j * nt], p1 = pts[(j + 1) * nt];
    const int32_t x = p1 > p0 ? (pr[p0] ^ pc[p0]) : 0;
    int n = 0;
    for (int p = p0 + threadIdx.x; p < p1; p += 256) {
        const double2 a = Elem<DT>::ld(pa, p), b = Elem<DT>::ld(pb, p);
        const bool ok = (pr[p] ^ pc[p]) == x && x != 0 && a.y == 0.0 && b.y == 0.0 &&
                        (a.x == 1.0 || a.x == -1.0) && (b.x == 1.0 || b.x == -1.0);
        n += ok ? 0 : 1;
    }
    for (int o = 32; o > 0; o >>= 1)
        n += __shfl_xor(n, o, 64);
    __shared__ int s[4];
    if ((threadIdx.x & 63) == 0)
        s[threadIdx.x >> 6] = n;
    __syncthreads();
    if (threadIdx.x == 0) {
        bad[j] = s[0] + s[1] + s[2] + s[3];
        xmask[j] = x;
    }
}

// word = r | (A[r,c] < 0) << 30 | (A[c,r] < 0) << 31
template <int DT>
__global__ void k_pair_compact(int64_t total, const int32_t *__restrict__ pr,
                               const void *__restrict__ pa, const void *__restrict__ pb,
                               uint32_t *__restrict__ words)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= total)
        return;
    const double a = Elem<DT>::ld(pa, p).x, b = Elem<DT>::ld(pb, p).x;
    words[p] = (uint32_t)pr[p] | (a < 0.0 ? (1u << 30) : 0u) | (b < 0.0 ? (1u << 31) : 0u);
}

template <int DT>
__global__ void __launch_bounds__(1024)
k_screen(const ScreenState *__restrict__ states, const PairTable *__restrict__ tables,
         const int4 *__restrict__ tasks)
{
    const int4 task = tasks[blockIdx.x];
    if (task.x < 0)
        return;
    const ScreenState st = states[task.x];
    if (VQE_SKIP(st))
        return;
    const PairTable tb = tables[st.table];
    const int t = task.y;
    // this workgroup's generators: order[range], order[range + n_ranges], ...
    // (order = descending pair count)
    const int range = task.z, n_ranges = task.w;
    const int n_mine = (tb.M - range + n_ranges - 1) / n_ranges;
    using T = typename Elem<DT>::T;
    extern __shared__ unsigned char smem[];
    const int64_t rows = (int64_t)tb.tile_rows < st.dim ? tb.tile_rows : st.dim;
    T *s_psi = reinterpret_cast<T *>(smem);
    T *s_sig = s_psi + rows;
    const int64_t base = (int64_t)t * tb.tile_rows;
    const T *psi = reinterpret_cast<const T *>(st.psi);
    const T *sig = reinterpret_cast<const T *>(st.sigma);
    // each thread issues the loads of SU rows before its LDS writes
    constexpr int SU = 8;
    for (int64_t i0 = threadIdx.x; i0 < rows; i0 += 1024 * SU) {
        T a[SU], b[SU];
#pragma unroll
        for (int u = 0; u < SU; u++)
            if (i0 + 1024 * u < rows) {
                a[u] = ldg(psi, base + i0 + 1024 * u);
                b[u] = ldg(sig, base + i0 + 1024 * u);
            }
#pragma unroll
        for (int u = 0; u < SU; u++)
            if (i0 + 1024 * u < rows) {
                s_psi[i0 + 1024 * u] = a[u];
                s_sig[i0 + 1024 * u] = b[u];
            }
    }
    __syncthreads();
    const double shift = st.shift;
    const T *pa = reinterpret_cast<const T *>(tb.pa);
    const T *pb = reinterpret_cast<const T *>(tb.pb);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    // one wave per generator (waves are independent: no barriers), four
    // pairs in flight per lane
    constexpr int U = 4;
    // wave w takes entries w, w + 16, ... of this workgroup's list, which is
    // ordered by descending pair count
    int widx = wid;
    auto next_op = [&]() -> int {
        const int idx = widx;
        widx += 16;
        return idx < n_mine ? gmem(tb.order)[range + idx * n_ranges] : -1;
    };
    if (tb.words) {
        for (int j = next_op(); j >= 0; j = next_op()) {
            const int p0 = gmem(tb.pts)[j * tb.nt + t], p1 = gmem(tb.pts)[j * tb.nt + t + 1];
            const int64_t x = gmem(tb.xmask)[j];
            double acc = 0.0;
            for (int pbase = p0 + lane; pbase < p1; pbase += U * 64) {
                uint32_t w[U];
#pragma unroll
                for (int u = 0; u < U; u++) {
                    const int p = pbase + u * 64;
                    w[u] = p < p1 ? gmem(tb.words)[p] : 0xffffffffu;
                }
#pragma unroll
                for (int u = 0; u < U; u++) {
                    if (pbase + u * 64 >= p1)
                        continue;
                    const int64_t r = w[u] & 0x3fffffffu;
                    const int64_t c = r ^ x;
                    const T pr_ = s_psi[r - base], qr_ = s_sig[r - base];
                    T pc_, qc_;
                    if (c >= base && c - base < rows) {
                        pc_ = s_psi[c - base];
                        qc_ = s_sig[c - base];
                    } else {
                        pc_ = ldg(psi, c);
                        qc_ = ldg(sig, c);
                    }
                    const double prx = pr_.x, pry = pr_.y, pcx = pc_.x, pcy = pc_.y;
                    const double srx = (double)qr_.x + shift * prx, sry = (double)qr_.y + shift * pry;
                    const double scx = (double)qc_.x + shift * pcx, scy = (double)qc_.y + shift * pcy;
                    const double t1 = srx * pcx + sry * pcy;   // Re conj(sigma_r) psi_c
                    const double t2 = scx * prx + scy * pry;   // Re conj(sigma_c) psi_r
                    acc += ((w[u] >> 30) & 1u ? -t1 : t1) + (w[u] >> 31 ? -t2 : t2);
                }
            }
            acc = wave_sum(acc);
            if (lane == 0)
                gmem(st.partials)[(int64_t)j * tb.nt + t] = acc;
        }
        return;
    }
    for (int j = next_op(); j >= 0; j = next_op()) {
        const int p0 = gmem(tb.pts)[j * tb.nt + t], p1 = gmem(tb.pts)[j * tb.nt + t + 1];
        double acc = 0.0;
        for (int pbase = p0 + lane; pbase < p1; pbase += U * 64) {
            int64_t r[U], c[U];
            T av[U], bv[U];
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int p = pbase + u * 64;
                if (p < p1) {
                    r[u] = gmem(tb.pr)[p];
                    c[u] = gmem(tb.pc)[p];
                    av[u] = ldg(pa, p);
                    bv[u] = ldg(pb, p);
                } else {
                    r[u] = -1;
                }
            }
#pragma unroll
            for (int u = 0; u < U; u++) {
                if (r[u] < 0)
                    continue;
                const T pr_ = s_psi[r[u] - base], qr_ = s_sig[r[u] - base];
                T pc_, qc_;
                if (c[u] >= base && c[u] - base < rows) {
                    pc_ = s_psi[c[u] - base];
                    qc_ = s_sig[c[u] - base];
                } else {
                    pc_ = ldg(psi, c[u]);
                    qc_ = ldg(sig, c[u]);
                }
                const double prx = pr_.x, pry = pr_.y, pcx = pc_.x, pcy = pc_.y;
                const double srx = (double)qr_.x + shift * prx, sry = (double)qr_.y + shift * pry;
                const double scx = (double)qc_.x + shift * pcx, scy = (double)qc_.y + shift * pcy;
                const double ax = av[u].x, ay = av[u].y, bx = bv[u].x, by = bv[u].y;
                const double wr = ax * pcx - ay * pcy, wi = ax * pcy + ay * pcx;
                const double ur = bx * prx - by * pry, ui = bx * pry + by * prx;
                acc += (srx * wr + sry * wi) + (scx * ur + scy * ui);
            }
        }
        acc = wave_sum(acc);
        if (lane == 0)
            gmem(st.partials)[(int64_t)j * tb.nt + t] = acc;
    }
}

// One workgroup per state.
__global__ void __launch_bounds__(256)
k_step_fin(const SpmvState *__restrict__ spmv, const ScreenState *__restrict__ screen,
           const PairTable *__restrict__ tables, const SelectState *__restrict__ sel,
           int do_grad, int do_select, double rel_tie)
{
    const int s = blockIdx.x;
    const SpmvState hs = spmv[s];
    if (VQE_SKIP(hs))
        return;
    (void)step_fin_block(hs, screen, tables, sel[s], s, do_grad != 0, do_select != 0, rel_tie, true);
}

}  // namespace

int32_t screen_tile_rows(int64_t dim, int dtype)
{
    int64_t rows = (int64_t)SCREEN_LDS_BYTES / (2 * (int64_t)vqe_elem_bytes(dtype));
    int64_t p = 1;
    while (p * 2 <= rows)
        p *= 2;
    return (int32_t)(p < dim ? p : dim);
}

// Build the pair table of one pool (setup; synchronises the stream).  mem_out
// receives two allocations (the full table, and the compact one or null).
int pair_table_build(vqe_ctx *ctx, const vqe_pool *pool, int64_t dim, PairTable *tb,
                     void **mem_out, size_t *bytes_out)
{
    hipStream_t s = ctx->stream;
    const int M = pool->M;
    const int32_t tile = screen_tile_rows(dim, pool->dtype);
    const int32_t nt = (int32_t)((dim + tile - 1) / tile);
    const size_t n_cnt = (size_t)M * nt;
    int32_t *d_cnt = nullptr;
    VQE_HIP(ctx, hipMalloc((void **)&d_cnt, (n_cnt + 1) * sizeof(int32_t)));
    k_pair_count<<<(unsigned)n_cnt, 256, 0, s>>>(pool->ops, nt, tile, d_cnt);
    std::vector<int32_t> cnt(n_cnt);
    hipError_t e = hipMemcpyAsync(cnt.data(), d_cnt, n_cnt * sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipFree(d_cnt);
        return vqe_fail(ctx, VQE_EHIP, "pair table count: %s", hipGetErrorString(e));
    }
    std::vector<int32_t> pts(n_cnt + 1, 0);
    int64_t total = 0;
    for (size_t i = 0; i < n_cnt; i++) {
        pts[i] = (int32_t)total;
        total += cnt[i];
    }
    if (total > 0x7fffffff) {
        (void)hipFree(d_cnt);
        return vqe_fail(ctx, VQE_ESIZE, "pair table too large");
    }
    pts[n_cnt] = (int32_t)total;
    // generators by descending pair count (ties by index), for load balance
    std::vector<int32_t> order(M);
    std::vector<int64_t> per_op(M, 0);
    for (int j = 0; j < M; j++) {
        order[j] = j;
        for (int t = 0; t < nt; t++)
            per_op[j] += cnt[(size_t)j * nt + t];
    }
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return per_op[a] > per_op[b]; });
    const size_t eb = vqe_elem_bytes(pool->dtype);
    const size_t o_ord = vqe_align((n_cnt + 1) * 4);
    const size_t o_pts = 0, o_pr = o_ord + vqe_align((size_t)M * 4), o_pc = o_pr + vqe_align(total * 4 + 4);
    const size_t o_pa = o_pc + vqe_align(total * 4 + 4), o_pb = o_pa + vqe_align(total * eb + eb);
    const size_t bytes = o_pb + vqe_align(total * eb + eb);
    char *mem = nullptr;
    e = hipMalloc((void **)&mem, bytes);
    if (e != hipSuccess) {
        (void)hipFree(d_cnt);
        (void)hipGetLastError();
        return vqe_fail(ctx, VQE_ENOMEM, "pair table allocation failed");
    }
    e = hipMemcpyAsync(mem + o_pts, pts.data(), pts.size() * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && M > 0)
        e = hipMemcpyAsync(mem + o_ord, order.data(), (size_t)M * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        if (pool->dtype == VQE_C128)
            k_pair_fill<VQE_C128><<<(unsigned)n_cnt, 256, 0, s>>>(
                pool->ops, nt, tile, (const int32_t *)(mem + o_pts), (int32_t *)(mem + o_pr),
                (int32_t *)(mem + o_pc), mem + o_pa, mem + o_pb);
        else
            k_pair_fill<VQE_C64><<<(unsigned)n_cnt, 256, 0, s>>>(
                pool->ops, nt, tile, (const int32_t *)(mem + o_pts), (int32_t *)(mem + o_pr),
                (int32_t *)(mem + o_pc), mem + o_pa, mem + o_pb);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    (void)hipFree(d_cnt);
    if (e != hipSuccess) {
        (void)hipFree(mem);
        return vqe_fail(ctx, VQE_EHIP, "pair table fill: %s", hipGetErrorString(e));
    }
    // compact form when every generator qualifies
    int32_t *d_x = nullptr;
    uint32_t *d_words = nullptr;
    bool compact = false;
    if (M > 0 && total > 0) {
        int32_t *d_chk = nullptr;
        e = hipMalloc((void **)&d_chk, 2 * (size_t)M * sizeof(int32_t));
        if (e != hipSuccess) {
            (void)hipFree(mem);
            (void)hipGetLastError();
            return vqe_fail(ctx, VQE_ENOMEM, "pair table check allocation failed");
        }
        if (pool->dtype == VQE_C128)
            k_pair_check<VQE_C128><<<(unsigned)M, 256, 0, s>>>(
                nt, (const int32_t *)(mem + o_pts), (const int32_t *)(mem + o_pr),
                (const int32_t *)(mem + o_pc), mem + o_pa, mem + o_pb, d_chk, d_chk + M);
        else
            k_pair_check<VQE_C64><<<(unsigned)M, 256, 0, s>>>(
                nt, (const int32_t *)(mem + o_pts), (const int32_t *)(mem + o_pr),
                (const int32_t *)(mem + o_pc), mem + o_pa, mem + o_pb, d_chk, d_chk + M);
        std::vector<int32_t> chk(2 * (size_t)M);
        e = hipMemcpyAsync(chk.data(), d_chk, chk.size() * 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipStreamSynchronize(s);
        if (e == hipSuccess) {
            compact = true;
            for (int j = 0; j < M; j++)
                compact = compact && chk[M + j] == 0;
        }
        if (compact) {
            // the compact words and masks get an allocation of their own
            e = hipMalloc((void **)&d_words, (size_t)total * 4 + (size_t)M * 4 + 256);
            if (e == hipSuccess) {
                d_x = (int32_t *)((char *)d_words + vqe_align((size_t)total * 4));
                e = hipMemcpyAsync(d_x, d_chk, (size_t)M * 4, hipMemcpyDeviceToDevice, s);
            }
            if (e == hipSuccess) {
                const unsigned g = (unsigned)((total + 255) / 256);
                if (pool->dtype == VQE_C128)
                    k_pair_compact<VQE_C128><<<g, 256, 0, s>>>(total, (const int32_t *)(mem + o_pr),
                                                                mem + o_pa, mem + o_pb, d_words);
                else
                    k_pair_compact<VQE_C64><<<g, 256, 0, s>>>(total, (const int32_t *)(mem + o_pr),
                                                               mem + o_pa, mem + o_pb, d_words);
                e = hipGetLastError();
            }
            if (e == hipSuccess)
                e = hipStreamSynchronize(s);
        }
        (void)hipFree(d_chk);
        if (e != hipSuccess) {
            if (d_words)
                (void)hipFree(d_words);
            (void)hipFree(mem);
            return vqe_fail(ctx, VQE_EHIP, "pair table compaction: %s", hipGetErrorString(e));
        }
    }
    tb->pts = (const int32_t *)(mem + o_pts);
    tb->order = (const int32_t *)(mem + o_ord);
    tb->pr = (const int32_t *)(mem + o_pr);
    tb->pc = (const int32_t *)(mem + o_pc);
    tb->pa = mem + o_pa;
    tb->pb = mem + o_pb;
    tb->M = M;
    tb->nt = nt;
    tb->tile_rows = tile;
    tb->words = compact ? d_words : nullptr;
    tb->xmask = compact ? d_x : nullptr;
    mem_out[0] = mem;
    mem_out[1] = compact ? (void *)d_words : nullptr;
    *bytes_out = bytes + (compact ? (size_t)total * 4 + (size_t)M * 4 : 0);
    return VQE_OK;
}

void launch_step_fin(const SpmvState *spmv, const ScreenState *screen, const PairTable *tables,
                     const SelectState *sel, unsigned n_states, bool grad, bool select,
                     double rel_tie, hipStream_t s)
{
    k_step_fin<<<n_states, 256, 0, s>>>(spmv, screen, tables, sel, grad ? 1 : 0, select ? 1 : 0,
                                        rel_tie);
}

void launch_screen(int dtype, const ScreenState *states, const PairTable *tables,
                   const int4 *tasks, unsigned grid, unsigned n_states, size_t lds, hipStream_t s)
{
    if (dtype == VQE_C128) {
        (void)hipFuncSetAttribute((const void *)k_screen<VQE_C128>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        k_screen<VQE_C128><<<grid, 1024, lds, s>>>(states, tables, tasks);
    } else {
        (void)hipFuncSetAttribute((const void *)k_screen<VQE_C64>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        k_screen<VQE_C64><<<grid, 1024, lds, s>>>(states, tables, tasks);
    }
    (void)n_states;
}
