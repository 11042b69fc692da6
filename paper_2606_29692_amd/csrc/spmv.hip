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

#include <algorithm>

// The LDS schedules hold the state in LDS, so one 16-wave workgroup fills a
// CU (4 waves per SIMD): the register allocator may use the whole budget.
#define VQE_LDS_OCCUPANCY __attribute__((amdgpu_waves_per_eu(4, 4)))

namespace {

// V = entries per lane per pass.  V = 1: lane l of the sub-group takes
// entries k0 + l, k0 + l + L, ...  V = 4: lanes take aligned groups of four
// consecutive entries (one 16-byte index load and 32- or 64-byte value loads),
// masked to the row; a 64-lane sub-group covers 256 entries per pass.
template <int DT, int V> struct RowLoad;

template <int DT> struct RowLoad<DT, 1> {
    using T = typename Elem<DT>::T;
    static __device__ __forceinline__ void load(const int32_t *col, const T *val, int k, int k0,
                                                int k1, int64_t nnz, int c[1], T v[1])
    {
        (void)k0;
        (void)nnz;
        if (k < k1) {
            c[0] = __builtin_nontemporal_load(gmem(col) + k);
            v[0] = ldg(val, k);
        } else {
            c[0] = -1;
        }
    }
};

// Four consecutive values from a 32-byte (c64) or 64-byte (c128) aligned address.
__device__ __forceinline__ void load4(const float2 *p, float2 v[4])
{
    const vqe_v4f a = gmem(reinterpret_cast<const vqe_v4f *>(p))[0];
    const vqe_v4f b = gmem(reinterpret_cast<const vqe_v4f *>(p))[1];
    v[0] = make_float2(a.x, a.y);
    v[1] = make_float2(a.z, a.w);
    v[2] = make_float2(b.x, b.y);
    v[3] = make_float2(b.z, b.w);
}

__device__ __forceinline__ void load4(const double2 *p, double2 v[4])
{
#pragma unroll
    for (int u = 0; u < 4; u++)
        v[u] = ldg(p, u);
}

template <int DT> struct RowLoad<DT, 4> {
    using T = typename Elem<DT>::T;
    static __device__ __forceinline__ void load(const int32_t *col, const T *val, int k, int k0,
                                                int k1, int64_t nnz, int c[4], T v[4])
    {
        if (k >= k1) {
            // the whole group lies past the row: no load at all
#pragma unroll
            for (int u = 0; u < 4; u++)
                c[u] = -1;
            return;
        }
        if ((int64_t)k + 3 < nnz) {
            typedef int v4i __attribute__((ext_vector_type(4)));
            const v4i c4 = __builtin_nontemporal_load(gmem(reinterpret_cast<const v4i *>(col + k)));
            c[0] = c4.x;
            c[1] = c4.y;
            c[2] = c4.z;
            c[3] = c4.w;
            load4(val + k, v);
        } else {
#pragma unroll
            for (int u = 0; u < 4; u++) {
                if ((int64_t)(k + u) < nnz) {
                    c[u] = gmem(col)[k + u];
                    v[u] = ldg(val, k + u);
                } else {
                    c[u] = -1;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < 4; u++)
            if (k + u < k0 || k + u >= k1)
                c[u] = -1;
    }
};

template <int DT, int L, int V, bool BATCH>
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
        if (VQE_SKIP(st))
            return;
    } else {
        st = single;
        blk = blockIdx.x;
    }
    constexpr int G = VQE_WAVE / L;
    constexpr int RPB = spmv_rows_per_block(L);
    constexpr int U = V == 1 ? 4 : 1;     // passes issued together
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int sub = lane / L, sl = lane % L;
    const int32_t *__restrict__ rowptr = st.rowptr;
    const int32_t *__restrict__ col = st.col;
    using T = typename Elem<DT>::T;
    const T *__restrict__ val = reinterpret_cast<const T *>(st.val);
    double e_re = 0.0, e_im = 0.0, e_n2 = 0.0;
#pragma unroll
    for (int it = 0; it < SPMV_RPT; it++) {
        const int64_t r = (int64_t)blk * RPB + (it * 4 + wid) * G + sub;
        double are = 0.0, aim = 0.0;
        if (r < st.dim) {
            const int k0 = gmem(rowptr)[r], k1 = gmem(rowptr)[r + 1];
            const int first = V == 1 ? k0 + sl : (k0 & ~3) + 4 * sl;
            for (int k = first; k < k1; k += U * V * L) {
                int c[U * V];
                T v[U * V];
#pragma unroll
                for (int u = 0; u < U; u++)
                    RowLoad<DT, V>::load(col, val, k + u * V * L, k0, k1, st.nnz, c + u * V,
                                         v + u * V);
#pragma unroll
                for (int u = 0; u < U * V; u++) {
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
        gmem(st.partials)[(int64_t)blk * 3 + q] = v;
    }
}

// Loads of the LDS schedules: four consecutive entries from an aligned group
// k (16-byte index load, 32- or 64-byte value load).  Entries outside the
// row [k0, k1) get column zc, the index of a zero element kept after the
// state in LDS, so the multiply needs no per-entry select: their values are
// finite (entries of a neighbouring row, or zero) and multiply that zero.
// Only groups that reach past the end of the arrays (k + 4 > nnz) take the
// entry-by-entry path.  All index arithmetic is 32-bit (nnz < 2^31).
template <int DT>
__device__ __forceinline__ void lds_group_load(const int32_t *col, const typename Elem<DT>::T *val,
                                               int k, int k0, int k1, int nnz, int zc, int c[4],
                                               typename Elem<DT>::T v[4])
{
    using T = typename Elem<DT>::T;
    if (k >= k1) {
        // the whole group lies past the row: no load at all
#pragma unroll
        for (int u = 0; u < 4; u++) {
            c[u] = zc;
            v[u] = T{};
        }
        return;
    }
    if (k + 4 <= nnz) {
        typedef int v4i __attribute__((ext_vector_type(4)));
        const v4i c4 = __builtin_nontemporal_load(gmem(reinterpret_cast<const v4i *>(col + k)));
        c[0] = c4.x;
        c[1] = c4.y;
        c[2] = c4.z;
        c[3] = c4.w;
        load4(val + k, v);
    } else {
#pragma unroll
        for (int u = 0; u < 4; u++) {
            if (k + u < nnz) {
                c[u] = gmem(col)[k + u];
                v[u] = ldg(val, k + u);
            } else {
                c[u] = zc;
                v[u] = T{};
            }
        }
    }
    // entry k + u belongs to the row iff 0 <= k + u - k0 < k1 - k0
    const unsigned len = (unsigned)(k1 - k0);
#pragma unroll
    for (int u = 0; u < 4; u++)
        c[u] = (unsigned)(k + u - k0) < len ? c[u] : zc;
}

// Gathers from the LDS copy of the state and FP64 multiply-accumulate.  All
// LDS reads issue back to back behind a single wait; masked entries read the
// zero element.
__device__ __forceinline__ float2 stage_load(const float2 *p, int64_t i) { return ldg(p, i); }
__device__ __forceinline__ double2 stage_load(const double2 *p, int64_t i) { return ldg(p, i); }
__device__ __forceinline__ int32_t stage_load(const int32_t *p, int64_t i) { return gmem(p)[i]; }

// Copy n elements from global memory to LDS with the workgroup's 1024
// threads: each thread issues SB loads before the batch's LDS writes, so it
// waits for memory once per batch instead of once per element.
template <int SB, typename T>
__device__ __forceinline__ void stage_lds(T *dst, const T *src, int64_t n, int tid)
{
    for (int64_t i0 = tid; i0 < n; i0 += 1024 * SB) {
        T v[SB];
#pragma unroll
        for (int u = 0; u < SB; u++) {
            const int64_t i = i0 + 1024 * (int64_t)u;
            if (i < n)
                v[u] = stage_load(src, i);
        }
#pragma unroll
        for (int u = 0; u < SB; u++) {
            const int64_t i = i0 + 1024 * (int64_t)u;
            if (i < n)
                dst[i] = v[u];
        }
    }
}

// The real parts of a state staged in LDS as FP64; returns nonzero when an
// element of this thread's share has a nonzero imaginary part.
template <int SB, typename T>
__device__ __forceinline__ int stage_real(double *dst, const T *src, int64_t n, int tid)
{
    int cplx = 0;
    for (int64_t i0 = tid; i0 < n; i0 += 1024 * SB) {
        T v[SB];
#pragma unroll
        for (int u = 0; u < SB; u++) {
            const int64_t i = i0 + (int64_t)u * 1024;
            if (i < n)
                v[u] = stage_load(src, i);
        }
#pragma unroll
        for (int u = 0; u < SB; u++) {
            const int64_t i = i0 + (int64_t)u * 1024;
            if (i < n) {
                dst[i] = (double)v[u].x;
                cplx |= v[u].y != 0;
            }
        }
    }
    return cplx;
}

// The real parts of a state staged in LDS in a given precision (FP32 real
// parts of FP32 storage stay exact); returns nonzero when an element of this
// thread's share has a nonzero imaginary part.
template <int SB, typename R, typename T>
__device__ __forceinline__ int stage_real_as(R *dst, const T *src, int64_t n, int tid)
{
    int cplx = 0;
    for (int64_t i0 = tid; i0 < n; i0 += 1024 * SB) {
        T v[SB];
#pragma unroll
        for (int u = 0; u < SB; u++) {
            const int64_t i = i0 + (int64_t)u * 1024;
            if (i < n)
                v[u] = stage_load(src, i);
        }
#pragma unroll
        for (int u = 0; u < SB; u++) {
            const int64_t i = i0 + (int64_t)u * 1024;
            if (i < n) {
                dst[i] = (R)v[u].x;
                cplx |= v[u].y != 0;
            }
        }
    }
    return cplx;
}

// One entry's product a * x added to (are, aim) in FP64: a complex value, or
// the real part alone when the operator is stored with real values.
template <typename T>
__device__ __forceinline__ void entry_fma(const float2 a, const T x, double &are, double &aim)
{
    const double ar = (double)a.x, ai = (double)a.y, xr = (double)x.x, xi = (double)x.y;
    are += ar * xr - ai * xi;
    aim += ar * xi + ai * xr;
}
template <typename T>
__device__ __forceinline__ void entry_fma(const double2 a, const T x, double &are, double &aim)
{
    const double ar = a.x, ai = a.y, xr = (double)x.x, xi = (double)x.y;
    are += ar * xr - ai * xi;
    aim += ar * xi + ai * xr;
}
template <typename T>
__device__ __forceinline__ void entry_fma(const float a, const T x, double &are, double &aim)
{
    are += (double)a * (double)x.x;
    aim += (double)a * (double)x.y;
}
template <typename T>
__device__ __forceinline__ void entry_fma(const double a, const T x, double &are, double &aim)
{
    are += a * (double)x.x;
    aim += a * (double)x.y;
}

// Entries against a real state (its real parts in FP64): the imaginary sum
// stays zero.
__device__ __forceinline__ void entry_fma(const float a, const double x, double &are, double &aim)
{
    (void)aim;
    are += (double)a * x;
}
__device__ __forceinline__ void entry_fma(const double a, const double x, double &are, double &aim)
{
    (void)aim;
    are += a * x;
}
__device__ __forceinline__ void entry_fma(const float a, const float x, double &are, double &aim)
{
    (void)aim;
    are += (double)a * (double)x;
}

// A row's terms of <psi|sigma> and <psi|psi> from its state element.
template <typename T>
__device__ __forceinline__ void energy_terms(const T ps, double are, double aim, double &e_re,
                                             double &e_im, double &e_n2)
{
    const double px = (double)ps.x, py = (double)ps.y;
    e_re += px * are + py * aim;
    e_im += px * aim - py * are;
    e_n2 += px * px + py * py;
}
__device__ __forceinline__ void energy_terms(const double px, double are, double aim, double &e_re,
                                             double &e_im, double &e_n2)
{
    (void)aim;
    (void)e_im;
    e_re += px * are;
    e_n2 += px * px;
}

template <typename T, typename V, int N>
__device__ __forceinline__ void lds_gather_fma(const T *s_x, const int c[N], const V v[N],
                                               double &are, double &aim)
{
    T xs[N];
#pragma unroll
    for (int u = 0; u < N; u++)
        xs[u] = s_x[c[u]];
#pragma unroll
    for (int u = 0; u < N; u++)
        entry_fma(v[u], xs[u], are, aim);
}

// The whole state vector staged in LDS (one 128 KB copy for 14 qubits in
// FP32 storage), so every gather of the product is an LDS read instead of an
// L2 request.  A workgroup of 16 waves owns SPMV_LDS_ROWS consecutive rows of
// one state; sub-groups of L lanes read their rows with the four-entry wide
// loads, U passes in flight.
template <int DT, int L, int U, bool BATCH>
__global__ void __launch_bounds__(1024) VQE_LDS_OCCUPANCY
k_spmv_lds(SpmvState single, const SpmvState *__restrict__ states, const int2 *__restrict__ tasks)
{
    SpmvState st;
    int blk;
    if (BATCH) {
        int2 t = tasks[blockIdx.x];
        if (t.x < 0)
            return;
        st = states[t.x];
        blk = t.y;
        if (VQE_SKIP(st))
            return;
    } else {
        st = single;
        blk = blockIdx.x;
    }
    using T = typename Elem<DT>::T;
    extern __shared__ unsigned char smem[];
    T *s_x = reinterpret_cast<T *>(smem);
    const int tid = threadIdx.x;
    const int64_t dim = st.dim;
    const T *__restrict__ psi = reinterpret_cast<const T *>(st.psi);
    const int64_t r0 = (int64_t)blk * SPMV_LDS_ROWS;
    const int64_t r1 = r0 + SPMV_LDS_ROWS < dim ? r0 + SPMV_LDS_ROWS : dim;
    // the state, one zero element (index dim), then the workgroup's row pointers
    int32_t *s_rp = reinterpret_cast<int32_t *>(smem + (size_t)(dim + 1) * sizeof(T));
    stage_lds<8>(s_x, psi, dim, tid);
    if (tid == 0)
        s_x[dim] = T{};
    stage_lds<4>(s_rp, st.rowptr + r0, r1 - r0 + 1, tid);
    __syncthreads();

    constexpr int G = VQE_WAVE / L;
    const int lane = tid & 63, wid = tid >> 6;
    const int sub = lane / L, sl = lane % L;
    const int32_t *__restrict__ col = st.col;
    const T *__restrict__ val = reinterpret_cast<const T *>(st.val);
    const int nnz = (int)st.nnz, zc = (int)dim;
    double e_re = 0.0, e_im = 0.0, e_n2 = 0.0;
    for (int64_t base = r0 + wid * G; base < r1; base += 16 * G) {
        const int64_t r = base + sub;
        double are = 0.0, aim = 0.0;
        if (r < r1) {
            const int k0 = s_rp[r - r0], k1 = s_rp[r - r0 + 1];
            for (int k = (k0 & ~3) + 4 * sl; k < k1; k += U * 4 * L) {
                int c[U * 4];
                T v[U * 4];
#pragma unroll
                for (int u = 0; u < U; u++)
                    lds_group_load<DT>(col, val, k + u * 4 * L, k0, k1, nnz, zc, c + 4 * u,
                                       v + 4 * u);
                lds_gather_fma<T, T, U * 4>(s_x, c, v, are, aim);
            }
        }
        are = group_sum<L>(are);
        aim = group_sum<L>(aim);
        if (sl == 0 && r < r1) {
            Elem<DT>::st(st.sigma, r, make_double2(are, aim));
            const T ps = s_x[r];
            const double px = (double)ps.x, py = (double)ps.y;
            e_re += px * are + py * aim;
            e_im += px * aim - py * are;
            e_n2 += px * px + py * py;
        }
    }
    __shared__ double s_part[16][3];
    e_re = wave_sum(e_re);
    e_im = wave_sum(e_im);
    e_n2 = wave_sum(e_n2);
    if (lane == 0) {
        s_part[wid][0] = e_re;
        s_part[wid][1] = e_im;
        s_part[wid][2] = e_n2;
    }
    __syncthreads();
    if (tid < 3) {
        double v = 0.0;
        for (int w = 0; w < 16; w++)
            v += s_part[w][tid];
        gmem(st.partials)[(int64_t)blk * 3 + tid] = v;
    }
}

// Raw buffer resources (gfx9 descriptor word 3): a load whose offset lies at
// or past num_records returns zero and makes no memory request.
#define VQE_BUF_WORD3 0x00020000
#define VQE_BUF_OOB 0x80000000u

// Value streamed per entry: the complex value, or its real part alone (RV)
// when the plan stores the operator's real parts (an operator whose entries
// are all real).
template <int DT, bool RV> struct ValOf { using T = typename Elem<DT>::T; };
template <> struct ValOf<VQE_C64, true> { using T = float; };
template <> struct ValOf<VQE_C128, true> { using T = double; };

__device__ __forceinline__ float2 ldv(const float2 *p, int64_t i) { return ldg(p, i); }
__device__ __forceinline__ double2 ldv(const double2 *p, int64_t i) { return ldg(p, i); }
__device__ __forceinline__ float ldv(const float *p, int64_t i) { return gmem(p)[i]; }
__device__ __forceinline__ double ldv(const double *p, int64_t i) { return gmem(p)[i]; }

template <int DT, bool RV> struct BufVal;
template <> struct BufVal<VQE_C64, false> {
    // four consecutive complex64 values: two 16-byte loads
    static __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t r, unsigned off, float2 v[4])
    {
        typedef float v4f __attribute__((ext_vector_type(4)));
        const v4f a = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
        const v4f b = __builtin_amdgcn_raw_buffer_load_b128(r, off + 16, 0, 0);
        v[0] = make_float2(a.x, a.y);
        v[1] = make_float2(a.z, a.w);
        v[2] = make_float2(b.x, b.y);
        v[3] = make_float2(b.z, b.w);
    }
};
template <> struct BufVal<VQE_C128, false> {
    static __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t r, unsigned off, double2 v[4])
    {
        typedef double v2d __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const v2d a = __builtin_amdgcn_raw_buffer_load_b128(r, off + 16 * u, 0, 0);
            v[u] = make_double2(a.x, a.y);
        }
    }
};
template <> struct BufVal<VQE_C64, true> {
    // four consecutive real FP32 values: one 16-byte load
    static __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t r, unsigned off, float v[4])
    {
        typedef float v4f __attribute__((ext_vector_type(4)));
        const v4f a = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
        v[0] = a.x;
        v[1] = a.y;
        v[2] = a.z;
        v[3] = a.w;
    }
};
template <> struct BufVal<VQE_C128, true> {
    static __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t r, unsigned off, double v[4])
    {
        typedef double v2d __attribute__((ext_vector_type(2)));
        const v2d a = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
        const v2d b = __builtin_amdgcn_raw_buffer_load_b128(r, off + 16, 0, 0);
        v[0] = a.x;
        v[1] = a.y;
        v[2] = b.x;
        v[3] = b.y;
    }
};

// Real parts of an operator's values (for operators whose entries are all real).
template <int DT>
__global__ void __launch_bounds__(256)
k_val_real(const void *__restrict__ val, void *__restrict__ out, int64_t nnz)
{
    using T = typename Elem<DT>::T;
    using R = typename ValOf<DT, true>::T;
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k < nnz)
        reinterpret_cast<R *>(out)[k] = ldg(reinterpret_cast<const T *>(val), k).x;
}

// Column codes of the 16-bit form: one wave per row, lanes over its entries.
__global__ void __launch_bounds__(256)
k_col_xor16(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
            uint16_t *__restrict__ col16, int64_t dim)
{
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= dim)
        return;
    const int32_t k1 = rowptr[r + 1];
    for (int32_t k = rowptr[r] + (int32_t)(threadIdx.x & 63); k < k1; k += 64)
        col16[k] = (uint16_t)((uint32_t)col[k] ^ (uint32_t)r);
}

// Row pointers of the padded layout, in which every row's length is rounded up
// to a multiple of SPMV_PAD.  One workgroup: each thread takes a contiguous run of
// rows, the workgroup scans the run totals, and each thread writes its run.
__global__ void __launch_bounds__(1024)
k_pad_rowptr(const int32_t *__restrict__ rowptr, int32_t *__restrict__ prow, int64_t dim)
{
    __shared__ int64_t s_sum[1024];
    const int tid = threadIdx.x;
    const int64_t per = (dim + 1023) / 1024;
    const int64_t a = (int64_t)tid * per < dim ? (int64_t)tid * per : dim;
    const int64_t b = a + per < dim ? a + per : dim;
    int64_t tot = 0;
    // the run's row pointers a batch at a time (independent loads)
    constexpr int NB = 16;
    for (int64_t r0 = a; r0 < b; r0 += NB) {
        int32_t p[NB + 1];
#pragma unroll
        for (int i = 0; i <= NB; i++)
            p[i] = r0 + i <= b ? rowptr[r0 + i] : 0;
#pragma unroll
        for (int i = 0; i < NB; i++)
            if (r0 + i < b)
                tot += (p[i + 1] - p[i] + SPMV_PAD - 1) & ~(SPMV_PAD - 1);
    }
    s_sum[tid] = tot;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t v = tid >= off ? s_sum[tid - off] : 0;
        __syncthreads();
        s_sum[tid] += v;
        __syncthreads();
    }
    int64_t run = s_sum[tid] - tot;
    for (int64_t r0 = a; r0 < b; r0 += NB) {
        int32_t p[NB + 1];
#pragma unroll
        for (int i = 0; i <= NB; i++)
            p[i] = r0 + i <= b ? rowptr[r0 + i] : 0;
#pragma unroll
        for (int i = 0; i < NB; i++)
            if (r0 + i < b) {
                prow[r0 + i] = (int32_t)run;
                run += (p[i + 1] - p[i] + SPMV_PAD - 1) & ~(SPMV_PAD - 1);
            }
    }
    if (tid == 1023)
        prow[dim] = (int32_t)s_sum[1023];
}

// Column codes and values in the padded layout, one wave per row: the real
// parts (RVAL) or the complex values themselves; a row's pad entries repeat
// its last column with the value zero.
template <int DT, bool RVAL>
__global__ void __launch_bounds__(256)
k_pad_fill(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
           const void *__restrict__ val, const int32_t *__restrict__ prow,
           uint16_t *__restrict__ code, void *__restrict__ vpad, int64_t dim)
{
    using T = typename Elem<DT>::T;
    using R = typename ValOf<DT, RVAL>::T;
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= dim)
        return;
    const int32_t k0 = rowptr[r], len = rowptr[r + 1] - k0;
    const int32_t p0 = prow[r], plen = prow[r + 1] - p0;
    for (int32_t j = (int32_t)(threadIdx.x & 63); j < plen; j += 64) {
        const int32_t k = k0 + (j < len ? j : len - 1);
        code[p0 + j] = (uint16_t)((uint32_t)col[k] ^ (uint32_t)r);
        R v{};
        if (j < len) {
            if constexpr (RVAL)
                v = (R)ldg(reinterpret_cast<const T *>(val), k).x;
            else
                v = ldg(reinterpret_cast<const T *>(val), k);
        }
        reinterpret_cast<R *>(vpad)[p0 + j] = v;
    }
}

// Pipelined variant of the LDS schedule.  A sub-group of L lanes covers a row
// of up to U * GE * L = 256 entries in one pass (GE entries per lane group: 4,
// or 8 in the padded layout) and keeps the loads of its next
// D rows in flight: after a row's products it refills that row's registers
// with the row D sweeps ahead.  The loads are raw buffer loads issued by every
// lane without branches: groups past the row (or past the last whole group of
// the arrays) get an out-of-range offset and return zero without a memory
// request.  Because the number of loads per row is fixed, the wait before one
// row's products leaves the other rows' loads outstanding (the scheduling
// barriers keep each refill issued before the next row is consumed).  Rows
// longer than one pass finish with further passes, and the last nnz % 4
// entries of the arrays are added entry by entry.  With X16 the column of
// entry k of row r is read as the 16-bit code col16[k] = col[k] ^ r (8 bytes
// per group of four instead of 16), for states of at most 2^16 rows.  With
// PL the codes and values are the plan's padded layout: each row starts at a
// multiple of eight and is padded with zero values to whole groups (row
// pointers st.prow), so no entry needs a row mask and there is no tail, and a
// lane takes eight entries with one 16-byte code load.  With RV (operators
// whose entries are all real; always in the padded layout) the values are the
// real parts, 4 instead of 8 bytes per entry in FP32 storage, and a workgroup
// whose staged state has no imaginary part multiplies in real arithmetic (RX).  The kernel, k_spmv_lds_pf, stages
// and then runs pf_rows.

// The rows [r0, r1) of one workgroup of the pipelined LDS schedule, the state
// already staged in LDS at smem (complex, or with RX its real parts in FP64)
// and the row pointers at s_rp; writes sigma and the workgroup's energy
// partials.
template <int DT, int L, int D, bool X16, bool RV, bool RX, bool PL>
__device__ __forceinline__ void pf_rows(const SpmvState &st, int blk, const unsigned char *smem,
                                        const int32_t *s_rp, int64_t r0, int64_t r1)
{
    static_assert(!RV || PL, "real values come in the padded layout");
    using T = typename Elem<DT>::T;
    using X = typename std::conditional<RX, double, T>::type;
    // a lane's group: 4 entries, or 8 in the padded layout (one 16-byte code
    // load and 16-byte value loads)
    constexpr int GE = PL ? SPMV_PAD : 4;
    constexpr int U = 256 / (L * GE) > 0 ? 256 / (L * GE) : 1;
    constexpr int W = U * GE;                // entries per lane per pass
    constexpr int PASS = W * L;              // entries per sub-group per pass
    using V = typename ValOf<DT, RV>::T;
    constexpr unsigned EB = sizeof(V);
    const X *s_x = reinterpret_cast<const X *>(smem);
    const int tid = threadIdx.x;
    const int64_t dim = st.dim;
    constexpr int G = VQE_WAVE / L;
    const int lane = tid & 63, wid = tid >> 6;
    const int sub = lane / L, sl = lane % L;
    // the padded layout (PL) holds whole groups only, up to st.cap entries
    const int nnz = (int)(PL ? st.cap : st.nnz), zc = (int)dim;
    const int whole = PL ? 0x7fffffff : nnz & ~3;   // groups starting below this are whole
    const __amdgpu_buffer_rsrc_t rc =
        X16 ? __builtin_amdgcn_make_buffer_rsrc((void *)st.col16, (short)0, nnz * 2, VQE_BUF_WORD3)
            : __builtin_amdgcn_make_buffer_rsrc((void *)st.col, (short)0, nnz * 4, VQE_BUF_WORD3);
    const __amdgpu_buffer_rsrc_t rv =
        __builtin_amdgcn_make_buffer_rsrc((void *)(PL ? st.vre : st.val), (short)0, (int)(nnz * EB),
                                          VQE_BUF_WORD3);
    double e_re = 0.0, e_im = 0.0, e_n2 = 0.0;

    // issue the loads of the pass starting at group kb of a row [k0, k1)
    auto issue = [&](int kb, int k1, int c[W], V v[W]) {
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int k = kb + u * GE * L;
            const bool ok = k < k1 && k < whole;
            if (X16 && GE == 8) {
                typedef unsigned v4u __attribute__((ext_vector_type(4)));
                const v4u c4 = __builtin_amdgcn_raw_buffer_load_b128(rc, ok ? (unsigned)k * 2u : VQE_BUF_OOB, 0, 0);
                const unsigned cw[4] = {c4.x, c4.y, c4.z, c4.w};
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    c[GE * u + 2 * q] = (int)(cw[q] & 0xffffu);
                    c[GE * u + 2 * q + 1] = (int)(cw[q] >> 16);
                }
            } else if (X16) {
                typedef unsigned v2u __attribute__((ext_vector_type(2)));
                const v2u c2 = __builtin_amdgcn_raw_buffer_load_b64(rc, ok ? (unsigned)k * 2u : VQE_BUF_OOB, 0, 0);
                c[GE * u + 0] = (int)(c2.x & 0xffffu);
                c[GE * u + 1] = (int)(c2.x >> 16);
                c[GE * u + 2] = (int)(c2.y & 0xffffu);
                c[GE * u + 3] = (int)(c2.y >> 16);
            } else {
                typedef int v4i __attribute__((ext_vector_type(4)));
                const v4i c4 = __builtin_amdgcn_raw_buffer_load_b128(rc, ok ? (unsigned)k * 4u : VQE_BUF_OOB, 0, 0);
                c[GE * u + 0] = c4.x;
                c[GE * u + 1] = c4.y;
                c[GE * u + 2] = c4.z;
                c[GE * u + 3] = c4.w;
            }
#pragma unroll
            for (int h = 0; h < GE / 4; h++)
                BufVal<DT, RV>::load(rv, ok ? (unsigned)(k + 4 * h) * EB : VQE_BUF_OOB, v + GE * u + 4 * h);
        }
    };
    // products of one pass of row r; entries outside [k0, k1) read the zero
    // element
    auto consume = [&](int64_t r, int kb, int k0, int k1, const int c[W], const V v[W],
                       double &are, double &aim) {
        int cm[W];
        const unsigned len = (unsigned)(k1 - k0);
        const int rx = (int)r;
#pragma unroll
        for (int u = 0; u < U; u++)
#pragma unroll
            for (int q = 0; q < GE; q++) {
                const int k = kb + u * GE * L + q;
                const int col = X16 ? (rx ^ c[GE * u + q]) : c[GE * u + q];
                cm[GE * u + q] = PL || (unsigned)(k - k0) < len ? col : zc;
            }
        lds_gather_fma<X, V, W>(s_x, cm, v, are, aim);
    };
    auto row_bounds = [&](int64_t r, int &k0, int &k1) {
        if (r < r1) {
            k0 = s_rp[r - r0];
            k1 = s_rp[r - r0 + 1];
        } else {
            k0 = k1 = 0;
        }
    };
    auto finish = [&](int64_t r, int k0, int k1, double are, double aim) {
        // further passes of a long row
        for (int kb = (k0 & ~(GE - 1)) + GE * sl + PASS; kb - GE * sl < k1; kb += PASS) {
            int c[W];
            V v[W];
            issue(kb, k1, c, v);
            consume(r, kb, k0, k1, c, v, are, aim);
        }
        // the entries after the last whole group of the arrays
        if (k1 > whole) {
            const int k = (k0 > whole ? k0 : whole) + sl;
            if (k < k1) {
                const V a = ldv(reinterpret_cast<const V *>(PL ? st.vre : st.val), k);
                const int col = X16 ? ((int)r ^ (int)gmem(st.col16)[k]) : gmem(st.col)[k];
                entry_fma(a, s_x[col], are, aim);
            }
        }
        are = group_sum<L>(are);
        if (!RX)
            aim = group_sum<L>(aim);
        if (sl == 0 && r < r1) {
            Elem<DT>::st(st.sigma, r, make_double2(are, aim));
            energy_terms(s_x[r], are, aim, e_re, e_im, e_n2);
        }
    };

    // D rows per sub-group in flight: each row's buffer is consumed and then
    // refilled with the sub-group's row D sweeps later
    int cb[D][W];
    V vb[D][W];
    int kb0[D], kb1[D];
    int64_t rr[D];
#pragma unroll
    for (int d = 0; d < D; d++) {
        rr[d] = r0 + (wid + 16 * d) * G + sub;
        row_bounds(rr[d], kb0[d], kb1[d]);
        issue((kb0[d] & ~(GE - 1)) + GE * sl, kb1[d], cb[d], vb[d]);
    }
    __builtin_amdgcn_sched_barrier(0);
    for (int64_t base = r0 + wid * G; base < r1; base += 16 * D * G) {
#pragma unroll
        for (int d = 0; d < D; d++) {
            {
                double are = 0.0, aim = 0.0;
                consume(rr[d], (kb0[d] & ~(GE - 1)) + GE * sl, kb0[d], kb1[d], cb[d], vb[d], are, aim);
                finish(rr[d], kb0[d], kb1[d], are, aim);
            }
            rr[d] += 16 * D * G;
            row_bounds(rr[d], kb0[d], kb1[d]);
            issue((kb0[d] & ~(GE - 1)) + GE * sl, kb1[d], cb[d], vb[d]);
            // keep the refill ahead of the next row's products
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    __shared__ double s_part[16][3];
    e_re = wave_sum(e_re);
    e_im = wave_sum(e_im);
    e_n2 = wave_sum(e_n2);
    if (lane == 0) {
        s_part[wid][0] = e_re;
        s_part[wid][1] = e_im;
        s_part[wid][2] = e_n2;
    }
    __syncthreads();
    if (tid < 3) {
        double v = 0.0;
        for (int w = 0; w < 16; w++)
            v += s_part[w][tid];
        gmem(st.partials)[(int64_t)blk * 3 + tid] = v;
    }
}

// The pipelined LDS schedule's kernel (described above pf_rows): one
// workgroup per (state, block of rows).
template <int DT, int L, int D, bool BATCH, bool X16, bool RV, bool PL>
__global__ void __launch_bounds__(1024) VQE_LDS_OCCUPANCY
k_spmv_lds_pf(SpmvState single, const SpmvState *__restrict__ states,
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
        if (VQE_SKIP(st))
            return;
    } else {
        st = single;
        blk = blockIdx.x;
    }
    using T = typename Elem<DT>::T;
    extern __shared__ unsigned char smem[];
    T *s_x = reinterpret_cast<T *>(smem);
    const int tid = threadIdx.x;
    const int64_t dim = st.dim;
    const T *__restrict__ psi = reinterpret_cast<const T *>(st.psi);
    const int64_t r0 = (int64_t)blk * SPMV_LDS_ROWS;
    const int64_t r1 = r0 + SPMV_LDS_ROWS < dim ? r0 + SPMV_LDS_ROWS : dim;
    int32_t *s_rp = reinterpret_cast<int32_t *>(smem + (size_t)(dim + 1) * sizeof(T));
    stage_lds<4>(s_rp, (PL ? st.prow : st.rowptr) + r0, r1 - r0 + 1, tid);
    if constexpr (RV) {
        // a real state (every imaginary part zero) runs in real arithmetic
        double *s_xr = reinterpret_cast<double *>(smem);
        const int cplx = stage_real<8>(s_xr, psi, dim, tid);
        if (tid == 0)
            s_xr[dim] = 0.0;
        if (!__syncthreads_or(cplx)) {
            pf_rows<DT, L, D, X16, RV, true, PL>(st, blk, smem, s_rp, r0, r1);
            return;
        }
    }
    stage_lds<8>(s_x, psi, dim, tid);
    if (tid == 0)
        s_x[dim] = T{};
    __syncthreads();
    pf_rows<DT, L, D, X16, RV, false, PL>(st, blk, smem, s_rp, r0, r1);
}


// ------------------------------------------------------------------ sliced layout
// VQE_SPMV_SLICED: one row per wave lane (the layout is described with
// SpmvState::scode).  Rows of a block are sorted by length so that the 64 rows
// of a slice are nearly equally long (the pads are a few percent of the
// entries at 14 qubits); a lane's loads of E entries sit next to its
// neighbours' (one contiguous run per wave and load), every lane sums its row
// in the CSR's column order with no cross-lane reduction, and the slice's
// length is uniform over the wave, so the loop has no row masks.

typedef unsigned sell_v2u __attribute__((ext_vector_type(2)));
typedef unsigned sell_v4u __attribute__((ext_vector_type(4)));
typedef int sell_v2i __attribute__((ext_vector_type(2)));

// Sort each block's rows by length, longest first (ties by row), and give
// each slice its length rounded up to E; one workgroup per block.
__global__ void __launch_bounds__(1024)
k_sell_sort(const int32_t *__restrict__ rowptr, int64_t dim, int E, uint16_t *__restrict__ srow,
            int32_t *__restrict__ slen)
{
    __shared__ uint32_t key[SPMV_LDS_ROWS];
    const int tid = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * SPMV_LDS_ROWS;
    const int n = (int)(dim - r0 < SPMV_LDS_ROWS ? dim - r0 : SPMV_LDS_ROWS);
    for (int i = tid; i < SPMV_LDS_ROWS; i += 1024) {
        uint32_t k = 0xffffffffu;   // no row: sorts last
        if (i < n) {
            const uint32_t len = (uint32_t)(gmem(rowptr)[r0 + i + 1] - gmem(rowptr)[r0 + i]);
            k = ((0xffffu - len) << 16) | (uint32_t)i;
        }
        key[i] = k;
    }
    __syncthreads();
    // bitonic sort, ascending keys
    for (int k = 2; k <= SPMV_LDS_ROWS; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = tid; i < SPMV_LDS_ROWS; i += 1024) {
                const int q = i ^ j;
                if (q > i) {
                    const uint32_t a = key[i], b = key[q];
                    if ((a > b) == ((i & k) == 0)) {
                        key[i] = b;
                        key[q] = a;
                    }
                }
            }
            __syncthreads();
        }
    for (int i = tid; i < n; i += 1024)
        srow[r0 + i] = (uint16_t)(key[i] & 0xffffu);
    if (tid < SPMV_SLICES_PER_BLOCK) {
        int len = 0;
        if (tid * VQE_WAVE < n) {
            len = (int)(0xffffu - (key[tid * VQE_WAVE] >> 16));
            len = (len + E - 1) / E * E;
        }
        slen[(int64_t)blockIdx.x * SPMV_SLICES_PER_BLOCK + tid] = len;
    }
}

// Slice starts (entries) in slice order and the total; one thread (a state
// that fits LDS has at most a few hundred slices).
__global__ void k_sell_scan(const int32_t *__restrict__ slen, int64_t ns, int2 *__restrict__ sslice,
                            int64_t *__restrict__ total)
{
    if (threadIdx.x != 0 || blockIdx.x != 0)
        return;
    int64_t at = 0;
    for (int64_t c = 0; c < ns; c++) {
        const int len = slen[c];
        sslice[c] = make_int2((int)at, len);
        at += (int64_t)len * VQE_WAVE;
    }
    *total = at;
}

// Codes and values of one slice per wave (pads: column dim, value zero); RV:
// the values' real parts (an operator whose entries are all real).
template <int DT, bool RV>
__global__ void __launch_bounds__(64)
k_sell_fill(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
            const void *__restrict__ val, int64_t dim, int E, const uint16_t *__restrict__ srow,
            const int2 *__restrict__ sslice, uint16_t *__restrict__ code, void *__restrict__ sval)
{
    using T = typename Elem<DT>::T;
    using V = typename ValOf<DT, RV>::T;
    const int64_t c = blockIdx.x;
    const int64_t r0 = (c / SPMV_SLICES_PER_BLOCK) * SPMV_LDS_ROWS;
    const int n = (int)(dim - r0 < SPMV_LDS_ROWS ? dim - r0 : SPMV_LDS_ROWS);
    const int lane = threadIdx.x;
    const int i = (int)(c % SPMV_SLICES_PER_BLOCK) * VQE_WAVE + lane;
    const int2 sl = sslice[c];
    int64_t k0 = 0;
    int len = 0;
    if (i < n) {
        const int64_t row = r0 + srow[r0 + i];
        k0 = rowptr[row];
        len = rowptr[row + 1] - (int32_t)k0;
    }
    V *out = reinterpret_cast<V *>(sval);
    const T *in = reinterpret_cast<const T *>(val);
    for (int j = 0; j < sl.y; j++) {
        const int64_t at = (int64_t)sl.x + ((int64_t)(j / E) * VQE_WAVE + lane) * E + j % E;
        code[at] = j < len ? (uint16_t)col[k0 + j] : (uint16_t)dim;
        if constexpr (RV)
            out[at] = j < len ? in[k0 + j].x : V{};
        else
            out[at] = j < len ? in[k0 + j] : V{};
    }
}

// Flip-mask index form (VQE_SPMV_XIDX): the masks x = col ^ row an operator
// uses (Eq. 3: every Pauli string maps r to r ^ x), numbered in ascending
// order, and the slices' entries stored as those numbers.
__global__ void __launch_bounds__(256)
k_sell_xclear(uint32_t *__restrict__ mark, int64_t dim)
{
    const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (x < dim)
        mark[x] = 0u;
}

// mark[x] = 1 for every mask the operator uses; one thread per row (col and
// row are below dim = 2^N, so is their XOR).
__global__ void __launch_bounds__(256)
k_sell_xmark(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col, int64_t dim,
             uint32_t *__restrict__ mark)
{
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= dim)
        return;
    for (int k = rowptr[r]; k < rowptr[r + 1]; k++)
        mark[(uint32_t)col[k] ^ (uint32_t)r] = 1u;
}

// The masks' numbers xmap[x] (ascending x), the table xtab[number] = x for
// the first SPMV_XIDX_MAX numbers and the count; one workgroup (dim <= 2^16).
__global__ void __launch_bounds__(1024)
k_sell_xscan(const uint32_t *__restrict__ mark, int64_t dim, uint16_t *__restrict__ xmap,
             uint16_t *__restrict__ xtab, int64_t *__restrict__ nx)
{
    __shared__ int part[1024];
    const int tid = threadIdx.x;
    const int64_t per = (dim + 1023) / 1024;
    const int64_t lo = (int64_t)tid * per < dim ? (int64_t)tid * per : dim;
    const int64_t hi = lo + per < dim ? lo + per : dim;
    int c = 0;
    for (int64_t x = lo; x < hi; x++)
        c += mark[x] != 0u;
    part[tid] = c;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int at = part[tid] - c;
    for (int64_t x = lo; x < hi; x++)
        if (mark[x]) {
            xmap[x] = (uint16_t)at;
            if (at < SPMV_XIDX_MAX)
                xtab[at] = (uint16_t)x;
            at++;
        }
    if (tid == 1023)
        *nx = part[1023];
}

// Indices and values of one slice per wave (E = 3 or 6 entries per group,
// E / 3 words; pads: index 0, value zero); RV: the values' real parts.
template <int DT, bool RV, int E>
__global__ void __launch_bounds__(64)
k_sell_fill_x(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
              const void *__restrict__ val, int64_t dim, const uint16_t *__restrict__ srow,
              const int2 *__restrict__ sslice, const uint16_t *__restrict__ xmap,
              uint32_t *__restrict__ code, void *__restrict__ sval)
{
    using T = typename Elem<DT>::T;
    using V = typename ValOf<DT, RV>::T;
    static_assert(E == 3 || E == 6, "three indices to a word");
    const int64_t c = blockIdx.x;
    const int64_t r0 = (c / SPMV_SLICES_PER_BLOCK) * SPMV_LDS_ROWS;
    const int n = (int)(dim - r0 < SPMV_LDS_ROWS ? dim - r0 : SPMV_LDS_ROWS);
    const int lane = threadIdx.x;
    const int i = (int)(c % SPMV_SLICES_PER_BLOCK) * VQE_WAVE + lane;
    const int2 sl = sslice[c];
    int64_t k0 = 0, row = 0;
    int len = 0;
    if (i < n) {
        row = r0 + srow[r0 + i];
        k0 = rowptr[row];
        len = rowptr[row + 1] - (int32_t)k0;
    }
    V *out = reinterpret_cast<V *>(sval);
    const T *in = reinterpret_cast<const T *>(val);
    for (int g = 0; g < sl.y / E; g++) {
        // the group's first entry: a multiple of E, so its words start at a
        // multiple of E / 3
        const int64_t at = (int64_t)sl.x + ((int64_t)g * VQE_WAVE + lane) * E;
        uint32_t w[E / 3] = {};
#pragma unroll
        for (int e = 0; e < E; e++) {
            const int j = g * E + e;
            const uint32_t idx = j < len ? xmap[(uint32_t)col[k0 + j] ^ (uint32_t)row] : 0u;
            w[e / 3] |= idx << (10 * (e % 3));
            if constexpr (RV)
                out[at + e] = j < len ? in[k0 + j].x : V{};
            else
                out[at + e] = j < len ? in[k0 + j] : V{};
        }
#pragma unroll
        for (int q = 0; q < E / 3; q++)
            code[at / 3 + q] = w[q];
    }
}

// One entry's product added to the row's sums in turn (each product with its
// own FMA): complex value and state; real value, complex state; real value,
// real state (FP64 real parts).
template <typename V, typename X>
__device__ __forceinline__ void sell_fma(const V a, const X x, double &are, double &aim)
{
    const double ar = (double)a.x, ai = (double)a.y, xr = (double)x.x, xi = (double)x.y;
    are = fma(ar, xr, are);
    are = fma(-ai, xi, are);
    aim = fma(ar, xi, aim);
    aim = fma(ai, xr, aim);
}
template <typename X>
__device__ __forceinline__ void sell_fma(const float a, const X x, double &are, double &aim)
{
    are = fma((double)a, (double)x.x, are);
    aim = fma((double)a, (double)x.y, aim);
}
template <typename X>
__device__ __forceinline__ void sell_fma(const double a, const X x, double &are, double &aim)
{
    are = fma(a, (double)x.x, are);
    aim = fma(a, (double)x.y, aim);
}
__device__ __forceinline__ void sell_fma(const float a, const double x, double &are, double &aim)
{
    (void)aim;
    are = fma((double)a, x, are);
}
__device__ __forceinline__ void sell_fma(const double a, const double x, double &are, double &aim)
{
    (void)aim;
    are = fma(a, x, are);
}

// E consecutive entries of one lane: their codes (two per word) and values
// (complex, or their real parts with RV).
template <int DT, int E, bool RV = false>
struct SellGroup {
    using T = typename Elem<DT>::T;
    using V = typename ValOf<DT, RV>::T;
    using C = uint16_t;     // the layout's code unit
    unsigned c[E / 2];
    V v[E];
    __device__ __forceinline__ void load(const uint16_t *__restrict__ code,
                                         const V *__restrict__ val, int64_t at)
    {
        if constexpr (E == 2) {
            c[0] = gmem(reinterpret_cast<const unsigned *>(code + at))[0];
        } else if constexpr (E == 4) {
            const sell_v2u w = gmem(reinterpret_cast<const sell_v2u *>(code + at))[0];
            c[0] = w.x;
            c[1] = w.y;
        } else {
            const sell_v4u w = gmem(reinterpret_cast<const sell_v4u *>(code + at))[0];
            c[0] = w.x;
            c[1] = w.y;
            c[2] = w.z;
            c[3] = w.w;
        }
        if constexpr (RV && DT == VQE_C64 && E == 2) {
            const vqe_v2f a = gmem(reinterpret_cast<const vqe_v2f *>(val + at))[0];
            v[0] = a.x;
            v[1] = a.y;
        } else if constexpr (RV && DT == VQE_C64) {
#pragma unroll
            for (int q = 0; q < E / 4; q++) {
                const vqe_v4f a = gmem(reinterpret_cast<const vqe_v4f *>(val + at))[q];
                v[4 * q] = a.x;
                v[4 * q + 1] = a.y;
                v[4 * q + 2] = a.z;
                v[4 * q + 3] = a.w;
            }
        } else if constexpr (RV) {
#pragma unroll
            for (int q = 0; q < E / 2; q++) {
                const vqe_v2d a = gmem(reinterpret_cast<const vqe_v2d *>(val + at))[q];
                v[2 * q] = a.x;
                v[2 * q + 1] = a.y;
            }
        } else if constexpr (DT == VQE_C64) {
#pragma unroll
            for (int q = 0; q < E / 2; q++) {
                const vqe_v4f a = gmem(reinterpret_cast<const vqe_v4f *>(val + at))[q];
                v[2 * q] = make_float2(a.x, a.y);
                v[2 * q + 1] = make_float2(a.z, a.w);
            }
        } else {
#pragma unroll
            for (int q = 0; q < E; q++)
                v[q] = ldg(val, at + q);
        }
    }
    // each product added to the row's sums in turn; X: the staged state's
    // element (complex, or the real parts in FP64)
    template <typename X>
    __device__ __forceinline__ void use(const X *s_x, double &are, double &aim) const
    {
#pragma unroll
        for (int q = 0; q < E; q++)
            sell_fma(v[q], s_x[(q & 1) ? c[q / 2] >> 16 : c[q / 2] & 0xffffu], are, aim);
    }
};

// The same for the flip-mask index form: E = 3 or 6 entries per lane, their
// indices in E / 3 32-bit words (three 10-bit fields each); an entry's column
// is the lane's row XOR the indexed mask.
template <int DT, bool RV, int E>
struct SellGroupX {
    using V = typename ValOf<DT, RV>::T;
    using C = uint32_t;
    static_assert(E == 3 || E == 6, "three indices to a word");
    unsigned c[E / 3];
    V v[E];
    // at: the group's first entry (a multiple of E: with E = 6 the words are
    // 8-byte and the values 16-byte aligned, 8-byte for FP32 real parts; with
    // E = 3 the values are aligned to their own size)
    __device__ __forceinline__ void load(const uint32_t *__restrict__ code, const V *__restrict__ val,
                                         int64_t at)
    {
        if constexpr (E == 3) {
            c[0] = gmem(code)[at / 3];
#pragma unroll
            for (int q = 0; q < E; q++) {
                if constexpr (RV)
                    v[q] = gmem(val)[at + q];
                else
                    v[q] = ldg(val, at + q);
            }
            return;
        }
        const sell_v2u w = gmem(reinterpret_cast<const sell_v2u *>(code + at / 3))[0];
        c[0] = w.x;
        c[1] = w.y;
        if constexpr (RV && DT == VQE_C64) {
#pragma unroll
            for (int q = 0; q < E / 2; q++) {
                const vqe_v2f a = gmem(reinterpret_cast<const vqe_v2f *>(val + at))[q];
                v[2 * q] = a.x;
                v[2 * q + 1] = a.y;
            }
        } else if constexpr (RV) {
#pragma unroll
            for (int q = 0; q < E / 2; q++) {
                const vqe_v2d a = gmem(reinterpret_cast<const vqe_v2d *>(val + at))[q];
                v[2 * q] = a.x;
                v[2 * q + 1] = a.y;
            }
        } else if constexpr (DT == VQE_C64) {
#pragma unroll
            for (int q = 0; q < E / 2; q++) {
                const vqe_v4f a = gmem(reinterpret_cast<const vqe_v4f *>(val + at))[q];
                v[2 * q] = make_float2(a.x, a.y);
                v[2 * q + 1] = make_float2(a.z, a.w);
            }
        } else {
#pragma unroll
            for (int q = 0; q < E; q++)
                v[q] = ldg(val, at + q);
        }
    }
    // each product added to the row's sums in turn; s_xt: the masks staged in
    // LDS, row: the lane's row
    template <typename X>
    __device__ __forceinline__ void use(const X *s_x, const uint16_t *s_xt, uint32_t row, double &are,
                                        double &aim) const
    {
#pragma unroll
        for (int q = 0; q < E; q++)
            sell_fma(v[q], s_x[row ^ (uint32_t)s_xt[(c[q / 3] >> (10 * (q % 3))) & 1023u]], are, aim);
    }
};

// One wave's share of a block of the sliced layout: slices A = wid and
// B = wid + 16 (those the block has), taken as one stream of groups (A's,
// then B's) so that B's first groups load while A finishes; D groups of E
// entries per lane in flight.  Every load is issued (past the stream's end
// it repeats the last group, which is in cache), so no load sits under a
// branch and each group's wait leaves the later groups' loads in flight.
template <int DT, int E, int D, bool RV, bool XI = false>
struct SellWave {
    using V = typename ValOf<DT, RV>::T;
    using G = typename std::conditional<XI, SellGroupX<DT, RV, E>, SellGroup<DT, E, RV>>::type;
    static constexpr int64_t STEP = (int64_t)VQE_WAVE * E;
    const typename G::C *code;
    const V *val;
    int64_t r0, ata, atb;
    int n, ns, nga, ngb, ng, ra, rb;   // ra, rb: block-local rows of this lane
    G g[D];

    __device__ __forceinline__ void init(const SpmvState &st, int blk, int lane, int wid)
    {
        code = reinterpret_cast<const typename G::C *>(st.scode);
        val = reinterpret_cast<const V *>(st.sval);
        r0 = (int64_t)blk * SPMV_LDS_ROWS;
        n = (int)(st.dim - r0 < SPMV_LDS_ROWS ? st.dim - r0 : SPMV_LDS_ROWS);
        ns = (n + VQE_WAVE - 1) / VQE_WAVE;
        const int ka = wid, kb = wid + 16;
        const sell_v2i *sls = reinterpret_cast<const sell_v2i *>(st.sslice) + (int64_t)blk * SPMV_SLICES_PER_BLOCK;
        sell_v2i a = {0, 0}, b = {0, 0};
        if (ka < ns)
            a = gmem(sls)[ka];
        if (kb < ns)
            b = gmem(sls)[kb];
        nga = __builtin_amdgcn_readfirstlane(a.y) / E;
        ngb = __builtin_amdgcn_readfirstlane(b.y) / E;
        ng = nga + ngb;
        ata = (int64_t)__builtin_amdgcn_readfirstlane(a.x) + lane * E;
        atb = (int64_t)__builtin_amdgcn_readfirstlane(b.x) + lane * E - (int64_t)nga * STEP;
        const int ia = ka * VQE_WAVE + lane, ib = kb * VQE_WAVE + lane;
        ra = gmem(st.srow)[r0 + (ia < n ? ia : n - 1)];
        rb = gmem(st.srow)[r0 + (ib < n ? ib : n - 1)];
    }
    // stream group p (clamped to the last) and its first entry for this lane
    __device__ __forceinline__ int64_t addr(int p) const
    {
        const int pc = p < ng ? p : ng - 1;
        return (pc < nga ? ata : atb) + (int64_t)pc * STEP;
    }
    // the stream's first groups (a wave with groups only)
    __device__ __forceinline__ void prefetch()
    {
#pragma unroll
        for (int d = 0; d < D; d++)
            g[d].load(code, val, addr(d));
    }
    // the rows' sums for A and B against the staged state s_x (X: complex, or
    // the real parts in FP64 for a real state; s_xt: the staged flip masks of
    // the index form); prefetch() came first
    template <typename X>
    __device__ __forceinline__ void run(const X *s_x, const uint16_t *s_xt, double2 &sa, double2 &sb)
    {
        double are = 0.0, aim = 0.0;
        sa = make_double2(0.0, 0.0);
        sb = make_double2(0.0, 0.0);
        if (ng == 0)
            return;
        uint32_t row = (uint32_t)(r0 + ra);
        auto use = [&](const G &gr) {
            if constexpr (XI)
                gr.use(s_x, s_xt, row, are, aim);
            else
                gr.use(s_x, are, aim);
        };
        int q = 0;
        for (; q + D <= ng; q += D) {
#pragma unroll
            for (int d = 0; d < D; d++) {
                if (q + d == nga) {     // B's first group: A's sums are done
                    sa = make_double2(are, aim);
                    are = aim = 0.0;
                    row = (uint32_t)(r0 + rb);
                }
                use(g[d]);
                g[d].load(code, val, addr(q + D + d));
                // keep the refill ahead of the next group's products
                __builtin_amdgcn_sched_barrier(0);
            }
        }
#pragma unroll
        for (int d = 0; d < D; d++)
            if (q + d < ng) {
                if (q + d == nga) {
                    sa = make_double2(are, aim);
                    are = aim = 0.0;
                    row = (uint32_t)(r0 + rb);
                }
                use(g[d]);
            }
        if (ngb == 0)
            sa = make_double2(are, aim);
        else
            sb = make_double2(are, aim);
    }
};

// The block's rows from a wave's sums: sigma (FP32 storage: gathered in LDS
// and stored in row order), the energy terms and the block's partials.
template <int DT, int E, int D, bool RV, bool XI, typename X>
__device__ __forceinline__ void sell_finish(const SpmvState &st, int blk, const SellWave<DT, E, D, RV, XI> &w,
                                            const X *s_x, float2 *s_sig, double2 sa, double2 sb)
{
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    double e_re = 0.0, e_im = 0.0, e_n2 = 0.0;
#pragma unroll
    for (int h = 0; h < 2; h++) {
        const int k = wid + 16 * h;
        const int i = k * VQE_WAVE + lane;
        if (k < w.ns && i < w.n) {
            const int64_t row = w.r0 + (h ? w.rb : w.ra);
            const double2 a = h ? sb : sa;
            if constexpr (DT == VQE_C64)
                s_sig[row - w.r0] = make_float2((float)a.x, (float)a.y);
            else
                Elem<DT>::st(st.sigma, row, a);
            energy_terms(s_x[row], a.x, a.y, e_re, e_im, e_n2);
        }
    }
    if constexpr (DT == VQE_C64) {
        // the block's results leave in row order
        __syncthreads();
        for (int i = tid; i < w.n; i += 1024)
            stg(reinterpret_cast<float2 *>(st.sigma), w.r0 + i, s_sig[i]);
    }
    __shared__ double s_part[16][3];
    e_re = wave_sum(e_re);
    e_im = wave_sum(e_im);
    e_n2 = wave_sum(e_n2);
    if (lane == 0) {
        s_part[wid][0] = e_re;
        s_part[wid][1] = e_im;
        s_part[wid][2] = e_n2;
    }
    __syncthreads();
    if (tid < 3) {
        double v = 0.0;
        for (int q = 0; q < 16; q++)
            v += s_part[q][tid];
        gmem(st.partials)[(int64_t)blk * 3 + tid] = v;
    }
}

// One workgroup per (state, block of SPMV_LDS_ROWS rows): the state staged in
// LDS (plus the zero element), then the block's slices; each wave's first
// groups are loaded together with the staged state.  With RV (the real parts
// of a real H) a state whose imaginary parts are all zero is staged as FP64
// real parts and multiplied in real arithmetic; any other state takes the
// complex staging in the same launch.  XI: the flip-mask index form, its
// masks staged after the block's results (every one of the SPMV_XIDX_MAX
// slots written, zero past the operator's count, so every index gives a
// column below dim).
template <int DT, int E, int D, bool RV, bool XI>
__global__ void __launch_bounds__(1024) VQE_LDS_OCCUPANCY
k_spmv_sell(const SpmvState *__restrict__ states, const int2 *__restrict__ tasks)
{
    const int2 t = tasks[blockIdx.x];
    if (t.x < 0)
        return;
    const SpmvState st = states[t.x];
    if (VQE_SKIP(st))
        return;
    using T = typename Elem<DT>::T;
    extern __shared__ unsigned char smem[];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t dim = st.dim;
    const T *psi = reinterpret_cast<const T *>(st.psi);
    // FP32 storage: the block's results gather in LDS after the state
    float2 *s_sig = reinterpret_cast<float2 *>(smem + (size_t)(dim + 1) * sizeof(T));
    uint16_t *s_xt = reinterpret_cast<uint16_t *>(
        smem + (size_t)(dim + 1) * sizeof(T) + (DT == VQE_C64 ? SPMV_LDS_ROWS * sizeof(float2) : 0));
    SellWave<DT, E, D, RV, XI> w;
    w.init(st, t.y, lane, wid);
    if constexpr (XI) {
        static_assert(SPMV_XIDX_MAX <= 1024, "one mask per thread");
        s_xt[tid] = tid < st.nx ? gmem(st.sxtab)[tid] : (uint16_t)0;
    }
    double2 sa, sb;
    if constexpr (RV) {
        if (w.ng > 0)
            w.prefetch();
        double *s_xr = reinterpret_cast<double *>(smem);
        const int cplx = stage_real<8>(s_xr, psi, dim, tid);
        if (tid == 0)
            s_xr[dim] = 0.0;
        if (!__syncthreads_or(cplx)) {
            w.run(s_xr, s_xt, sa, sb);
            sell_finish(st, t.y, w, s_xr, s_sig, sa, sb);
            return;
        }
    }
    // the state in 16-byte chunks (dim * sizeof(T) is a multiple of 16 and
    // psi 16-byte aligned): the first SP per thread loaded before the wave's
    // first groups, so both latencies overlap
    T *s_x = reinterpret_cast<T *>(smem);
    constexpr int SP = 8;
    const int64_t nch = dim * (int64_t)sizeof(T) / 16;
    const vqe_v4f *src = reinterpret_cast<const vqe_v4f *>(psi);
    vqe_v4f *dst = reinterpret_cast<vqe_v4f *>(s_x);
    vqe_v4f pre[SP];
#pragma unroll
    for (int u = 0; u < SP; u++) {
        const int64_t c = tid + 1024 * u;
        if (c < nch)
            pre[u] = gmem(src)[c];
    }
    if (!RV && w.ng > 0)
        w.prefetch();
#pragma unroll
    for (int u = 0; u < SP; u++) {
        const int64_t c = tid + 1024 * u;
        if (c < nch)
            dst[c] = pre[u];
    }
    for (int64_t c = tid + 1024 * SP; c < nch; c += 1024)
        dst[c] = gmem(src)[c];
    if (tid == 0)
        s_x[dim] = T{};
    __syncthreads();
    w.run(s_x, s_xt, sa, sb);
    sell_finish(st, t.y, w, s_x, s_sig, sa, sb);
}

// Column-tiled variant of the pipelined LDS schedule, for states larger than
// LDS.  A workgroup takes one block of rows and one column tile: it stages
// that tile of the state (SPMV_TILE_BYTES) and, per row, streams only the
// row's entries in the tile -- a contiguous sub-range, since columns are
// sorted within a row, bounded by the per-tile row pointers.  The row sums of
// a tile go to an FP64 partial array; the tile-sum kernel adds the tiles in
// ascending order and applies the energy epilogue.

// The rows [r0, r1) of one column tile t of the column-tiled schedule, the
// columns [c_lo, c_lo + tc) staged in LDS at smem (complex, or with RX the
// real parts in storage precision) and the rows' tile bounds at s_k0, s_k1;
// entries outside those columns are masked.  Writes the FP64 tile partials,
// or adds to them (accumulate).
template <int DT, int L, int D, int U, bool X16, bool RV, bool RX>
__device__ __forceinline__ void tiled_rows(const SpmvState &st, int t, int c_lo, int tc,
                                           bool accumulate, const unsigned char *smem,
                                           const int32_t *s_k0, const int32_t *s_k1, int64_t r0,
                                           int64_t r1)
{
    using X = typename std::conditional<RX, typename ValOf<DT, true>::T,
                                        typename Elem<DT>::T>::type;
    constexpr int W = U * 4;
    constexpr int PASS = W * L;
    using V = typename ValOf<DT, RV>::T;
    constexpr unsigned EB = sizeof(V);
    const X *s_x = reinterpret_cast<const X *>(smem);
    const int tid = threadIdx.x;
    const int64_t dim = st.dim;
    constexpr int G = VQE_WAVE / L;
    const int lane = tid & 63, wid = tid >> 6;
    const int sub = lane / L, sl = lane % L;
    const int nnz = (int)st.nnz, zc = tc;
    const int whole = nnz & ~3;
    const __amdgpu_buffer_rsrc_t rc =
        X16 ? __builtin_amdgcn_make_buffer_rsrc((void *)st.col16, (short)0, nnz * 2, VQE_BUF_WORD3)
            : __builtin_amdgcn_make_buffer_rsrc((void *)st.col, (short)0, nnz * 4, VQE_BUF_WORD3);
    const __amdgpu_buffer_rsrc_t rv =
        __builtin_amdgcn_make_buffer_rsrc((void *)(RV ? st.vre : st.val), (short)0, (int)(nnz * EB),
                                          VQE_BUF_WORD3);
    double *__restrict__ part = st.tile_part + (int64_t)t * dim * 2;

    auto issue = [&](int kb, int k1, int c[W], V v[W]) {
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int k = kb + u * 4 * L;
            const bool ok = k < k1 && k < whole;
            if (X16) {
                typedef unsigned v2u __attribute__((ext_vector_type(2)));
                const v2u c2 = __builtin_amdgcn_raw_buffer_load_b64(rc, ok ? (unsigned)k * 2u : VQE_BUF_OOB, 0, 0);
                c[4 * u + 0] = (int)(c2.x & 0xffffu);
                c[4 * u + 1] = (int)(c2.x >> 16);
                c[4 * u + 2] = (int)(c2.y & 0xffffu);
                c[4 * u + 3] = (int)(c2.y >> 16);
            } else {
                typedef int v4i __attribute__((ext_vector_type(4)));
                const v4i c4 = __builtin_amdgcn_raw_buffer_load_b128(rc, ok ? (unsigned)k * 4u : VQE_BUF_OOB, 0, 0);
                c[4 * u + 0] = c4.x;
                c[4 * u + 1] = c4.y;
                c[4 * u + 2] = c4.z;
                c[4 * u + 3] = c4.w;
            }
            BufVal<DT, RV>::load(rv, ok ? (unsigned)k * EB : VQE_BUF_OOB, v + 4 * u);
        }
    };
    // entries outside [k0, k1) (or not loaded) read the zero element; the
    // column test keeps every LDS index inside the tile
    auto consume = [&](int64_t r, int kb, int k0, int k1, const int c[W], const V v[W],
                       double &are, double &aim) {
        int cm[W];
        const unsigned len = (unsigned)(k1 - k0);
        const int rx = (int)r;
#pragma unroll
        for (int u = 0; u < U; u++)
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int k = kb + u * 4 * L + q;
                const int cl = (X16 ? (rx ^ c[4 * u + q]) : c[4 * u + q]) - c_lo;
                cm[4 * u + q] = ((unsigned)(k - k0) < len && (unsigned)cl < (unsigned)tc) ? cl : zc;
            }
        lds_gather_fma<X, V, W>(s_x, cm, v, are, aim);
    };
    auto row_bounds = [&](int64_t r, int &k0, int &k1) {
        if (r < r1) {
            k0 = s_k0[r - r0];
            k1 = s_k1[r - r0];
        } else {
            k0 = k1 = 0;
        }
    };
    auto finish = [&](int64_t r, int k0, int k1, double are, double aim) {
        for (int kb = (k0 & ~3) + 4 * sl + PASS; kb - 4 * sl < k1; kb += PASS) {
            int c[W];
            V v[W];
            issue(kb, k1, c, v);
            consume(r, kb, k0, k1, c, v, are, aim);
        }
        if (k1 > whole) {
            const int k = (k0 > whole ? k0 : whole) + sl;
            if (k < k1) {
                const V a = ldv(reinterpret_cast<const V *>(RV ? st.vre : st.val), k);
                const int col = X16 ? ((int)r ^ (int)gmem(st.col16)[k]) : gmem(st.col)[k];
                if ((unsigned)(col - c_lo) < (unsigned)tc)
                    entry_fma(a, s_x[col - c_lo], are, aim);
            }
        }
        are = group_sum<L>(are);
        if (!RX)
            aim = group_sum<L>(aim);
        if (sl == 0 && r < r1) {
            if (accumulate) {
                are += gmem(part)[2 * r];
                aim += gmem(part)[2 * r + 1];
            }
            gmem(part)[2 * r] = are;
            gmem(part)[2 * r + 1] = aim;
        }
    };

    int cb[D][W];
    V vb[D][W];
    int kb0[D], kb1[D];
    int64_t rr[D];
#pragma unroll
    for (int d = 0; d < D; d++) {
        rr[d] = r0 + (wid + 16 * d) * G + sub;
        row_bounds(rr[d], kb0[d], kb1[d]);
        issue((kb0[d] & ~3) + 4 * sl, kb1[d], cb[d], vb[d]);
    }
    __builtin_amdgcn_sched_barrier(0);
    for (int64_t base = r0 + wid * G; base < r1; base += 16 * D * G) {
#pragma unroll
        for (int d = 0; d < D; d++) {
            {
                double are = 0.0, aim = 0.0;
                consume(rr[d], (kb0[d] & ~3) + 4 * sl, kb0[d], kb1[d], cb[d], vb[d], are, aim);
                finish(rr[d], kb0[d], kb1[d], are, aim);
            }
            rr[d] += 16 * D * G;
            row_bounds(rr[d], kb0[d], kb1[d]);
            issue((kb0[d] & ~3) + 4 * sl, kb1[d], cb[d], vb[d]);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}


template <int DT, int L, int D, int U, bool X16, bool RV>
__global__ void __launch_bounds__(1024) VQE_LDS_OCCUPANCY
k_spmv_tiled(const SpmvState *__restrict__ states, const int2 *__restrict__ tasks)
{
    const int2 task = tasks[blockIdx.x];
    if (task.x < 0)
        return;
    const SpmvState st = states[task.x];
    if (VQE_SKIP(st))
        return;
    const int blk = task.y >> 8, t = task.y & 0xff;
    using T = typename Elem<DT>::T;
    extern __shared__ unsigned char smem[];
    T *s_x = reinterpret_cast<T *>(smem);
    const int tid = threadIdx.x;
    const int64_t dim = st.dim;
    const int tc = st.tile_cols;
    const int c_lo = t * tc;
    const T *__restrict__ psi = reinterpret_cast<const T *>(st.psi);
    const int64_t r0 = (int64_t)blk * SPMV_LDS_ROWS;
    const int64_t r1 = r0 + SPMV_LDS_ROWS < dim ? r0 + SPMV_LDS_ROWS : dim;
    // the tile, one zero element (index tc), then the block's tile bounds.
    // With real values (RV) the plan's tiles are twice as wide: a tile with no
    // imaginary part is staged as its real parts in storage precision; a
    // complex one runs as two half-width passes (complex elements), each over
    // the rows' whole segments with the columns outside its half masked, the
    // second adding to the first's partials
    const size_t x_bytes = (size_t)((RV ? tc / 2 : tc) + 1) * sizeof(T);
    int32_t *s_k0 = reinterpret_cast<int32_t *>(smem + x_bytes);
    int32_t *s_k1 = s_k0 + SPMV_LDS_ROWS;
    stage_lds<2>(s_k0, st.tptr + (int64_t)t * dim + r0, r1 - r0, tid);
    stage_lds<2>(s_k1, st.tptr + (int64_t)(t + 1) * dim + r0, r1 - r0, tid);
    if constexpr (RV) {
        using R = typename ValOf<DT, true>::T;
        R *s_xr = reinterpret_cast<R *>(smem);
        const int cplx = stage_real_as<8, R>(s_xr, psi + c_lo, (int64_t)tc, tid);
        if (tid == 0)
            s_xr[tc] = (R)0;
        if (!__syncthreads_or(cplx)) {
            tiled_rows<DT, L, D, U, X16, RV, true>(st, t, c_lo, tc, false, smem, s_k0, s_k1, r0, r1);
            return;
        }
        const int th = tc / 2;
        for (int h = 0; h < 2; h++) {
            stage_lds<8>(s_x, psi + c_lo + h * th, (int64_t)th, tid);
            if (tid == 0)
                s_x[th] = T{};
            __syncthreads();
            tiled_rows<DT, L, D, U, X16, RV, false>(st, t, c_lo + h * th, th, h == 1, smem, s_k0,
                                                    s_k1, r0, r1);
            __syncthreads();      // every wave is done with this half
        }
        return;
    }
    stage_lds<8>(s_x, psi + c_lo, (int64_t)tc, tid);
    if (tid == 0)
        s_x[tc] = T{};
    __syncthreads();
    tiled_rows<DT, L, D, U, X16, RV, false>(st, t, c_lo, tc, false, smem, s_k0, s_k1, r0, r1);
}

// sigma_r = sum over tiles (ascending) of the tile partials; the energy sums.
template <int DT>
__global__ void __launch_bounds__(256)
k_spmv_tile_sum(const SpmvState *__restrict__ states, const int2 *__restrict__ tasks)
{
    const int2 task = tasks[blockIdx.x];
    if (task.x < 0)
        return;
    const SpmvState st = states[task.x];
    if (VQE_SKIP(st))
        return;
    const int64_t dim = st.dim;
    const int64_t r0 = (int64_t)task.y * SPMV_SUM_ROWS;
    const int64_t r1 = r0 + SPMV_SUM_ROWS < dim ? r0 + SPMV_SUM_ROWS : dim;
    double e_re = 0.0, e_im = 0.0, e_n2 = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) {
        double sr = 0.0, si = 0.0;
        for (int t = 0; t < st.ntiles; t++) {
            sr += gmem(st.tile_part)[((int64_t)t * dim + r) * 2];
            si += gmem(st.tile_part)[((int64_t)t * dim + r) * 2 + 1];
        }
        Elem<DT>::st(st.sigma, r, make_double2(sr, si));
        const double2 p = Elem<DT>::ld(st.psi, r);
        e_re += p.x * sr + p.y * si;
        e_im += p.x * si - p.y * sr;
        e_n2 += p.x * p.x + p.y * p.y;
    }
    __shared__ double s_part[4][3];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
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
        gmem(st.partials)[(int64_t)task.y * 3 + q] =
            ((s_part[0][q] + s_part[1][q]) + s_part[2][q]) + s_part[3][q];
    }
}

// ------------------------------------------------------------------ blocked layout
// The column-tiled product of states larger than LDS, blocked: the plan lays
// H out per (row block, column tile) slab (the entries of the block's rows
// whose columns fall in the tile, rows in order, each slab starting at a
// multiple of four entries), with 16-bit tile-local column codes (any state
// size, since a tile holds fewer than 2^16 columns) and the values (complex,
// interleaved).  One workgroup owns a row block and walks every tile in
// ascending order: it stages the tile of the state and the slab's row
// pointers in LDS, streams the slab with the pipelined row loop, and adds each
// row's sum to the row's FP64 accumulator in LDS; after the last tile it
// writes sigma and the energy partials.  Each slab is one contiguous stream,
// so no line is shared between two workgroups' reads, and no per-tile partial
// sums go through device memory.

// first k in [lo, hi) with col[k] >= lim (columns ascend within a row)
__device__ __forceinline__ int first_col_at_least(const int32_t *col, int lo, int hi, int64_t lim)
{
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((int64_t)col[mid] < lim)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// Step 1: the number of entries of row r in tile t, stored in the slab's
// row-pointer slot i + 1 (i = r - block * R); one thread per (row, tile),
// tiles fastest.  The slots start zeroed.
__global__ void __launch_bounds__(256)
k_blk_count(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col, int64_t dim,
            int32_t nt, int32_t tc, int32_t R, int32_t *__restrict__ brp)
{
    const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (gid >= dim * nt)
        return;
    const int64_t r = gid / nt;
    const int t = (int)(gid - r * nt);
    const int k0 = rowptr[r], k1 = rowptr[r + 1];
    const int lo = first_col_at_least(col, k0, k1, (int64_t)t * tc);
    const int hi = first_col_at_least(col, lo, k1, (int64_t)(t + 1) * tc);
    const int64_t b = r / R, i = r - b * R;
    brp[(b * nt + t) * (R + 1) + i + 1] = hi - lo;
}

// Step 2: per slab (one 256-thread workgroup), the row lengths in slots
// 1..R become the rows' starts (inclusive prefix sums: slot i = start of row
// i, slot R = the slab's length); the slab's length rounded up to four entries
// goes to blen.
__global__ void __launch_bounds__(256)
k_blk_scan(int32_t *__restrict__ brp, int32_t R, int64_t *__restrict__ blen)
{
    __shared__ int32_t s_tot[256];
    const int tid = threadIdx.x;
    int32_t *p = brp + (int64_t)blockIdx.x * (R + 1);
    const int per = (R + 255) / 256;
    const int a = 1 + tid * per;
    const int e = a + per < R + 1 ? a + per : R + 1;
    int32_t sum = 0;
    for (int i = a; i < e; i++)
        sum += p[i];
    s_tot[tid] = sum;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int32_t v = tid >= off ? s_tot[tid - off] : 0;
        __syncthreads();
        s_tot[tid] += v;
        __syncthreads();
    }
    int32_t run = s_tot[tid] - sum;
    for (int i = a; i < e; i++) {
        run += p[i];
        p[i] = run;
    }
    if (tid == 0)
        p[0] = 0;
    if (tid == 255)
        blen[blockIdx.x] = ((int64_t)s_tot[255] + 3) & ~(int64_t)3;
}

// Step 3: slab starts, the exclusive prefix sums of the rounded lengths
// (boff[n] = the total); one workgroup, each thread a contiguous run.
__global__ void __launch_bounds__(1024)
k_blk_offsets(const int64_t *__restrict__ blen, int64_t n, int64_t *__restrict__ boff)
{
    __shared__ int64_t s_sum[1024];
    const int tid = threadIdx.x;
    const int64_t per = (n + 1023) / 1024;
    const int64_t a = (int64_t)tid * per < n ? (int64_t)tid * per : n;
    const int64_t e = a + per < n ? a + per : n;
    int64_t tot = 0;
    for (int64_t i = a; i < e; i++)
        tot += blen[i];
    s_sum[tid] = tot;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t v = tid >= off ? s_sum[tid - off] : 0;
        __syncthreads();
        s_sum[tid] += v;
        __syncthreads();
    }
    int64_t run = s_sum[tid] - tot;
    for (int64_t i = a; i < e; i++) {
        boff[i] = run;
        run += blen[i];
    }
    if (tid == 1023)
        boff[n] = s_sum[1023];
}

// Step 4: copy row r's entries of tile t into its slab (codes col - t * tc),
// one thread per (row, tile); the entries between one slab's end and the next
// slab's start are set to zero by the thread of the block's last row.
template <int DT>
__global__ void __launch_bounds__(256)
k_blk_fill(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
           const void *__restrict__ val, int64_t dim, int32_t nt, int32_t tc, int32_t R,
           const int32_t *__restrict__ brp, const int64_t *__restrict__ boff,
           uint16_t *__restrict__ bcode, void *__restrict__ bval)
{
    using T = typename Elem<DT>::T;
    const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (gid >= dim * nt)
        return;
    const int64_t r = gid / nt;
    const int t = (int)(gid - r * nt);
    const int k0 = rowptr[r], k1 = rowptr[r + 1];
    const int lo = first_col_at_least(col, k0, k1, (int64_t)t * tc);
    const int hi = first_col_at_least(col, lo, k1, (int64_t)(t + 1) * tc);
    const int64_t b = r / R, i = r - b * R;
    const int64_t slab = b * nt + t;
    const int32_t *rp = brp + slab * (R + 1);
    const int64_t dst = boff[slab] + rp[i];
    const T *v = reinterpret_cast<const T *>(val);
    T *bv = reinterpret_cast<T *>(bval);
    for (int k = lo; k < hi; k++) {
        bcode[dst + (k - lo)] = (uint16_t)(col[k] - t * tc);
        bv[dst + (k - lo)] = v[k];
    }
    const int64_t rows = dim - b * R < R ? dim - b * R : R;
    if (i == rows - 1)
        for (int64_t k = boff[slab] + rp[rows]; k < boff[slab + 1]; k++) {
            bcode[k] = 0;
            bv[k] = T{};
        }
}

// The rows of one slab of a blocked state (tile of the state at s_x, its
// zero element at index w; the slab's row pointers at s_rp): the pipelined row
// loop of the LDS schedule with L lanes per row, U groups of four entries per
// lane per pass and D rows in flight per sub-group; each row's sum is added to
// its FP64 accumulator in LDS.
template <int DT, int L, int D, int U>
__device__ __forceinline__ void blk_rows(const SpmvState &st, int64_t slab, int w,
                                         const typename Elem<DT>::T *s_x, const int32_t *s_rp,
                                         double2 *s_acc, int nrows)
{
    using T = typename Elem<DT>::T;
    constexpr int W = U * 4;                 // entries per lane per pass
    constexpr int PASS = W * L;              // entries per sub-group per pass
    constexpr unsigned EB = sizeof(T);
    constexpr int G = VQE_WAVE / L;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
    const int sub = lane / L, sl = lane % L;
    const int64_t base = st.boff[slab];
    const int nrec = (s_rp[nrows] + 3) & ~3;   // the slab's entries, whole groups
    const __amdgpu_buffer_rsrc_t rc = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(st.bcode + base), (short)0, nrec * 2, VQE_BUF_WORD3);
    const __amdgpu_buffer_rsrc_t rv = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(reinterpret_cast<const T *>(st.bval) + base), (short)0, (int)(nrec * EB),
        VQE_BUF_WORD3);

    auto issue = [&](int kb, int k1, int c[W], T v[W]) {
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int k = kb + u * 4 * L;
            const bool ok = k < k1;
            typedef unsigned v2u __attribute__((ext_vector_type(2)));
            const v2u c2 = __builtin_amdgcn_raw_buffer_load_b64(rc, ok ? (unsigned)k * 2u : VQE_BUF_OOB, 0, 0);
            c[4 * u + 0] = (int)(c2.x & 0xffffu);
            c[4 * u + 1] = (int)(c2.x >> 16);
            c[4 * u + 2] = (int)(c2.y & 0xffffu);
            c[4 * u + 3] = (int)(c2.y >> 16);
            BufVal<DT, false>::load(rv, ok ? (unsigned)k * EB : VQE_BUF_OOB, v + 4 * u);
        }
    };
    // entries outside the row [k0, k1) read the zero element
    auto consume = [&](int kb, int k0, int k1, const int c[W], const T v[W], double &are,
                       double &aim) {
        int cm[W];
        const unsigned len = (unsigned)(k1 - k0);
#pragma unroll
        for (int u = 0; u < U; u++)
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int k = kb + u * 4 * L + q;
                cm[4 * u + q] = (unsigned)(k - k0) < len ? c[4 * u + q] : w;
            }
        lds_gather_fma<T, T, W>(s_x, cm, v, are, aim);
    };
    auto row_bounds = [&](int i, int &k0, int &k1) {
        if (i < nrows) {
            k0 = s_rp[i];
            k1 = s_rp[i + 1];
        } else {
            k0 = k1 = 0;
        }
    };
    auto finish = [&](int i, int k0, int k1, double are, double aim) {
        for (int kb = (k0 & ~3) + 4 * sl + PASS; kb - 4 * sl < k1; kb += PASS) {
            int c[W];
            T v[W];
            issue(kb, k1, c, v);
            consume(kb, k0, k1, c, v, are, aim);
        }
        are = group_sum<L>(are);
        aim = group_sum<L>(aim);
        if (sl == 0 && i < nrows) {
            const double2 a = s_acc[i];
            s_acc[i] = make_double2(a.x + are, a.y + aim);
        }
    };

    int cb[D][W];
    T vb[D][W];
    int kb0[D], kb1[D], rr[D];
#pragma unroll
    for (int d = 0; d < D; d++) {
        rr[d] = (wid + 16 * d) * G + sub;
        row_bounds(rr[d], kb0[d], kb1[d]);
        issue((kb0[d] & ~3) + 4 * sl, kb1[d], cb[d], vb[d]);
    }
    __builtin_amdgcn_sched_barrier(0);
    for (int row = wid * G; row < nrows; row += 16 * D * G) {
#pragma unroll
        for (int d = 0; d < D; d++) {
            {
                double are = 0.0, aim = 0.0;
                consume((kb0[d] & ~3) + 4 * sl, kb0[d], kb1[d], cb[d], vb[d], are, aim);
                finish(rr[d], kb0[d], kb1[d], are, aim);
            }
            rr[d] += 16 * D * G;
            row_bounds(rr[d], kb0[d], kb1[d]);
            issue((kb0[d] & ~3) + 4 * sl, kb1[d], cb[d], vb[d]);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// The blocked product's kernel: one workgroup per (state, row block).
template <int DT, int L, int D, int U>
__global__ void __launch_bounds__(1024) VQE_LDS_OCCUPANCY
k_spmv_blk(const SpmvState *__restrict__ states, const int2 *__restrict__ tasks)
{
    const int2 task = tasks[blockIdx.x];
    if (task.x < 0)
        return;
    const SpmvState st = states[task.x];
    if (VQE_SKIP(st))
        return;
    using T = typename Elem<DT>::T;
    extern __shared__ unsigned char smem[];
    const int tid = threadIdx.x;
    const int64_t dim = st.dim;
    const int R = st.blk_rows, tc = st.tile_cols, nt = st.ntiles;
    const int b = task.y;
    const int64_t r0 = (int64_t)b * R;
    const int nrows = (int)(dim - r0 < R ? dim - r0 : R);
    // LDS: the rows' accumulators, the tile (and its zero element), the
    // slab's row pointers
    double2 *s_acc = reinterpret_cast<double2 *>(smem);
    T *s_x = reinterpret_cast<T *>(smem + (size_t)R * sizeof(double2));
    int32_t *s_rp = reinterpret_cast<int32_t *>(smem + (size_t)R * sizeof(double2) +
                                                (size_t)(tc + 1) * sizeof(T));
    const T *__restrict__ psi = reinterpret_cast<const T *>(st.psi);
    for (int i = tid; i < nrows; i += 1024)
        s_acc[i] = make_double2(0.0, 0.0);
    for (int t = 0; t < nt; t++) {
        const int64_t c_lo = (int64_t)t * tc;
        const int w = (int)(dim - c_lo < tc ? dim - c_lo : tc);
        const int64_t slab = (int64_t)b * nt + t;
        __syncthreads();      // every wave is done with the previous tile
        stage_lds<2>(s_rp, st.brp + slab * (R + 1), nrows + 1, tid);
        stage_lds<8>(s_x, psi + c_lo, w, tid);
        if (tid == 0)
            s_x[w] = T{};
        __syncthreads();
        blk_rows<DT, L, D, U>(st, slab, w, s_x, s_rp, s_acc, nrows);
    }
    __syncthreads();
    double e_re = 0.0, e_im = 0.0, e_n2 = 0.0;
    for (int i = tid; i < nrows; i += 1024) {
        const double2 a = s_acc[i];
        Elem<DT>::st(st.sigma, r0 + i, a);
        energy_terms(ldg(psi, r0 + i), a.x, a.y, e_re, e_im, e_n2);
    }
    __shared__ double s_part[16][3];
    const int lane = tid & 63, wid = tid >> 6;
    e_re = wave_sum(e_re);
    e_im = wave_sum(e_im);
    e_n2 = wave_sum(e_n2);
    if (lane == 0) {
        s_part[wid][0] = e_re;
        s_part[wid][1] = e_im;
        s_part[wid][2] = e_n2;
    }
    __syncthreads();
    if (tid < 3) {
        double v = 0.0;
        for (int q = 0; q < 16; q++)
            v += s_part[q][tid];
        gmem(st.partials)[(int64_t)b * 3 + tid] = v;
    }
}

// Per-tile row bounds: the first entry of row r with column >= t * tile_cols.
__global__ void __launch_bounds__(256)
k_tile_bounds(const SpmvState *__restrict__ states, const int2 *__restrict__ tasks)
{
    const int2 task = tasks[blockIdx.x];
    if (task.x < 0)
        return;
    const SpmvState st = states[task.x];
    const int64_t r = (int64_t)task.y * 256 + threadIdx.x;
    if (r >= st.dim)
        return;
    const int k0 = st.rowptr[r], k1 = st.rowptr[r + 1];
    int32_t *tp = const_cast<int32_t *>(st.tptr);
    tp[r] = k0;
    for (int t = 1; t < st.ntiles; t++) {
        const int lim = t * st.tile_cols;
        int lo = k0, hi = k1;   // first k in [k0, k1) with col[k] >= lim
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (st.col[mid] < lim)
                lo = mid + 1;
            else
                hi = mid;
        }
        tp[(int64_t)t * st.dim + r] = lo;
    }
    tp[(int64_t)st.ntiles * st.dim + r] = k1;
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
    if (VQE_SKIP(st))
        return;
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

template <int DT, int L, int V>
static void launch_spmv_t(const SpmvState &single, const SpmvState *states, const int2 *tasks,
                          unsigned grid, hipStream_t s)
{
    if (tasks)
        k_spmv_energy<DT, L, V, true><<<grid, 256, 0, s>>>(single, states, tasks);
    else
        k_spmv_energy<DT, L, V, false><<<grid, 256, 0, s>>>(single, states, tasks);
}

template <int DT, int L, int U>
static void launch_spmv_lds_t(const SpmvState &single, const SpmvState *states, const int2 *tasks,
                              unsigned grid, hipStream_t s, size_t lds)
{
    if (tasks) {
        auto k = k_spmv_lds<DT, L, U, true>;
        (void)hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds);
        k<<<grid, 1024, lds, s>>>(single, states, tasks);
    } else {
        auto k = k_spmv_lds<DT, L, U, false>;
        (void)hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds);
        k<<<grid, 1024, lds, s>>>(single, states, tasks);
    }
}

template <int DT, int L, int D, bool X16 = false, bool RV = false, bool PL = RV>
static void launch_spmv_pf_t(const SpmvState &single, const SpmvState *states, const int2 *tasks,
                             unsigned grid, hipStream_t s, size_t lds)
{
    if (tasks) {
        auto k = k_spmv_lds_pf<DT, L, D, true, X16, RV, PL>;
        (void)hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds);
        k<<<grid, 1024, lds, s>>>(single, states, tasks);
    } else {
        auto k = k_spmv_lds_pf<DT, L, D, false, false, false, false>;
        (void)hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds);
        k<<<grid, 1024, lds, s>>>(single, states, tasks);
    }
}

// Sliced schedules: E entries per lane and load group, D groups in flight;
// rv: the real parts of the values (VQE_SPMV_REAL).
template <int DT, int E, int D, bool XI = false>
static void launch_sell_t(const SpmvState *states, const int2 *tasks, unsigned grid, hipStream_t s,
                          size_t lds, bool rv)
{
    // the state (with its zero element; lds counts it with the row pointers
    // of the other LDS schedules), in FP32 storage a block of results, and
    // the flip masks of the index form
    lds = lds - (SPMV_LDS_ROWS + 1) * sizeof(int32_t) +
          (DT == VQE_C64 ? SPMV_LDS_ROWS * sizeof(float2) : 0) + (XI ? SPMV_XIDX_MAX * sizeof(uint16_t) : 0);
    auto k = rv ? k_spmv_sell<DT, E, D, true, XI> : k_spmv_sell<DT, E, D, false, XI>;
    (void)hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    k<<<grid, 1024, lds, s>>>(states, tasks);
}

template <int DT>
static void launch_spmv_dt(int sched, const SpmvState &single, const SpmvState *states,
                           const int2 *tasks, unsigned grid, hipStream_t s, size_t lds)
{
    if ((sched & VQE_SPMV_SLICED) && tasks) {
        // the sliced layout exists only in batch plans; E = 2, 4 or 8
        // (FP64 values keep half as many groups in flight: the registers)
        constexpr bool W = DT == VQE_C128;
        const bool rv = (sched & VQE_SPMV_REAL) != 0;
        if (sched & VQE_SPMV_XIDX) {
            if ((sched & 0xff) == 3)
                launch_sell_t<DT, 3, W ? 2 : 6, true>(states, tasks, grid, s, lds, rv);
            else
                launch_sell_t<DT, 6, W ? 1 : 3, true>(states, tasks, grid, s, lds, rv);
            return;
        }
        switch (sched & 0xff) {
        case 2: launch_sell_t<DT, 2, W ? 2 : 4>(states, tasks, grid, s, lds, rv); return;
        case 8: launch_sell_t<DT, 8, W ? 1 : 2>(states, tasks, grid, s, lds, rv); return;
        default: launch_sell_t<DT, 4, W ? 2 : 3>(states, tasks, grid, s, lds, rv); return;
        }
    }
    constexpr int D = VQE_SPMV_LDS | VQE_SPMV_DEEP;
    constexpr int P = VQE_SPMV_LDS | VQE_SPMV_PREFETCH;
    constexpr int X = P | VQE_SPMV_X16;
    constexpr int R = X | VQE_SPMV_REAL;
    constexpr int Q = X | VQE_SPMV_PAD;
    switch (sched) {
    // the 16-bit column form, the padded layout and the real values exist
    // only in batch plans (tasks non-null)
    case 16 | Q: launch_spmv_pf_t<DT, 16, 2, true, false, true>(single, states, tasks, grid, s, lds); return;
    case 32 | Q: launch_spmv_pf_t<DT, 32, 2, true, false, true>(single, states, tasks, grid, s, lds); return;
    case 64 | Q: launch_spmv_pf_t<DT, 64, 2, true, false, true>(single, states, tasks, grid, s, lds); return;
    case 32 | Q | VQE_SPMV_DEEP: launch_spmv_pf_t<DT, 32, 3, true, false, true>(single, states, tasks, grid, s, lds); return;
    case 64 | Q | VQE_SPMV_DEEP: launch_spmv_pf_t<DT, 64, 3, true, false, true>(single, states, tasks, grid, s, lds); return;
    case 16 | R: launch_spmv_pf_t<DT, 16, 2, true, true>(single, states, tasks, grid, s, lds); return;
    case 32 | R: launch_spmv_pf_t<DT, 32, 2, true, true>(single, states, tasks, grid, s, lds); return;
    case 64 | R: launch_spmv_pf_t<DT, 64, 2, true, true>(single, states, tasks, grid, s, lds); return;
    case 32 | R | VQE_SPMV_DEEP: launch_spmv_pf_t<DT, 32, 3, true, true>(single, states, tasks, grid, s, lds); return;
    case 64 | R | VQE_SPMV_DEEP: launch_spmv_pf_t<DT, 64, 3, true, true>(single, states, tasks, grid, s, lds); return;
    case 32 | X: launch_spmv_pf_t<DT, 32, 2, true>(single, states, tasks, grid, s, lds); return;
    case 64 | X: launch_spmv_pf_t<DT, 64, 2, true>(single, states, tasks, grid, s, lds); return;
    case 32 | X | VQE_SPMV_DEEP: launch_spmv_pf_t<DT, 32, 3, true>(single, states, tasks, grid, s, lds); return;
    case 64 | X | VQE_SPMV_DEEP: launch_spmv_pf_t<DT, 64, 3, true>(single, states, tasks, grid, s, lds); return;
    case 32 | P: launch_spmv_pf_t<DT, 32, 2>(single, states, tasks, grid, s, lds); return;
    case 64 | P: launch_spmv_pf_t<DT, 64, 2>(single, states, tasks, grid, s, lds); return;
    case 32 | P | VQE_SPMV_DEEP: launch_spmv_pf_t<DT, 32, 3>(single, states, tasks, grid, s, lds); return;
    case 64 | P | VQE_SPMV_DEEP: launch_spmv_pf_t<DT, 64, 3>(single, states, tasks, grid, s, lds); return;
    default: break;
    }
    switch (sched) {
    case 8 | VQE_SPMV_LDS: launch_spmv_lds_t<DT, 8, 2>(single, states, tasks, grid, s, lds); return;
    case 16 | VQE_SPMV_LDS: launch_spmv_lds_t<DT, 16, 2>(single, states, tasks, grid, s, lds); return;
    case 32 | VQE_SPMV_LDS: launch_spmv_lds_t<DT, 32, 2>(single, states, tasks, grid, s, lds); return;
    case 64 | VQE_SPMV_LDS: launch_spmv_lds_t<DT, 64, 1>(single, states, tasks, grid, s, lds); return;
    case 8 | D: launch_spmv_lds_t<DT, 8, 4>(single, states, tasks, grid, s, lds); return;
    case 16 | D: launch_spmv_lds_t<DT, 16, 4>(single, states, tasks, grid, s, lds); return;
    case 32 | D: launch_spmv_lds_t<DT, 32, 4>(single, states, tasks, grid, s, lds); return;
    case 64 | D: launch_spmv_lds_t<DT, 64, 2>(single, states, tasks, grid, s, lds); return;
    default: break;
    }
    switch (sched) {
    case 8: launch_spmv_t<DT, 8, 1>(single, states, tasks, grid, s); break;
    case 16: launch_spmv_t<DT, 16, 1>(single, states, tasks, grid, s); break;
    case 32: launch_spmv_t<DT, 32, 1>(single, states, tasks, grid, s); break;
    case 64: launch_spmv_t<DT, 64, 1>(single, states, tasks, grid, s); break;
    case 16 | VQE_SPMV_VEC4: launch_spmv_t<DT, 16, 4>(single, states, tasks, grid, s); break;
    case 32 | VQE_SPMV_VEC4: launch_spmv_t<DT, 32, 4>(single, states, tasks, grid, s); break;
    default: launch_spmv_t<DT, 64, 4>(single, states, tasks, grid, s); break;
    }
}

// ------------------------------------------------------------------ sliced, column-tiled
// VQE_SPMV_SLICED on a state larger than LDS: slabs of a block of
// SPMV_SELLT_ROWS rows against one column tile of SPMV_SELLT_TILE_BYTES are
// each sorted and sliced like the sliced layout, by the rows' segment lengths
// in the tile.  srow[slab * R + i] is the
// block-local row at sorted position i of the slab; sslice[slab *
// SPMV_SLICES_PER_BLOCK + k] = (start relative to the slab's boff[slab],
// entries per lane); codes are tile-local (col - t * tile_cols); a pad takes
// the column of its slice's first entry (so it reads a staged element) and
// the value zero.  One workgroup per row block walks the tiles with its rows'
// FP64 sums in LDS, as the blocked product.

// Layout step 1: per (row block, tile), the row's entries in the tile; one
// thread per row (tiles in turn; columns ascending).
__global__ void __launch_bounds__(256)
k_sellt_count(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col, int64_t dim,
              int32_t nt, int32_t tc, int32_t R, uint16_t *__restrict__ cnt)
{
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= dim)
        return;
    const int64_t b = r / R, i = r - b * R;
    int k = rowptr[r];
    const int k1 = rowptr[r + 1];
    for (int t = 0; t < nt; t++) {
        const int k2 = first_col_at_least(col, k, k1, (int64_t)(t + 1) * tc);
        cnt[(b * nt + t) * R + i] = (uint16_t)(k2 - k);
        k = k2;
    }
}

// Step 2: one workgroup per slab sorts the block's rows by their entries in
// the tile (longest first, ties by row; in place: the counts become the row
// order) and writes the slab's slices (start in the slab, length rounded up
// to E) and its total entries, and clears its part mask.
__global__ void __launch_bounds__(1024)
k_sellt_sort(int64_t dim, int32_t nt, int E, uint16_t *__restrict__ cnt_row,
             int2 *__restrict__ sslice, int64_t *__restrict__ stot, uint32_t *__restrict__ smask)
{
    constexpr int R = SPMV_SELLT_ROWS, RK = 2048;   // rows, keys (a power of two)
    static_assert(R <= RK && (RK + VQE_WAVE - 1) / VQE_WAVE <= SPMV_SLICES_PER_BLOCK, "block size");
    __shared__ uint32_t key[RK];
    const int tid = threadIdx.x;
    const int64_t slab = blockIdx.x;
    const int64_t r0 = (slab / nt) * R;
    const int n = (int)(dim - r0 < R ? dim - r0 : R);
    uint16_t *c = cnt_row + slab * R;
    for (int i = tid; i < RK; i += 1024)
        key[i] = i < n ? ((0xffffu - (uint32_t)c[i]) << 16) | (uint32_t)i : 0xffffffffu;
    __syncthreads();
    for (int k = 2; k <= RK; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = tid; i < RK; i += 1024) {
                const int q = i ^ j;
                if (q > i) {
                    const uint32_t a = key[i], b = key[q];
                    if ((a > b) == ((i & k) == 0)) {
                        key[i] = b;
                        key[q] = a;
                    }
                }
            }
            __syncthreads();
        }
    for (int i = tid; i < n; i += 1024)
        c[i] = (uint16_t)(key[i] & 0xffffu);
    if (tid == 0) {
        int at = 0;
        for (int k = 0; k < SPMV_SLICES_PER_BLOCK; k++) {
            int len = 0;
            if (k * VQE_WAVE < n) {
                len = (int)(0xffffu - (key[k * VQE_WAVE] >> 16));
                len = (len + E - 1) / E * E;
            }
            sslice[slab * SPMV_SLICES_PER_BLOCK + k] = make_int2(at, len);
            at += len * VQE_WAVE;
        }
        stot[slab] = at;
        smask[slab] = 0;     // the fill sets the parts the codes reach
    }
}

// Step 3: the slabs' starts (exclusive prefix of their totals) and the
// layout's total entries; one workgroup.
__global__ void __launch_bounds__(1024)
k_sellt_scan(const int64_t *__restrict__ stot, int64_t nslab, int64_t *__restrict__ sbase,
             int64_t *__restrict__ total)
{
    __shared__ int64_t part[1024];
    const int tid = threadIdx.x;
    const int64_t per = (nslab + 1023) / 1024;
    const int64_t lo = (int64_t)tid * per < nslab ? (int64_t)tid * per : nslab;
    const int64_t hi = lo + per < nslab ? lo + per : nslab;
    int64_t sum = 0;
    for (int64_t j = lo; j < hi; j++)
        sum += stot[j];
    part[tid] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int64_t at = part[tid] - sum;
    for (int64_t j = lo; j < hi; j++) {
        sbase[j] = at;
        at += stot[j];
    }
    if (tid == 1023)
        *total = part[1023];
}

// Step 4: codes and values, one wave per slice (empty slices return), and
// the tile parts the slice's columns reach, ORed into its slab's mask.
template <int DT>
__global__ void __launch_bounds__(64)
k_sellt_fill(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
             const void *__restrict__ val, int64_t dim, int32_t nt, int32_t tc, int E,
             const uint16_t *__restrict__ srow, const int2 *__restrict__ sslice,
             const int64_t *__restrict__ sbase, uint16_t *__restrict__ code, void *__restrict__ sval,
             uint32_t *__restrict__ smask)
{
    using T = typename Elem<DT>::T;
    constexpr int R = SPMV_SELLT_ROWS;
    const int64_t q = blockIdx.x;
    const int2 sl = sslice[q];
    if (sl.y == 0)
        return;
    const int64_t slab = q / SPMV_SLICES_PER_BLOCK;
    const int k = (int)(q - slab * SPMV_SLICES_PER_BLOCK);
    const int64_t b = slab / nt;
    const int t = (int)(slab - b * nt);
    const int64_t r0 = b * R;
    const int n = (int)(dim - r0 < R ? dim - r0 : R);
    const int lane = threadIdx.x;
    const int i = k * VQE_WAVE + lane;
    const int64_t c_lo = (int64_t)t * tc;
    int k0 = 0, len = 0;
    if (i < n) {
        const int64_t row = r0 + srow[slab * R + i];
        const int a = rowptr[row], e = rowptr[row + 1];
        k0 = first_col_at_least(col, a, e, c_lo);
        len = first_col_at_least(col, k0, e, c_lo + tc) - k0;
    }
    T *out = reinterpret_cast<T *>(sval);
    const T *in = reinterpret_cast<const T *>(val);
    const int64_t base = sbase[slab] + sl.x;
    constexpr int PART = SPMV_SELLT_PART_BYTES / (int)sizeof(T);
    // the pads' column: the slice's first entry (lane 0 holds its longest row)
    const int cpad = __shfl(len > 0 ? col[k0] - (int)c_lo : 0, 0);
    uint32_t parts = 0;
    for (int j = 0; j < sl.y; j++) {
        const int64_t at = base + ((int64_t)(j / E) * VQE_WAVE + lane) * E + j % E;
        const int c = j < len ? col[k0 + j] - (int)c_lo : cpad;
        code[at] = (uint16_t)c;
        out[at] = j < len ? in[k0 + j] : T{};
        if (j < len)
            parts |= 1u << (c / PART);
    }
    for (int off = VQE_WAVE / 2; off > 0; off >>= 1)
        parts |= (uint32_t)__shfl_xor((int)parts, off);
    if (lane == 0 && parts)
        atomicOr(smask + slab, parts);
}

// The product: one workgroup per (state, row block); per tile with entries,
// the parts of the tile that the slab reaches staged in LDS, each wave takes
// two of the slab's slices, every lane sums its
// row's segment with D groups of E entries in flight and adds it to the row's
// FP64 sums in LDS (each row once per slab, tiles in ascending order).
template <int DT, int E, int D, bool PF>
__global__ void __launch_bounds__(1024) VQE_LDS_OCCUPANCY
k_spmv_sellt(const SpmvState *__restrict__ states, const int2 *__restrict__ tasks)
{
    const int2 task = tasks[blockIdx.x];
    if (task.x < 0)
        return;
    const SpmvState st = states[task.x];
    if (VQE_SKIP(st))
        return;
    using T = typename Elem<DT>::T;
    constexpr int R = SPMV_SELLT_ROWS;
    extern __shared__ unsigned char smem[];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t dim = st.dim;
    const int tc = st.tile_cols, nt = st.ntiles;
    const int b = task.y;
    const int64_t r0 = (int64_t)b * R;
    const int n = (int)(dim - r0 < R ? dim - r0 : R);
    double2 *s_acc = reinterpret_cast<double2 *>(smem);
    T *s_x = reinterpret_cast<T *>(smem + (size_t)R * sizeof(double2));
    const T *__restrict__ psi = reinterpret_cast<const T *>(st.psi);
    const uint16_t *__restrict__ code = st.scode;
    const T *__restrict__ val = reinterpret_cast<const T *>(st.sval);
    for (int i = tid; i < n; i += 1024)
        s_acc[i] = make_double2(0.0, 0.0);
    constexpr int64_t STEP = (int64_t)VQE_WAVE * E;
    // A tile is loaded into registers (16 bytes per thread and part) and
    // written to LDS between the tiles' barriers, only the parts of the tile
    // that the slab's columns reach; with PF the next tile's loads are issued
    // while the current tile is multiplied.  A tile's bytes are a multiple of
    // 16 (dim and the tile width are even) and start 16-byte aligned.
    constexpr int SP = SPMV_SELLT_TILE_BYTES / SPMV_SELLT_PART_BYTES;
    static_assert(SPMV_SELLT_PART_BYTES == 16 * 1024 && SP <= 32, "a part is 16 bytes per thread");
    vqe_v4f pre[SP];
    auto fetch = [&](int t, uint32_t parts) {
        const int64_t c_lo = (int64_t)t * tc;
        const int64_t nbytes = (dim - c_lo < tc ? dim - c_lo : tc) * (int64_t)sizeof(T);
        const vqe_v4f *src = reinterpret_cast<const vqe_v4f *>(psi + c_lo);
#pragma unroll
        for (int u = 0; u < SP; u++) {
            const int c = tid + 1024 * u;
            if (((parts >> u) & 1u) && (int64_t)c * 16 < nbytes)
                pre[u] = gmem(src)[c];
        }
        return nbytes;
    };
    // the slabs' part masks, 64 tiles at a time one per lane, and the tiles
    // with entries in this block as a bit mask of that window
    int win = -1;
    uint32_t pv = 0u;
    uint64_t live = 0ull;
    auto load_window = [&](int w) {
        win = w;
        const int tl = w * 64 + lane;
        pv = tl < nt ? gmem(st.smask)[(int64_t)b * nt + tl] : 0u;
        live = __builtin_amdgcn_ballot_w64(pv != 0u);
    };
    // the first tile at or after t with entries in this block (nt: none)
    auto next_tile = [&](int t) {
        while (t < nt) {
            if ((t >> 6) != win)
                load_window(t >> 6);
            const uint64_t m = live & (~0ull << (t & 63));
            if (m)
                return win * 64 + (int)__builtin_ctzll(m);
            t = (win + 1) * 64;
        }
        return nt;
    };
    auto parts_at = [&](int t) {   // t in the current window
        return (uint32_t)__builtin_amdgcn_readlane((int)pv, t & 63);
    };
    // wave w takes slices w and 31 - w of each slab (longest with shortest:
    // the slices are sorted longest first)
    static_assert(SPMV_SLICES_PER_BLOCK == 32, "two slices per wave");
    const int ka = wid, kb = SPMV_SLICES_PER_BLOCK - 1 - wid;
    int t = next_tile(0);
    uint32_t parts = 0u;
    int64_t staged = 0;
    if (PF && t < nt) {
        parts = parts_at(t);
        staged = fetch(t, parts);
    }
    while (t < nt) {
        const int64_t slab = (int64_t)b * nt + t;
        const uint32_t here = PF ? parts : parts_at(t);
        if (!PF)
            staged = fetch(t, here);
        // the slab's tables, loaded before the barriers: its start, the two
        // slices and the rows their lanes take (clamped to the block)
        const sell_v2i *sls = reinterpret_cast<const sell_v2i *>(st.sslice) + slab * SPMV_SLICES_PER_BLOCK;
        const int64_t base = gmem(st.boff)[slab];
        const sell_v2i sl2[2] = {gmem(sls)[ka], gmem(sls)[kb]};
        const uint16_t *srow = st.srow + slab * R;
        const int ia = ka * VQE_WAVE + lane, ib = kb * VQE_WAVE + lane;
        const int rl2[2] = {gmem(srow)[ia < n ? ia : n - 1], gmem(srow)[ib < n ? ib : n - 1]};
        __syncthreads();      // every wave is done with the previous tile
#pragma unroll
        for (int u = 0; u < SP; u++) {
            const int c = tid + 1024 * u;
            if (((here >> u) & 1u) && (int64_t)c * 16 < staged)
                reinterpret_cast<vqe_v4f *>(s_x)[c] = pre[u];
        }
        __syncthreads();
        const int tn = next_tile(t + 1);
        if (PF && tn < nt) {
            parts = parts_at(tn);
            staged = fetch(tn, parts);
        }
        // the wave's two slices as one stream of groups (the first slice's,
        // then the second's), so that the second slice's first groups load
        // while the first one finishes; each slice sums into its own pair
        const int nga = __builtin_amdgcn_readfirstlane(sl2[0].y) / E;
        const int ngb = __builtin_amdgcn_readfirstlane(sl2[1].y) / E;
        if (nga > 0) {
            const int ng = nga + ngb;
            const int64_t ata = base + __builtin_amdgcn_readfirstlane(sl2[0].x) + lane * E;
            const int64_t atb = base + __builtin_amdgcn_readfirstlane(sl2[1].x) + lane * E - (int64_t)nga * STEP;
            // stream group p (clamped to the last) and its address
            auto addr = [&](int p) {
                const int pc = p < ng ? p : ng - 1;
                return (pc < nga ? ata : atb) + (int64_t)pc * STEP;
            };
            // one running sum; at the second slice's first group the first
            // slice's sum is set aside and the sum restarts
            double are = 0.0, aim = 0.0;
            double2 sa = make_double2(0.0, 0.0), sb;
            SellGroup<DT, E> g[D];
#pragma unroll
            for (int d = 0; d < D; d++)
                g[d].load(code, val, addr(d));
            int q = 0;
            for (; q + D <= ng; q += D) {
#pragma unroll
                for (int d = 0; d < D; d++) {
                    if (q + d == nga) {
                        sa = make_double2(are, aim);
                        are = aim = 0.0;
                    }
                    g[d].use(s_x, are, aim);
                    g[d].load(code, val, addr(q + D + d));
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
#pragma unroll
            for (int d = 0; d < D; d++)
                if (q + d < ng) {
                    if (q + d == nga) {
                        sa = make_double2(are, aim);
                        are = aim = 0.0;
                    }
                    g[d].use(s_x, are, aim);
                }
            if (ngb == 0)
                sa = make_double2(are, aim);
            sb = make_double2(are, aim);
            if (ka * VQE_WAVE + lane < n) {
                double2 a = s_acc[rl2[0]];
                a.x += sa.x;
                a.y += sa.y;
                s_acc[rl2[0]] = a;
            }
            if (ngb > 0 && kb * VQE_WAVE + lane < n) {
                double2 a = s_acc[rl2[1]];
                a.x += sb.x;
                a.y += sb.y;
                s_acc[rl2[1]] = a;
            }
        }
        t = tn;
    }
    __syncthreads();
    double e_re = 0.0, e_im = 0.0, e_n2 = 0.0;
    for (int i = tid; i < n; i += 1024) {
        const double2 a = s_acc[i];
        Elem<DT>::st(st.sigma, r0 + i, a);
        energy_terms(ldg(psi, r0 + i), a.x, a.y, e_re, e_im, e_n2);
    }
    // the waves' energy sums in the tile's space (the tiles are done): the
    // rows' sums and one tile fill the LDS
    double (*s_part)[3] = reinterpret_cast<double (*)[3]>(s_x);
    e_re = wave_sum(e_re);
    e_im = wave_sum(e_im);
    e_n2 = wave_sum(e_n2);
    if (lane == 0) {
        s_part[wid][0] = e_re;
        s_part[wid][1] = e_im;
        s_part[wid][2] = e_n2;
    }
    __syncthreads();
    if (tid < 3) {
        double v = 0.0;
        for (int q = 0; q < 16; q++)
            v += s_part[q][tid];
        gmem(st.partials)[(int64_t)b * 3 + tid] = v;
    }
}

int32_t spmv_blk_tile_cols(int dtype) { return (int32_t)(SPMV_BLK_TILE_BYTES / vqe_elem_bytes(dtype)); }
int32_t spmv_sellt_tile_cols(int dtype) { return (int32_t)(SPMV_SELLT_TILE_BYTES / vqe_elem_bytes(dtype)); }

size_t spmv_blk_lds(int dtype)
{
    return (size_t)SPMV_BLK_ROWS * 2 * sizeof(double) +
           (size_t)(spmv_blk_tile_cols(dtype) + 1) * vqe_elem_bytes(dtype) +
           (size_t)(SPMV_BLK_ROWS + 1) * sizeof(int32_t);
}

// Blocked schedules: L lanes per row (4, 8, 16, 32 or 64); VQE_SPMV_X16 gives
// each lane two groups of four entries per pass instead of one; VQE_SPMV_DEEP
// keeps four rows per sub-group in flight instead of two (short segments carry
// few bytes per row, so narrow sub-groups need many rows in flight).
template <int DT, int L, int D, int U>
static void launch_blk_t(const SpmvState *states, const int2 *tasks, unsigned grid, hipStream_t s)
{
    const size_t lds = spmv_blk_lds(DT);
    auto k = k_spmv_blk<DT, L, D, U>;
    (void)hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    k<<<grid, 1024, lds, s>>>(states, tasks);
}

template <int DT, int L>
static void launch_blk_l(int sched, const SpmvState *states, const int2 *tasks, unsigned grid,
                         hipStream_t s)
{
    const bool deep = (sched & VQE_SPMV_DEEP) != 0, wide = (sched & VQE_SPMV_X16) != 0;
    if (deep)
        wide ? launch_blk_t<DT, L, 4, 2>(states, tasks, grid, s)
             : launch_blk_t<DT, L, 4, 1>(states, tasks, grid, s);
    else
        wide ? launch_blk_t<DT, L, 2, 2>(states, tasks, grid, s)
             : launch_blk_t<DT, L, 2, 1>(states, tasks, grid, s);
}

template <int DT>
static void launch_blk_dt(int sched, const SpmvState *states, const int2 *tasks, unsigned grid,
                          hipStream_t s)
{
    switch (sched & 0xff) {
    case 4: launch_blk_l<DT, 4>(sched, states, tasks, grid, s); break;
    case 8: launch_blk_l<DT, 8>(sched, states, tasks, grid, s); break;
    case 16: launch_blk_l<DT, 16>(sched, states, tasks, grid, s); break;
    case 64: launch_blk_l<DT, 64>(sched, states, tasks, grid, s); break;
    default: launch_blk_l<DT, 32>(sched, states, tasks, grid, s); break;
    }
}

// Sliced schedules of column-tiled states: E entries per lane and load group,
// D groups in flight (FP64 values: half as many, the registers).
template <int DT, int E, int D>
static void launch_sellt_t(const SpmvState *states, const int2 *tasks, unsigned grid, hipStream_t s,
                           bool pf)
{
    const size_t lds = (size_t)SPMV_SELLT_ROWS * sizeof(double2) +
                       (size_t)spmv_sellt_tile_cols(DT) * vqe_elem_bytes(DT);
    auto k = pf ? k_spmv_sellt<DT, E, D, true> : k_spmv_sellt<DT, E, D, false>;
    (void)hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    k<<<grid, 1024, lds, s>>>(states, tasks);
}

template <int DT>
static void launch_sellt_dt(int sched, const SpmvState *states, const int2 *tasks, unsigned grid,
                            hipStream_t s)
{
    constexpr bool W = DT == VQE_C128;
    // VQE_SPMV_DEEP: the next column tile's loads in flight during each tile
    const bool pf = (sched & VQE_SPMV_DEEP) != 0;
    switch (sched & 0xff) {
    case 2: launch_sellt_t<DT, 2, W ? 2 : 4>(states, tasks, grid, s, pf); break;
    case 8: launch_sellt_t<DT, 8, W ? 1 : 2>(states, tasks, grid, s, pf); break;
    default: launch_sellt_t<DT, 4, W ? 2 : 3>(states, tasks, grid, s, pf); break;
    }
}

void launch_spmv_blk(int dtype, int sched, const SpmvState *states, const int2 *tasks,
                     unsigned grid, hipStream_t s)
{
    if (sched & VQE_SPMV_SLICED) {
        if (dtype == VQE_C128)
            launch_sellt_dt<VQE_C128>(sched, states, tasks, grid, s);
        else
            launch_sellt_dt<VQE_C64>(sched, states, tasks, grid, s);
        return;
    }
    if (dtype == VQE_C128)
        launch_blk_dt<VQE_C128>(sched, states, tasks, grid, s);
    else
        launch_blk_dt<VQE_C64>(sched, states, tasks, grid, s);
}

namespace {
__global__ void __launch_bounds__(256) k_zero_i32(int32_t *__restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        p[i] = 0;
}
}  // namespace

void launch_blk_layout(const vqe_csr *H, int32_t nt, int32_t tc, int32_t R, int32_t *brp,
                       int64_t *blen, int64_t *boff, uint16_t *bcode, void *bval, hipStream_t s)
{
    const int64_t dim = H->dim;
    const int64_t nb = (dim + R - 1) / R;
    const int64_t nslab = nb * nt;
    const int64_t nrp = nslab * (R + 1);
    const unsigned zgrid = (unsigned)std::min<int64_t>((nrp + 255) / 256, 65536);
    k_zero_i32<<<zgrid, 256, 0, s>>>(brp, nrp);
    const unsigned g = (unsigned)((dim * nt + 255) / 256);
    k_blk_count<<<g, 256, 0, s>>>(H->rowptr, H->col, dim, nt, tc, R, brp);
    k_blk_scan<<<(unsigned)nslab, 256, 0, s>>>(brp, R, blen);
    k_blk_offsets<<<1, 1024, 0, s>>>(blen, nslab, boff);
    if (H->dtype == VQE_C128)
        k_blk_fill<VQE_C128><<<g, 256, 0, s>>>(H->rowptr, H->col, H->val, dim, nt, tc, R, brp, boff,
                                               bcode, bval);
    else
        k_blk_fill<VQE_C64><<<g, 256, 0, s>>>(H->rowptr, H->col, H->val, dim, nt, tc, R, brp, boff,
                                              bcode, bval);
}

void launch_sell_layout(const vqe_csr *H, int E, uint16_t *srow, int32_t *slen, int2 *sslice,
                        int64_t *total, hipStream_t s)
{
    const int64_t nb = (H->dim + SPMV_LDS_ROWS - 1) / SPMV_LDS_ROWS;
    k_sell_sort<<<(unsigned)nb, 1024, 0, s>>>(H->rowptr, H->dim, E, srow, slen);
    k_sell_scan<<<1, 64, 0, s>>>(slen, nb * SPMV_SLICES_PER_BLOCK, sslice, total);
}

void launch_sell_xtab(const vqe_csr *H, uint32_t *mark, uint16_t *xmap, uint16_t *xtab, int64_t *nx,
                      hipStream_t s)
{
    const unsigned g = (unsigned)((H->dim + 255) / 256);
    k_sell_xclear<<<g, 256, 0, s>>>(mark, H->dim);
    k_sell_xmark<<<g, 256, 0, s>>>(H->rowptr, H->col, H->dim, mark);
    k_sell_xscan<<<1, 1024, 0, s>>>(mark, H->dim, xmap, xtab, nx);
}

template <int E>
static void launch_sell_fill_x_e(const vqe_csr *H, bool real, const uint16_t *srow, const int2 *sslice,
                                 const uint16_t *xmap, uint32_t *code, void *val, hipStream_t s)
{
    const int64_t nb = (H->dim + SPMV_LDS_ROWS - 1) / SPMV_LDS_ROWS;
    const unsigned g = (unsigned)(nb * SPMV_SLICES_PER_BLOCK);
    auto k = H->dtype == VQE_C128
                 ? (real ? k_sell_fill_x<VQE_C128, true, E> : k_sell_fill_x<VQE_C128, false, E>)
                 : (real ? k_sell_fill_x<VQE_C64, true, E> : k_sell_fill_x<VQE_C64, false, E>);
    k<<<g, 64, 0, s>>>(H->rowptr, H->col, H->val, H->dim, srow, sslice, xmap, code, val);
}

void launch_sell_fill_x(const vqe_csr *H, int E, bool real, const uint16_t *srow, const int2 *sslice,
                        const uint16_t *xmap, uint32_t *code, void *val, hipStream_t s)
{
    if (E == 3)
        launch_sell_fill_x_e<3>(H, real, srow, sslice, xmap, code, val, s);
    else
        launch_sell_fill_x_e<6>(H, real, srow, sslice, xmap, code, val, s);
}

void launch_sellt_layout(const vqe_csr *H, int32_t nt, int32_t tc, int E, uint16_t *srow,
                         int2 *sslice, int64_t *stot, int64_t *sbase, int64_t *total, uint32_t *smask,
                         hipStream_t s)
{
    const int64_t nb = (H->dim + SPMV_SELLT_ROWS - 1) / SPMV_SELLT_ROWS, nslab = nb * nt;
    k_sellt_count<<<(unsigned)((H->dim + 255) / 256), 256, 0, s>>>(H->rowptr, H->col, H->dim, nt, tc,
                                                                  SPMV_SELLT_ROWS, srow);
    k_sellt_sort<<<(unsigned)nslab, 1024, 0, s>>>(H->dim, nt, E, srow, sslice, stot, smask);
    k_sellt_scan<<<1, 1024, 0, s>>>(stot, nslab, sbase, total);
}

void launch_sellt_fill(const vqe_csr *H, int32_t nt, int32_t tc, int E, const uint16_t *srow,
                       const int2 *sslice, const int64_t *sbase, uint16_t *code, void *val,
                       uint32_t *smask, hipStream_t s)
{
    const int64_t nb = (H->dim + SPMV_SELLT_ROWS - 1) / SPMV_SELLT_ROWS;
    const unsigned g = (unsigned)(nb * nt * SPMV_SLICES_PER_BLOCK);
    if (H->dtype == VQE_C128)
        k_sellt_fill<VQE_C128><<<g, 64, 0, s>>>(H->rowptr, H->col, H->val, H->dim, nt, tc, E, srow,
                                                sslice, sbase, code, val, smask);
    else
        k_sellt_fill<VQE_C64><<<g, 64, 0, s>>>(H->rowptr, H->col, H->val, H->dim, nt, tc, E, srow,
                                               sslice, sbase, code, val, smask);
}

void launch_sell_fill(const vqe_csr *H, int E, bool real, const uint16_t *srow,
                      const int2 *sslice, uint16_t *code, void *val, hipStream_t s)
{
    const int64_t nb = (H->dim + SPMV_LDS_ROWS - 1) / SPMV_LDS_ROWS;
    const unsigned g = (unsigned)(nb * SPMV_SLICES_PER_BLOCK);
    auto k = H->dtype == VQE_C128 ? (real ? k_sell_fill<VQE_C128, true> : k_sell_fill<VQE_C128, false>)
                                  : (real ? k_sell_fill<VQE_C64, true> : k_sell_fill<VQE_C64, false>);
    k<<<g, 64, 0, s>>>(H->rowptr, H->col, H->val, H->dim, E, srow, sslice, code, val);
}

void launch_spmv(int dtype, int sched, const SpmvState &single, const SpmvState *states,
                 const int2 *tasks, unsigned grid, hipStream_t s, int64_t max_dim)
{
    const size_t lds = (size_t)(max_dim + 1) * vqe_elem_bytes(dtype) + (SPMV_LDS_ROWS + 1) * sizeof(int32_t);
    if (dtype == VQE_C128)
        launch_spmv_dt<VQE_C128>(sched, single, states, tasks, grid, s, lds);
    else
        launch_spmv_dt<VQE_C64>(sched, single, states, tasks, grid, s, lds);
}

int32_t spmv_tile_cols(int dtype) { return (int32_t)(SPMV_TILE_BYTES / vqe_elem_bytes(dtype)); }
int32_t spmv_tile_cols_real(int dtype) { return 2 * spmv_tile_cols(dtype); }

// Tile passes see short row segments, so narrow sub-groups keep two groups of
// four entries per lane (U = 2) instead of covering 256 entries per pass.
// The real-value form comes only with the 16-bit codes.
template <int DT, int L, int D>
static void launch_tiled_t(const SpmvState *states, const int2 *tasks, unsigned grid, hipStream_t s,
                           bool x16, bool rv)
{
    const size_t lds = (size_t)(spmv_tile_cols(DT) + 1) * vqe_elem_bytes(DT) +
                       2 * SPMV_LDS_ROWS * sizeof(int32_t);
    constexpr int U = L >= 32 ? 64 / L : 2;
    auto k = rv ? k_spmv_tiled<DT, L, D, U, true, true>
                : x16 ? k_spmv_tiled<DT, L, D, U, true, false> : k_spmv_tiled<DT, L, D, U, false, false>;
    (void)hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    k<<<grid, 1024, lds, s>>>(states, tasks);
}

template <int DT>
static void launch_tiled_dt(int sched, const SpmvState *states, const int2 *tasks, unsigned grid,
                            const int2 *sum_tasks, unsigned sum_grid, hipStream_t s)
{
    const bool deep = (sched & VQE_SPMV_DEEP) != 0;
    const bool x = (sched & VQE_SPMV_X16) != 0;
    const bool r = (sched & VQE_SPMV_REAL) != 0;
    switch (sched & 0xff) {
    case 8: deep ? launch_tiled_t<DT, 8, 3>(states, tasks, grid, s, x, r)
                 : launch_tiled_t<DT, 8, 2>(states, tasks, grid, s, x, r); break;
    case 16: deep ? launch_tiled_t<DT, 16, 3>(states, tasks, grid, s, x, r)
                  : launch_tiled_t<DT, 16, 2>(states, tasks, grid, s, x, r); break;
    case 64: deep ? launch_tiled_t<DT, 64, 3>(states, tasks, grid, s, x, r)
                  : launch_tiled_t<DT, 64, 2>(states, tasks, grid, s, x, r); break;
    default: deep ? launch_tiled_t<DT, 32, 3>(states, tasks, grid, s, x, r)
                  : launch_tiled_t<DT, 32, 2>(states, tasks, grid, s, x, r); break;
    }
    k_spmv_tile_sum<DT><<<sum_grid, 256, 0, s>>>(states, sum_tasks);
}

void launch_spmv_tiled(int dtype, int sched, const SpmvState *states, const int2 *tasks,
                       unsigned grid, const int2 *sum_tasks, unsigned sum_grid, hipStream_t s)
{
    if (dtype == VQE_C128)
        launch_tiled_dt<VQE_C128>(sched, states, tasks, grid, sum_tasks, sum_grid, s);
    else
        launch_tiled_dt<VQE_C64>(sched, states, tasks, grid, sum_tasks, sum_grid, s);
}

void launch_tile_bounds(const SpmvState *states, const int2 *tasks, unsigned grid, hipStream_t s)
{
    k_tile_bounds<<<grid, 256, 0, s>>>(states, tasks);
}

bool vqe_valid_schedule(int sched)
{
    switch (sched) {
    case 8: case 16: case 32: case 64:
    case 16 | VQE_SPMV_VEC4: case 32 | VQE_SPMV_VEC4: case 64 | VQE_SPMV_VEC4:
    case 8 | VQE_SPMV_LDS: case 16 | VQE_SPMV_LDS: case 32 | VQE_SPMV_LDS: case 64 | VQE_SPMV_LDS:
    case 8 | VQE_SPMV_LDS | VQE_SPMV_DEEP: case 16 | VQE_SPMV_LDS | VQE_SPMV_DEEP:
    case 32 | VQE_SPMV_LDS | VQE_SPMV_DEEP: case 64 | VQE_SPMV_LDS | VQE_SPMV_DEEP:
    case 32 | VQE_SPMV_LDS | VQE_SPMV_PREFETCH: case 64 | VQE_SPMV_LDS | VQE_SPMV_PREFETCH:
    case 32 | VQE_SPMV_LDS | VQE_SPMV_PREFETCH | VQE_SPMV_DEEP:
    case 64 | VQE_SPMV_LDS | VQE_SPMV_PREFETCH | VQE_SPMV_DEEP:
    // 8 and 16 lanes: pipelined only in the column-tiled form (else plain LDS)
    case 8 | VQE_SPMV_LDS | VQE_SPMV_PREFETCH: case 16 | VQE_SPMV_LDS | VQE_SPMV_PREFETCH:
    case 16 | VQE_SPMV_LDS | VQE_SPMV_PREFETCH | VQE_SPMV_DEEP:
    case 32 | VQE_SPMV_LDS | VQE_SPMV_PREFETCH | VQE_SPMV_X16:
    case 64 | VQE_SPMV_LDS | VQE_SPMV_PREFETCH | VQE_SPMV_X16:
    case 32 | VQE_SPMV_LDS | VQE_SPMV_PREFETCH | VQE_SPMV_DEEP | VQE_SPMV_X16:
    case 64 | VQE_SPMV_LDS | VQE_SPMV_PREFETCH | VQE_SPMV_DEEP | VQE_SPMV_X16:
    case 16 | VQE_SPMV_LDS | VQE_SPMV_PREFETCH | VQE_SPMV_X16 | VQE_SPMV_REAL:
    case 32 | VQE_SPMV_LDS | VQE_SPMV_PREFETCH | VQE_SPMV_X16 | VQE_SPMV_REAL:
    case 64 | VQE_SPMV_LDS | VQE_SPMV_PREFETCH | VQE_SPMV_X16 | VQE_SPMV_REAL:
    case 32 | VQE_SPMV_LDS | VQE_SPMV_PREFETCH | VQE_SPMV_DEEP | VQE_SPMV_X16 | VQE_SPMV_REAL:
    case 64 | VQE_SPMV_LDS | VQE_SPMV_PREFETCH | VQE_SPMV_DEEP | VQE_SPMV_X16 | VQE_SPMV_REAL:
    // narrow pipelined schedules with the codes (plain LDS for states that
    // fit, with at least eight lanes; the blocked product's narrow forms for
    // larger states)
    case 4 | VQE_SPMV_LDS | VQE_SPMV_PREFETCH:
    case 4 | VQE_SPMV_LDS | VQE_SPMV_PREFETCH | VQE_SPMV_DEEP:
    case 4 | VQE_SPMV_LDS | VQE_SPMV_PREFETCH | VQE_SPMV_X16:
    case 4 | VQE_SPMV_LDS | VQE_SPMV_PREFETCH | VQE_SPMV_DEEP | VQE_SPMV_X16:
    case 8 | VQE_SPMV_LDS | VQE_SPMV_PREFETCH | VQE_SPMV_DEEP:
    case 8 | VQE_SPMV_LDS | VQE_SPMV_PREFETCH | VQE_SPMV_X16:
    case 8 | VQE_SPMV_LDS | VQE_SPMV_PREFETCH | VQE_SPMV_DEEP | VQE_SPMV_X16:
    case 16 | VQE_SPMV_LDS | VQE_SPMV_PREFETCH | VQE_SPMV_X16:
    case 16 | VQE_SPMV_LDS | VQE_SPMV_PREFETCH | VQE_SPMV_DEEP | VQE_SPMV_X16:
    case 16 | VQE_SPMV_LDS | VQE_SPMV_PREFETCH | VQE_SPMV_X16 | VQE_SPMV_PAD:
    case 32 | VQE_SPMV_LDS | VQE_SPMV_PREFETCH | VQE_SPMV_X16 | VQE_SPMV_PAD:
    case 64 | VQE_SPMV_LDS | VQE_SPMV_PREFETCH | VQE_SPMV_X16 | VQE_SPMV_PAD:
    case 32 | VQE_SPMV_LDS | VQE_SPMV_PREFETCH | VQE_SPMV_DEEP | VQE_SPMV_X16 | VQE_SPMV_PAD:
    case 64 | VQE_SPMV_LDS | VQE_SPMV_PREFETCH | VQE_SPMV_DEEP | VQE_SPMV_X16 | VQE_SPMV_PAD:
    case 2 | VQE_SPMV_LDS | VQE_SPMV_SLICED:
    case 4 | VQE_SPMV_LDS | VQE_SPMV_SLICED:
    case 8 | VQE_SPMV_LDS | VQE_SPMV_SLICED:
    case 2 | VQE_SPMV_LDS | VQE_SPMV_SLICED | VQE_SPMV_DEEP:
    case 4 | VQE_SPMV_LDS | VQE_SPMV_SLICED | VQE_SPMV_DEEP:
    case 8 | VQE_SPMV_LDS | VQE_SPMV_SLICED | VQE_SPMV_DEEP:
    case 2 | VQE_SPMV_LDS | VQE_SPMV_SLICED | VQE_SPMV_REAL:
    case 4 | VQE_SPMV_LDS | VQE_SPMV_SLICED | VQE_SPMV_REAL:
    case 8 | VQE_SPMV_LDS | VQE_SPMV_SLICED | VQE_SPMV_REAL:
    case 3 | VQE_SPMV_LDS | VQE_SPMV_SLICED | VQE_SPMV_XIDX:
    case 3 | VQE_SPMV_LDS | VQE_SPMV_SLICED | VQE_SPMV_XIDX | VQE_SPMV_REAL:
    case 6 | VQE_SPMV_LDS | VQE_SPMV_SLICED | VQE_SPMV_XIDX:
    case 6 | VQE_SPMV_LDS | VQE_SPMV_SLICED | VQE_SPMV_XIDX | VQE_SPMV_REAL:
        return true;
    default:
        return false;
    }
}

// Wide loads need 16-byte aligned column and 32-byte aligned value arrays; the
// LDS schedule also needs the state to fit in LDS.  Otherwise the plain
// schedule with the same lanes is used.
int vqe_effective_schedule(const vqe_csr *H, int sched)
{
    // the sliced layout needs a state that fits LDS (with its 16-bit columns);
    // otherwise the 32-lane pipelined schedule with the codes stands in
    if (sched & VQE_SPMV_SLICED) {
        if (H->dim * (int64_t)vqe_elem_bytes(H->dtype) > SPMV_LDS_MAX_BYTES || H->dim >= 65536)
            return vqe_effective_schedule(H, 32 | VQE_SPMV_LDS | VQE_SPMV_PREFETCH | VQE_SPMV_X16);
        // the index form stages its masks too (states of up to 128 KiB)
        if ((sched & VQE_SPMV_XIDX) &&
            (H->dim + 1) * (int64_t)vqe_elem_bytes(H->dtype) + SPMV_LDS_ROWS * (int64_t)sizeof(float2) +
                    SPMV_XIDX_MAX * (int64_t)sizeof(uint16_t) > 160 * 1024)
            sched = (sched & ~(VQE_SPMV_XIDX | 0xff)) | 4;
        // the real values need an operator flagged real
        return sched & (VQE_SPMV_SLICED | VQE_SPMV_LDS | VQE_SPMV_XIDX | 0xff |
                        ((H->flags & VQE_REAL) ? VQE_SPMV_REAL : 0));
    }
    // four lanes per row exist only in the blocked product of states larger
    // than LDS; elsewhere the same schedule runs with eight
    if ((sched & 0xff) == 4)
        sched = (sched & ~0xff) | 8;
    // the real-value form needs an operator flagged real, and the codes
    if (!(H->flags & VQE_REAL))
        sched &= ~VQE_SPMV_REAL;
    const bool wide = (sched & (VQE_SPMV_VEC4 | VQE_SPMV_LDS)) != 0;
    if (wide && ((((uintptr_t)H->col) & 15) != 0 || (((uintptr_t)H->val) & 31) != 0))
        return sched & 0xff;
    if ((sched & VQE_SPMV_LDS) && H->dim * (int64_t)vqe_elem_bytes(H->dtype) > SPMV_LDS_MAX_BYTES)
        return (sched & 0xff) == 8 ? 16 | VQE_SPMV_VEC4 : (sched & 0xff) | VQE_SPMV_VEC4;
    // the pipelined schedule addresses the arrays with 31-bit buffer offsets,
    // and runs with 32 or 64 lanes when the state fits LDS
    if ((sched & VQE_SPMV_PREFETCH) &&
        (!(sched & VQE_SPMV_LDS) || H->nnz * (int64_t)vqe_elem_bytes(H->dtype) > 0x7fffff00LL ||
         (sched & 0xff) < ((sched & (VQE_SPMV_REAL | VQE_SPMV_PAD)) ? 16 : 32)))
        return sched & ~(VQE_SPMV_PREFETCH | VQE_SPMV_DEEP | VQE_SPMV_X16 | VQE_SPMV_REAL |
                         VQE_SPMV_PAD);
    // the 16-bit column form needs column XOR row below 2^16; the padded
    // layout comes with it; the real values imply the padded layout
    if ((sched & VQE_SPMV_X16) && H->dim > SPMV_X16_MAX_DIM)
        return sched & ~(VQE_SPMV_X16 | VQE_SPMV_REAL | VQE_SPMV_PAD);
    if (!(sched & VQE_SPMV_X16))
        sched &= ~VQE_SPMV_PAD;
    if (sched & VQE_SPMV_REAL)
        sched &= ~VQE_SPMV_PAD;
    return sched;
}

// In a batch plan, a pipelined LDS schedule on a state too large for LDS
// becomes the column-tiled schedule with the same lanes and depth.
int vqe_batch_schedule(const vqe_csr *H, int sched)
{
    const bool big = H->dim * (int64_t)vqe_elem_bytes(H->dtype) > SPMV_LDS_MAX_BYTES;
    // a sliced schedule runs a state larger than LDS in the slabs of the
    // blocked layout, each sorted and sliced
    if ((sched & VQE_SPMV_SLICED) && big) {
        // (the index form's states fit LDS; larger ones take two entries per group)
        if (sched & VQE_SPMV_XIDX)
            sched = (sched & ~(VQE_SPMV_XIDX | 0xff)) | 2;
        return (sched & (0xff | VQE_SPMV_LDS | VQE_SPMV_SLICED | VQE_SPMV_DEEP)) | VQE_SPMV_TILED |
               VQE_SPMV_BLOCKED;
    }
    const bool aligned = ((((uintptr_t)H->col) & 15) == 0) && ((((uintptr_t)H->val) & 31) == 0);
    if (big && (sched & VQE_SPMV_LDS) && (sched & VQE_SPMV_PREFETCH) && H->dim <= ((int64_t)1 << 30)) {
        // the real-value form keeps the column-tiled CSR (16-bit col ^ row
        // codes, real parts, per-tile row bounds) where it applies
        if ((sched & VQE_SPMV_REAL) && (sched & VQE_SPMV_X16) && (H->flags & VQE_REAL) && aligned &&
            H->dim <= SPMV_X16_MAX_DIM && H->nnz * (int64_t)vqe_elem_bytes(H->dtype) <= 0x7fffff00LL)
            return (sched & ~VQE_SPMV_PAD) | VQE_SPMV_TILED;
        // otherwise the blocked layout (complex values, tile-local codes;
        // VQE_SPMV_X16 and VQE_SPMV_DEEP select the pass width and depth)
        return (sched & (0xff | VQE_SPMV_LDS | VQE_SPMV_PREFETCH | VQE_SPMV_DEEP | VQE_SPMV_X16)) |
               VQE_SPMV_TILED | VQE_SPMV_BLOCKED;
    }
    return vqe_effective_schedule(H, sched);
}

void launch_val_real(const vqe_csr *H, void *out, hipStream_t s)
{
    const unsigned grid = (unsigned)((H->nnz + 255) / 256);
    if (grid == 0)
        return;
    if (H->dtype == VQE_C128)
        k_val_real<VQE_C128><<<grid, 256, 0, s>>>(H->val, out, H->nnz);
    else
        k_val_real<VQE_C64><<<grid, 256, 0, s>>>(H->val, out, H->nnz);
}

void launch_pad_layout(const vqe_csr *H, int32_t *prow, uint16_t *code, void *vpad, bool real,
                       hipStream_t s)
{
    k_pad_rowptr<<<1, 1024, 0, s>>>(H->rowptr, prow, H->dim);
    const unsigned grid = (unsigned)((H->dim + 3) / 4);
    if (H->dtype == VQE_C128) {
        if (real)
            k_pad_fill<VQE_C128, true><<<grid, 256, 0, s>>>(H->rowptr, H->col, H->val, prow, code, vpad, H->dim);
        else
            k_pad_fill<VQE_C128, false><<<grid, 256, 0, s>>>(H->rowptr, H->col, H->val, prow, code, vpad, H->dim);
    } else {
        if (real)
            k_pad_fill<VQE_C64, true><<<grid, 256, 0, s>>>(H->rowptr, H->col, H->val, prow, code, vpad, H->dim);
        else
            k_pad_fill<VQE_C64, false><<<grid, 256, 0, s>>>(H->rowptr, H->col, H->val, prow, code, vpad, H->dim);
    }
}

void launch_col_xor16(const vqe_csr *H, uint16_t *col16, hipStream_t s)
{
    const unsigned grid = (unsigned)((H->dim + 3) / 4);
    k_col_xor16<<<grid, 256, 0, s>>>(H->rowptr, H->col, col16, H->dim);
}

int64_t spmv_blocks(int64_t dim, int sched)
{
    const int64_t rpb = (sched & VQE_SPMV_LDS) ? SPMV_LDS_ROWS : spmv_rows_per_block(sched);
    return (dim + rpb - 1) / rpb;
}

extern "C" int32_t vqe_default_schedule(const vqe_csr *H)
{
    if (!H || H->dim <= 0)
        return 32;
    const double avg = (double)H->nnz / (double)H->dim;
    if (avg >= 96.0)
        return 64 | VQE_SPMV_VEC4;
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
    if (lanes & VQE_SPMV_SLICED)   // batch plans only
        lanes = 32 | VQE_SPMV_LDS | VQE_SPMV_PREFETCH;
    lanes = vqe_effective_schedule(H, lanes);
    const int64_t nblk = spmv_blocks(dim, lanes);
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
    st.nnz = H->nnz;
    launch_spmv(H->dtype, lanes, st, nullptr, nullptr, (unsigned)nblk, ctx->stream, dim);
    k_energy_finalize<<<1, 64, 0, ctx->stream>>>(st, nullptr, 1);
    VQE_LAUNCH_CHECK(ctx);
    return VQE_OK;
}

size_t vqe_spmv_partials_bytes(int64_t dim, int lanes)
{
    // the larger of the two block counts, so any schedule fits
    const int64_t a = spmv_blocks(dim, lanes & 0xff), b = spmv_blocks(dim, lanes);
    return vqe_align((size_t)(a > b ? a : b) * 3 * sizeof(double));
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
    return vqe_spmv_energy_launch(ctx, H, psi, sigma_out, out, vqe_default_schedule(H));
}

extern "C" int energy_noalloc(vqe_ctx *ctx, const vqe_csr *H, const void *psi, void *sigma_out,
                              double *out)
{
    if (!ctx)
        return VQE_EINVAL;
    int rc = check_csr(ctx, H, "energy_noalloc");
    if (rc)
        return rc;
    if (!psi || !sigma_out || !out)
        return vqe_fail(ctx, VQE_EINVAL, "energy_noalloc: null psi, sigma_out or out");
    const int lanes = vqe_default_schedule(H);
    const size_t need = vqe_spmv_partials_bytes(H->dim, lanes);
    if (need > VQE_NOALLOC_SCRATCH_BYTES)
        return vqe_fail(ctx, VQE_ESIZE,
                        "energy_noalloc: the reduction of a %lld-row operator needs %zu bytes of "
                        "partial sums, more than the %u-byte scratch array",
                        (long long)H->dim, need, (unsigned)VQE_NOALLOC_SCRATCH_BYTES);
    if (!ctx->scratch)
        return vqe_fail(ctx, VQE_EHIP, "energy_noalloc: the scratch array's device address is "
                                       "unknown (%s)", ctx->err);
    return vqe_spmv_energy_core(ctx, H, psi, sigma_out, out, lanes, ctx->scratch);
}

extern "C" int vqe_time_spmv(vqe_ctx *ctx, const vqe_csr *H, const void *psi, void *sigma,
                             int32_t schedule, int32_t reps, float *ms_out)
{
    if (!ctx)
        return VQE_EINVAL;
    int rc = check_csr(ctx, H, "vqe_time_spmv");
    if (rc)
        return rc;
    if (!psi || !sigma || !ms_out || reps < 1)
        return vqe_fail(ctx, VQE_EINVAL, "vqe_time_spmv: bad arguments");
    if (!vqe_valid_schedule(schedule))
        return vqe_fail(ctx, VQE_EINVAL, "vqe_time_spmv: unknown schedule %d", schedule);
    // a single call has no 16-bit column codes, real values or sliced layout:
    // the same schedule without them (the 32-lane pipelined one for a sliced)
    const int lanes = (schedule & VQE_SPMV_SLICED) ? 32 | VQE_SPMV_LDS | VQE_SPMV_PREFETCH
                                                   : schedule & ~(VQE_SPMV_X16 | VQE_SPMV_REAL);
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
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms_out = ms / (float)reps;
    return rc;
}
