// Internal definitions shared by the HIP sources of libadaptvqe.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>

#include "adaptvqe.h"

#define VQE_WAVE 64

struct vqe_ctx {
    int device;
    hipStream_t stream;
    int n_cu;
    char name[256];
    char err[512];
    // Growable scratch for single-call entry points.
    void *ws;
    size_t ws_bytes;
    // Small pinned host buffer for scalar read-backs of the build phase.
    int64_t *host_scalars;
    // This device's copy of the library's static scratch array (the
    // allocation-free entry points), or null if its address is unknown.
    double *scratch;
};

// Record an error message on the context and return `status`.
static inline int vqe_fail(vqe_ctx *ctx, int status, const char *fmt, ...)
{
    if (ctx) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(ctx->err, sizeof(ctx->err), fmt, ap);
        va_end(ap);
    }
    return status;
}

#define VQE_HIP(ctx, expr)                                                              \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return vqe_fail((ctx), VQE_EHIP, "%s failed: %s (%s:%d)", #expr,           \
                            hipGetErrorString(e_), __FILE__, __LINE__);                 \
    } while (0)

#define VQE_LAUNCH_CHECK(ctx)                                                           \
    do {                                                                                \
        hipError_t e_ = hipGetLastError();                                              \
        if (e_ != hipSuccess)                                                           \
            return vqe_fail((ctx), VQE_EHIP, "kernel launch failed: %s (%s:%d)",       \
                            hipGetErrorString(e_), __FILE__, __LINE__);                 \
    } while (0)

// Ensure the context scratch holds at least `bytes` (256-byte aligned use).
int vqe_ws_reserve(vqe_ctx *ctx, size_t bytes);

__host__ __device__ static inline size_t vqe_align(size_t v) { return (v + 255) & ~(size_t)255; }

// ------------------------------------------------------------------ address spaces
// Pointers read from descriptor tables are generic; the compiler then emits
// flat loads, which count against both the memory and the LDS wait counters
// and so serialise LDS traffic behind global loads.  Every global access of
// the kernels goes through these casts to the global address space.
#define VQE_GLOBAL __attribute__((address_space(1)))

template <typename T> __device__ __forceinline__ const VQE_GLOBAL T *gmem(const T *p)
{
    return (const VQE_GLOBAL T *)p;
}
template <typename T> __device__ __forceinline__ VQE_GLOBAL T *gmem(T *p)
{
    return (VQE_GLOBAL T *)p;
}

// Element loads and stores through the global address space (clang vector
// types carry the address space; HIP's float2/double2 classes do not).
typedef double vqe_v2d __attribute__((ext_vector_type(2)));
typedef float vqe_v2f __attribute__((ext_vector_type(2)));
typedef float vqe_v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float2 ldg(const float2 *p, int64_t i)
{
    const vqe_v2f t = gmem(reinterpret_cast<const vqe_v2f *>(p))[i];
    return make_float2(t.x, t.y);
}
__device__ __forceinline__ double2 ldg(const double2 *p, int64_t i)
{
    const vqe_v2d t = gmem(reinterpret_cast<const vqe_v2d *>(p))[i];
    return make_double2(t.x, t.y);
}
__device__ __forceinline__ void stg(float2 *p, int64_t i, float2 v)
{
    vqe_v2f t;
    t.x = v.x;
    t.y = v.y;
    gmem(reinterpret_cast<vqe_v2f *>(p))[i] = t;
}
__device__ __forceinline__ void stg(double2 *p, int64_t i, double2 v)
{
    vqe_v2d t;
    t.x = v.x;
    t.y = v.y;
    gmem(reinterpret_cast<vqe_v2d *>(p))[i] = t;
}

// ------------------------------------------------------------------ complex I/O
// Elements are loaded into FP64 registers whatever the storage type.
template <int DT> struct Elem;

template <> struct Elem<VQE_C128> {
    using T = double2;
    static __device__ __forceinline__ double2 ld(const void *p, int64_t i)
    {
        return ldg(reinterpret_cast<const double2 *>(p), i);
    }
    static __device__ __forceinline__ void st(void *p, int64_t i, double2 v)
    {
        stg(reinterpret_cast<double2 *>(p), i, v);
    }
};

template <> struct Elem<VQE_C64> {
    using T = float2;
    static __device__ __forceinline__ double2 ld(const void *p, int64_t i)
    {
        const float2 v = ldg(reinterpret_cast<const float2 *>(p), i);
        return make_double2((double)v.x, (double)v.y);
    }
    static __device__ __forceinline__ void st(void *p, int64_t i, double2 v)
    {
        stg(reinterpret_cast<float2 *>(p), i, make_float2((float)v.x, (float)v.y));
    }
};

static inline size_t vqe_elem_bytes(int dtype) { return dtype == VQE_C64 ? 8 : 16; }

// ------------------------------------------------------------------ wave reductions
// Butterfly sums over the 64 lanes of a wave (fixed order: deterministic).
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, VQE_WAVE);
    return v;
}

// A double moved between lanes with a DPP pattern (two 32-bit moves).
// Every control used here has a valid source lane for every lane, so the
// moves need no previous destination value (bound_ctrl set).
template <int CTRL> __device__ __forceinline__ double dpp_f64(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

// Sum over aligned groups of `width` lanes; every lane of a group gets the
// same total (each step adds a partner's partial, a + b = b + a exactly, so
// the order is fixed and deterministic).  Within a 16-lane row the steps are
// DPP moves (two quad swaps, the half-row mirror, the row mirror), which stay
// out of the LDS pipeline; wider groups add cross-row shuffles.
template <int WIDTH> __device__ __forceinline__ double group_sum(double v)
{
    v += dpp_f64<0xB1>(v);                 // quad_perm [1,0,3,2]: lane ^ 1
    if (WIDTH > 2)
        v += dpp_f64<0x4E>(v);             // quad_perm [2,3,0,1]: lane ^ 2
    if (WIDTH > 4)
        v += dpp_f64<0x141>(v);            // row_half_mirror: the other quad of 8 lanes
    if (WIDTH > 8)
        v += dpp_f64<0x140>(v);            // row_mirror: the other half of 16 lanes
    if (WIDTH > 16)
        v += __shfl_xor(v, 16, VQE_WAVE);
    if (WIDTH > 32)
        v += __shfl_xor(v, 32, VQE_WAVE);
    return v;
}

// ------------------------------------------------------------------ internal entry points
// Defined in the individual sources; called by the C ABI layer.
int vqe_spmv_energy_launch(vqe_ctx *ctx, const vqe_csr *H, const void *psi, void *sigma,
                           double *out, int lanes);
int vqe_pool_grad_launch(vqe_ctx *ctx, const vqe_csr *H, const vqe_pool *pool, const void *psi,
                         const void *sigma, double *g_out);
int vqe_select_launch(vqe_ctx *ctx, int32_t M, const double *g, double rel_tie, int32_t *k_out,
                      double *gmax_out);
int vqe_taylor_launch(vqe_ctx *ctx, const vqe_csr *A, double theta, void *psi, int renorm,
                      double *norm2_out);
