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

// ------------------------------------------------------------------ complex I/O
// Elements are loaded into FP64 registers whatever the storage type.
template <int DT> struct Elem;

template <> struct Elem<VQE_C128> {
    using T = double2;
    static __device__ __forceinline__ double2 ld(const void *p, int64_t i)
    {
        return reinterpret_cast<const double2 *>(p)[i];
    }
    static __device__ __forceinline__ void st(void *p, int64_t i, double2 v)
    {
        reinterpret_cast<double2 *>(p)[i] = v;
    }
};

template <> struct Elem<VQE_C64> {
    using T = float2;
    static __device__ __forceinline__ double2 ld(const void *p, int64_t i)
    {
        float2 v = reinterpret_cast<const float2 *>(p)[i];
        return make_double2((double)v.x, (double)v.y);
    }
    static __device__ __forceinline__ void st(void *p, int64_t i, double2 v)
    {
        reinterpret_cast<float2 *>(p)[i] = make_float2((float)v.x, (float)v.y);
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

// Sum over aligned groups of `width` lanes; every lane of a group gets the total.
template <int WIDTH> __device__ __forceinline__ double group_sum(double v)
{
#pragma unroll
    for (int o = WIDTH / 2; o > 0; o >>= 1)
        v += __shfl_xor(v, o, VQE_WAVE);
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
