// C ABI: contexts, workspace, status strings and the batch planner.
//
// The batch planner turns B independent adaptive steps into a fixed list of
// launches over device task tables:
//   H products with the energy reduction (one launch per schedule in use),
//   the pool-gradient screen, one per-state kernel for the energy, the
//   gradient sums and the selection, the optional line search, the fused
//   pairing Taylor update and the renormalisation.
// States are assigned to the 8 XCDs of the device (balanced by H bytes) and
// every task table is interleaved so that workgroup i runs on XCD i % 8 and
// only touches states of that XCD: each state's psi and sigma stay in one L2.
// The launch list can be captured once into a HIP graph and replayed; theta,
// the selected index and every result live in caller-owned device buffers, so
// a replay needs no host round trip.
#include "kernels.hpp"
#include "step_fin.hpp"

#include <algorithm>
#include <cstdlib>
#include <cmath>
#include <map>
#include <mutex>
#include <numeric>
#include <vector>

static const int kXcd = 8;
#define VQE_RUN_GRAPHS 4   // multi-step graphs kept per plan

// Scratch of the allocation-free entry points: a static device array, one
// copy per GPU, held until the process ends.  In host code `scratch` names a
// host-side stand-in, never its device address: the address of each GPU's
// copy is taken once per device at context creation (with that device
// current) and used from then on.
static __device__ __align__(256) double scratch[VQE_NOALLOC_SCRATCH_BYTES / sizeof(double)];
static const int kMaxDevices = 64;
static double *g_scratch_dev[kMaxDevices];
static std::mutex g_scratch_mu;

static void scratch_setup(vqe_ctx *ctx)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (ctx->device >= kMaxDevices) {
        vqe_fail(ctx, VQE_EHIP, "device %d: no scratch slot (at most %d devices)", ctx->device,
                 kMaxDevices);
        return;
    }
    if (!g_scratch_dev[ctx->device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            vqe_fail(ctx, VQE_EHIP, "hipGetSymbolAddress(scratch) failed on device %d: %s",
                     ctx->device, hipGetErrorString(e));
            return;
        }
        g_scratch_dev[ctx->device] = (double *)p;
    }
    ctx->scratch = g_scratch_dev[ctx->device];
}

extern "C" const char *vqe_strerror(int status)
{
    switch (status) {
    case VQE_OK: return "success";
    case VQE_EINVAL: return "invalid argument";
    case VQE_ESIZE: return "size out of range";
    case VQE_ENOMEM: return "out of device memory";
    case VQE_EHIP: return "HIP runtime error";
    case VQE_ENOTSUP: return "not supported";
    default: return "unknown status";
    }
}

extern "C" const char *vqe_last_error(const vqe_ctx *ctx) { return ctx ? ctx->err : "no context"; }

extern "C" int vqe_create(int device, void *hip_stream, vqe_ctx **out)
{
    if (!out)
        return VQE_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n < 1)
        return VQE_EHIP;
    if (device < 0 || device >= n)
        return VQE_EINVAL;
    if (hipSetDevice(device) != hipSuccess)
        return VQE_EHIP;
    vqe_ctx *ctx = new (std::nothrow) vqe_ctx();
    if (!ctx)
        return VQE_ENOMEM;
    ctx->device = device;
    ctx->stream = (hipStream_t)hip_stream;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        delete ctx;
        return VQE_EHIP;
    }
    ctx->n_cu = prop.multiProcessorCount;
    snprintf(ctx->name, sizeof(ctx->name), "%s (%s)", prop.name, prop.gcnArchName);
    if (hipHostMalloc((void **)&ctx->host_scalars, 64, hipHostMallocDefault) != hipSuccess) {
        delete ctx;
        return VQE_ENOMEM;
    }
    // with the device current: this device's scratch address (a failure is
    // reported by the allocation-free entry points, which need it)
    scratch_setup(ctx);
    *out = ctx;
    return VQE_OK;
}

extern "C" int vqe_destroy(vqe_ctx *ctx)
{
    if (!ctx)
        return VQE_EINVAL;
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->ws)
        (void)hipFree(ctx->ws);
    if (ctx->host_scalars)
        (void)hipHostFree(ctx->host_scalars);
    delete ctx;
    return VQE_OK;
}

extern "C" int vqe_set_stream(vqe_ctx *ctx, void *hip_stream)
{
    if (!ctx)
        return VQE_EINVAL;
    ctx->stream = (hipStream_t)hip_stream;
    return VQE_OK;
}

extern "C" int vqe_device_info(const vqe_ctx *ctx, int32_t *n_cu, char *name, int32_t name_len)
{
    if (!ctx)
        return VQE_EINVAL;
    if (n_cu)
        *n_cu = ctx->n_cu;
    if (name && name_len > 0)
        snprintf(name, (size_t)name_len, "%s", ctx->name);
    return VQE_OK;
}

int vqe_ws_reserve(vqe_ctx *ctx, size_t bytes)
{
    if (bytes <= ctx->ws_bytes)
        return VQE_OK;
    // earlier work may still read the old scratch
    VQE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (ctx->ws) {
        (void)hipFree(ctx->ws);
        ctx->ws = nullptr;
        ctx->ws_bytes = 0;
    }
    size_t sz = std::max<size_t>(bytes, (size_t)1 << 20);
    if (hipMalloc(&ctx->ws, sz) != hipSuccess) {
        ctx->ws = nullptr;
        (void)hipGetLastError();
        return vqe_fail(ctx, VQE_ENOMEM, "workspace allocation of %zu bytes failed", sz);
    }
    ctx->ws_bytes = sz;
    return VQE_OK;
}

// ------------------------------------------------------------------ batch plan
struct vqe_batch {
    vqe_ctx *ctx = nullptr;
    int32_t B = 0;
    int32_t dtype = 0;
    double rel_tie = 0.0;
    char *dmem = nullptr;          // one allocation: tables + partials
    size_t dmem_bytes = 0;
    SpmvState *d_spmv = nullptr;
    struct SpmvLaunch {
        int lanes;
        int2 *tasks;
        unsigned grid;
        int64_t max_dim;
        int2 *sum_tasks;    // column-tiled schedules: the tile-sum tasks
        unsigned sum_grid;
    };
    int2 *d_bounds_tasks = nullptr;       // per-tile row bounds (tiled states)
    std::vector<std::pair<unsigned, unsigned>> bounds_range;   // per slot: first task, count
    std::vector<SpmvLaunch> spmv;
    ScreenState *d_screen = nullptr;
    PairTable *d_tables = nullptr;
    int4 *d_screen_tasks = nullptr;
    unsigned n_screen_tasks = 0;
    int32_t max_m = 0;          // largest pool of the plan
    int64_t max_gpart = 0;      // largest M x (screen tiles): the gradient partials per state
    size_t screen_lds = 0;
    // real-state screen (matrix-free pools of real anti-Hermitian generators
    // whose states fit one LDS tile as reals): tasks per (state, range)
    int4 *d_screen1_tasks = nullptr;
    unsigned n_screen1_tasks = 0;
    size_t screen1_lds = 0;
    std::vector<void *> table_mem;   // one allocation per distinct pool
    size_t table_bytes = 0;
    SelectState *d_sel = nullptr;
    TaylorState *d_tay = nullptr;
    int2 *d_tay_tasks = nullptr;
    unsigned n_tay_tasks = 0;
    int2 *d_norm_tasks = nullptr;
    unsigned n_norm_tasks = 0;
    hipGraphExec_t exec[32] = {};  // rest-of-step graphs by flag set (step_key)
    hipGraph_t graph[32] = {};
    bool compact_taylor = false;   // every pool has a compact pair table
    bool mf = false;               // every pool is matrix-free: screen and update from records
    // host image of the descriptors (for rebinding slots)
    std::vector<char> image;
    size_t o_spmv = 0, o_screen = 0, o_tay = 0;
    std::vector<int> sched;            // effective H-product schedule per slot
    std::vector<const void *> pool_ops;  // pool of each slot
    std::vector<int64_t> dims;
    hipGraphExec_t exec_spmv = nullptr;
    hipGraph_t graph_spmv = nullptr;
    hipGraphExec_t exec_all[32] = {};  // whole-step graphs by flag set (steps without events)
    hipGraph_t graph_all[32] = {};
    // multi-step graphs of vqe_batch_run, by (flags, steps, angle rows); the
    // least recently used one is replaced
    struct RunGraph {
        uint32_t flags = 0;
        int32_t n = 0;
        const double *rows = nullptr;
        hipGraph_t g = nullptr;
        hipGraphExec_t x = nullptr;
        uint64_t used = 0;
    };
    RunGraph runs[VQE_RUN_GRAPHS];
    uint64_t run_tick = 0;
    double *theta_io = nullptr;        // the caller's angle buffer [B]
    // line search (vqe_batch_set_line_search)
    std::vector<PairTable> tables_host;            // CSR mode: pair tables (host copy)
    std::vector<const vqe_mf_pool *> mf_host;      // mf mode: pool of each table
    std::vector<const vqe_mf_desc *> mf_desc_dev;  // mf mode: device descriptors of each table
    std::vector<int> table_idx;                    // table of each slot
    std::vector<int> xcd;                          // XCD of each slot
    int ls_checked = 0;                            // 0 unknown, 1 every generator has A^3 = -A, -1 not
    bool ls_ready = false;
    char *ls_mem = nullptr;
    size_t ls_bytes = 0;
    std::vector<char> ls_image;
    size_t o_ls = 0, o_ls1 = 0, o_ls2 = 0;
    LsState *d_ls = nullptr;
    SpmvState *d_ls1 = nullptr, *d_ls2 = nullptr;
    int2 *d_ls_tasks = nullptr;
    unsigned n_ls_tasks = 0;
    // per slot, the plan-owned forms of H its schedule reads: 16-bit column
    // codes (VQE_SPMV_X16), the values in the padded layout (real parts with
    // VQE_SPMV_REAL, complex with VQE_SPMV_PAD) and its row pointers;
    // capacities in bytes
    std::vector<void *> col16, vre, prow;
    std::vector<int64_t> col16_cap, vre_cap, prow_cap;
    // per slot, the blocked layout of a column-tiled H (VQE_SPMV_BLOCKED):
    // one allocation holding slab row pointers, slab lengths and starts,
    // codes and values; capacity in bytes
    std::vector<void *> blk;
    std::vector<int64_t> blk_cap;
    // per slot, the entries (pads included) of a sliced layout, else 0
    std::vector<int64_t> entries;
    // re-optimisation (vqe_batch_reoptimize): descriptors, three product
    // descriptor arrays, tasks, then per slot nine vectors and partials
    char *ro_mem = nullptr;
    size_t ro_bytes = 0;
    std::vector<char> ro_image;
    size_t o_ro = 0, o_roh[3] = {0, 0, 0};
    RoState *d_ro = nullptr;
    SpmvState *d_roh[3] = {nullptr, nullptr, nullptr};
    int2 *d_ro_tasks = nullptr;
    unsigned n_ro_tasks = 0;
};

namespace {

struct Arena {
    std::vector<char> host;
    size_t take(size_t bytes)
    {
        size_t o = host.size();
        host.resize(o + vqe_align(bytes), 0);
        return o;
    }
    template <class T> T *at(size_t off) { return reinterpret_cast<T *>(host.data() + off); }
};

// Interleave per-XCD task lists so that workgroup i belongs to XCD i % 8.
template <class T>
std::vector<T> interleave(const std::vector<std::vector<T>> &per, const T &pad)
{
    size_t longest = 0;
    for (auto &v : per)
        longest = std::max(longest, v.size());
    std::vector<T> out;
    out.reserve(longest * per.size());
    for (size_t i = 0; i < longest; i++)
        for (auto &v : per)
            out.push_back(i < v.size() ? v[i] : pad);
    return out;
}

// Grow one of slot s's plan-owned buffers to at least `need` bytes (the
// caller rebuilds the contents).
int grow_ctx(vqe_ctx *ctx, void **buf, int64_t *cap, int64_t need, const char *what, int s)
{
    if (*cap >= need)
        return VQE_OK;
    if (*buf) {
        VQE_HIP(ctx, hipStreamSynchronize(ctx->stream));
        (void)hipFree(*buf);
        *buf = nullptr;
        *cap = 0;
    }
    if (hipMalloc(buf, (size_t)need) != hipSuccess) {
        (void)hipGetLastError();
        *buf = nullptr;
        return vqe_fail(ctx, VQE_ENOMEM, "%s of slot %d: allocation failed", what, s);
    }
    *cap = need;
    return VQE_OK;
}

int grow(vqe_batch *p, void **buf, int64_t *cap, int64_t need, const char *what, int s)
{
    return grow_ctx(p->ctx, buf, cap, need, what, s);
}

// Buffers of a sliced layout (the slot's own, or a vqe_layout's): the slice
// or slab tables, the codes and the values, with their capacities in bytes.
struct SellBufs {
    void **meta, **code, **val;
    int64_t *meta_cap, *code_cap, *val_cap;
};

// (Re)build slot s's plan-owned forms of H for its schedule -- the 16-bit
// column codes, and with VQE_SPMV_REAL the real parts of the values, with
// VQE_SPMV_PAD the complex values, in the padded layout unless the slot is
// column-tiled -- and point the slot's host descriptor at them (the caller
// uploads the descriptor).
int codes_fill(vqe_batch *p, int s, const vqe_csr *H, int sched)
{
    vqe_ctx *ctx = p->ctx;
    SpmvState &st = reinterpret_cast<SpmvState *>(p->image.data() + p->o_spmv)[s];
    const int64_t rb = (int64_t)vqe_elem_bytes(H->dtype) / 2;
    int rc;
    if ((sched & (VQE_SPMV_REAL | VQE_SPMV_PAD)) && !(sched & VQE_SPMV_TILED)) {
        // the padded layout: real parts (VQE_SPMV_REAL) or complex values
        const bool real = (sched & VQE_SPMV_REAL) != 0;
        const int64_t vb = real ? rb : 2 * rb;
        const int64_t cap = H->nnz + (SPMV_PAD - 1) * H->dim + SPMV_PAD;
        if ((rc = grow(p, &p->col16[s], &p->col16_cap[s], cap * 2, "column codes", s)) ||
            (rc = grow(p, &p->vre[s], &p->vre_cap[s], cap * vb, "padded values", s)) ||
            (rc = grow(p, &p->prow[s], &p->prow_cap[s], (H->dim + 1) * 4, "row pointers", s)))
            return rc;
        launch_pad_layout(H, (int32_t *)p->prow[s], (uint16_t *)p->col16[s], p->vre[s], real,
                          ctx->stream);
        st.col16 = (const uint16_t *)p->col16[s];
        st.vre = p->vre[s];
        st.prow = (const int32_t *)p->prow[s];
        st.cap = cap;
        return VQE_OK;
    }
    const int64_t nnz = H->nnz > 0 ? H->nnz : 1;
    if ((rc = grow(p, &p->col16[s], &p->col16_cap[s], nnz * 2, "column codes", s)))
        return rc;
    launch_col_xor16(H, (uint16_t *)p->col16[s], ctx->stream);
    st.col16 = (const uint16_t *)p->col16[s];
    if (sched & VQE_SPMV_REAL) {
        if ((rc = grow(p, &p->vre[s], &p->vre_cap[s], nnz * rb, "real values", s)))
            return rc;
        launch_val_real(H, p->vre[s], ctx->stream);
        st.vre = p->vre[s];
    }
    return VQE_OK;
}

// Build the sliced layout of H (VQE_SPMV_SLICED) in the buffers b -- the
// slice table (row order, slice lengths and starts, the total) in meta, the
// codes in code, the values in val -- and point st's layout fields at it.
// The codes and values are sized from the table, so this waits for the
// context stream once.  s names the slot in messages (-1: a vqe_layout).
int sliced_build(vqe_ctx *ctx, const vqe_csr *H, int sched, const SellBufs &b, SpmvState &st,
                 int64_t *entries, int s)
{
    const int E = sched & 0xff;
    const bool xi = (sched & VQE_SPMV_XIDX) != 0;
    const int64_t nb = (H->dim + SPMV_LDS_ROWS - 1) / SPMV_LDS_ROWS;
    const int64_t ns = nb * SPMV_SLICES_PER_BLOCK;
    const size_t o_len = vqe_align((size_t)H->dim * sizeof(uint16_t));
    const size_t o_sl = o_len + vqe_align((size_t)ns * sizeof(int32_t));
    const size_t o_tot = o_sl + vqe_align((size_t)ns * sizeof(int2));
    // the index form: the masks' marks, numbers, table and count
    const size_t o_mark = o_tot + vqe_align(sizeof(int64_t));
    const size_t o_xmap = o_mark + vqe_align((size_t)H->dim * sizeof(uint32_t));
    const size_t o_xtab = o_xmap + vqe_align((size_t)H->dim * sizeof(uint16_t));
    const size_t o_nx = o_xtab + vqe_align((size_t)SPMV_XIDX_MAX * sizeof(uint16_t));
    const size_t need = xi ? o_nx + sizeof(int64_t) : o_tot + sizeof(int64_t);
    int rc = grow_ctx(ctx, b.meta, b.meta_cap, (int64_t)need, "slice table", s);
    if (rc)
        return rc;
    char *m = (char *)*b.meta;
    launch_sell_layout(H, E, (uint16_t *)m, (int32_t *)(m + o_len), (int2 *)(m + o_sl),
                       (int64_t *)(m + o_tot), ctx->stream);
    VQE_LAUNCH_CHECK(ctx);
    if (xi) {
        launch_sell_xtab(H, (uint32_t *)(m + o_mark), (uint16_t *)(m + o_xmap), (uint16_t *)(m + o_xtab),
                         (int64_t *)(m + o_nx), ctx->stream);
        VQE_LAUNCH_CHECK(ctx);
    }
    int64_t total = 0, nx = 0;
    VQE_HIP(ctx, hipMemcpyAsync(&total, m + o_tot, sizeof(total), hipMemcpyDeviceToHost, ctx->stream));
    if (xi)
        VQE_HIP(ctx, hipMemcpyAsync(&nx, m + o_nx, sizeof(nx), hipMemcpyDeviceToHost, ctx->stream));
    VQE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (total < 0 || total > 0x7fffffffLL)
        return vqe_fail(ctx, VQE_ESIZE, "sliced layout of slot %d: %lld entries", s, (long long)total);
    if (nx < 0 || nx > SPMV_XIDX_MAX)
        return vqe_fail(ctx, VQE_ENOTSUP, "sliced layout of slot %d: %lld flip masks, more than the "
                        "index form's %d", s, (long long)nx, SPMV_XIDX_MAX);
    const int64_t n = total > 0 ? total : 1;
    const bool real = (sched & VQE_SPMV_REAL) != 0;
    const int64_t vb = (int64_t)vqe_elem_bytes(H->dtype) / (real ? 2 : 1);
    // 16-bit columns, or one 32-bit word per three entries (whole groups)
    const int64_t cb = xi ? (n + 2) / 3 * 4 + 8 : n * 2;
    if ((rc = grow_ctx(ctx, b.code, b.code_cap, cb, "slice codes", s)) ||
        (rc = grow_ctx(ctx, b.val, b.val_cap, n * vb, "slice values", s)))
        return rc;
    if (xi)
        launch_sell_fill_x(H, E, real, (const uint16_t *)m, (const int2 *)(m + o_sl),
                           (const uint16_t *)(m + o_xmap), (uint32_t *)*b.code, *b.val, ctx->stream);
    else
        launch_sell_fill(H, E, real, (const uint16_t *)m, (const int2 *)(m + o_sl),
                         (uint16_t *)*b.code, *b.val, ctx->stream);
    VQE_LAUNCH_CHECK(ctx);
    st.scode = (const uint16_t *)*b.code;
    st.sval = *b.val;
    st.srow = (const uint16_t *)m;
    st.sslice = (const int2 *)(m + o_sl);
    st.sxtab = xi ? (const uint16_t *)(m + o_xtab) : nullptr;
    st.nx = (int32_t)nx;
    *entries = total;
    return VQE_OK;
}

// The same for a column-tiled H (VQE_SPMV_SLICED on a state larger than LDS):
// the slab tables (row order, slices, slab totals and starts, the total, the
// tile parts each slab reaches) in meta, the tile-local codes in code, the
// values in val.
int sliced_tiled_build(vqe_ctx *ctx, const vqe_csr *H, int sched, const SellBufs &b, SpmvState &st,
                       int64_t *entries, int s)
{
    const int E = sched & 0xff;
    const int32_t R = SPMV_SELLT_ROWS, tc = spmv_sellt_tile_cols(H->dtype);
    const int32_t nt = (int32_t)((H->dim + tc - 1) / tc);
    const int64_t nb = (H->dim + R - 1) / R, nslab = nb * nt;
    const size_t o_sl = vqe_align((size_t)nslab * R * sizeof(uint16_t));
    const size_t o_tot = o_sl + vqe_align((size_t)nslab * SPMV_SLICES_PER_BLOCK * sizeof(int2));
    const size_t o_base = o_tot + vqe_align((size_t)nslab * sizeof(int64_t));
    const size_t o_all = o_base + vqe_align((size_t)nslab * sizeof(int64_t));
    const size_t o_msk = o_all + vqe_align(sizeof(int64_t));
    int rc = grow_ctx(ctx, b.meta, b.meta_cap, (int64_t)(o_msk + (size_t)nslab * sizeof(uint32_t)),
                      "slab tables", s);
    if (rc)
        return rc;
    char *m = (char *)*b.meta;
    uint32_t *msk = (uint32_t *)(m + o_msk);
    launch_sellt_layout(H, nt, tc, E, (uint16_t *)m, (int2 *)(m + o_sl), (int64_t *)(m + o_tot),
                        (int64_t *)(m + o_base), (int64_t *)(m + o_all), msk, ctx->stream);
    VQE_LAUNCH_CHECK(ctx);
    int64_t total = 0;
    VQE_HIP(ctx, hipMemcpyAsync(&total, m + o_all, sizeof(total), hipMemcpyDeviceToHost, ctx->stream));
    VQE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (total < 0)
        return vqe_fail(ctx, VQE_EHIP, "sliced layout of slot %d: bad size", s);
    const int64_t n = total > 0 ? total : 1;
    if ((rc = grow_ctx(ctx, b.code, b.code_cap, n * 2, "slice codes", s)) ||
        (rc = grow_ctx(ctx, b.val, b.val_cap, n * (int64_t)vqe_elem_bytes(H->dtype), "slice values", s)))
        return rc;
    launch_sellt_fill(H, nt, tc, E, (const uint16_t *)m, (const int2 *)(m + o_sl),
                      (const int64_t *)(m + o_base), (uint16_t *)*b.code, *b.val, msk, ctx->stream);
    VQE_LAUNCH_CHECK(ctx);
    st.scode = (const uint16_t *)*b.code;
    st.sval = *b.val;
    st.srow = (const uint16_t *)m;
    st.sslice = (const int2 *)(m + o_sl);
    st.boff = (const int64_t *)(m + o_base);
    st.smask = msk;
    st.blk_rows = R;
    st.tile_cols = tc;
    st.ntiles = nt;
    st.nblocks = (int32_t)nb;
    *entries = total;
    return VQE_OK;
}

// (Re)build slot s's sliced layout (either form) in its plan-owned buffers --
// tables in prow, codes in col16, values in vre -- and point the slot's host
// descriptor at it (the caller uploads the descriptor).
int sliced_fill(vqe_batch *p, int s, const vqe_csr *H, int sched)
{
    SpmvState &st = reinterpret_cast<SpmvState *>(p->image.data() + p->o_spmv)[s];
    const SellBufs b{&p->prow[s], &p->col16[s], &p->vre[s], &p->prow_cap[s], &p->col16_cap[s],
                     &p->vre_cap[s]};
    return (sched & VQE_SPMV_BLOCKED) ? sliced_tiled_build(p->ctx, H, sched, b, st, &p->entries[s], s)
                                      : sliced_build(p->ctx, H, sched, b, st, &p->entries[s], s);
}

// (Re)build slot s's blocked layout of H (VQE_SPMV_BLOCKED) in its plan-owned
// allocation and point the slot's host descriptor at it (the caller uploads
// the descriptor).  The layout is built on the context stream from the CSR,
// which must stay valid while it runs.
int blocked_fill(vqe_batch *p, int s, const vqe_csr *H)
{
    SpmvState &st = reinterpret_cast<SpmvState *>(p->image.data() + p->o_spmv)[s];
    const int32_t R = SPMV_BLK_ROWS, tc = spmv_blk_tile_cols(H->dtype);
    const int32_t nt = (int32_t)((H->dim + tc - 1) / tc);
    const int64_t nb = (H->dim + R - 1) / R, nslab = nb * nt;
    const int64_t cap = H->nnz + 4 * nslab + 4;     // entries, with the slabs' alignment
    const size_t o_rp = 0, o_len = o_rp + vqe_align((size_t)nslab * (R + 1) * sizeof(int32_t));
    const size_t o_off = o_len + vqe_align((size_t)nslab * sizeof(int64_t));
    const size_t o_code = o_off + vqe_align((size_t)(nslab + 1) * sizeof(int64_t));
    const size_t o_val = o_code + vqe_align((size_t)cap * sizeof(uint16_t));
    const size_t bytes = o_val + vqe_align((size_t)cap * vqe_elem_bytes(H->dtype));
    int rc = grow(p, &p->blk[s], &p->blk_cap[s], (int64_t)bytes, "blocked layout", s);
    if (rc)
        return rc;
    char *m = (char *)p->blk[s];
    launch_blk_layout(H, nt, tc, R, (int32_t *)(m + o_rp), (int64_t *)(m + o_len),
                      (int64_t *)(m + o_off), (uint16_t *)(m + o_code), m + o_val, p->ctx->stream);
    VQE_LAUNCH_CHECK(p->ctx);
    st.brp = (const int32_t *)(m + o_rp);
    st.boff = (const int64_t *)(m + o_off);
    st.bcode = (const uint16_t *)(m + o_code);
    st.bval = m + o_val;
    st.blk_rows = R;
    st.tile_cols = tc;
    st.ntiles = nt;
    st.nblocks = (int32_t)nb;
    return VQE_OK;
}

// The step is two launch sequences: the H products (sequence A) and the rest
// (sequence B: screen, per-state finalisation and selection, Taylor update,
// renormalisation).  `ev` (nullable) receives the phase events.
void launch_products(vqe_batch *p, const SpmvState *states)
{
    SpmvState dummy{};
    for (auto &l : p->spmv) {
        if (l.lanes & VQE_SPMV_BLOCKED)
            launch_spmv_blk(p->dtype, l.lanes, states, l.tasks, l.grid, p->ctx->stream);
        else if (l.lanes & VQE_SPMV_TILED)
            launch_spmv_tiled(p->dtype, l.lanes, states, l.tasks, l.grid, l.sum_tasks, l.sum_grid,
                              p->ctx->stream);
        else
            launch_spmv(p->dtype, l.lanes, dummy, states, l.tasks, l.grid, p->ctx->stream, l.max_dim);
    }
}

int enqueue_spmv(vqe_batch *p)
{
    launch_products(p, p->d_spmv);
    VQE_LAUNCH_CHECK(p->ctx);
    return VQE_OK;
}

// theta_row (nullable, matrix-free plans): the update's angles from this
// device row instead of the plan's angle buffer (which the update then sets)
int enqueue_rest(vqe_batch *p, uint32_t flags, hipEvent_t *ev, const double *theta_row = nullptr)
{
    vqe_ctx *ctx = p->ctx;
    hipStream_t s = ctx->stream;
    auto mark = [&](int i) -> int {
        if (ev)
            VQE_HIP(ctx, hipEventRecord(ev[i], s));
        return VQE_OK;
    };
    // the screen, then one per-state kernel for the energy, the gradient sums
    // and the selection (the energy phase event coincides with the start)
    int rc = mark(2);
    const bool grad = p->mf || p->n_screen_tasks;
    if (p->mf && p->n_screen1_tasks && !(flags & VQE_STEP_TILED_SCREEN))
        launch_screen_mf_real(p->dtype, p->d_screen, p->d_screen1_tasks, p->n_screen1_tasks,
                              p->screen1_lds, s);
    else if (p->mf)
        launch_screen_mf(p->dtype, p->d_screen, p->d_screen_tasks, p->n_screen_tasks,
                         p->screen_lds, s);
    else if (p->n_screen_tasks)
        launch_screen(p->dtype, p->d_screen, p->d_tables, p->d_screen_tasks, p->n_screen_tasks,
                      (unsigned)p->B, p->screen_lds, s);
    // without a line search the matrix-free update does the finalisation
    // itself (one kernel boundary less)
    // (only while the screen's partial sums are few: every update block reads
    // all of its state's)
    const bool fused_fin = p->mf && p->max_m <= FIN_LDS_G && p->max_gpart <= FIN_FUSE_PARTIALS &&
                           !(flags & VQE_STEP_NO_UPDATE) &&
                           !(flags & VQE_STEP_LINESEARCH);
    if (!fused_fin)
        launch_step_fin(p->d_spmv, p->d_screen, p->d_tables, p->d_sel, (unsigned)p->B, grad,
                        !(flags & VQE_STEP_FORCED), p->rel_tie, s);
    rc = rc ? rc : mark(3);
    rc = rc ? rc : mark(4);
    if ((flags & VQE_STEP_LINESEARCH) && !(flags & VQE_STEP_NO_UPDATE)) {
        // v1 = A psi, v2 = A^2 psi; S v1 and S v2 with the plan's schedules;
        // Re<v1|S v2>; then the angle
        launch_ls_vectors(p->dtype, p->d_ls, p->d_ls_tasks, p->n_ls_tasks, s);
        launch_products(p, p->d_ls1);
        launch_products(p, p->d_ls2);
        launch_ls_dot(p->dtype, p->d_ls, p->d_ls_tasks, p->n_ls_tasks, s);
        launch_ls_solve(p->d_ls, (unsigned)p->B, s);
    }
    if (!(flags & VQE_STEP_NO_UPDATE)) {
        if (fused_fin)
            launch_taylor_mf_fin(p->dtype, p->d_tay, p->d_tay_tasks, p->n_tay_tasks, p->d_spmv,
                                 p->d_screen, p->d_tables, p->d_sel, !(flags & VQE_STEP_FORCED),
                                 p->rel_tie, theta_row, s);
        else if (p->mf)
            launch_taylor_mf(p->dtype, p->d_tay, p->d_tay_tasks, p->n_tay_tasks, theta_row, s);
        else if (p->compact_taylor)
            launch_taylor_compact(p->dtype, p->d_tay, p->d_tay_tasks, p->n_tay_tasks, s);
        else
            launch_taylor_pair(p->dtype, p->d_tay, p->d_tay_tasks, p->n_tay_tasks, s);
    }
    rc = rc ? rc : mark(5);
    if (!(flags & VQE_STEP_NO_UPDATE) && (flags & VQE_STEP_RENORM)) {
        if (p->mf)
            launch_norm_mf(p->dtype, p->d_tay, p->d_norm_tasks, p->n_norm_tasks, s);
        else
            launch_norm(p->dtype, p->d_tay, p->d_norm_tasks, p->n_norm_tasks, s);
    }
    rc = rc ? rc : mark(6);
    if (rc)
        return rc;
    VQE_LAUNCH_CHECK(ctx);
    return VQE_OK;
}

int enqueue_step(vqe_batch *p, uint32_t flags, hipEvent_t *ev = nullptr)
{
    if (ev)
        VQE_HIP(p->ctx, hipEventRecord(ev[0], p->ctx->stream));
    int rc = enqueue_spmv(p);
    if (rc)
        return rc;
    if (ev)
        VQE_HIP(p->ctx, hipEventRecord(ev[1], p->ctx->stream));
    return enqueue_rest(p, flags, ev);
}

// Capture `fn` on the context stream into an executable graph.
template <class F> int capture(vqe_ctx *ctx, F fn, hipGraph_t *g_out, hipGraphExec_t *x_out)
{
    if (!ctx->stream)
        return vqe_fail(ctx, VQE_EINVAL, "graph capture needs a non-null stream");
    VQE_HIP(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
    int rc = fn();
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(ctx->stream, &g);
    if (rc) {
        if (g)
            (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess)
        return vqe_fail(ctx, VQE_EHIP, "graph capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(x_out, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        *x_out = nullptr;
        return vqe_fail(ctx, VQE_EHIP, "graph instantiation failed: %s", hipGetErrorString(e));
    }
    *g_out = g;
    return VQE_OK;
}

// Graph launch of the step (graphs captured on first use).  Without events,
// one graph holds the whole step for this flag set; with events, sequence A
// and sequence B are separate graphs: events 0 and 1 bracket sequence A,
// event 2 follows sequence B.
int graph_step(vqe_batch *p, uint32_t flags, hipEvent_t *ev)
{
    vqe_ctx *ctx = p->ctx;
    const unsigned key = (flags & 7u) | ((flags & VQE_STEP_LINESEARCH) ? 8u : 0u) |
                         ((flags & VQE_STEP_TILED_SCREEN) ? 16u : 0u);
    int rc;
    if (!ev) {
        if (!p->exec_all[key] &&
            (rc = capture(ctx, [&] {
                 const int r = enqueue_spmv(p);
                 return r ? r : enqueue_rest(p, flags, nullptr);
             }, &p->graph_all[key], &p->exec_all[key])))
            return rc;
        VQE_HIP(ctx, hipGraphLaunch(p->exec_all[key], ctx->stream));
        return VQE_OK;
    }
    if (!p->exec_spmv && (rc = capture(ctx, [&] { return enqueue_spmv(p); }, &p->graph_spmv,
                                       &p->exec_spmv)))
        return rc;
    if (!p->exec[key] && (rc = capture(ctx, [&] { return enqueue_rest(p, flags, nullptr); },
                                       &p->graph[key], &p->exec[key])))
        return rc;
    if (ev)
        VQE_HIP(ctx, hipEventRecord(ev[0], ctx->stream));
    VQE_HIP(ctx, hipGraphLaunch(p->exec_spmv, ctx->stream));
    if (ev)
        VQE_HIP(ctx, hipEventRecord(ev[1], ctx->stream));
    VQE_HIP(ctx, hipGraphLaunch(p->exec[key], ctx->stream));
    if (ev)
        VQE_HIP(ctx, hipEventRecord(ev[2], ctx->stream));
    return VQE_OK;
}

// Eager step with three events: before the H products, after them, at the end.
int enqueue_step3(vqe_batch *p, uint32_t flags, hipEvent_t *ev)
{
    VQE_HIP(p->ctx, hipEventRecord(ev[0], p->ctx->stream));
    int rc = enqueue_spmv(p);
    if (rc)
        return rc;
    VQE_HIP(p->ctx, hipEventRecord(ev[1], p->ctx->stream));
    rc = enqueue_rest(p, flags, nullptr);
    if (rc)
        return rc;
    VQE_HIP(p->ctx, hipEventRecord(ev[2], p->ctx->stream));
    return VQE_OK;
}

}  // namespace

extern "C" int vqe_batch_create(vqe_ctx *ctx, int32_t B, const vqe_batch_item *items,
                                const vqe_batch_io *io, double rel_tie, vqe_batch **out)
{
    if (!ctx || !out)
        return VQE_EINVAL;
    *out = nullptr;
    if (B < 1 || !items || !io || !io->theta || !io->energy_out || !io->g_out ||
        !io->g_offset_host || !io->k_io || !io->gmax_out || !(rel_tie >= 0.0 && rel_tie < 1.0))
        return vqe_fail(ctx, VQE_EINVAL, "vqe_batch_create: bad arguments");
    const int dtype = items[0].H ? items[0].H->dtype : -1;
    for (int s = 0; s < B; s++) {
        const vqe_batch_item &it = items[s];
        int rc = check_csr(ctx, it.H, "vqe_batch_create");
        if (rc)
            return rc;
        if (it.H->dtype != dtype)
            return vqe_fail(ctx, VQE_EINVAL, "vqe_batch_create: states differ in dtype");
        if (!it.pool || it.pool->M < 1 || it.pool->n_qubits != it.H->n_qubits ||
            it.pool->dtype != dtype)
            return vqe_fail(ctx, VQE_EINVAL, "vqe_batch_create: bad pool for state %d", s);
        if (!(it.pool->mf ? true : false) != !(items[0].pool && items[0].pool->mf))
            return vqe_fail(ctx, VQE_EINVAL,
                            "vqe_batch_create: either every pool or none is matrix-free");
        if (it.pool->mf) {
            // the matrix-free screen stages row pairs with 16-byte loads
            if ((((uintptr_t)it.psi) & 15) || (((uintptr_t)it.sigma) & 15))
                return vqe_fail(ctx, VQE_EINVAL,
                                "vqe_batch_create: psi and sigma must be 16-byte aligned");
            if (vqe_mf_pool_size(it.pool->mf) != it.pool->M ||
                vqe_mf_pool_qubits(it.pool->mf) != it.pool->n_qubits)
                return vqe_fail(ctx, VQE_EINVAL,
                                "vqe_batch_create: matrix-free pool of state %d does not match", s);
        } else {
            if (!it.pool->ops || !it.pool->ops_host)
                return vqe_fail(ctx, VQE_EINVAL, "vqe_batch_create: bad pool for state %d", s);
            if (!it.pool->all_pairing)
                return vqe_fail(ctx, VQE_ENOTSUP,
                                "vqe_batch_create: state %d has a non-pairing generator", s);
        }
        if (!it.psi || !it.sigma)
            return vqe_fail(ctx, VQE_EINVAL, "vqe_batch_create: null psi or sigma");
        if (it.spmv_schedule != 0 && !vqe_valid_schedule(it.spmv_schedule))
            return vqe_fail(ctx, VQE_EINVAL, "vqe_batch_create: bad spmv_schedule");
    }

    vqe_batch *p = new (std::nothrow) vqe_batch();
    if (!p)
        return VQE_ENOMEM;
    p->ctx = ctx;
    p->theta_io = io->theta;
    p->B = B;
    p->dtype = dtype;
    p->rel_tie = rel_tie;

    // --- XCD assignment: largest H first onto the least loaded XCD
    std::vector<int> order(B), xcd_of(B);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return items[a].H->nnz > items[b].H->nnz; });
    std::vector<double> load(kXcd, 0.0);
    for (int s : order) {
        int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        xcd_of[s] = x;
        load[x] += (double)items[s].H->nnz * 12.0 + (double)items[s].H->dim * 20.0;
    }

    Arena A;
    const size_t o_spmv = A.take(sizeof(SpmvState) * B);
    const size_t o_sel = A.take(sizeof(SelectState) * B);
    const size_t o_tay = A.take(sizeof(TaylorState) * B);
    std::vector<int> lanes(B);
    std::vector<size_t> o_epart(B), o_npart(B), o_gpart(B);
    std::vector<size_t> o_tptr(B, 0), o_tpart(B, 0);
    std::vector<int> ntiles(B, 0), tcols(B, 0);
    for (int s = 0; s < B; s++) {
        const vqe_csr *H = items[s].H;
        const int req = items[s].spmv_schedule ? items[s].spmv_schedule : vqe_default_schedule(H);
        lanes[s] = vqe_batch_schedule(H, req);
        int64_t nblk = spmv_blocks(H->dim, lanes[s]);
        if (lanes[s] & VQE_SPMV_BLOCKED) {
            // the layout lives in the slot's own buffers (blocked_fill,
            // sliced_fill)
            const int64_t rb = (lanes[s] & VQE_SPMV_SLICED) ? SPMV_SELLT_ROWS : SPMV_BLK_ROWS;
            nblk = (H->dim + rb - 1) / rb;
        } else if (lanes[s] & VQE_SPMV_TILED) {
            // real-value tiles are twice as wide (real parts in storage precision)
            tcols[s] = (lanes[s] & VQE_SPMV_REAL) ? spmv_tile_cols_real(dtype) : spmv_tile_cols(dtype);
            ntiles[s] = (int)((H->dim + tcols[s] - 1) / tcols[s]);
            o_tptr[s] = A.take((size_t)(ntiles[s] + 1) * H->dim * sizeof(int32_t));
            o_tpart[s] = A.take((size_t)ntiles[s] * H->dim * 2 * sizeof(double));
            nblk = (H->dim + SPMV_SUM_ROWS - 1) / SPMV_SUM_ROWS;
        }
        o_epart[s] = A.take(std::max(vqe_spmv_partials_bytes(H->dim, lanes[s] & ~VQE_SPMV_TILED),
                                     (size_t)nblk * 3 * sizeof(double)));
        const int64_t nn = (H->dim + NORM_ROWS_PER_BLOCK - 1) / NORM_ROWS_PER_BLOCK;
        o_npart[s] = A.take(nn * sizeof(double));
    }

    // --- H product tasks, one table per lanes value
    std::map<int, std::vector<std::vector<int2>>> per_lanes, per_sum;
    std::vector<int2> bounds_list;
    std::vector<std::pair<unsigned, unsigned>> bounds_range(B, {0u, 0u});
    for (int s = 0; s < B; s++) {
        auto &per = per_lanes[lanes[s]];
        if (per.empty())
            per.resize(kXcd);
        const int64_t dim = items[s].H->dim;
        if (lanes[s] & VQE_SPMV_BLOCKED) {
            const int64_t rb = (lanes[s] & VQE_SPMV_SLICED) ? SPMV_SELLT_ROWS : SPMV_BLK_ROWS;
            const int nb = (int)((dim + rb - 1) / rb);
            for (int b = 0; b < nb; b++)
                per[xcd_of[s]].push_back(make_int2(s, b));
            continue;
        }
        if (lanes[s] & VQE_SPMV_TILED) {
            const int nb = (int)((dim + SPMV_LDS_ROWS - 1) / SPMV_LDS_ROWS);
            for (int b = 0; b < nb; b++)
                for (int t = 0; t < ntiles[s]; t++)
                    per[xcd_of[s]].push_back(make_int2(s, (b << 8) | t));
            auto &ps = per_sum[lanes[s]];
            if (ps.empty())
                ps.resize(kXcd);
            for (int b = 0; b < (int)((dim + SPMV_SUM_ROWS - 1) / SPMV_SUM_ROWS); b++)
                ps[xcd_of[s]].push_back(make_int2(s, b));
            bounds_range[s] = {(unsigned)bounds_list.size(), (unsigned)((dim + 255) / 256)};
            for (int b = 0; b < (int)((dim + 255) / 256); b++)
                bounds_list.push_back(make_int2(s, b));
            continue;
        }
        const int nb = (int)spmv_blocks(dim, lanes[s]);
        for (int b = 0; b < nb; b++)
            per[xcd_of[s]].push_back(make_int2(s, b));
    }
    std::vector<std::pair<int, size_t>> spmv_tab;
    std::vector<std::vector<int2>> spmv_lists, sum_lists;
    std::vector<size_t> sum_tab;
    std::vector<int64_t> spmv_maxdim;
    for (auto &kv : per_lanes) {
        auto flat = interleave(kv.second, make_int2(-1, 0));
        spmv_tab.push_back({kv.first, A.take(flat.size() * sizeof(int2))});
        spmv_lists.push_back(std::move(flat));
        std::vector<int2> sflat;
        if ((kv.first & VQE_SPMV_TILED) && !(kv.first & VQE_SPMV_BLOCKED))
            sflat = interleave(per_sum[kv.first], make_int2(-1, 0));
        sum_tab.push_back(A.take(sflat.size() * sizeof(int2) + 8));
        sum_lists.push_back(std::move(sflat));
        int64_t md = 0;
        for (int s = 0; s < B; s++)
            if (lanes[s] == kv.first)
                md = std::max<int64_t>(md, items[s].H->dim);
        spmv_maxdim.push_back(md);
    }
    const size_t o_btasks = A.take(bounds_list.size() * sizeof(int2) + 8);

    const bool mf_mode = items[0].pool->mf != nullptr;
    p->mf = mf_mode;
    // pool identity: the matrix-free object, or the CSR descriptor array
    auto pool_key = [&](const vqe_pool *pl) -> const void * {
        return mf_mode ? (const void *)pl->mf : (const void *)pl->ops;
    };
    auto fail_free = [&](int rc) {
        for (void *m : p->table_mem)
            (void)hipFree(m);
        delete p;
        return rc;
    };

    // --- gradient screen: one table per distinct pool (pair table, or the
    //     matrix-free records); tasks per (state, row tile, generator range),
    //     on the state's XCD
    std::map<const void *, int> table_of;
    std::vector<PairTable> tables;
    std::vector<const MfTable *> mf_dev;        // device header per table (mf mode)
    std::vector<const vqe_mf_desc *> mf_desc_ptrs;  // device descriptors per table (mf mode)
    std::vector<MfHostPlan> mf_plans, mf_plans1;
    std::vector<const MfTable *> mf_dev1;       // whole-state tables (real-state screen)
    // one allocation per table: header, tile records, whole-state records,
    // lists, descriptors, index tables
    auto upload_mf = [&](const MfHostPlan &hp, const vqe_mf_pool *pool, const MfTable **dev,
                 const vqe_mf_desc **ddesc) -> int {
    const size_t o_h = 0, o_t = vqe_align(sizeof(MfTable));
    const size_t o_f = o_t + vqe_align(hp.tile_recs.size() * sizeof(MfRec));
    const size_t o_l = o_f + vqe_align(hp.full_recs.size() * sizeof(MfRec));
    const size_t o_d = o_l + vqe_align(hp.lists.size() * sizeof(int32_t) + 4);
    const size_t o_x = o_d + vqe_align((size_t)hp.M * sizeof(vqe_mf_desc));
    const size_t o_i = o_x + vqe_align(hp.tabs.size() * sizeof(uint32_t) + 4);
    const size_t bytes = o_i + vqe_align(hp.list_info.size() * sizeof(int4) + 16);
    char *mem = nullptr;
    if (hipMalloc((void **)&mem, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return vqe_fail(ctx, VQE_ENOMEM, "vqe_batch_create: record allocation failed");
    }
    p->table_mem.push_back(mem);
    p->table_bytes += bytes;
    MfTable h{};
    h.tile_recs = (const MfRec *)(mem + o_t);
    h.full_recs = (const MfRec *)(mem + o_f);
    h.lists = (const int32_t *)(mem + o_l);
    h.desc = (const vqe_mf_desc *)(mem + o_d);
    h.tabs = (const uint32_t *)(mem + o_x);
    h.linfo = (const int4 *)(mem + o_i);
    h.nlists = (int32_t)hp.list_info.size();
    h.M = hp.M;
    h.ntile = hp.ntile;
    h.tile_rows = hp.tile_rows;
    hipError_t e = hipMemcpy(mem + o_h, &h, sizeof(h), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(mem + o_t, hp.tile_recs.data(), hp.tile_recs.size() * sizeof(MfRec),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(mem + o_f, hp.full_recs.data(), hp.full_recs.size() * sizeof(MfRec),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess && !hp.lists.empty())
        e = hipMemcpy(mem + o_l, hp.lists.data(), hp.lists.size() * sizeof(int32_t),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess && !hp.tabs.empty())
        e = hipMemcpy(mem + o_x, hp.tabs.data(), hp.tabs.size() * sizeof(uint32_t),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess && !hp.list_info.empty()) {
        std::vector<int4> li;
        for (const auto &L : hp.list_info)
            li.push_back(make_int4(L.off, L.len, L.v, 0));
        e = hipMemcpy(mem + o_i, li.data(), li.size() * sizeof(int4), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) {
        std::vector<vqe_mf_desc> dd(hp.M);
        for (int j = 0; j < hp.M; j++)
            (void)vqe_mf_pool_get(pool, j, &dd[j]);
        e = hipMemcpy(mem + o_d, dd.data(), dd.size() * sizeof(vqe_mf_desc),
                      hipMemcpyHostToDevice);
    }
    if (e != hipSuccess)
        return vqe_fail(ctx, VQE_EHIP, "vqe_batch_create: record upload: %s",
                        hipGetErrorString(e));
    *dev = (const MfTable *)(mem + o_h);
    *ddesc = (const vqe_mf_desc *)(mem + o_d);
    return VQE_OK;
    };

    // the real-state screen applies when every generator of every pool has a
    // real value and is anti-Hermitian (so the diagonal shift drops out) and
    // every state fits one LDS tile as reals
    bool real_screen = mf_mode;
    for (int s = 0; s < B && real_screen; s++) {
        real_screen = screen_real_lds(items[s].H->dim, dtype) <= SCREEN_LDS_BYTES;
        const vqe_mf_pool *pl = items[s].pool->mf;
        for (int j = 0; j < items[s].pool->M && real_screen; j++) {
            vqe_mf_desc d;
            real_screen = vqe_mf_pool_get(pl, j, &d) == VQE_OK && d.v_im == 0.0 &&
                          mf_antihermitian(d);
        }
    }
    for (int s = 0; s < B; s++) {
        const void *key = pool_key(items[s].pool);
        if (table_of.count(key))
            continue;
        PairTable tb{};
        if (mf_mode) {
            MfHostPlan hp;
            char err[160] = {0};
            const int32_t tile = screen_tile_rows(items[s].H->dim, dtype);
            int rc = mf_host_plan(items[s].pool->mf, tile, &hp, err, sizeof(err));
            if (rc)
                return fail_free(vqe_fail(ctx, rc, "vqe_batch_create: %s", err));
            const MfTable *dev = nullptr;
            const vqe_mf_desc *ddesc = nullptr;
            if ((rc = upload_mf(hp, items[s].pool->mf, &dev, &ddesc)))
                return fail_free(rc);
            // the real-state screen: the same records on one whole-state tile
            const MfTable *dev1 = nullptr;
            if (real_screen) {
                MfHostPlan hp1;
                if ((rc = mf_host_plan(items[s].pool->mf, items[s].H->dim, &hp1, err, sizeof(err))))
                    return fail_free(vqe_fail(ctx, rc, "vqe_batch_create: %s", err));
                const vqe_mf_desc *unused = nullptr;
                if ((rc = upload_mf(hp1, items[s].pool->mf, &dev1, &unused)))
                    return fail_free(rc);
                mf_plans1.push_back(std::move(hp1));
            } else {
                mf_plans1.emplace_back();
            }
            mf_dev1.push_back(dev1);
            tb.M = hp.M;
            tb.nt = hp.ntile;
            tb.tile_rows = hp.tile_rows;
            mf_dev.push_back(dev);
            mf_desc_ptrs.push_back(ddesc);
            mf_plans.push_back(std::move(hp));
        } else {
            void *mem[2] = {nullptr, nullptr};
            size_t bytes = 0;
            int rc = pair_table_build(ctx, items[s].pool, items[s].H->dim, &tb, mem, &bytes);
            if (rc)
                return fail_free(rc);
            for (void *m : mem)
                if (m)
                    p->table_mem.push_back(m);
            p->table_bytes += bytes;
        }
        table_of[key] = (int)tables.size();
        tables.push_back(tb);
    }
    const size_t o_tables = A.take(sizeof(PairTable) * tables.size());
    const size_t o_screen = A.take(sizeof(ScreenState) * B);
    std::vector<std::vector<int4>> screen_per(kXcd);
    const int n_ranges = 2;
    for (int s = 0; s < B; s++) {
        const int ti = table_of[pool_key(items[s].pool)];
        const PairTable &tb = tables[ti];
        const int M = tb.M;
        if (mf_mode) {
            // about eight workgroups per state, split over the lists by work
            const MfHostPlan &hp = mf_plans[ti];
            double W = 0.0;
            for (auto &L : hp.list_info)
                W += L.work;
            for (auto &L : hp.list_info) {
                const int nr = std::max(1, std::min({L.len, 255, (int)std::lround(8.0 * L.work / W)}));
                for (int r = 0; r < nr; r++)
                    screen_per[xcd_of[s]].push_back(make_int4(s, L.off, L.len, r | (nr << 8) | (L.v << 16)));
            }
            const size_t elem = 2 * vqe_elem_bytes(dtype);
            p->screen_lds = std::max(p->screen_lds, (size_t)hp.tile_rows * elem);
        } else {
            const int nr = std::min(n_ranges, M);
            for (int t = 0; t < tb.nt; t++)
                for (int r = 0; r < nr; r++)
                    screen_per[xcd_of[s]].push_back(make_int4(s, t, r, nr));
            const int64_t rows = std::min<int64_t>(tb.tile_rows, items[s].H->dim);
            p->screen_lds = std::max(p->screen_lds, (size_t)(2 * rows * vqe_elem_bytes(dtype)));
        }
        o_gpart[s] = A.take((size_t)M * tb.nt * sizeof(double));
    }
    auto screen_flat = interleave(screen_per, make_int4(-1, 0, 0, 0));
    const size_t o_stasks = A.take(screen_flat.size() * sizeof(int4));
    // real-state screen: four workgroups per state (one per CU for 64
    // states), generators dealt over them by descending cost; a complex state
    // runs the tiled screen's lists in the same workgroups, so the LDS holds
    // either form
    std::vector<std::vector<int4>> screen1_per(kXcd);
    // (ADAPTVQE_SCREEN_WG overrides the four, 1..64, for tuning)
    int split = 4;
    if (const char *e = std::getenv("ADAPTVQE_SCREEN_WG"))
        split = std::max(1, std::min(64, std::atoi(e)));
    if (real_screen)
        for (int s = 0; s < B; s++) {
            const MfHostPlan &hp1 = mf_plans1[table_of[pool_key(items[s].pool)]];
            for (auto &L : hp1.list_info) {
                const int nr = std::max(1, std::min(L.len, split));
                for (int r = 0; r < nr; r++)
                    screen1_per[xcd_of[s]].push_back(make_int4(s, L.off, L.len, r | (nr << 8)));
            }
            p->screen1_lds = std::max({p->screen1_lds, screen_real_lds(items[s].H->dim, dtype),
                                       p->screen_lds});
        }
    auto screen1_flat = interleave(screen1_per, make_int4(-1, 0, 0, 0));
    const size_t o_s1tasks = A.take(screen1_flat.size() * sizeof(int4) + 16);

    // --- Taylor and norm tasks (matrix-free records or compact tables: blocks
    //     cover the largest generator's pairs; otherwise the CSR rows)
    p->compact_taylor = !mf_mode;
    std::vector<int> max_pairs(tables.size(), 0);
    for (size_t i = 0; i < tables.size(); i++) {
        if (mf_mode) {
            for (const MfRec &r : mf_plans[i].full_recs)
                max_pairs[i] = std::max(max_pairs[i], r.nfree < 0 ? 0 : 1 << r.nfree);
            continue;
        }
        p->compact_taylor = p->compact_taylor && tables[i].words != nullptr;
        const PairTable &tb = tables[i];
        std::vector<int32_t> pts((size_t)tb.M * tb.nt + 1);
        if (hipMemcpy(pts.data(), tb.pts, pts.size() * 4, hipMemcpyDeviceToHost) != hipSuccess)
            return fail_free(vqe_fail(ctx, VQE_EHIP, "vqe_batch_create: reading the pair table failed"));
        for (int j = 0; j < tb.M; j++)
            max_pairs[i] = std::max(max_pairs[i], pts[(size_t)(j + 1) * tb.nt] - pts[(size_t)j * tb.nt]);
    }
    std::vector<std::vector<int2>> tay_per(kXcd), norm_per(kXcd);
    std::vector<size_t> o_taypart(B, 0);
    std::vector<int32_t> ntay(B, 0);
    for (int s = 0; s < B; s++) {
        const int64_t dim = items[s].H->dim;
        const int mp = max_pairs[table_of[pool_key(items[s].pool)]];
        const int nt = (mf_mode || p->compact_taylor)
                           ? std::max(1, (mp + TAYLOR_ROWS_PER_BLOCK - 1) / TAYLOR_ROWS_PER_BLOCK)
                           : (int)((dim + TAYLOR_ROWS_PER_BLOCK - 1) / TAYLOR_ROWS_PER_BLOCK);
        const int nn = (int)((dim + NORM_ROWS_PER_BLOCK - 1) / NORM_ROWS_PER_BLOCK);
        for (int b = 0; b < nt; b++)
            tay_per[xcd_of[s]].push_back(make_int2(s, b));
        if (mf_mode) {
            // the update blocks' changes of |psi|^2, for the renormalisation
            o_taypart[s] = A.take((size_t)nt * sizeof(double));
            ntay[s] = nt;
        }
        for (int b = 0; b < nn; b++)
            norm_per[xcd_of[s]].push_back(make_int2(s, b));
    }
    auto tay_flat = interleave(tay_per, make_int2(-1, 0));
    auto norm_flat = interleave(norm_per, make_int2(-1, 0));
    const size_t o_ttasks = A.take(tay_flat.size() * sizeof(int2));
    const size_t o_ntasks = A.take(norm_flat.size() * sizeof(int2));

    // --- allocate, then fill the host image with device addresses
    p->dmem_bytes = A.host.size();
    if (hipMalloc((void **)&p->dmem, p->dmem_bytes) != hipSuccess) {
        (void)hipGetLastError();
        for (void *m : p->table_mem)
            (void)hipFree(m);
        delete p;
        return vqe_fail(ctx, VQE_ENOMEM, "vqe_batch_create: allocation failed");
    }
    char *D = p->dmem;
    for (int s = 0; s < B; s++) {
        const vqe_batch_item &it = items[s];
        SpmvState &st = A.at<SpmvState>(o_spmv)[s];
        st.rowptr = it.H->rowptr;
        st.col = it.H->col;
        st.val = it.H->val;
        st.psi = it.psi;
        st.sigma = it.sigma;
        st.partials = (double *)(D + o_epart[s]);
        st.energy_out = io->energy_out + 3 * s;
        st.dim = it.H->dim;
        st.shift = it.H->diag_shift;
        st.nblocks = (int32_t)spmv_blocks(it.H->dim, lanes[s]);
        st.lanes = lanes[s];
        if (lanes[s] & VQE_SPMV_BLOCKED) {
            const int64_t rb = (lanes[s] & VQE_SPMV_SLICED) ? SPMV_SELLT_ROWS : SPMV_BLK_ROWS;
            st.nblocks = (int32_t)((it.H->dim + rb - 1) / rb);
        } else if (lanes[s] & VQE_SPMV_TILED) {
            st.tptr = (const int32_t *)(D + o_tptr[s]);
            st.tile_part = (double *)(D + o_tpart[s]);
            st.ntiles = ntiles[s];
            st.tile_cols = tcols[s];
            st.nblocks = (int32_t)((it.H->dim + SPMV_SUM_ROWS - 1) / SPMV_SUM_ROWS);
        }
        st.nnz = it.H->nnz;
        st.active = io->active ? io->active + s : nullptr;

        SelectState &se = A.at<SelectState>(o_sel)[s];
        se.g = io->g_out + io->g_offset_host[s];
        se.M = it.pool->M;
        se.k_out = io->k_io + s;
        se.gmax_out = io->gmax_out + s;
        se.active = io->active ? io->active + s : nullptr;

        TaylorState &ts = A.at<TaylorState>(o_tay)[s];
        ts.ops = it.pool->ops;
        ts.k = io->k_io + s;
        ts.M = it.pool->M;
        ts.theta = io->theta + s;
        ts.psi = it.psi;
        ts.dim = it.H->dim;
        ts.norm_partials = (double *)(D + o_npart[s]);
        ts.norm2_out = nullptr;
        ts.nblocks = (int32_t)((it.H->dim + NORM_ROWS_PER_BLOCK - 1) / NORM_ROWS_PER_BLOCK);
        ts.renorm = 1;
        ts.table = (const PairTable *)(D + o_tables) + table_of[pool_key(it.pool)];
        ts.active = io->active ? io->active + s : nullptr;
        ts.mf = mf_mode ? mf_dev[table_of[pool_key(it.pool)]] : nullptr;
        if (mf_mode) {
            // |psi|^2 before the update: this step's energy reduction
            ts.n2_prev = io->energy_out + 3 * s + 1;
            ts.tay_partials = (double *)(D + o_taypart[s]);
            ts.ntay = ntay[s];
        }
    }
    std::copy(tables.begin(), tables.end(), A.at<PairTable>(o_tables));
    for (int s = 0; s < B; s++) {
        ScreenState &ss = A.at<ScreenState>(o_screen)[s];
        ss.psi = items[s].psi;
        ss.sigma = items[s].sigma;
        ss.shift = items[s].H->diag_shift;
        ss.partials = (double *)(D + o_gpart[s]);
        ss.g_out = io->g_out + io->g_offset_host[s];
        ss.dim = items[s].H->dim;
        ss.table = table_of[pool_key(items[s].pool)];
        ss.active = io->active ? io->active + s : nullptr;
        ss.mf = mf_mode ? mf_dev[table_of[pool_key(items[s].pool)]] : nullptr;
        ss.mf_ntile = tables[table_of[pool_key(items[s].pool)]].nt;
        ss.mf1 = real_screen ? mf_dev1[table_of[pool_key(items[s].pool)]] : nullptr;
    }
    for (size_t i = 0; i < spmv_tab.size(); i++) {
        std::copy(spmv_lists[i].begin(), spmv_lists[i].end(), A.at<int2>(spmv_tab[i].second));
        std::copy(sum_lists[i].begin(), sum_lists[i].end(), A.at<int2>(sum_tab[i]));
        p->spmv.push_back({spmv_tab[i].first, (int2 *)(D + spmv_tab[i].second),
                           (unsigned)spmv_lists[i].size(), spmv_maxdim[i],
                           (int2 *)(D + sum_tab[i]), (unsigned)sum_lists[i].size()});
    }
    std::copy(bounds_list.begin(), bounds_list.end(), A.at<int2>(o_btasks));
    std::copy(screen_flat.begin(), screen_flat.end(), A.at<int4>(o_stasks));
    std::copy(screen1_flat.begin(), screen1_flat.end(), A.at<int4>(o_s1tasks));
    std::copy(tay_flat.begin(), tay_flat.end(), A.at<int2>(o_ttasks));
    std::copy(norm_flat.begin(), norm_flat.end(), A.at<int2>(o_ntasks));
    p->d_spmv = (SpmvState *)(D + o_spmv);
    p->d_sel = (SelectState *)(D + o_sel);
    p->d_tay = (TaylorState *)(D + o_tay);
    p->d_tables = (PairTable *)(D + o_tables);
    p->d_screen = (ScreenState *)(D + o_screen);
    p->d_screen_tasks = (int4 *)(D + o_stasks);
    p->n_screen_tasks = (unsigned)screen_flat.size();
    p->d_screen1_tasks = (int4 *)(D + o_s1tasks);
    p->n_screen1_tasks = (unsigned)screen1_flat.size();
    p->d_tay_tasks = (int2 *)(D + o_ttasks);
    p->n_tay_tasks = (unsigned)tay_flat.size();
    p->d_norm_tasks = (int2 *)(D + o_ntasks);
    p->n_norm_tasks = (unsigned)norm_flat.size();
    p->o_spmv = o_spmv;
    p->o_screen = o_screen;
    p->o_tay = o_tay;
    p->sched = lanes;
    for (int s = 0; s < B; s++) {
        p->pool_ops.push_back(pool_key(items[s].pool));
        p->dims.push_back(items[s].H->dim);
        p->table_idx.push_back(table_of[pool_key(items[s].pool)]);
        p->xcd.push_back(xcd_of[s]);
    }
    p->tables_host = tables;
    for (const PairTable &t : tables)
        p->max_m = std::max(p->max_m, t.M);
    for (const PairTable &t : tables)
        p->max_gpart = std::max<int64_t>(p->max_gpart, (int64_t)t.M * t.nt);
    if (mf_mode) {
        p->mf_host.assign(tables.size(), nullptr);
        for (int s = 0; s < B; s++)
            p->mf_host[table_of[pool_key(items[s].pool)]] = items[s].pool->mf;
        p->mf_desc_dev = mf_desc_ptrs;
    }
    hipError_t e = hipMemcpyAsync(p->dmem, A.host.data(), p->dmem_bytes, hipMemcpyHostToDevice,
                                  ctx->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        (void)hipFree(p->dmem);
        for (void *m : p->table_mem)
            (void)hipFree(m);
        delete p;
        return vqe_fail(ctx, VQE_EHIP, "vqe_batch_create: %s", hipGetErrorString(e));
    }
    p->image = std::move(A.host);
    // 16-bit column codes for the slots whose schedule reads them
    for (auto *v : {&p->col16, &p->vre, &p->prow})
        v->assign(B, nullptr);
    for (auto *v : {&p->col16_cap, &p->vre_cap, &p->prow_cap})
        v->assign(B, 0);
    p->blk.assign(B, nullptr);
    p->blk_cap.assign(B, 0);
    p->entries.assign(B, 0);
    bool any16 = false;
    for (int s = 0; s < B; s++) {
        if (!(lanes[s] & (VQE_SPMV_X16 | VQE_SPMV_BLOCKED | VQE_SPMV_SLICED)))
            continue;
        any16 = true;
        const bool sl = (lanes[s] & VQE_SPMV_SLICED) != 0, bl = (lanes[s] & VQE_SPMV_BLOCKED) != 0;
        const int rc16 = sl   ? sliced_fill(p, s, items[s].H, lanes[s])
                         : bl ? blocked_fill(p, s, items[s].H)
                              : codes_fill(p, s, items[s].H, lanes[s]);
        if (rc16) {
            vqe_batch_destroy(p);
            return rc16;
        }
    }
    if (any16) {
        e = hipMemcpyAsync(p->dmem + p->o_spmv, p->image.data() + p->o_spmv, sizeof(SpmvState) * B,
                           hipMemcpyHostToDevice, ctx->stream);
        if (e == hipSuccess)
            e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) {
            vqe_batch_destroy(p);
            return vqe_fail(ctx, VQE_EHIP, "vqe_batch_create: %s", hipGetErrorString(e));
        }
    }
    if (!bounds_list.empty()) {
        p->d_bounds_tasks = (int2 *)(D + o_btasks);
        p->bounds_range = bounds_range;
        launch_tile_bounds(p->d_spmv, p->d_bounds_tasks, (unsigned)bounds_list.size(), ctx->stream);
        e = hipGetLastError();
        if (e == hipSuccess)
            e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) {
            const int rc = vqe_fail(ctx, VQE_EHIP, "vqe_batch_create: tile bounds: %s",
                                    hipGetErrorString(e));
            vqe_batch_destroy(p);
            return rc;
        }
    }
    *out = p;
    return VQE_OK;
}

namespace {
void ls_fill_slot(vqe_batch *p, int s, double theta_max, char *D);
}

// A sliced layout of one operator, built once (vqe_layout_create) and pointed
// to by batch slots (vqe_batch_rebind_layout).
struct vqe_layout {
    vqe_ctx *ctx = nullptr;
    int32_t sched = 0;          // the effective batch schedule it was built for
    int32_t dtype = 0;
    int64_t dim = 0;
    const vqe_csr *H = nullptr; // identity check only
    void *meta = nullptr, *code = nullptr, *val = nullptr;
    int64_t meta_cap = 0, code_cap = 0, val_cap = 0;
    SpmvState st{};             // the layout's fields of a slot descriptor
    int64_t entries = 0;
};

namespace {
int rebind_impl(vqe_batch *p, int32_t slot, const vqe_batch_item *it, const vqe_layout *layout,
                const char *who)
{
    if (!p)
        return VQE_EINVAL;
    vqe_ctx *ctx = p->ctx;
    if (slot < 0 || slot >= p->B || !it)
        return vqe_fail(ctx, VQE_EINVAL, "%s: bad slot or item", who);
    int rc = check_csr(ctx, it->H, who);
    if (rc)
        return rc;
    if (!it->pool || !it->psi || !it->sigma || it->H->dtype != p->dtype ||
        it->H->dim != p->dims[slot] ||
        (p->mf ? (const void *)it->pool->mf : (const void *)it->pool->ops) != p->pool_ops[slot])
        return vqe_fail(ctx, VQE_EINVAL, "%s: item does not match slot %d", who, slot);
    if ((((uintptr_t)it->psi) & 15) || (((uintptr_t)it->sigma) & 15))
        return vqe_fail(ctx, VQE_EINVAL, "%s: psi and sigma must be 16-byte aligned", who);
    const int sched = vqe_batch_schedule(
        it->H, it->spmv_schedule ? it->spmv_schedule : vqe_default_schedule(it->H));
    if (sched != p->sched[slot])
        return vqe_fail(ctx, VQE_EINVAL, "%s: schedule differs from slot %d", who, slot);
    if (layout && (layout->sched != sched || layout->dim != it->H->dim ||
                   layout->dtype != it->H->dtype || layout->H != it->H))
        return vqe_fail(ctx, VQE_EINVAL, "%s: the layout was not built for this operator and schedule",
                        who);
    SpmvState *st = reinterpret_cast<SpmvState *>(p->image.data() + p->o_spmv) + slot;
    st->rowptr = it->H->rowptr;
    st->col = it->H->col;
    st->val = it->H->val;
    st->psi = it->psi;
    st->sigma = it->sigma;
    st->shift = it->H->diag_shift;
    st->nnz = it->H->nnz;
    ScreenState *ss = reinterpret_cast<ScreenState *>(p->image.data() + p->o_screen) + slot;
    ss->psi = it->psi;
    ss->sigma = it->sigma;
    ss->shift = it->H->diag_shift;
    TaylorState *ts = reinterpret_cast<TaylorState *>(p->image.data() + p->o_tay) + slot;
    ts->psi = it->psi;
    if (layout) {
        // a prebuilt sliced layout of this H: the slot points to its buffers,
        // taking the fields the builder writes (the column-tiled form also
        // fixes the slab geometry; otherwise the slot keeps its block count)
        st->scode = layout->st.scode;
        st->sval = layout->st.sval;
        st->srow = layout->st.srow;
        st->sslice = layout->st.sslice;
        st->sxtab = layout->st.sxtab;
        st->nx = layout->st.nx;
        if (sched & VQE_SPMV_BLOCKED) {
            st->boff = layout->st.boff;
            st->smask = layout->st.smask;
            st->blk_rows = layout->st.blk_rows;
            st->tile_cols = layout->st.tile_cols;
            st->ntiles = layout->st.ntiles;
            st->nblocks = layout->st.nblocks;
        }
        p->entries[slot] = layout->entries;
    } else if (sched & VQE_SPMV_SLICED) {
        rc = sliced_fill(p, slot, it->H, sched);
        if (rc)
            return rc;
    } else if (sched & VQE_SPMV_BLOCKED) {
        rc = blocked_fill(p, slot, it->H);
        if (rc)
            return rc;
    } else if (sched & VQE_SPMV_X16) {
        rc = codes_fill(p, slot, it->H, sched);
        if (rc)
            return rc;
    }
    hipStream_t s = ctx->stream;
    VQE_HIP(ctx, hipMemcpyAsync(p->dmem + ((char *)st - p->image.data()), st, sizeof(*st),
                                hipMemcpyHostToDevice, s));
    VQE_HIP(ctx, hipMemcpyAsync(p->dmem + ((char *)ss - p->image.data()), ss, sizeof(*ss),
                                hipMemcpyHostToDevice, s));
    VQE_HIP(ctx, hipMemcpyAsync(p->dmem + ((char *)ts - p->image.data()), ts, sizeof(*ts),
                                hipMemcpyHostToDevice, s));
    if (p->bounds_range.size() > (size_t)slot && p->bounds_range[slot].second > 0) {
        // the new H's per-tile row bounds
        launch_tile_bounds(p->d_spmv, p->d_bounds_tasks + p->bounds_range[slot].first,
                           p->bounds_range[slot].second, s);
        VQE_LAUNCH_CHECK(ctx);
    }
    if (p->ls_mem) {
        const double tm = reinterpret_cast<LsState *>(p->ls_image.data() + p->o_ls)[slot].theta_max;
        ls_fill_slot(p, slot, tm, p->ls_mem);
        const size_t offs[3] = {p->o_ls + slot * sizeof(LsState), p->o_ls1 + slot * sizeof(SpmvState),
                                p->o_ls2 + slot * sizeof(SpmvState)};
        const size_t sizes[3] = {sizeof(LsState), sizeof(SpmvState), sizeof(SpmvState)};
        for (int i = 0; i < 3; i++)
            VQE_HIP(ctx, hipMemcpyAsync(p->ls_mem + offs[i], p->ls_image.data() + offs[i], sizes[i],
                                        hipMemcpyHostToDevice, s));
    }
    return VQE_OK;
}
}  // namespace

extern "C" int vqe_batch_rebind(vqe_batch *p, int32_t slot, const vqe_batch_item *it)
{
    return rebind_impl(p, slot, it, nullptr, "vqe_batch_rebind");
}

extern "C" int vqe_batch_rebind_layout(vqe_batch *p, int32_t slot, const vqe_batch_item *it,
                                       const vqe_layout *layout)
{
    if (p && !layout)
        return vqe_fail(p->ctx, VQE_EINVAL, "vqe_batch_rebind_layout: null layout");
    return rebind_impl(p, slot, it, layout, "vqe_batch_rebind_layout");
}

extern "C" int vqe_layout_create(vqe_ctx *ctx, const vqe_csr *H, int32_t schedule, vqe_layout **out)
{
    if (!ctx)
        return VQE_EINVAL;
    if (!out)
        return vqe_fail(ctx, VQE_EINVAL, "vqe_layout_create: null out");
    *out = nullptr;
    int rc = check_csr(ctx, H, "vqe_layout_create");
    if (rc)
        return rc;
    if (schedule != 0 && !vqe_valid_schedule(schedule))
        return vqe_fail(ctx, VQE_EINVAL, "vqe_layout_create: unknown schedule %d", schedule);
    const int sched = vqe_batch_schedule(H, schedule ? schedule : vqe_default_schedule(H));
    if (!(sched & VQE_SPMV_SLICED))
        return vqe_fail(ctx, VQE_ENOTSUP, "vqe_layout_create: schedule %d has no sliced layout "
                        "for this operator", schedule);
    vqe_layout *L = new (std::nothrow) vqe_layout();
    if (!L)
        return vqe_fail(ctx, VQE_ENOMEM, "vqe_layout_create: allocation failed");
    L->ctx = ctx;
    L->sched = sched;
    L->dtype = H->dtype;
    L->dim = H->dim;
    L->H = H;
    const SellBufs b{&L->meta, &L->code, &L->val, &L->meta_cap, &L->code_cap, &L->val_cap};
    rc = (sched & VQE_SPMV_BLOCKED) ? sliced_tiled_build(ctx, H, sched, b, L->st, &L->entries, -1)
                                    : sliced_build(ctx, H, sched, b, L->st, &L->entries, -1);
    if (rc) {
        vqe_layout_destroy(L);
        return rc;
    }
    *out = L;
    return VQE_OK;
}

extern "C" int vqe_layout_destroy(vqe_layout *L)
{
    if (!L)
        return VQE_EINVAL;
    (void)hipStreamSynchronize(L->ctx->stream);
    for (void *m : {L->meta, L->code, L->val})
        if (m)
            (void)hipFree(m);
    delete L;
    return VQE_OK;
}

extern "C" int64_t vqe_layout_bytes(const vqe_layout *L)
{
    return L ? L->meta_cap + L->code_cap + L->val_cap : 0;
}

extern "C" int vqe_batch_step(vqe_batch *p, uint32_t flags)
{
    if (!p)
        return VQE_EINVAL;
    if (flags & ~(uint32_t)(VQE_STEP_RENORM | VQE_STEP_FORCED | VQE_STEP_NO_UPDATE | VQE_STEP_GRAPH |
                            VQE_STEP_LINESEARCH | VQE_STEP_TILED_SCREEN))
        return vqe_fail(p->ctx, VQE_EINVAL, "vqe_batch_step: unknown flags");
    if ((flags & VQE_STEP_LINESEARCH) && !p->ls_ready)
        return vqe_fail(p->ctx, VQE_EINVAL,
                        "vqe_batch_step: line search not enabled (vqe_batch_set_line_search)");
    if (flags & VQE_STEP_GRAPH)
        return graph_step(p, flags, nullptr);
    return enqueue_step(p, flags);
}

extern "C" int vqe_batch_run(vqe_batch *p, uint32_t flags, const double *theta_rows, int32_t n_steps)
{
    if (!p)
        return VQE_EINVAL;
    vqe_ctx *ctx = p->ctx;
    if (flags & ~(uint32_t)(VQE_STEP_RENORM | VQE_STEP_FORCED | VQE_STEP_GRAPH | VQE_STEP_TILED_SCREEN |
                            VQE_STEP_LINESEARCH))
        return vqe_fail(ctx, VQE_EINVAL, "vqe_batch_run: unknown flags, or a flag a run of updates "
                        "does not take");
    const bool ls = (flags & VQE_STEP_LINESEARCH) != 0;
    if (n_steps < 0 || n_steps > VQE_RUN_MAX_STEPS || (n_steps > 0 && !ls && !theta_rows) ||
        (ls && theta_rows))
        return vqe_fail(ctx, VQE_EINVAL, "vqe_batch_run: bad steps (%d), or angle rows given with "
                        "a line search or missing without one", n_steps);
    if (ls && !p->ls_ready)
        return vqe_fail(ctx, VQE_EINVAL,
                        "vqe_batch_run: line search not enabled (vqe_batch_set_line_search)");
    if (n_steps == 0)
        return VQE_OK;
    const uint32_t sflags = flags & ~(uint32_t)VQE_STEP_GRAPH;
    // each step with its row of angles: the matrix-free update reads the row
    // itself; otherwise the row is first copied into the plan's angle buffer;
    // with a line search each step chooses its own angles
    auto enqueue = [&]() -> int {
        for (int32_t i = 0; i < n_steps; i++) {
            const double *row = ls ? nullptr : theta_rows + (size_t)i * p->B;
            int rc;
            if (ls) {
                rc = enqueue_step(p, sflags);
            } else if (p->mf) {
                rc = enqueue_spmv(p);
                rc = rc ? rc : enqueue_rest(p, sflags, nullptr, row);
            } else {
                launch_theta_row(row, p->theta_io, p->B, ctx->stream);
                rc = enqueue_step(p, sflags);
            }
            if (rc)
                return rc;
        }
        return VQE_OK;
    };
    if (!(flags & VQE_STEP_GRAPH))
        return enqueue();
    vqe_batch::RunGraph *hit = nullptr, *lru = &p->runs[0];
    for (auto &r : p->runs) {
        if (r.x && r.flags == sflags && r.n == n_steps && r.rows == theta_rows)
            hit = &r;
        if (r.used < lru->used)
            lru = &r;
    }
    if (!hit) {
        hipGraph_t g = nullptr;
        hipGraphExec_t x = nullptr;
        const int rc = capture(ctx, enqueue, &g, &x);
        if (rc)
            return rc;
        if (lru->x)
            (void)hipGraphExecDestroy(lru->x);
        if (lru->g)
            (void)hipGraphDestroy(lru->g);
        lru->flags = sflags;
        lru->n = n_steps;
        lru->rows = theta_rows;
        lru->g = g;
        lru->x = x;
        hit = lru;
    }
    hit->used = ++p->run_tick;
    VQE_HIP(ctx, hipGraphLaunch(hit->x, ctx->stream));
    return VQE_OK;
}

extern "C" int vqe_batch_step_timed(vqe_batch *p, uint32_t flags, void **events,
                                    int32_t n_events)
{
    if (!p)
        return VQE_EINVAL;
    if (!events || (n_events != 3 && n_events != 7) ||
        (n_events == 7 && (flags & VQE_STEP_GRAPH)) ||
        (flags & ~(uint32_t)(VQE_STEP_RENORM | VQE_STEP_FORCED | VQE_STEP_NO_UPDATE | VQE_STEP_GRAPH |
                             VQE_STEP_LINESEARCH | VQE_STEP_TILED_SCREEN)) ||
        ((flags & VQE_STEP_LINESEARCH) && !p->ls_ready))
        return vqe_fail(p->ctx, VQE_EINVAL, "vqe_batch_step_timed: bad flags or events");
    for (int i = 0; i < n_events; i++)
        if (!events[i])
            return vqe_fail(p->ctx, VQE_EINVAL, "vqe_batch_step_timed: null event");
    hipEvent_t *ev = reinterpret_cast<hipEvent_t *>(events);
    if (flags & VQE_STEP_GRAPH)
        return graph_step(p, flags, ev);
    if (n_events == 3)
        return enqueue_step3(p, flags, ev);
    return enqueue_step(p, flags, ev);
}

extern "C" int vqe_batch_layout_entries(const vqe_batch *p, int32_t slot, int64_t *entries_out)
{
    if (!p || !entries_out)
        return VQE_EINVAL;
    if (slot < 0 || slot >= p->B)
        return vqe_fail(p->ctx, VQE_EINVAL, "vqe_batch_layout_entries: bad slot %d", slot);
    *entries_out = p->entries[slot];
    return VQE_OK;
}

extern "C" int vqe_batch_time_products(vqe_batch *p, int32_t reps, float *ms_out)
{
    if (!p)
        return VQE_EINVAL;
    vqe_ctx *ctx = p->ctx;
    if (reps < 1 || !ms_out)
        return vqe_fail(ctx, VQE_EINVAL, "vqe_batch_time_products: bad arguments");
    hipEvent_t e0, e1;
    VQE_HIP(ctx, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return vqe_fail(ctx, VQE_EHIP, "vqe_batch_time_products: event creation failed");
    }
    hipError_t e = hipEventRecord(e0, ctx->stream);
    for (int i = 0; i < reps && e == hipSuccess; i++) {
        launch_products(p, p->d_spmv);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipEventRecord(e1, ctx->stream);
    if (e == hipSuccess)
        e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess)
        e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess)
        return vqe_fail(ctx, VQE_EHIP, "vqe_batch_time_products: %s", hipGetErrorString(e));
    *ms_out = ms / (float)reps;
    return VQE_OK;
}

extern "C" int vqe_batch_destroy(vqe_batch *p)
{
    if (!p)
        return VQE_EINVAL;
    (void)hipStreamSynchronize(p->ctx->stream);
    for (int i = 0; i < 32; i++) {
        if (p->exec[i])
            (void)hipGraphExecDestroy(p->exec[i]);
        if (p->graph[i])
            (void)hipGraphDestroy(p->graph[i]);
    }
    for (int i = 0; i < 32; i++) {
        if (p->exec_all[i])
            (void)hipGraphExecDestroy(p->exec_all[i]);
        if (p->graph_all[i])
            (void)hipGraphDestroy(p->graph_all[i]);
    }
    for (auto &r : p->runs) {
        if (r.x)
            (void)hipGraphExecDestroy(r.x);
        if (r.g)
            (void)hipGraphDestroy(r.g);
    }
    if (p->exec_spmv)
        (void)hipGraphExecDestroy(p->exec_spmv);
    if (p->graph_spmv)
        (void)hipGraphDestroy(p->graph_spmv);
    if (p->dmem)
        (void)hipFree(p->dmem);
    if (p->ls_mem)
        (void)hipFree(p->ls_mem);
    if (p->ro_mem)
        (void)hipFree(p->ro_mem);
    for (const auto *v : {&p->col16, &p->vre, &p->prow, &p->blk})
        for (void *m : *v)
            if (m)
                (void)hipFree(m);
    for (void *m : p->table_mem)
        (void)hipFree(m);
    delete p;
    return VQE_OK;
}

extern "C" int64_t vqe_batch_workspace_bytes(const vqe_batch *p)
{
    if (!p)
        return -1;
    int64_t c16 = 0;
    for (const auto *v : {&p->col16_cap, &p->vre_cap, &p->prow_cap, &p->blk_cap})
        for (int64_t c : *v)
            c16 += c;
    return (int64_t)(p->dmem_bytes + p->table_bytes + p->ls_bytes + p->ro_bytes) + c16;
}

namespace {

// Every generator of every pool of the plan satisfies A^2 = -(projector on
// its support), i.e. A[r, c] A[c, r] = -1 on every pair.
int ls_check(vqe_batch *p)
{
    if (p->ls_checked)
        return p->ls_checked > 0 ? VQE_OK : VQE_ENOTSUP;
    bool ok = true;
    if (p->mf) {
        for (const vqe_mf_pool *mp : p->mf_host) {
            for (int j = 0; mp && j < vqe_mf_pool_size(mp) && ok; j++) {
                vqe_mf_desc d;
                (void)vqe_mf_pool_get(mp, j, &d);
                // A[r,c] A[c,r] = v^2 (-1)^{|zsign & x|}
                const double sg = (__builtin_popcountll(d.zsign & d.x) & 1) ? -1.0 : 1.0;
                ok = sg * (d.v_re * d.v_re - d.v_im * d.v_im) == -1.0 && d.v_re * d.v_im == 0.0;
            }
        }
    } else {
        for (const PairTable &tb : p->tables_host) {
            const int64_t n = [&] {
                int32_t last = 0;
                (void)hipMemcpy(&last, tb.pts + (size_t)tb.M * tb.nt, 4, hipMemcpyDeviceToHost);
                return (int64_t)last;
            }();
            const size_t eb = vqe_elem_bytes(p->dtype);
            std::vector<char> a(n * eb), b(n * eb);
            if (n > 0 && (hipMemcpy(a.data(), tb.pa, n * eb, hipMemcpyDeviceToHost) != hipSuccess ||
                          hipMemcpy(b.data(), tb.pb, n * eb, hipMemcpyDeviceToHost) != hipSuccess))
                return vqe_fail(p->ctx, VQE_EHIP, "vqe_batch_set_line_search: reading the pair table");
            for (int64_t i = 0; i < n && ok; i++) {
                double ar, ai, br, bi;
                if (p->dtype == VQE_C128) {
                    ar = ((const double *)a.data())[2 * i];
                    ai = ((const double *)a.data())[2 * i + 1];
                    br = ((const double *)b.data())[2 * i];
                    bi = ((const double *)b.data())[2 * i + 1];
                } else {
                    ar = ((const float *)a.data())[2 * i];
                    ai = ((const float *)a.data())[2 * i + 1];
                    br = ((const float *)b.data())[2 * i];
                    bi = ((const float *)b.data())[2 * i + 1];
                }
                ok = ar * br - ai * bi == -1.0 && ar * bi + ai * br == 0.0;
            }
        }
    }
    p->ls_checked = ok ? 1 : -1;
    return ok ? VQE_OK : VQE_ENOTSUP;
}

// Line-search descriptors of slot s from the plan's descriptors.
void ls_fill_slot(vqe_batch *p, int s, double theta_max, char *D)
{
    const SpmvState &hs = reinterpret_cast<const SpmvState *>(p->image.data() + p->o_spmv)[s];
    const TaylorState &ts = reinterpret_cast<const TaylorState *>(p->image.data() + p->o_tay)[s];
    LsState &ls = reinterpret_cast<LsState *>(p->ls_image.data() + p->o_ls)[s];
    SpmvState &s1 = reinterpret_cast<SpmvState *>(p->ls_image.data() + p->o_ls1)[s];
    SpmvState &s2 = reinterpret_cast<SpmvState *>(p->ls_image.data() + p->o_ls2)[s];
    // vectors and partials keep the addresses assigned at allocation
    void *v1 = ls.v1, *v2 = ls.v2, *w2 = ls.w2;
    void *w1 = s1.sigma;
    double *pv = ls.part_vec, *pd = ls.part_dot;
    double *h1 = const_cast<double *>(ls.part_h1), *h2 = const_cast<double *>(ls.part_h2);
    ls.psi = hs.psi;
    ls.sigma = hs.sigma;
    ls.v1 = v1;
    ls.v2 = v2;
    ls.w2 = w2;
    ls.k = ts.k;
    ls.theta = const_cast<double *>(ts.theta);
    ls.energy = hs.energy_out;
    ls.shift = hs.shift;
    ls.dim = hs.dim;
    ls.ops = ts.ops;
    ls.mf = p->mf ? p->mf_desc_dev[p->table_idx[s]] : nullptr;
    ls.M = ts.M;
    ls.nb_rows = (int32_t)((hs.dim + LS_ROWS_PER_BLOCK - 1) / LS_ROWS_PER_BLOCK);
    ls.part_vec = pv;
    ls.part_dot = pd;
    ls.part_h1 = h1;
    ls.part_h2 = h2;
    ls.nb_spmv = hs.nblocks;
    ls.theta_max = theta_max;
    ls.active = hs.active;
    s1 = hs;
    s1.psi = v1;
    s1.sigma = w1;
    s1.partials = h1;
    s1.energy_out = nullptr;
    s2 = hs;
    s2.psi = v2;
    s2.sigma = w2;
    s2.partials = h2;
    s2.energy_out = nullptr;
    (void)D;
}

}  // namespace

extern "C" int vqe_batch_set_line_search(vqe_batch *p, double theta_max)
{
    if (!p)
        return VQE_EINVAL;
    vqe_ctx *ctx = p->ctx;
    if (!(theta_max >= 0.0) || !std::isfinite(theta_max))
        return vqe_fail(ctx, VQE_EINVAL, "vqe_batch_set_line_search: bad theta_max");
    if (theta_max == 0.0) {
        p->ls_ready = false;
        return VQE_OK;
    }
    int rc = ls_check(p);
    if (rc)
        return rc == VQE_ENOTSUP
                   ? vqe_fail(ctx, VQE_ENOTSUP,
                              "vqe_batch_set_line_search: a generator does not satisfy A^3 = -A")
                   : rc;
    const int B = p->B;
    if (!p->ls_mem) {
        // layout: descriptors, tasks, then per slot v1, v2, w1, w2 and partials
        Arena A;
        p->o_ls = A.take(sizeof(LsState) * B);
        p->o_ls1 = A.take(sizeof(SpmvState) * B);
        p->o_ls2 = A.take(sizeof(SpmvState) * B);
        std::vector<std::vector<int2>> per(kXcd);
        for (int s = 0; s < B; s++) {
            const int nb = (int)((p->dims[s] + LS_ROWS_PER_BLOCK - 1) / LS_ROWS_PER_BLOCK);
            for (int b = 0; b < nb; b++)
                per[p->xcd[s]].push_back(make_int2(s, b));
        }
        auto flat = interleave(per, make_int2(-1, 0));
        const size_t o_tasks = A.take(flat.size() * sizeof(int2));
        const size_t eb = vqe_elem_bytes(p->dtype);
        std::vector<size_t> o_vec(B), o_part(B);
        for (int s = 0; s < B; s++) {
            const SpmvState &hs = reinterpret_cast<const SpmvState *>(p->image.data() + p->o_spmv)[s];
            const int64_t nb = (p->dims[s] + LS_ROWS_PER_BLOCK - 1) / LS_ROWS_PER_BLOCK;
            o_vec[s] = A.take(4 * vqe_align(p->dims[s] * eb));
            o_part[s] = A.take(((size_t)nb * (LS_NVEC + 1) + 2 * (size_t)hs.nblocks * 3) * sizeof(double));
        }
        p->ls_bytes = A.host.size();
        if (hipMalloc((void **)&p->ls_mem, p->ls_bytes) != hipSuccess) {
            (void)hipGetLastError();
            p->ls_mem = nullptr;
            p->ls_bytes = 0;
            return vqe_fail(ctx, VQE_ENOMEM, "vqe_batch_set_line_search: allocation failed");
        }
        char *D = p->ls_mem;
        std::copy(flat.begin(), flat.end(), A.at<int2>(o_tasks));
        for (int s = 0; s < B; s++) {
            const SpmvState &hs = reinterpret_cast<const SpmvState *>(p->image.data() + p->o_spmv)[s];
            const int64_t nb = (p->dims[s] + LS_ROWS_PER_BLOCK - 1) / LS_ROWS_PER_BLOCK;
            const size_t vb = vqe_align(p->dims[s] * eb);
            LsState &ls = A.at<LsState>(p->o_ls)[s];
            SpmvState &s1 = A.at<SpmvState>(p->o_ls1)[s];
            ls.v1 = D + o_vec[s];
            ls.v2 = D + o_vec[s] + vb;
            s1.sigma = D + o_vec[s] + 2 * vb;   // w1
            ls.w2 = D + o_vec[s] + 3 * vb;
            double *pp = (double *)(D + o_part[s]);
            ls.part_vec = pp;
            ls.part_dot = pp + nb * LS_NVEC;
            ls.part_h1 = pp + nb * (LS_NVEC + 1);
            ls.part_h2 = pp + nb * (LS_NVEC + 1) + (size_t)hs.nblocks * 3;
        }
        p->ls_image = std::move(A.host);
        p->d_ls = (LsState *)(D + p->o_ls);
        p->d_ls1 = (SpmvState *)(D + p->o_ls1);
        p->d_ls2 = (SpmvState *)(D + p->o_ls2);
        p->d_ls_tasks = (int2 *)(D + o_tasks);
        p->n_ls_tasks = (unsigned)flat.size();
    }
    for (int s = 0; s < B; s++)
        ls_fill_slot(p, s, theta_max, p->ls_mem);
    VQE_HIP(ctx, hipMemcpyAsync(p->ls_mem, p->ls_image.data(), p->ls_image.size(),
                                hipMemcpyHostToDevice, ctx->stream));
    VQE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    p->ls_ready = true;
    return VQE_OK;
}

extern "C" int vqe_batch_reoptimize(vqe_batch *p, const int32_t *ks, double *thetas, int32_t ld,
                                    int32_t n, const void *const *refs, int32_t sweeps,
                                    double theta_max, double *energies_out)
{
    if (!p)
        return VQE_EINVAL;
    vqe_ctx *ctx = p->ctx;
    if (n < 0 || ld < n || sweeps < 0 || !(theta_max > 0.0) || !std::isfinite(theta_max) ||
        (n > 0 && (!ks || !thetas || !refs)))
        return vqe_fail(ctx, VQE_EINVAL, "vqe_batch_reoptimize: bad arguments");
    const int B = p->B;
    for (int s = 0; s < B && n > 0; s++)
        if (!refs[s])
            return vqe_fail(ctx, VQE_EINVAL, "vqe_batch_reoptimize: null reference for slot %d", s);
    if (n == 0 || sweeps == 0)
        return VQE_OK;
    int rc = ls_check(p);
    if (rc)
        return rc == VQE_ENOTSUP
                   ? vqe_fail(ctx, VQE_ENOTSUP,
                              "vqe_batch_reoptimize: a generator does not satisfy A^3 = -A")
                   : rc;
    const size_t eb = vqe_elem_bytes(p->dtype);
    const SpmvState *hsv = reinterpret_cast<const SpmvState *>(p->image.data() + p->o_spmv);
    const TaylorState *tsv = reinterpret_cast<const TaylorState *>(p->image.data() + p->o_tay);
    std::vector<size_t> o_vec(B), o_part(B), o_hp(B);
    if (!p->ro_mem) {
        Arena A;
        p->o_ro = A.take(sizeof(RoState) * B);
        for (int i = 0; i < 3; i++)
            p->o_roh[i] = A.take(sizeof(SpmvState) * B);
        std::vector<std::vector<int2>> per(kXcd);
        for (int s = 0; s < B; s++) {
            const int nb = (int)((p->dims[s] + LS_ROWS_PER_BLOCK - 1) / LS_ROWS_PER_BLOCK);
            for (int b = 0; b < nb; b++)
                per[p->xcd[s]].push_back(make_int2(s, b));
        }
        auto flat = interleave(per, make_int2(-1, 0));
        const size_t o_tasks = A.take(flat.size() * sizeof(int2));
        for (int s = 0; s < B; s++) {
            const int64_t nb = (p->dims[s] + LS_ROWS_PER_BLOCK - 1) / LS_ROWS_PER_BLOCK;
            o_vec[s] = A.take(9 * vqe_align(p->dims[s] * eb));
            o_part[s] = A.take((size_t)nb * RO_NDOT * sizeof(double));
            o_hp[s] = A.take(3 * (size_t)hsv[s].nblocks * 3 * sizeof(double));
        }
        p->ro_bytes = A.host.size();
        if (hipMalloc((void **)&p->ro_mem, p->ro_bytes) != hipSuccess) {
            (void)hipGetLastError();
            p->ro_mem = nullptr;
            p->ro_bytes = 0;
            return vqe_fail(ctx, VQE_ENOMEM, "vqe_batch_reoptimize: allocation failed");
        }
        char *D = p->ro_mem;
        std::copy(flat.begin(), flat.end(), A.at<int2>(o_tasks));
        // fixed addresses: vectors and partials
        for (int s = 0; s < B; s++) {
            const size_t vb = vqe_align(p->dims[s] * eb);
            RoState &ro = A.at<RoState>(p->o_ro)[s];
            char *v = D + o_vec[s];
            ro.L = v;
            ro.v1 = v + vb;
            ro.v2 = v + 2 * vb;
            for (int i = 0; i < 3; i++) {
                ro.w[i] = v + (3 + i) * vb;
                ro.h[i] = v + (6 + i) * vb;
                SpmvState &hs = A.at<SpmvState>(p->o_roh[i])[s];
                hs.partials = (double *)(D + o_hp[s]) + (size_t)i * hsv[s].nblocks * 3;
            }
            ro.part = (double *)(D + o_part[s]);
        }
        p->ro_image = std::move(A.host);
        p->d_ro = (RoState *)(D + p->o_ro);
        for (int i = 0; i < 3; i++)
            p->d_roh[i] = (SpmvState *)(D + p->o_roh[i]);
        p->d_ro_tasks = (int2 *)(D + o_tasks);
        p->n_ro_tasks = (unsigned)flat.size();
    }
    // this call's descriptors (the plan's current slots, the caller's arrays)
    for (int s = 0; s < B; s++) {
        const SpmvState &hs = hsv[s];
        const TaylorState &ts = tsv[s];
        RoState &ro = reinterpret_cast<RoState *>(p->ro_image.data() + p->o_ro)[s];
        ro.psi = const_cast<void *>(hs.psi);
        ro.ks = ks + (size_t)s * ld;
        ro.thetas = thetas + (size_t)s * ld;
        ro.e_out = energies_out ? energies_out + s : nullptr;
        ro.shift = hs.shift;
        ro.dim = hs.dim;
        ro.ops = ts.ops;
        ro.mf = p->mf ? p->mf_desc_dev[p->table_idx[s]] : nullptr;
        ro.M = ts.M;
        ro.nb_rows = (int32_t)((hs.dim + LS_ROWS_PER_BLOCK - 1) / LS_ROWS_PER_BLOCK);
        ro.theta_max = theta_max;
        ro.active = hs.active;
        for (int i = 0; i < 3; i++) {
            SpmvState &h = reinterpret_cast<SpmvState *>(p->ro_image.data() + p->o_roh[i])[s];
            double *part = h.partials;
            h = hs;
            h.psi = ro.w[i];
            h.sigma = const_cast<void *>(ro.h[i]);
            h.partials = part;
            h.energy_out = nullptr;
        }
    }
    hipStream_t st = ctx->stream;
    VQE_HIP(ctx, hipMemcpyAsync(p->ro_mem, p->ro_image.data(), p->ro_image.size(),
                                hipMemcpyHostToDevice, st));
    VQE_HIP(ctx, hipStreamSynchronize(st));
    const RoState *ro_host = reinterpret_cast<const RoState *>(p->ro_image.data() + p->o_ro);
    for (int sw = 0; sw < sweeps; sw++) {
        // every sweep starts from the reference
        for (int s = 0; s < B; s++)
            VQE_HIP(ctx, hipMemcpyAsync(ro_host[s].L, refs[s], p->dims[s] * eb,
                                        hipMemcpyDeviceToDevice, st));
        for (int m = 0; m < n; m++) {
            launch_ro_vectors(p->dtype, p->d_ro, p->d_ro_tasks, p->n_ro_tasks, m, st);
            for (int q = m + 1; q < n; q++)
                launch_ro_taylor(p->dtype, p->d_ro, p->d_ro_tasks, p->n_ro_tasks, q, false, st);
            for (int i = 0; i < 3; i++)
                launch_products(p, p->d_roh[i]);
            launch_ro_dots(p->dtype, p->d_ro, p->d_ro_tasks, p->n_ro_tasks, st);
            launch_ro_solve(p->d_ro, (unsigned)B, m, st);
            launch_ro_taylor(p->dtype, p->d_ro, p->d_ro_tasks, p->n_ro_tasks, m, true, st);
        }
    }
    launch_ro_finish(p->dtype, p->d_ro, p->d_ro_tasks, p->n_ro_tasks, st);
    launch_norm(p->dtype, p->d_tay, p->d_norm_tasks, p->n_norm_tasks, st);
    VQE_LAUNCH_CHECK(ctx);
    return VQE_OK;
}
