// C ABI: contexts, workspace, status strings and the batch planner.
//
// The batch planner turns B independent adaptive steps into a fixed list of
// launches over device task tables:
//   H products with the energy reduction (one launch per lanes-per-row value),
//   energy finalisation, pool gradients, gradient finalisation, selection,
//   the fused pairing Taylor update and the renormalisation.
// States are assigned to the 8 XCDs of the device (balanced by H bytes) and
// every task table is interleaved so that workgroup i runs on XCD i % 8 and
// only touches states of that XCD: each state's psi and sigma stay in one L2.
// The launch list can be captured once into a HIP graph and replayed; theta,
// the selected index and every result live in caller-owned device buffers, so
// a replay needs no host round trip.
#include "kernels.hpp"

#include <algorithm>
#include <map>
#include <numeric>
#include <vector>

static const int kXcd = 8;

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
    };
    std::vector<SpmvLaunch> spmv;
    ScreenState *d_screen = nullptr;
    PairTable *d_tables = nullptr;
    int4 *d_screen_tasks = nullptr;
    unsigned n_screen_tasks = 0;
    size_t screen_lds = 0;
    std::vector<void *> table_mem;   // one allocation per distinct pool
    size_t table_bytes = 0;
    SelectState *d_sel = nullptr;
    TaylorState *d_tay = nullptr;
    int2 *d_tay_tasks = nullptr;
    unsigned n_tay_tasks = 0;
    int2 *d_norm_tasks = nullptr;
    unsigned n_norm_tasks = 0;
    hipGraphExec_t exec[16] = {};
    hipGraph_t graph[16] = {};
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

// The step is two launch sequences: the H products (sequence A) and the rest
// (sequence B: energy finalisation, screen, selection, Taylor update,
// renormalisation).  `ev` (nullable) receives the phase events.
int enqueue_spmv(vqe_batch *p)
{
    SpmvState dummy{};
    for (auto &l : p->spmv)
        launch_spmv(p->dtype, l.lanes, dummy, p->d_spmv, l.tasks, l.grid, p->ctx->stream, l.max_dim);
    VQE_LAUNCH_CHECK(p->ctx);
    return VQE_OK;
}

int enqueue_rest(vqe_batch *p, uint32_t flags, hipEvent_t *ev)
{
    vqe_ctx *ctx = p->ctx;
    hipStream_t s = ctx->stream;
    auto mark = [&](int i) -> int {
        if (ev)
            VQE_HIP(ctx, hipEventRecord(ev[i], s));
        return VQE_OK;
    };
    SpmvState dummy{};
    k_energy_finalize<<<(unsigned)p->B, 64, 0, s>>>(dummy, p->d_spmv, p->B);
    int rc = mark(2);
    if (p->mf) {
        launch_screen_mf(p->dtype, p->d_screen, p->d_screen_tasks, p->n_screen_tasks,
                         p->screen_lds, s);
        launch_screen_fin(p->d_screen, p->d_tables, (unsigned)p->B, s);
    } else if (p->n_screen_tasks) {
        launch_screen(p->dtype, p->d_screen, p->d_tables, p->d_screen_tasks, p->n_screen_tasks,
                      (unsigned)p->B, p->screen_lds, s);
    }
    rc = rc ? rc : mark(3);
    if (!(flags & VQE_STEP_FORCED))
        launch_select(p->d_sel, (unsigned)p->B, p->rel_tie, s);
    rc = rc ? rc : mark(4);
    if (!(flags & VQE_STEP_NO_UPDATE)) {
        if (p->mf)
            launch_taylor_mf(p->dtype, p->d_tay, p->d_tay_tasks, p->n_tay_tasks, s);
        else if (p->compact_taylor)
            launch_taylor_compact(p->dtype, p->d_tay, p->d_tay_tasks, p->n_tay_tasks, s);
        else
            launch_taylor_pair(p->dtype, p->d_tay, p->d_tay_tasks, p->n_tay_tasks, s);
    }
    rc = rc ? rc : mark(5);
    if (!(flags & VQE_STEP_NO_UPDATE) && (flags & VQE_STEP_RENORM))
        launch_norm(p->dtype, p->d_tay, p->d_norm_tasks, p->n_norm_tasks, s);
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

// Graph launch of the step: sequence A, then sequence B for this flag set
// (each captured on first use).  Events 0 and 1 bracket sequence A, event 2
// follows sequence B.
int graph_step(vqe_batch *p, uint32_t flags, hipEvent_t *ev)
{
    vqe_ctx *ctx = p->ctx;
    const unsigned key = flags & 7u;
    int rc;
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
    for (int s = 0; s < B; s++) {
        const vqe_csr *H = items[s].H;
        lanes[s] = vqe_effective_schedule(
            H, items[s].spmv_schedule ? items[s].spmv_schedule : vqe_default_schedule(H));
        o_epart[s] = A.take(vqe_spmv_partials_bytes(H->dim, lanes[s]));
        const int64_t nn = (H->dim + NORM_ROWS_PER_BLOCK - 1) / NORM_ROWS_PER_BLOCK;
        o_npart[s] = A.take(nn * sizeof(double));
    }

    // --- H product tasks, one table per lanes value
    std::map<int, std::vector<std::vector<int2>>> per_lanes;
    for (int s = 0; s < B; s++) {
        auto &per = per_lanes[lanes[s]];
        if (per.empty())
            per.resize(kXcd);
        const int nb = (int)spmv_blocks(items[s].H->dim, lanes[s]);
        for (int b = 0; b < nb; b++)
            per[xcd_of[s]].push_back(make_int2(s, b));
    }
    std::vector<std::pair<int, size_t>> spmv_tab;
    std::vector<std::vector<int2>> spmv_lists;
    std::vector<int64_t> spmv_maxdim;
    for (auto &kv : per_lanes) {
        auto flat = interleave(kv.second, make_int2(-1, 0));
        spmv_tab.push_back({kv.first, A.take(flat.size() * sizeof(int2))});
        spmv_lists.push_back(std::move(flat));
        int64_t md = 0;
        for (int s = 0; s < B; s++)
            if (lanes[s] == kv.first)
                md = std::max<int64_t>(md, items[s].H->dim);
        spmv_maxdim.push_back(md);
    }

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
    std::vector<MfHostPlan> mf_plans;
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
            // one allocation: header, tile records, whole-state records, lists
            const size_t o_h = 0, o_t = vqe_align(sizeof(MfTable));
            const size_t o_f = o_t + vqe_align(hp.tile_recs.size() * sizeof(MfRec));
            const size_t o_l = o_f + vqe_align(hp.full_recs.size() * sizeof(MfRec));
            const size_t bytes = o_l + vqe_align(hp.lists.size() * sizeof(int32_t) + 4);
            char *mem = nullptr;
            if (hipMalloc((void **)&mem, bytes) != hipSuccess) {
                (void)hipGetLastError();
                return fail_free(vqe_fail(ctx, VQE_ENOMEM, "vqe_batch_create: record allocation failed"));
            }
            p->table_mem.push_back(mem);
            p->table_bytes += bytes;
            MfTable h{};
            h.tile_recs = (const MfRec *)(mem + o_t);
            h.full_recs = (const MfRec *)(mem + o_f);
            h.lists = (const int32_t *)(mem + o_l);
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
            if (e != hipSuccess)
                return fail_free(vqe_fail(ctx, VQE_EHIP, "vqe_batch_create: record upload: %s",
                                          hipGetErrorString(e)));
            tb.M = hp.M;
            tb.nt = hp.ntile;
            tb.tile_rows = hp.tile_rows;
            mf_dev.push_back((const MfTable *)(mem + o_h));
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
    for (int s = 0; s < B; s++) {
        const int64_t dim = items[s].H->dim;
        const int mp = max_pairs[table_of[pool_key(items[s].pool)]];
        const int nt = (mf_mode || p->compact_taylor)
                           ? std::max(1, (mp + TAYLOR_ROWS_PER_BLOCK - 1) / TAYLOR_ROWS_PER_BLOCK)
                           : (int)((dim + TAYLOR_ROWS_PER_BLOCK - 1) / TAYLOR_ROWS_PER_BLOCK);
        const int nn = (int)((dim + NORM_ROWS_PER_BLOCK - 1) / NORM_ROWS_PER_BLOCK);
        for (int b = 0; b < nt; b++)
            tay_per[xcd_of[s]].push_back(make_int2(s, b));
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
    }
    for (size_t i = 0; i < spmv_tab.size(); i++) {
        std::copy(spmv_lists[i].begin(), spmv_lists[i].end(), A.at<int2>(spmv_tab[i].second));
        p->spmv.push_back({spmv_tab[i].first, (int2 *)(D + spmv_tab[i].second),
                           (unsigned)spmv_lists[i].size(), spmv_maxdim[i]});
    }
    std::copy(screen_flat.begin(), screen_flat.end(), A.at<int4>(o_stasks));
    std::copy(tay_flat.begin(), tay_flat.end(), A.at<int2>(o_ttasks));
    std::copy(norm_flat.begin(), norm_flat.end(), A.at<int2>(o_ntasks));
    p->d_spmv = (SpmvState *)(D + o_spmv);
    p->d_sel = (SelectState *)(D + o_sel);
    p->d_tay = (TaylorState *)(D + o_tay);
    p->d_tables = (PairTable *)(D + o_tables);
    p->d_screen = (ScreenState *)(D + o_screen);
    p->d_screen_tasks = (int4 *)(D + o_stasks);
    p->n_screen_tasks = (unsigned)screen_flat.size();
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
    *out = p;
    return VQE_OK;
}

extern "C" int vqe_batch_rebind(vqe_batch *p, int32_t slot, const vqe_batch_item *it)
{
    if (!p)
        return VQE_EINVAL;
    vqe_ctx *ctx = p->ctx;
    if (slot < 0 || slot >= p->B || !it)
        return vqe_fail(ctx, VQE_EINVAL, "vqe_batch_rebind: bad slot or item");
    int rc = check_csr(ctx, it->H, "vqe_batch_rebind");
    if (rc)
        return rc;
    if (!it->pool || !it->psi || !it->sigma || it->H->dtype != p->dtype ||
        it->H->dim != p->dims[slot] ||
        (p->mf ? (const void *)it->pool->mf : (const void *)it->pool->ops) != p->pool_ops[slot])
        return vqe_fail(ctx, VQE_EINVAL, "vqe_batch_rebind: item does not match slot %d", slot);
    const int sched = vqe_effective_schedule(
        it->H, it->spmv_schedule ? it->spmv_schedule : vqe_default_schedule(it->H));
    if (sched != p->sched[slot])
        return vqe_fail(ctx, VQE_EINVAL, "vqe_batch_rebind: schedule differs from slot %d", slot);
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
    hipStream_t s = ctx->stream;
    VQE_HIP(ctx, hipMemcpyAsync(p->dmem + ((char *)st - p->image.data()), st, sizeof(*st),
                                hipMemcpyHostToDevice, s));
    VQE_HIP(ctx, hipMemcpyAsync(p->dmem + ((char *)ss - p->image.data()), ss, sizeof(*ss),
                                hipMemcpyHostToDevice, s));
    VQE_HIP(ctx, hipMemcpyAsync(p->dmem + ((char *)ts - p->image.data()), ts, sizeof(*ts),
                                hipMemcpyHostToDevice, s));
    return VQE_OK;
}

extern "C" int vqe_batch_step(vqe_batch *p, uint32_t flags)
{
    if (!p)
        return VQE_EINVAL;
    if (flags & ~(uint32_t)(VQE_STEP_RENORM | VQE_STEP_FORCED | VQE_STEP_NO_UPDATE | VQE_STEP_GRAPH))
        return vqe_fail(p->ctx, VQE_EINVAL, "vqe_batch_step: unknown flags");
    if (flags & VQE_STEP_GRAPH)
        return graph_step(p, flags, nullptr);
    return enqueue_step(p, flags);
}

extern "C" int vqe_batch_step_timed(vqe_batch *p, uint32_t flags, void **events,
                                    int32_t n_events)
{
    if (!p)
        return VQE_EINVAL;
    if (!events || (n_events != 3 && n_events != 7) ||
        (n_events == 7 && (flags & VQE_STEP_GRAPH)) ||
        (flags & ~(uint32_t)(VQE_STEP_RENORM | VQE_STEP_FORCED | VQE_STEP_NO_UPDATE | VQE_STEP_GRAPH)))
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

extern "C" int vqe_batch_destroy(vqe_batch *p)
{
    if (!p)
        return VQE_EINVAL;
    (void)hipStreamSynchronize(p->ctx->stream);
    for (int i = 0; i < 16; i++) {
        if (p->exec[i])
            (void)hipGraphExecDestroy(p->exec[i]);
        if (p->graph[i])
            (void)hipGraphDestroy(p->graph[i]);
    }
    if (p->exec_spmv)
        (void)hipGraphExecDestroy(p->exec_spmv);
    if (p->graph_spmv)
        (void)hipGraphDestroy(p->graph_spmv);
    if (p->dmem)
        (void)hipFree(p->dmem);
    for (void *m : p->table_mem)
        (void)hipFree(m);
    delete p;
    return VQE_OK;
}

extern "C" int64_t vqe_batch_workspace_bytes(const vqe_batch *p)
{
    return p ? (int64_t)(p->dmem_bytes + p->table_bytes) : -1;
}
