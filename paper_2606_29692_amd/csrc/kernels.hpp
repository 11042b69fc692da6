// Device-side descriptors and launch helpers shared by the kernel sources and
// the batch planner.
#pragma once

#include "common.hpp"

// True when a batch slot is switched off for this step (uniform per workgroup).
#define VQE_SKIP(st) ((st).active && !*gmem((st).active))

// Rows per wave pass handled by one sub-group, and passes per workgroup.
#define SPMV_RPT 2

// A schedule is the lanes per row (8, 16, 32, 64), optionally | VQE_SPMV_VEC4
// or | VQE_SPMV_LDS.  The LDS schedule gives each workgroup SPMV_LDS_ROWS rows.
#ifndef SPMV_LDS_ROWS
#define SPMV_LDS_ROWS 2048
#endif
// state bytes that fit next to the staged row pointers
#define SPMV_LDS_MAX_BYTES (147 * 1024)
__host__ __device__ constexpr int spmv_rows_per_block(int sched)
{
    return 4 * (VQE_WAVE / (sched & 0xff)) * SPMV_RPT;
}

// One state of an H product with the energy reduction.
struct SpmvState {
    const int32_t *rowptr;
    const int32_t *col;
    const void *val;
    const void *psi;
    void *sigma;
    double *partials;     // [nblocks * 3]
    double *energy_out;   // [3]
    int64_t dim;
    int64_t nnz;
    double shift;
    const int32_t *active;     // batch slot flag (nullable): 0 = skip this state
    int32_t nblocks;
    int32_t lanes;
};

// Rows of a pool operator handled by one workgroup of the gradient kernel.
#define GRAD_CHUNK_ROWS 1024
#define GRAD_MAX_GROUP 8

// One group of states that share a pool and a dimension (gradient kernel).
struct GradGroup {
    const vqe_csr *ops;        // device array of the pool's descriptors
    int32_t M;
    int32_t n_states;          // <= GRAD_MAX_GROUP
    int32_t nchunks;
    int32_t chunk_rows;
    int64_t dim;
    const void *psi[GRAD_MAX_GROUP];
    const void *sigma[GRAD_MAX_GROUP];
    double shift[GRAD_MAX_GROUP];
    double *partials[GRAD_MAX_GROUP];   // per state: [M * nchunks]
    double *g_out[GRAD_MAX_GROUP];      // per state: [M]
};

struct PairTable;

// One state of the Taylor update.
struct TaylorState {
    const vqe_csr *ops;        // pool descriptors (device) when the index comes from k
    const int32_t *k;          // device index into ops (nullable: use `op`)
    int32_t M;                 // number of descriptors in ops (k outside [0, M) -> no update)
    int32_t pad0;
    vqe_csr op;                // the operator when k is null
    const double *theta;       // device angle (nullable: use theta_value)
    double theta_value;
    void *psi;
    int64_t dim;
    double *norm_partials;     // [nblocks]
    double *norm2_out;         // nullable
    const PairTable *table;    // device pair table of the pool (compact form), nullable
    const int32_t *active;     // batch slot flag (nullable): 0 = skip this state
    int32_t nblocks;
    int32_t renorm;
};

// Per-state argmax.
struct SelectState {
    const double *g;
    int32_t M;
    int32_t *k_out;
    double *gmax_out;
    const int32_t *active;     // batch slot flag (nullable): 0 = skip this state
};

// Pair table of a pool of pairing generators (built once per batch plan).
#define SCREEN_LDS_BYTES (128 * 1024)
struct PairTable {
    const int32_t *pts;     // [M * nt + 1]: start of (generator j, tile t)
    const int32_t *pr;      // lower row of each pair
    const int32_t *pc;      // partner row
    const void *pa;         // A[r, c]
    const void *pb;         // A[c, r] (0 when c == r)
    const uint32_t *words;  // compact form (nullable): r | sign(A[r,c]) << 30 | sign(A[c,r]) << 31
    const int32_t *xmask;   // compact form: per generator, c = r ^ xmask[j]
    const int32_t *order;   // generators by descending pair count
    int32_t M;
    int32_t nt;             // row tiles
    int32_t tile_rows;
    int32_t pad;
};

struct ScreenState {
    const void *psi;
    const void *sigma;
    double shift;
    double *partials;       // [M * nt]
    double *g_out;          // [M]
    int64_t dim;
    const int32_t *active;  // batch slot flag (nullable): 0 = skip this state
    int32_t table;          // index into the plan's PairTable array
    int32_t pad;
};

int32_t screen_tile_rows(int64_t dim, int dtype);
int pair_table_build(vqe_ctx *ctx, const vqe_pool *pool, int64_t dim, PairTable *tb,
                     void **mem_out, size_t *bytes_out);
void launch_screen(int dtype, const ScreenState *states, const PairTable *tables,
                   const int4 *tasks, unsigned grid, unsigned n_states, size_t lds, hipStream_t s);

#define TAYLOR_ROWS_PER_BLOCK 256
#define NORM_ROWS_PER_BLOCK 2048

int check_csr(vqe_ctx *ctx, const vqe_csr *M, const char *what);
int vqe_spmv_energy_core(vqe_ctx *ctx, const vqe_csr *H, const void *psi, void *sigma,
                         double *out, int lanes, double *partials);
size_t vqe_spmv_partials_bytes(int64_t dim, int lanes);
bool vqe_valid_schedule(int sched);
int vqe_effective_schedule(const vqe_csr *H, int sched);

void launch_spmv(int dtype, int lanes, const SpmvState &single, const SpmvState *states,
                 const int2 *tasks, unsigned grid, hipStream_t s, int64_t max_dim);
int64_t spmv_blocks(int64_t dim, int sched);
__global__ void k_energy_finalize(SpmvState single, const SpmvState *states, int n_states);

void launch_pool_grad(int dtype, const GradGroup *groups, const int4 *tasks, unsigned grid,
                      hipStream_t s);
void launch_grad_finalize(const GradGroup *groups, const int2 *items, unsigned n_items,
                          hipStream_t s);
void launch_select(const SelectState *states, unsigned n, double rel_tie, hipStream_t s);

void launch_taylor_pair(int dtype, const TaylorState *states, const int2 *tasks, unsigned grid,
                        hipStream_t s);
void launch_norm(int dtype, const TaylorState *states, const int2 *tasks, unsigned grid,
                 hipStream_t s);
void launch_taylor_compact(int dtype, const TaylorState *states, const int2 *tasks,
                           unsigned grid, hipStream_t s);
