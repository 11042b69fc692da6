// Device-side descriptors and launch helpers shared by the kernel sources and
// the batch planner.
#pragma once

#include "common.hpp"
#include "spmv.hpp"

#include <vector>

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
struct MfTable;

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
    const MfTable *mf;         // matrix-free records of the pool (nullable)
    // renormalisation after the matrix-free update (nullable): |psi|^2 before
    // the update, and the update blocks' changes of |psi|^2 [ntay]
    const double *n2_prev;
    double *tay_partials;
    int32_t ntay;
    int32_t pad1;
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
    int32_t mf_ntile;       // row tiles of the matrix-free screen (partials per generator)
    const MfTable *mf;      // matrix-free records of the pool (nullable)
    // real-state screen (nullable): the pool's records on one whole-state tile
    const MfTable *mf1;
};

// Matrix-free enumeration of a generator's pairs {r, c = r ^ x} on a row set
// (one row tile of the screen, or the whole state for the update).  The
// owner rows r (bit h = top bit of x clear) of the row set are
//     r = D(e) ^ P(D(e)) ^ base,  e in [0, 2^nfree),
// where D deposits the bits of e into the free bit positions, base holds the
// tile's fixed bits, and P sets every pivot bit piv_i to k_i ^ |beta_i & r|.
#define MF_LANE_BITS 8     // screen: 64 lanes x 4 elements cover the lowest free bits
#define MF_MAX_TB 8         // screen row tiles: at most 2^8 (states of up to 21 qubits in FP32 storage)
struct MfRec {
    uint32_t x, zsign;      // flip mask, sign mask: A[r ^ x, r] = v (-1)^{|zsign & r|}
    uint32_t cx;            // x with the tile bits removed (LDS index offset)
    uint32_t ex;            // |zsign & x| mod 2
    uint32_t base;          // fixed tile bits of this row set
    uint32_t free_mask;     // all free bits
    uint32_t hi_mask;       // free bits above the lowest nlow
    int32_t nfree;          // owner rows on the row set = 2^nfree; -1: none
    int32_t nlow;           // min(nfree, MF_LANE_BITS)
    int32_t ncon;           // pivots
    uint32_t kbits;
    int32_t j;              // generator index
    int32_t ntb;            // tile bits
    int32_t antiherm;       // A[c, r] = -conj(A[r, c]) on every pair
    uint8_t lowpos[MF_LANE_BITS];   // positions of the lowest nlow free bits
    uint8_t piv[VQE_MF_MAX_CON];
    uint8_t tbpos[MF_MAX_TB];   // tile bit positions, descending
    uint32_t tab_off;       // tile records: offset of the screen's index tables
    uint32_t beta[VQE_MF_MAX_CON];
    double v_re, v_im;
};

struct MfTable {
    const MfRec *tile_recs;   // [M * ntile]: generator j on tile v at j * ntile + v
    const MfRec *full_recs;   // [M]: generator j on the whole state
    const int32_t *lists;     // generator indices per (tile-bit group, tile), by descending cost
    const vqe_mf_desc *desc;  // [M]: the descriptors (support tests)
    // screen index tables of the tile records (see MF_TAB_ITER): per record,
    // MF_TAB_ITER entries then one per loop iteration; an entry is a
    // compressed (tile) row index part with its sign parity in bit 31
    const uint32_t *tabs;
    const int4 *linfo;        // per list: offset into lists, length, tile, 0
    int32_t M, ntile, tile_rows, nlists;
};
// table layout of one tile record: 64 lane parts, MF_LANE_UNROLL unroll parts,
// then the iteration parts
#define MF_TAB_ITER (64 + 4)

// One state of the line search over the selected generator's angle.
#define LS_ROWS_PER_BLOCK 2048
#define LS_NVEC 7             // partial sums of the vector kernel
#define LS_GRID 256           // angles of the coarse search
struct LsState {
    const void *psi;
    const void *sigma;        // stored S psi
    void *v1, *v2;            // A psi, A^2 psi
    void *w2;                 // S v2
    const int32_t *k;         // selected generator
    double *theta;            // out: the chosen angle
    const double *energy;     // this step's (E, <psi|psi>, Im)
    double shift;
    int64_t dim;
    const vqe_csr *ops;       // CSR pool (device descriptors), or
    const vqe_mf_desc *mf;    // matrix-free descriptors
    int32_t M;
    int32_t nb_rows;          // blocks of the vector and dot kernels
    double *part_vec;         // [nb_rows * LS_NVEC]
    double *part_dot;         // [nb_rows]
    const double *part_h1;    // partial triples of S v1 [nb_spmv * 3]
    const double *part_h2;    // partial triples of S v2
    int32_t nb_spmv;
    int32_t pad;
    double theta_max;
    const int32_t *active;
};

// Re-optimisation of every angle of one slot's ansatz (cyclic coordinate line
// search over the updates ks[0..n), angles thetas[0..n)).
#define RO_NDOT 12            // partial sums of the inner-product kernel
struct RoState {
    void *psi;                // out: the slot's state at the final angles
    void *L;                  // the state before the visited update
    void *v1, *v2;            // A L, A^2 L
    void *w[3];               // (L, A L, A^2 L) with the later updates applied
    const void *h[3];         // S w_i (written by the H products)
    const int32_t *ks;        // [n] generator of each update
    double *thetas;           // [n] angles (in/out)
    double *e_out;            // energy after the last visit (nullable)
    double shift;
    int64_t dim;
    const vqe_csr *ops;       // CSR pool (device descriptors), or
    const vqe_mf_desc *mf;    // matrix-free descriptors
    int32_t M;
    int32_t nb_rows;          // blocks of the vector, update and dot kernels
    double *part;             // [nb_rows * RO_NDOT]
    double theta_max;
    const int32_t *active;
};
void launch_ls_vectors(int dtype, const LsState *states, const int2 *tasks, unsigned grid,
                       hipStream_t s);
void launch_ls_dot(int dtype, const LsState *states, const int2 *tasks, unsigned grid,
                   hipStream_t s);
void launch_ro_vectors(int dtype, const RoState *states, const int2 *tasks, unsigned grid, int m,
                       hipStream_t s);
void launch_ro_taylor(int dtype, const RoState *states, const int2 *tasks, unsigned grid, int m,
                      bool advance, hipStream_t s);
void launch_ro_dots(int dtype, const RoState *states, const int2 *tasks, unsigned grid,
                    hipStream_t s);
void launch_ro_solve(const RoState *states, unsigned n_states, int m, hipStream_t s);
void launch_ro_finish(int dtype, const RoState *states, const int2 *tasks, unsigned grid,
                      hipStream_t s);
void launch_ls_solve(const LsState *states, unsigned n_states, hipStream_t s);

struct vqe_mf_pool;
// Host: records of every generator of a pool for a state of 2^n rows whose
// screen tiles hold tile_rows rows.  Returns VQE_OK or VQE_ENOTSUP.
struct MfHostPlan {
    std::vector<MfRec> tile_recs, full_recs;
    std::vector<uint32_t> tabs;                    // screen index tables of tile_recs
    std::vector<int32_t> lists;                    // concatenated
    struct List { int32_t off, len, v; double work; };
    std::vector<List> list_info;
    int32_t M = 0, ntile = 1, tile_rows = 0;
};
int mf_host_plan(const vqe_mf_pool *pool, int64_t tile_rows, MfHostPlan *out, char *err, size_t n_err);
bool mf_antihermitian(const vqe_mf_desc &d);
void launch_screen_mf(int dtype, const ScreenState *states, const int4 *tasks, unsigned grid,
                      size_t lds, hipStream_t s);
void launch_screen_mf_real(int dtype, const ScreenState *states, const int4 *tasks, unsigned grid,
                           size_t lds, hipStream_t s);
// LDS bytes of the real-state screen's whole-state tile (psi.re, sigma.re)
inline size_t screen_real_lds(int64_t dim, int dtype)
{
    return (size_t)dim * (dtype == VQE_C64 ? 2 * sizeof(float) : 2 * sizeof(double));
}
// (theta_row, nullable: state s takes the angle theta_row[s] and stores it as
// its angle, instead of reading its angle)
void launch_taylor_mf(int dtype, const TaylorState *states, const int2 *tasks, unsigned grid,
                      const double *theta_row, hipStream_t s);
// the matrix-free update with the step's finalisation (launch_step_fin) done
// by every update workgroup for its state (pools of at most 2048 generators)
void launch_taylor_mf_fin(int dtype, const TaylorState *states, const int2 *tasks, unsigned grid,
                          const SpmvState *spmv, const ScreenState *screen,
                          const PairTable *tables, const SelectState *sel, bool select,
                          double rel_tie, const double *theta_row, hipStream_t s);
// renormalisation after launch_taylor_mf from the pre-update norm and the
// update's changes (states with n2_prev and tay_partials set)
// dst[0..n) = src[0..n): one row of a caller's angle schedule into a plan's
// angle buffer (a kernel, so that it can sit in a captured graph)
void launch_theta_row(const double *src, double *dst, int n, hipStream_t s);
void launch_norm_mf(int dtype, const TaylorState *states, const int2 *tasks, unsigned grid,
                    hipStream_t s);

int32_t screen_tile_rows(int64_t dim, int dtype);
int pair_table_build(vqe_ctx *ctx, const vqe_pool *pool, int64_t dim, PairTable *tb,
                     void **mem_out, size_t *bytes_out);
void launch_screen(int dtype, const ScreenState *states, const PairTable *tables,
                   const int4 *tasks, unsigned grid, unsigned n_states, size_t lds, hipStream_t s);
// Per-state energy finalisation, gradient sums (grad) and selection (select).
void launch_step_fin(const SpmvState *spmv, const ScreenState *screen, const PairTable *tables,
                     const SelectState *sel, unsigned n_states, bool grad, bool select,
                     double rel_tie, hipStream_t s);
int32_t vqe_mf_pool_size(const vqe_mf_pool *pool);
int32_t vqe_mf_pool_qubits(const vqe_mf_pool *pool);

#define TAYLOR_ROWS_PER_BLOCK 256
#define NORM_ROWS_PER_BLOCK 2048

int check_csr(vqe_ctx *ctx, const vqe_csr *M, const char *what);
int vqe_spmv_energy_core(vqe_ctx *ctx, const vqe_csr *H, const void *psi, void *sigma,
                         double *out, int lanes, double *partials);
size_t vqe_spmv_partials_bytes(int64_t dim, int lanes);
bool vqe_valid_schedule(int sched);
int vqe_effective_schedule(const vqe_csr *H, int sched);
int vqe_batch_schedule(const vqe_csr *H, int sched);

void launch_spmv(int dtype, int lanes, const SpmvState &single, const SpmvState *states,
                 const int2 *tasks, unsigned grid, hipStream_t s, int64_t max_dim);
// column-tiled schedule: the tile passes (tasks {state, block << 8 | tile}),
// then the fixed-order tile sum with the energy epilogue (tasks {state, block})
void launch_spmv_tiled(int dtype, int sched, const SpmvState *states, const int2 *tasks,
                       unsigned grid, const int2 *sum_tasks, unsigned sum_grid, hipStream_t s);
void launch_tile_bounds(const SpmvState *states, const int2 *tasks, unsigned grid, hipStream_t s);
// blocked layout of a column-tiled state (VQE_SPMV_BLOCKED): tile width and
// LDS bytes of the product's workgroups; the product itself (tasks {state,
// row block}); and the layout's build from the CSR (slab row pointers brp
// [nb * nt * (R + 1)], scratch blen [nb * nt], slab starts boff [nb * nt + 1],
// codes and values with room for nnz + 4 nb nt + 4 entries)
int32_t spmv_blk_tile_cols(int dtype);
// columns per tile of the sliced column-tiled layout (SPMV_SELLT_TILE_BYTES)
int32_t spmv_sellt_tile_cols(int dtype);
size_t spmv_blk_lds(int dtype);
void launch_spmv_blk(int dtype, int sched, const SpmvState *states, const int2 *tasks,
                     unsigned grid, hipStream_t s);
void launch_blk_layout(const vqe_csr *H, int32_t nt, int32_t tc, int32_t R, int32_t *brp,
                       int64_t *blen, int64_t *boff, uint16_t *bcode, void *bval, hipStream_t s);
int32_t spmv_tile_cols(int dtype);
// tile width of the column-tiled form with real values (VQE_SPMV_REAL): twice
// as many columns, since a real tile holds storage-precision real parts
int32_t spmv_tile_cols_real(int dtype);
int64_t spmv_blocks(int64_t dim, int sched);
// col16[k] = col[k] ^ row(k) for every entry of H (dim <= SPMV_X16_MAX_DIM)
void launch_col_xor16(const vqe_csr *H, uint16_t *col16, hipStream_t s);
// out[k] = Re val[k] (FP32 or FP64 by H's dtype) for every entry of H
void launch_val_real(const vqe_csr *H, void *out, hipStream_t s);
// padded layout of H (dim <= SPMV_X16_MAX_DIM): prow[dim + 1], the 16-bit
// codes and the values -- their real parts (real) or the complex values --
// with every row rounded up to a multiple of SPMV_PAD entries (room for
// nnz + (SPMV_PAD - 1) dim entries)
void launch_pad_layout(const vqe_csr *H, int32_t *prow, uint16_t *code, void *vpad, bool real,
                       hipStream_t s);
// sliced layout of H (a state that fits LDS; VQE_SPMV_SLICED with E entries
// per lane and load group): the per-block row order srow [dim], the slice
// lengths slen [blocks * SPMV_SLICES_PER_BLOCK], the slices (start, length)
// sslice [same] and *total, the entries of all slices (device int64) ...
void launch_sell_layout(const vqe_csr *H, int E, uint16_t *srow, int32_t *slen, int2 *sslice,
                        int64_t *total, hipStream_t s);
// ... then, with room for total entries, the codes and the values (their real
// parts with real)
void launch_sell_fill(const vqe_csr *H, int E, bool real, const uint16_t *srow,
                      const int2 *sslice, uint16_t *code, void *val, hipStream_t s);
// flip-mask index form (VQE_SPMV_XIDX): the masks col ^ row the operator
// uses, numbered ascending (xmap [dim], with mark [dim] as scratch), the
// first SPMV_XIDX_MAX of them in xtab and their count in *nx ...
void launch_sell_xtab(const vqe_csr *H, uint32_t *mark, uint16_t *xmap, uint16_t *xtab, int64_t *nx,
                      hipStream_t s);
// ... then, with room for the slices' entries, the packed indices (one
// 32-bit word per three entries) and the values
void launch_sell_fill_x(const vqe_csr *H, int E, bool real, const uint16_t *srow, const int2 *sslice,
                        const uint16_t *xmap, uint32_t *code, void *val, hipStream_t s);
// sliced layout of a column-tiled state (VQE_SPMV_SLICED on a state larger
// than LDS): per slab of the blocked layout (nt tiles of tc columns) the row
// order srow [slabs * SPMV_SELLT_ROWS] (first the rows' entry counts), the
// slices sslice [slabs * SPMV_SLICES_PER_BLOCK] (start in the slab, length),
// the slab totals stot and starts sbase [slabs], *total, and the part masks
// smask [slabs] cleared ...
void launch_sellt_layout(const vqe_csr *H, int32_t nt, int32_t tc, int E, uint16_t *srow,
                         int2 *sslice, int64_t *stot, int64_t *sbase, int64_t *total, uint32_t *smask,
                         hipStream_t s);
// ... then, with room for total entries, the tile-local codes, the values and
// the tile parts each slab's codes reach (smask)
void launch_sellt_fill(const vqe_csr *H, int32_t nt, int32_t tc, int E, const uint16_t *srow,
                       const int2 *sslice, const int64_t *sbase, uint16_t *code, void *val,
                       uint32_t *smask, hipStream_t s);
__global__ void k_energy_finalize(SpmvState single, const SpmvState *states, int n_states);

void launch_pool_grad(int dtype, const GradGroup *groups, const int4 *tasks, unsigned grid,
                      hipStream_t s);
void launch_grad_finalize(const GradGroup *groups, const int2 *items, unsigned n_items,
                          hipStream_t s);

void launch_taylor_pair(int dtype, const TaylorState *states, const int2 *tasks, unsigned grid,
                        hipStream_t s);
void launch_norm(int dtype, const TaylorState *states, const int2 *tasks, unsigned grid,
                 hipStream_t s);
void launch_taylor_compact(int dtype, const TaylorState *states, const int2 *tasks,
                           unsigned grid, hipStream_t s);
