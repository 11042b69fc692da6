/*
 * adaptvqe.h -- C ABI of the MI355X (gfx950) adaptive-VQE hot path.
 *
 * The library evaluates, on one GPU, the classical core of an adaptive
 * variational eigensolver step:
 *   - compilation of a Pauli-sum operator (Sec. II-A, Eq. 3) into CSR
 *     (the on-the-fly sparse compilation of Sec. III-E);
 *   - the energy, a Rayleigh quotient <psi|H|psi>/<psi|psi> (Eq. 1), whose cost
 *     is one sparse product with H;
 *   - the pool-gradient screen g_j = <psi|[H, A_j]|psi> (Eq. 5), evaluated as
 *     2 Re <H psi | A_j psi> for anti-Hermitian generators A_j;
 *   - the selection of the largest |g_j| (Sec. III-D);
 *   - the fifth-order Taylor state update of Eq. 6, i.e. the five chained
 *     sparse products v_n = A v_{n-1} of Eq. 7 and the accumulation of Eq. 8.
 * Batch plans run that step for many independent states per launch sequence
 * (optionally through captured HIP graphs), with the angle chosen by line
 * search and every angle of the ansatz re-optimised on request (the
 * parameter optimisation of Sec. III-D); pools can be applied matrix-free,
 * straight from their Pauli terms; and a pool can be split into commuting
 * families (Sec. III-F, Alg. 1).
 *
 * Conventions shared by every entry point
 *   - Complex numbers are interleaved (re, im) pairs: VQE_C128 uses two
 *     doubles per element, VQE_C64 two floats.
 *   - A state vector has dim = 2^n_qubits elements; basis index bit q is qubit q.
 *   - All array pointers are DEVICE pointers owned by the caller unless an
 *     argument says "host".  The library never frees caller memory; memory it
 *     allocates for itself (workspace, plans) belongs to the context or plan.
 *   - Work is enqueued on the context's HIP stream and is asynchronous; results
 *     are valid after the stream is synchronised.  The sizing phase of
 *     csr_build_from_pauli is the one exception: it synchronises the stream.
 *   - Every call returns VQE_OK (0) or a negative status.  No C++ exception
 *     crosses the ABI.  vqe_last_error() gives a message for the last failure.
 *   - A context is not thread-safe: use one per host thread (or stream).
 *   - Results do not depend on how many states share a launch: the order of
 *     every floating-point sum is fixed by the operator's size alone.
 */
#ifndef ADAPTVQE_H
#define ADAPTVQE_H

#include <stdint.h>

#if defined(__GNUC__)
#define VQE_API __attribute__((visibility("default")))
#else
#define VQE_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status */
enum {
    VQE_OK = 0,
    VQE_EINVAL = -1,   /* bad argument: null pointer, n_qubits out of range,
                          mask bit >= n_qubits, non-finite theta, dtype mismatch */
    VQE_ESIZE = -2,    /* nnz > INT32_MAX, or a row longer than the builder supports */
    VQE_ENOMEM = -3,   /* device workspace allocation failed */
    VQE_EHIP = -4,     /* HIP runtime error (text in vqe_last_error) */
    VQE_ENOTSUP = -5   /* operation not supported for this operator */
};

typedef enum { VQE_C128 = 0, VQE_C64 = 1 } vqe_dtype;

/* Opaque context: device, HIP stream, workspace (created by vqe_create). */
typedef struct vqe_ctx vqe_ctx;

/* vqe_csr.flags, set by csr_build_from_pauli */
#define VQE_PAIRING 1u   /* every row holds at most one entry and col(col(r)) = r:
                            true of every fermionic single or double excitation
                            generator under JW or BK.  Enables the fused
                            register-resident Taylor kernel. */
#define VQE_REAL 2u      /* every entry is real: each term's c_t i^{|x_t & z_t|}
                            is real (Eq. 3 with the real coefficients of a
                            molecular Hamiltonian: strings with an even number
                            of Y factors).  Set from the terms, exactly; a
                            caller that sets it on a CSR of its own asserts
                            that every imaginary part is zero.  Enables
                            VQE_SPMV_REAL. */

/*
 * A square CSR operator of dimension dim = 2^n_qubits.  Device arrays:
 *   rowptr[dim+1] (int32, rowptr[0] = 0), col[nnz] (int32, strictly ascending
 *   within a row), val[nnz] (complex of the given dtype).
 * The stored matrix is S = M - diag_shift * I, where M is the operator itself.
 * diag_shift is 0 for VQE_C128; for VQE_C64 it is the FP64 reference value
 * subtracted before rounding to FP32 so that large diagonal entries lose no
 * accuracy.  When diag_shift != 0 every row stores its diagonal entry.
 */
typedef struct vqe_csr {
    int32_t n_qubits;
    int32_t dtype;        /* vqe_dtype */
    int64_t dim;
    int64_t nnz;
    int32_t *rowptr;
    int32_t *col;
    void *val;
    double diag_shift;
    uint32_t flags;
    uint32_t reserved;
} vqe_csr;

/* ------------------------------------------------------------------ matrix-free generators */
/*
 * Matrix-free form of a generator given as a Pauli sum A = sum_t c_t P(x_t, z_t)
 * (Eq. 3), for the on-the-fly treatment of Sec. III-E carried one step further:
 * the operator is applied straight from its Pauli terms, with no CSR.
 *
 * It applies when every term flips the same bits x != 0.  Column c then has
 * the single entry A[c ^ x, c] = f(c) = sum_t c_t i^{|x & z_t|} (-1)^{|z_t & c|};
 * f depends on c only through the parities y_i = |beta_i & c| mod 2 for a
 * basis beta_1..beta_d of span{z_t ^ z_0}, times the sign (-1)^{|z_0 & c|}.
 * When f vanishes on every parity pattern but one (k), the operator is
 *     A[c ^ x, c] = v * (-1)^{|zsign & c|}   if |beta_i & c| = k_i mod 2 for all i,
 *                   0                          otherwise,
 * with zsign = z_0 and v the value of the sum on pattern k.  Every fermionic
 * single or double excitation generator under JW or BK has this form (d = 1
 * or 3 under JW).  The value is the same ordered FP64 sum as the CSR builder's
 * (term order, from +0.0, up to a sign flip that is exact) and the same drop
 * rule decides which patterns vanish, so the represented entries equal
 * csr_build_from_pauli's bit for bit.
 */
#define VQE_MF_MAX_CON 8
typedef struct vqe_mf_desc {
    uint64_t x;                      /* common flip mask */
    uint64_t zsign;                  /* sign mask (z of the first term) */
    double v_re, v_im;               /* value on the support */
    int32_t n_qubits;
    int32_t n_con;                   /* d, at most VQE_MF_MAX_CON */
    uint64_t beta[VQE_MF_MAX_CON];   /* support constraints (reduced echelon form) */
    uint32_t kbits;                  /* bit i = required parity k_i */
    uint32_t reserved;
} vqe_mf_desc;
/*
 * Derive the matrix-free form of one generator from its Pauli terms (HOST
 * arrays: xmask, zmask [n_terms], coeff [2*n_terms] interleaved re, im).
 * A pattern's value is dropped when |re| <= drop_tol and |im| <= drop_tol.
 * Host computation only (no device, no context).  Errors: VQE_EINVAL (bad
 * arguments, a mask bit >= n_qubits); VQE_ENOTSUP (terms with different x,
 * x = 0, more than VQE_MF_MAX_CON constraints, zero or several nonvanishing
 * patterns, or a support not closed under c -> c ^ x).
 */
VQE_API int vqe_mf_describe(int32_t n_qubits, int64_t n_terms, const uint64_t *xmask,
                            const uint64_t *zmask, const double *coeff, double drop_tol,
                            vqe_mf_desc *out);
/*
 * A pool in matrix-free form: M generators, generator j made of the terms
 * [term_offset[j], term_offset[j+1]) of the HOST arrays xmask, zmask, coeff.
 * drop_tol: host double[M], or NULL for 1e-12 * max_t |c_t| per generator.
 * The object holds host descriptors only; plans that use it build their
 * device records.  Errors as vqe_mf_describe (the message names the generator).
 */
typedef struct vqe_mf_pool vqe_mf_pool;
VQE_API int vqe_mf_pool_create(int32_t n_qubits, int32_t M, const int64_t *term_offset,
                               const uint64_t *xmask, const uint64_t *zmask, const double *coeff,
                               const double *drop_tol, vqe_mf_pool **out);
VQE_API int vqe_mf_pool_destroy(vqe_mf_pool *pool);
/* Copy generator j's descriptor (host); VQE_EINVAL if j is out of range. */
VQE_API int vqe_mf_pool_get(const vqe_mf_pool *pool, int32_t j, vqe_mf_desc *out);
/*
 * Host mirror of the device enumeration, for checking without a GPU: the
 * owner rows r (the lower row of each pair {r, r ^ x}) of generator j on row
 * tile `tile` of a screen whose tiles hold tile_rows rows (tile = -1: the
 * whole state, as the update enumerates them), in the order the device visits
 * them.  *count receives the number of rows; rows_out (host uint32[*count],
 * nullable) the rows; lds_index_out (nullable) each row's index in the tile.
 */
VQE_API int vqe_mf_owner_rows(const vqe_mf_pool *pool, int32_t j, int64_t tile_rows, int32_t tile,
                              int64_t *count, uint32_t *rows_out, uint32_t *lds_index_out);

/*
 * Commuting-family partition (Sec. III-F, Alg. 1).
 * vqe_mf_noncommutation: the complementary graph of Alg. 1 for a matrix-free
 * pool, adj[i*M + j] = 1 iff [A_i, A_j] != 0 as operators (full commutation),
 * 0 otherwise and on the diagonal.  adj is a DEVICE uint8[M*M]; the call
 * returns after the kernel has finished.  Exact integer work: A_i A_j and
 * A_j A_i map column c to the same basis state, and the generators commute
 * iff for every c both terms are absent or both present with equal sign.
 * vqe_partition_greedy (host only): Alg. 1 on a HOST uint8[M*M] adjacency:
 * vertices by descending degree (ties by index), each to the lowest-indexed
 * family holding none of its neighbours, else a new family; family[v]
 * (host int32[M]) and *n_families receive the result.
 */
VQE_API int vqe_mf_noncommutation(vqe_ctx *ctx, const vqe_mf_pool *pool, uint8_t *adj);
VQE_API int vqe_partition_greedy(int32_t M, const uint8_t *adj, int32_t *family,
                                 int32_t *n_families);

/*
 * An operator pool (Sec. III-A): M generators of one dimension and dtype.
 * ops is a DEVICE array of M descriptors (each pointing to device CSR
 * arrays); ops_host is the same array in host memory (read for sizes and
 * flags, never dereferenced on the device).  Both are owned by the caller.
 * mf (nullable) is the same pool in matrix-free form; a batch plan then
 * screens and updates from it and reads no pool CSR, so ops and ops_host may
 * be NULL when mf is set.
 */
typedef struct vqe_pool {
    int32_t M;
    int32_t n_qubits;
    int32_t dtype;
    int32_t all_pairing;  /* 1 if every generator has VQE_PAIRING */
    const vqe_csr *ops;
    const vqe_csr *ops_host;
    const vqe_mf_pool *mf;
} vqe_pool;

/* ------------------------------------------------------------------ context */
/* Create a context bound to HIP device `device` and stream `hip_stream`
 * (a hipStream_t, or NULL for the null stream).  Returns VQE_EINVAL for a bad
 * device, VQE_EHIP if the device cannot be used. */
VQE_API int vqe_create(int device, void *hip_stream, vqe_ctx **out);
/* Destroy a context.  Every batch plan created on it must be destroyed first
 * (a plan uses its context's stream until vqe_batch_destroy returns). */
VQE_API int vqe_destroy(vqe_ctx *ctx);
/* Re-bind the context to another stream of the same device. */
VQE_API int vqe_set_stream(vqe_ctx *ctx, void *hip_stream);
VQE_API const char *vqe_strerror(int status);
VQE_API const char *vqe_last_error(const vqe_ctx *ctx);
/* Number of compute units and the device name (for reports). */
VQE_API int vqe_device_info(const vqe_ctx *ctx, int32_t *n_cu, char *name, int32_t name_len);

/* ------------------------------------------------------------------ build */
/*
 * Compile sum_t c_t P(x_t, z_t) into CSR (Eq. 3, Sec. III-E).
 * xmask, zmask: HOST uint64[n_terms]; bit q of (x, z) selects the factor on
 * qubit q: (0,0)=I, (1,0)=X, (0,1)=Z, (1,1)=Y.  coeff: HOST double[2*n_terms]
 * (complex c_t, interleaved).  P(x,z)|c> = i^{|x&z|} (-1)^{|z&c|} |c^x>, so
 * term t adds to entry (r, r^x_t) the value c_t i^{|x_t&z_t|} (-1)^{|z_t&(r^x_t)|}.
 * Contributions to one entry are summed in ascending t from +0.0 in FP64
 * with plain additions; an entry is dropped when |re| <= drop_tol and
 * |im| <= drop_tol (it is kept regardless when it is a diagonal entry and
 * diag_shift != 0).  Columns are ascending within each row.
 *
 * Two phases on the same `inout` descriptor:
 *   1. inout->rowptr set (device int32[dim+1]), inout->col == inout->val ==
 *      NULL: fills rowptr, sets nnz, flags, n_qubits, dim, dtype, diag_shift,
 *      writes *nnz_out and synchronises the stream.
 *   2. the caller allocates col[nnz] and val[nnz] (of `dtype`), stores them in
 *      inout, and calls again with the same arguments: fills col and val.
 * VQE_C64 values are fp32(value - diag_shift * [r == c]).
 * Errors: VQE_EINVAL (n_qubits outside [1, 30], mask bit >= n_qubits, null
 * pointers, n_terms < 0); VQE_ESIZE (nnz > INT32_MAX, or a row with more than
 * 2048 entries); VQE_EHIP.
 */
VQE_API int csr_build_from_pauli(vqe_ctx *ctx, int32_t n_qubits, int64_t n_terms,
                         const uint64_t *xmask, const uint64_t *zmask, const double *coeff,
                         double drop_tol, int32_t dtype, double diag_shift,
                         vqe_csr *inout, int64_t *nnz_out);

/* ------------------------------------------------------------------ hot path */
/*
 * Fifth-order Taylor update (Eq. 6): psi <- sum_{n=0..5} (theta A)^n psi / n!,
 * evaluated as v_n = A v_{n-1} (Eq. 7) and psi + sum_n theta^n/n! v_n (Eq. 8),
 * in place on psi (device, dim elements of A->dtype).  Arithmetic is FP64 in
 * registers for both dtypes.  For VQE_PAIRING operators one fused kernel runs
 * all five products; other operators use a fused single-workgroup kernel
 * when small and five chained launches otherwise.
 * renormalize != 0 rescales psi to unit norm afterwards (FP64 norm).
 * norm2_out (device double[1], nullable) receives the squared norm of the raw
 * Eq. 8 result.  A must have diag_shift == 0.
 * Errors: VQE_EINVAL (non-finite theta, null pointers, diag_shift != 0).
 */
VQE_API int taylor5_apply(vqe_ctx *ctx, const vqe_csr *A, double theta, void *psi,
                  int32_t renormalize, double *norm2_out);

/*
 * Energy (Eq. 1).  sigma = S psi is written to sigma_out (device, dim elements
 * of H->dtype; nullable -> workspace), where S = H - diag_shift I is the
 * stored matrix.  out (device double[3]) receives
 *   out[0] = diag_shift + Re<psi|S psi> / <psi|psi>   (the Rayleigh quotient),
 *   out[1] = <psi|psi>,
 *   out[2] = Im<psi|S psi>                             (zero for Hermitian H).
 * Products are accumulated in FP64; the reductions are FP64 in a fixed order.
 */
VQE_API int energy(vqe_ctx *ctx, const vqe_csr *H, const void *psi, void *sigma_out, double *out);

/*
 * Energy without allocation.  For callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  Same computation, kernels and results as energy(), bit for bit;
 * the FP64 block partial sums of the reduction are held in a static device
 * array of the library (VQE_NOALLOC_SCRATCH_BYTES, one copy per GPU, reserved
 * on every GPU the library runs on until the process ends) instead of the
 * context's growable workspace.  sigma_out is required (device, dim elements
 * of H->dtype).  The call makes no device allocation and synchronises
 * nothing.  Every call on one GPU shares that GPU's array, which keeps the
 * last call's partial sums (each call writes every sum it reads, so nothing
 * needs clearing): calls that overlap on one GPU (other streams, other
 * contexts, other host threads) race and must be ordered by the caller.
 * Errors: as energy(); VQE_EINVAL for a null sigma_out; VQE_ESIZE when the
 * reduction needs more than VQE_NOALLOC_SCRATCH_BYTES (three doubles per
 * block of the default schedule: every operator of up to 2^20 rows fits);
 * VQE_EHIP when the array's device address could not be obtained at
 * vqe_create (vqe_last_error gives the reason).
 */
#define VQE_NOALLOC_SCRATCH_BYTES (4u << 20)
VQE_API int energy_noalloc(vqe_ctx *ctx, const vqe_csr *H, const void *psi, void *sigma_out,
                           double *out);

/*
 * Pool-gradient screen (Eq. 5): g_j = 2 Re sum_r conj(sigma_r) (A_j psi)_r for
 * j = 0..M-1, with sigma = H psi.  `sigma` (device, nullable) is the stored
 * product S psi returned by energy(); when NULL it is computed here.  The
 * shift is added back, sigma = S psi + diag_shift psi, so g is exact for any
 * pool.  g_out: device double[M].  FP64 accumulation, fixed order.
 */
VQE_API int pool_gradients(vqe_ctx *ctx, const vqe_csr *H, const vqe_pool *pool, const void *psi,
                   const void *sigma, double *g_out);

/*
 * Selection (Sec. III-D): gmax = max_j |g_j|; the chosen index is the lowest
 * j with |g_j| >= gmax * (1 - rel_tie).  g, k_out (int32[1]) and gmax_out
 * (double[1]) are device pointers.  Convergence (gmax < eps) is the caller's
 * test on gmax_out.
 */
VQE_API int vqe_select(vqe_ctx *ctx, int32_t M, const double *g, double rel_tie,
               int32_t *k_out, double *gmax_out);

/* ------------------------------------------------------------------ batching */
/*
 * A batch plan runs one adaptive step for B independent states in a fixed
 * sequence of launches (replayable as one HIP graph):
 *   sigma_s = S_s psi_s and E_s (Eq. 1); g_s over the state's pool (Eq. 5);
 *   k_s = argmax |g_s| (or a caller-given index); psi_s <- T5(theta_s A_{k_s}) psi_s
 *   (Eq. 6-8); optional renormalisation.
 * States may differ in size and pool.  All buffers are the caller's device
 * memory and must stay valid for the life of the plan:
 *   psi, sigma        per state, dim_s elements of the plan dtype
 *   theta             double[B]
 *   energy_out        double[3*B] (as energy() out, per state)
 *   g_out             double[sum_s M_s], state s at offset g_offset[s]
 *   k_io              int32[B]  (output of the selection, or the input index
 *                     when the step is run with VQE_STEP_FORCED)
 *   gmax_out          double[B]
 * Each state's pool must consist of VQE_PAIRING generators.
 */
typedef struct vqe_batch_item {
    const vqe_csr *H;       /* host pointer to the state's Hamiltonian descriptor */
    const vqe_pool *pool;   /* host pointer to the state's pool */
    void *psi;
    void *sigma;
    int32_t spmv_schedule;  /* H product schedule: 0 = default, else lanes per row
                               (8, 16, 32, 64) with the VQE_SPMV_* options of the
                               tuning section below */
    int32_t reserved;
} vqe_batch_item;

typedef struct vqe_batch_io {
    double *theta;
    double *energy_out;
    double *g_out;
    const int64_t *g_offset_host;   /* host int64[B]: offset of state s in g_out */
    int32_t *k_io;
    double *gmax_out;
    const int32_t *active;          /* device int32[B], nullable: a slot whose flag is 0
                                       is skipped by every kernel of the step (its
                                       outputs keep their previous values) */
} vqe_batch_io;

#define VQE_STEP_RENORM 1u      /* renormalise every state after its update */
#define VQE_STEP_FORCED 2u      /* take k from k_io instead of selecting */
#define VQE_STEP_NO_UPDATE 4u   /* screen only: energy, gradients, selection */
#define VQE_STEP_GRAPH 8u       /* launch through captured HIP graphs, captured on
                                   first use and then replayed: one per flag set
                                   holding the whole step (vqe_batch_step), or one
                                   for the H products and one per flag set for the
                                   rest, with the events between them
                                   (vqe_batch_step_timed) */
#define VQE_STEP_LINESEARCH 16u /* choose each state's angle by line search before
                                   the update (see vqe_batch_set_line_search); the
                                   chosen angle is written to theta */
#define VQE_STEP_TILED_SCREEN 32u /* matrix-free plans: screen every state on row
                                   tiles of its complex psi and sigma (the screen
                                   used for states with imaginary parts), skipping
                                   the plan's screen of real states on one
                                   whole-state tile of real parts, which sends a
                                   state with imaginary parts through the same row
                                   tiles from inside its own launch, with fewer
                                   workgroups.  For callers whose states are
                                   complex.  The same sums for a complex state,
                                   bit for bit; for a real state the same sums
                                   formed in complex arithmetic per row tile,
                                   equal to the rounding of FP64 sums */

typedef struct vqe_batch vqe_batch;

VQE_API int vqe_batch_create(vqe_ctx *ctx, int32_t B, const vqe_batch_item *items,
                     const vqe_batch_io *io, double rel_tie, vqe_batch **out);
VQE_API int vqe_batch_step(vqe_batch *plan, uint32_t flags);
/*
 * n_steps adaptive steps of the plan in one call (Sec. III-D's loop of
 * screen, selection and Eq. 6-8 update, repeated), the angles given: step i
 * runs as vqe_batch_step with its angles from row i of theta_rows (DEVICE
 * float64 [n_steps][B], row-major, read when that step runs); the plan's
 * angle buffer (io->theta) receives each row, so afterwards it holds the
 * last row for every active slot.  With VQE_STEP_LINESEARCH (after
 * vqe_batch_set_line_search) theta_rows must be NULL and every step chooses
 * its angles by line search, as vqe_batch_step does: n_steps whole adaptive
 * iterations with no host work between them.  flags: VQE_STEP_RENORM,
 * VQE_STEP_FORCED, VQE_STEP_TILED_SCREEN, VQE_STEP_LINESEARCH as for
 * vqe_batch_step, and VQE_STEP_GRAPH: the n_steps steps form ONE captured
 * graph, launched once (no host work and no launch gap between the steps);
 * it is captured on first use for its (flags, n_steps, theta_rows) and kept
 * (up to 4 per plan, the least recently used replaced), so a caller that
 * refills the same rows replays it.  The per-step outputs (energies,
 * gradients, selection) are those of the last step.  Errors: VQE_EINVAL for
 * another flag (VQE_STEP_NO_UPDATE), n_steps outside [0, VQE_RUN_MAX_STEPS],
 * theta_rows NULL with n_steps > 0 and no line search, theta_rows given with
 * one, or a line search not enabled; n_steps = 0 does nothing.
 */
#define VQE_RUN_MAX_STEPS 1024
VQE_API int vqe_batch_run(vqe_batch *plan, uint32_t flags, const double *theta_rows, int32_t n_steps);
/*
 * Bind another state to slot `slot` of a plan (continuous batching): the new
 * item must have the same dimension, dtype and H-product schedule as the
 * slot's state at creation and use the same pool (same ops array).  The new
 * descriptors are copied on the context stream, so they apply to every step
 * enqueued afterwards, graph replays included; steps already enqueued keep
 * the old binding.  Errors: VQE_EINVAL (slot out of range, mismatch, psi or
 * sigma not 16-byte aligned).
 */
VQE_API int vqe_batch_rebind(vqe_batch *plan, int32_t slot, const vqe_batch_item *item);
/*
 * A sliced layout (VQE_SPMV_SLICED) of one operator, built once so that batch
 * slots can point to it: a serving loop builds it when it admits a run, and
 * binding the run to a slot later (vqe_batch_rebind_layout) copies no data
 * and waits for nothing.  vqe_layout_create builds the layout of H (the same
 * content as a slot's own: the sort, slices, codes and values of the Eq. 1
 * product) for `schedule` (0: the default) as a batch plan would resolve it
 * for H; it waits for the context stream once, and the contents are
 * written on that stream (ready for work enqueued there afterwards).
 * VQE_ENOTSUP when that schedule has no sliced layout for H, VQE_EINVAL for
 * a bad operator or schedule, VQE_ENOMEM when the device memory runs out.
 * The layout belongs to the caller (vqe_layout_destroy, which waits for the
 * context stream), must outlive every slot bound to it and be destroyed
 * before its context; it reads H only while it is built.
 * vqe_layout_bytes: its device bytes.
 */
typedef struct vqe_layout vqe_layout;
VQE_API int vqe_layout_create(vqe_ctx *ctx, const vqe_csr *H, int32_t schedule, vqe_layout **out);
VQE_API int vqe_layout_destroy(vqe_layout *layout);
VQE_API int64_t vqe_layout_bytes(const vqe_layout *layout);
/*
 * vqe_batch_rebind with a layout built for item->H (the same vqe_csr
 * descriptor) and the slot's schedule: the slot points to the layout instead
 * of rebuilding its own.  VQE_EINVAL if the layout was built for another
 * operator, size, dtype or schedule.  The results equal those of
 * vqe_batch_rebind, bit for bit.
 */
VQE_API int vqe_batch_rebind_layout(vqe_batch *plan, int32_t slot, const vqe_batch_item *item,
                                    const vqe_layout *layout);
/*
 * The same step while recording caller-created HIP events (hipEvent_t) on the
 * context stream.  n_events = 3: [0] before the H products, [1] after them,
 * [2] at the end of the step (eager, or with VQE_STEP_GRAPH the H-product
 * graph and the rest-of-step graph with the events between them).
 * n_events = 7 (eager only): [0] before the H products, [1] after them,
 * [2] after the energy finalisation, [3] after the gradient screen, [4] after
 * the selection, [5] after the Taylor update, [6] after the renormalisation;
 * skipped phases record their events back to back.
 */
VQE_API int vqe_batch_step_timed(vqe_batch *plan, uint32_t flags, void **events, int32_t n_events);
/*
 * Time the plan's H products alone (Eq. 1's sigma = S psi with the energy
 * partials of every active slot, the kernels a step runs first): `reps`
 * back-to-back launches of them bracketed by two HIP events on the context
 * stream, so that the events' and the launches' own cost is spread over the
 * launches; *ms_out = average milliseconds per launch.  psi is read only;
 * sigma and the energy partials are rewritten (the same values each time).
 * Waits for the context stream.  For measurement.
 */
VQE_API int vqe_batch_time_products(vqe_batch *plan, int32_t reps, float *ms_out);
/*
 * Entries (pads included) of slot `slot`'s sliced layout (VQE_SPMV_SLICED),
 * the entries its H product streams per launch; 0 for the other schedules.
 * VQE_EINVAL for a bad slot.
 */
VQE_API int vqe_batch_layout_entries(const vqe_batch *plan, int32_t slot, int64_t *entries_out);
/*
 * Parameter optimisation (the adaptive loop of Sec. III-D leaves the choice of
 * the angle open).  Enables steps with VQE_STEP_LINESEARCH: after the
 * selection, each state's angle is the theta in [-theta_max, theta_max] that
 * minimises the energy (Eq. 1) of the renormalised fifth-order update
 * (Eq. 6-8).  For generators with A^3 = -A (every fermionic single or double
 * excitation) the update is psi + s(theta) A psi + c(theta) A^2 psi with
 * s = theta - theta^3/6 + theta^5/120 and c = theta^2/2 - theta^4/24, so the
 * energy is a ratio of quadratic forms in (1, s, c) built from psi, A psi,
 * A^2 psi and two more H products per state; it is minimised in FP64 over a
 * 256-point grid and refined by golden-section search.  The chosen angle is
 * written to the plan's theta before the update.  Allocates the plan's
 * line-search workspace (4 vectors per state) on first use; theta_max = 0
 * disables.  Errors: VQE_EINVAL (bad theta_max), VQE_ENOTSUP (a generator of
 * a pool does not satisfy A[r,c] A[c,r] = -1 on every pair), VQE_ENOMEM.
 */
VQE_API int vqe_batch_set_line_search(vqe_batch *plan, double theta_max);
/*
 * Re-optimisation of every angle of each slot's adaptive ansatz (the
 * parameter optimisation of the adaptive loop, Sec. III-D, over the updates
 * of Eq. 6-8).  The ansatz state of slot s is
 *     psi = T5(t_{n-1} A_{k_{n-1}}) ... T5(t_0 A_{k_0}) ref_s   (renormalised),
 * and each sweep visits m = 0, 1, ..., n-1 in order, replacing t_m by the
 * angle in [-theta_max, theta_max] that minimises the energy (Eq. 1) with
 * the other angles held (cyclic coordinate descent; the angles before m are
 * already the sweep's new ones).  As in the line search, with L the state
 * before update m and R the later updates, the ansatz is
 * R L + s(t) R A L + c(t) R A^2 L, so each visit costs three H products and
 * the later updates applied to three vectors; the energy ratio is minimised
 * in FP64 (256-point grid, golden-section refinement; the current angle is
 * kept unless something is lower).
 *   ks      DEVICE int32 [B * ld]: row s holds slot s's generator indices
 *           (indices outside [0, M) leave that update out)
 *   thetas  DEVICE FP64 [B * ld]: the angles, updated in place
 *   ld, n   row stride and number of updates per slot, 0 <= n <= ld
 *   refs    HOST array of B DEVICE pointers: each slot's reference state
 *           (dim elements of the plan's dtype; read only)
 *   sweeps  number of sweeps (0: nothing is done)
 *   energies_out  DEVICE FP64 [B] (nullable): the energy after the last visit
 * On completion (stream order) each slot's psi holds the renormalised ansatz
 * state at the new angles; sigma and the plan's energy buffers are left for
 * the next step to recompute.  Slots switched off by the plan's active flags
 * are left unchanged.  Every generator of every pool must satisfy
 * A[r,c] A[c,r] = -1 on its pairs (VQE_ENOTSUP otherwise).  Allocates nine
 * state vectors per slot on the first call (VQE_ENOMEM); synchronises the
 * stream once to upload the call's descriptors, otherwise asynchronous.
 * Errors: VQE_EINVAL (null plan arrays, n > ld, bad theta_max or sweeps).
 */
VQE_API int vqe_batch_reoptimize(vqe_batch *plan, const int32_t *ks, double *thetas, int32_t ld,
                                 int32_t n, const void *const *refs, int32_t sweeps,
                                 double theta_max, double *energies_out);
VQE_API int vqe_batch_destroy(vqe_batch *plan);
/* Bytes of device workspace the plan owns (for footprint accounting). */
VQE_API int64_t vqe_batch_workspace_bytes(const vqe_batch *plan);

/* ------------------------------------------------------------------ tuning */
/*
 * H product schedules.  A schedule is the number of wave lanes that share one
 * CSR row (8, 16, 32 or 64); with VQE_SPMV_VEC4 each lane reads four
 * consecutive entries per pass with 16-byte index loads (16, 32 or 64 lanes;
 * needs 16-byte aligned col and 32-byte aligned val, else the plain schedule
 * with the same lanes is used).  The schedule fixes the summation order.
 */
#define VQE_SPMV_VEC4 0x100
/* VQE_SPMV_LDS: wide loads plus the whole state vector staged in LDS by each
 * workgroup (8, 16, 32 or 64 lanes; VQE_SPMV_DEEP doubles the loads kept in
 * flight per lane); needs dim * element size <= 147 KiB, else the VEC4
 * schedule with the same lanes (16 for 8) is used. */
#define VQE_SPMV_LDS 0x200
#define VQE_SPMV_DEEP 0x400
/* VQE_SPMV_PREFETCH (with VQE_SPMV_LDS): each sub-group keeps the loads of its
 * next rows in flight while it multiplies the current one (two rows, or three
 * with VQE_SPMV_DEEP); needs nnz * element size below 2^31 bytes (raw buffer
 * offsets), else the LDS schedule is used.  32 or 64 lanes when the state fits
 * LDS (8 or 16 lanes then run the plain LDS schedule).
 * In a batch plan, a state larger than the LDS limit runs such a schedule
 * column-tiled: per 128 KiB tile of the state, every row's entries in that
 * tile (a contiguous sub-range of the row) against the tile staged in LDS,
 * with FP64 per-tile row sums added in ascending tile order (8, 16, 32 or 64
 * lanes).  The plan keeps per-tile row bounds ((tiles + 1) * dim int32) and
 * the per-tile sums (tiles * dim complex FP64) for such states.
 * That column-tiled CSR form serves the real-value schedules (VQE_SPMV_REAL)
 * of states of at most 2^16 rows.  Every other pipelined schedule runs a
 * larger-than-LDS state in the blocked layout instead: the plan copies H into
 * slabs of (2048-row block, 96 KiB column tile), each the block's entries in
 * the tile with 16-bit tile-local column codes and the complex values (about
 * nnz * (2 + value bytes) plus 4 bytes per row per tile of slab row
 * pointers, plan-owned, rebuilt by vqe_batch_rebind), and one workgroup per
 * row block walks the tiles with its rows' FP64 sums in LDS; any state size
 * and any nnz below 2^31.  There the lanes (4, 8, 16, 32 or 64; four only
 * there, elsewhere a four-lane schedule runs with eight) set the
 * sub-group width, VQE_SPMV_X16 two groups of four entries per lane and pass
 * instead of one, and VQE_SPMV_DEEP four rows in flight per sub-group instead
 * of two. */
#define VQE_SPMV_PREFETCH 0x800
/* VQE_SPMV_X16 (with VQE_SPMV_LDS | VQE_SPMV_PREFETCH, 32 or 64 lanes; batch
 * plans only): the product reads each column as the 16-bit code
 * col[k] ^ row, which the plan derives from the CSR once (2 bytes per entry,
 * plan-owned, rebuilt by vqe_batch_rebind), instead of the 4-byte index:
 * 10 instead of 12 bytes per entry in FP32 storage; the column-tiled form of
 * larger-than-LDS states reads them too.  States with more than 2^16 rows
 * use the schedule without it; single calls (vqe_time_spmv) ignore it. */
#define VQE_SPMV_X16 0x4000
/* VQE_SPMV_REAL (with VQE_SPMV_X16, and then also with 16 lanes; batch
 * plans only): for an H flagged
 * VQE_REAL the product streams the real parts of its values, which the plan
 * copies from the CSR once (4 bytes per entry in FP32 storage, 8 in FP64;
 * plan-owned, rebuilt by vqe_batch_rebind): 6 instead of 10 bytes per entry
 * in FP32 storage.  For a state that fits LDS the plan lays the codes and
 * values out with every row padded to a multiple of eight entries (zero
 * values; at most 7 pads per row, plus dim + 1 int32 row pointers), so the
 * product needs no row masks and reads each lane's eight codes at once.
 * A column-tiled state keeps the CSR order and the per-tile row bounds, with
 * tiles twice as wide (real parts in storage precision).  Whether the state
 * is real is decided at run time: a state (or, column-tiled, a tile) whose
 * imaginary parts are all zero multiplies in real arithmetic; any other runs
 * the same launch in complex arithmetic (a wide tile as two half-width
 * passes).  Dropped for an H without the flag and
 * wherever the codes are dropped; single calls (vqe_time_spmv) ignore it.
 * The row sums are the same FP64 sums of exact-in-FP64 products as without
 * it, grouped over the lanes differently in the padded layout: results agree
 * to the rounding of FP64 sums (bit for bit in the column-tiled form with
 * FP32 storage). */
#define VQE_SPMV_REAL 0x8000
/* VQE_SPMV_PAD (with VQE_SPMV_X16, 16, 32 or 64 lanes; batch plans only):
 * the padded layout of VQE_SPMV_REAL with the complex values themselves
 * (interleaved, 8 bytes per entry in FP32 storage): every row of the plan's
 * copy of the codes and values starts at a multiple of eight entries and is
 * padded with zero values (at most 7 pads per row, plus dim + 1 int32 row
 * pointers), so a lane reads its eight codes with one 16-byte load and no
 * entry needs a row mask.  Plan-owned, rebuilt by vqe_batch_rebind.  Dropped
 * with the codes, for column-tiled states and where VQE_SPMV_REAL applies.
 * The row sums are the same FP64 sums of exact-in-FP64 products, grouped over
 * the lanes differently: results agree to the rounding of FP64 sums. */
#define VQE_SPMV_PAD 0x10000
/* VQE_SPMV_SLICED (with VQE_SPMV_LDS and E = 2, 4 or 8 in place of the lanes,
 * or E = 3 or 6 with VQE_SPMV_XIDX below;
 * batch plans only): one row per wave lane.  The plan sorts each block of
 * 2048 rows by length (longest first, ties by row) and stores every 64
 * consecutive sorted rows as a slice in which lane i's j-th entry sits at
 * ((j / E) * 64 + i) * E + j mod E, so that each load of E entries is
 * contiguous over the wave; a slice is padded to its longest row, rounded up
 * to E, with zero values (a few percent of the entries for the molecular
 * Hamiltonians at 14 qubits).  Columns are stored as 16-bit indices beside
 * the complex values (about nnz * (2 + value bytes) plus 2 bytes per row and
 * 8 per slice; plan-owned, rebuilt by vqe_batch_rebind, which then waits for
 * the layout's size; vqe_batch_layout_entries reports the entries).  Each
 * lane sums its row in the CSR's column order.  A state larger than LDS is
 * cut into slabs (2048-row block, 128 KiB column tile aligned to a power of
 * two of columns), each slab sorted and sliced by the rows' entries in its tile, with
 * tile-local codes and 2 bytes per row and tile of row order; one workgroup
 * per row block walks the tiles with its rows' FP64 sums in LDS, and a row
 * sums its tiles in ascending order; there VQE_SPMV_DEEP keeps the next
 * tile's loads in flight while a tile is multiplied (ignored for states that
 * fit LDS).  With VQE_SPMV_REAL (an H flagged real; states that fit LDS) the
 * slices hold the values' real parts (6 bytes per entry in FP32 storage) and
 * a state whose imaginary parts are all zero is multiplied in real
 * arithmetic (checked per workgroup at run time); the sums are the complex
 * form's, bit for bit.  Single calls (vqe_time_spmv) run the
 * 32-lane pipelined schedule.  Results agree with the other schedules to the
 * rounding of FP64 sums. */
#define VQE_SPMV_SLICED 0x40000
/*
 * With VQE_SPMV_SLICED and E = 3 or 6, for a state that fits LDS: every entry's
 * column is row ^ x with x one of the operator's flip masks (Eq. 3: a Pauli
 * string maps basis state r to r ^ x), so the slices store the index of x in
 * a per-operator table of at most 1024 masks (ascending; 2 bytes each, staged
 * in LDS beside the state) instead of the 16-bit column: three 10-bit indices
 * to a 32-bit word (E / 3 words per group), 1.33 bytes per entry instead of 2.  Pads take index 0
 * and the value zero.  The plan (or vqe_layout_create) reports VQE_ENOTSUP
 * for an operator with more than 1024 distinct flip masks; a state larger
 * than LDS runs the column-tiled sliced product with E = 2.  Each lane adds
 * its row's entries in the order of the 16-bit column form, so the results
 * equal that form's bit for bit (the pads add zeros).
 */
#define VQE_SPMV_XIDX 0x80000
/*
 * Time the H product (sigma = S psi with the energy reduction) with the given
 * schedule: `reps` back-to-back launches bracketed by HIP events on the
 * context stream; *ms_out = average milliseconds per launch.
 */
VQE_API int vqe_time_spmv(vqe_ctx *ctx, const vqe_csr *H, const void *psi, void *sigma,
                  int32_t schedule, int32_t reps, float *ms_out);
/* Schedule used for an operator when none is given (energy(), pool_gradients()). */
VQE_API int32_t vqe_default_schedule(const vqe_csr *H);

#ifdef __cplusplus
}
#endif

#endif /* ADAPTVQE_H */
