// Descriptors and constants of the H product (the kernels of spmv.hip and
// the batch planner).
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
    // column-tiled schedule (states larger than LDS): per tile t the entries of
    // row r with columns in tile t are [tptr[t*dim + r], tptr[(t+1)*dim + r])
    const int32_t *tptr;       // [(ntiles + 1) * dim]
    double *tile_part;         // [ntiles * dim] FP64 complex partial rows
    int32_t ntiles;            // 0: not tiled
    int32_t tile_cols;
    // 16-bit column form (schedules with VQE_SPMV_X16): col16[k] = col[k] ^ row
    const uint16_t *col16;
    // real parts of val (schedules with VQE_SPMV_REAL): FP32 or FP64.  For
    // the column-tiled form [nnz], with col16 in the CSR's layout; otherwise
    // col16 and vre hold the padded layout (rows rounded up to a multiple of
    // SPMV_PAD entries, zero values in the pads) with row pointers
    // prow[dim + 1] and room for cap entries.  With VQE_SPMV_PAD (complex
    // values) vre holds the complex values in the same padded layout.
    const void *vre;
    const int32_t *prow;
    int64_t cap;
    // blocked layout (column-tiled states of schedules without VQE_SPMV_REAL):
    // per (row block b, column tile t) a slab of the block's entries with
    // columns in the tile, rows in order, starting at entry boff[b * ntiles + t]
    // (a multiple of four; the few entries between slabs are zero); row i of
    // the block is [brp[(b * ntiles + t) * (blk_rows + 1) + i], ... + i + 1)
    // relative to the slab; codes are the tile-local columns col - t * tile_cols
    const uint16_t *bcode;
    const void *bval;
    const int32_t *brp;
    const int64_t *boff;
    int32_t blk_rows;
    // sliced layout (VQE_SPMV_SLICED), for a state that fits LDS: per block
    // of SPMV_LDS_ROWS rows, srow[block start + i] is the block-local row
    // taken by sorted position i (rows by length, longest first), and slice k
    // of block b (sorted positions 64k ... 64k + 63) starts at entry
    // sslice[b * SPMV_SLICES_PER_BLOCK + k].x with .y entries per lane; lane
    // i's j-th entry is at start + ((j / E) * 64 + i) * E + j % E, with the
    // absolute 16-bit column in scode and the value (or its real part with
    // VQE_SPMV_REAL) in sval (pads: column dim, value zero).  For a
    // column-tiled state the same per slab (SPMV_SELLT_ROWS-row block b,
    // tile t; slab = b * ntiles + t): srow[slab * SPMV_SELLT_ROWS + i], the
    // slices' starts relative to the slab's start boff[slab], tile-local
    // columns (pads: the column of the slice's first entry, value zero), and
    // per slab smask[slab] with bit u set when
    // the slab's codes reach part u of the tile (SPMV_SELLT_PART_BYTES each,
    // the parts the product stages)
    const uint16_t *scode;
    const void *sval;
    const uint16_t *srow;
    const int2 *sslice;
    const uint32_t *smask;
    // flip-mask index form (VQE_SPMV_XIDX, E = 3 or 6): the operator's flip
    // masks, ascending, sxtab[0 .. nx); scode then holds 32-bit words of three
    // 10-bit indices, word (start + ((j / E) * 64 + i) * E) / 3 + (j % E) / 3
    // holding entry j of lane i in bits 10 * (j % 3)
    const uint16_t *sxtab;
    int32_t nx;
};

// Column-tiled H product: tile width (state elements staged in LDS per pass)
// and rows per workgroup of the tile-sum kernel.
#define VQE_SPMV_TILED 0x1000
// Blocked layout of a column-tiled state (with VQE_SPMV_TILED): one
// workgroup per block of SPMV_BLK_ROWS rows walks every column tile of
// SPMV_BLK_TILE_BYTES, keeping its rows' FP64 sums in LDS.
#define VQE_SPMV_BLOCKED 0x20000
#define SPMV_BLK_ROWS 2048
#define SPMV_BLK_TILE_BYTES (96 * 1024)
// Sliced column-tiled layout: rows per block (their FP64 sums and one tile
// fill the LDS exactly; a pad's code is a column its slice reaches, so no
// zero element is staged) and tile bytes (a power of two of columns, so that
// a block, whose rows share their high bits, meets only the tiles its rows'
// flip masks reach)
#define SPMV_SELLT_ROWS 2048
#define SPMV_SELLT_TILE_BYTES (128 * 1024)
// a tile is staged in parts of 16 bytes per thread of a 1024-thread workgroup;
// a slab stages only the parts its columns reach
#define SPMV_SELLT_PART_BYTES (16 * 1024)
// Sliced layout: slices of one wave's rows per block of SPMV_LDS_ROWS rows.
#define SPMV_SLICES_PER_BLOCK (SPMV_LDS_ROWS / VQE_WAVE)
// flip-mask index form: table entries (10-bit indices)
#define SPMV_XIDX_MAX 1024
// largest dimension whose column XOR row fits 16 bits
#define SPMV_X16_MAX_DIM 65536
// row length granule of the padded layout (real values, states that fit LDS)
#define SPMV_PAD 8
#define SPMV_TILE_BYTES (128 * 1024)
#define SPMV_SUM_ROWS 1024
