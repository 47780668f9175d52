/*
 * spleaf: leaf kernels of distributed sparse tensor algebra on one AMD
 * Instinct MI355X (gfx950).
 *
 * The library evaluates the tensor-index-notation statements of the SpDISTAL
 * paper's evaluation (Sec. VI-A) on one GPU's share of the data: sparse
 * operands stored with Dense and Compressed levels (Sec. II-B, III-B), split
 * into tiles by the paper's two partition kinds (Sec. II-B): a universe
 * partition of the row coordinates ("row split") or a non-zero partition of
 * the fused coordinates ("non-zero split"), plus an equal split of the merged
 * row-end/position sequence ("merge split").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every pointer inside spl_sparse and spl_dense, every output array, every
 *   workspace and every tile-bound array is a DEVICE pointer on the context's
 *   GPU, owned by the caller.  The library never frees or keeps them.
 *   Pointers documented as "host" are host memory.
 * - A Compressed level l stores pos[l] (parent count + 1 entries, int32,
 *   pos[l][0] = 0, non-decreasing) and crd[l] (int32, one per stored
 *   coordinate).  The coordinates of parent entry e are crd[l][pos[l][e]] ..
 *   crd[l][pos[l][e+1]-1] (Sec. III-B; the paper's inclusive (lo, hi) pairs are
 *   lo = pos[e], hi = pos[e+1]-1).  Coordinates must be strictly increasing
 *   within each segment.  Only CSR = (Dense, Compressed) and
 *   CSF = (Dense, Compressed, Compressed) are accepted.
 * - Dense operands are row-major with leading dimension ld (in elements).
 * - Outputs are overwritten (assignment semantics of Sec. II-A): every output
 *   entry is written, an empty row gives +0.0.
 * - Calls are asynchronous on `stream` (a hipStream_t) unless documented
 *   otherwise.  Metadata (shapes, dtypes, formats, null pointers) is checked
 *   on the host before anything is launched; the CONTENTS of pos/crd are
 *   checked only by spl_validate, and a kernel call on invalid contents is
 *   undefined.  HIP launch errors are reported as SPL_ERR_HIP; errors of
 *   earlier asynchronous work surface at the next call or at spl_sync.
 * - `workspace` may be NULL: the context then uses a device buffer of its own,
 *   grown on demand (the grow synchronizes the device).  A caller-supplied
 *   workspace of fewer bytes than spl_workspace_query reports is rejected
 *   with SPL_ERR_WORKSPACE.
 * - No C++ exception crosses this interface.  A context is not thread-safe;
 *   use one per host thread.  Results are deterministic: no floating-point
 *   atomics are used, so repeated calls give identical bits.
 */
#ifndef SPLEAF_H
#define SPLEAF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum spl_status {
    SPL_OK = 0,
    SPL_ERR_ARG = 1,         /* null pointer, negative size, bad enum value   */
    SPL_ERR_FORMAT = 2,      /* level formats other than (D,C) / (D,C,C)      */
    SPL_ERR_SHAPE = 3,       /* operand dimensions do not match               */
    SPL_ERR_DTYPE = 4,       /* dtype combination not provided                */
    SPL_ERR_UNSUPPORTED = 5, /* valid request this library does not implement */
    SPL_ERR_WORKSPACE = 6,   /* caller workspace smaller than required        */
    SPL_ERR_NOMEM = 7,       /* device allocation failed                      */
    SPL_ERR_HIP = 8,         /* HIP runtime error                             */
    SPL_ERR_INVALID = 9      /* spl_validate found malformed pos/crd          */
} spl_status;

typedef enum spl_dtype { SPL_F64 = 0, SPL_F32 = 1, SPL_BF16 = 2 } spl_dtype;

typedef enum spl_level_format { SPL_DENSE = 0, SPL_COMPRESSED = 1 } spl_level_format;

/* Element type of the pos arrays of a sparse operand. */
typedef enum spl_index_type { SPL_I32 = 0, SPL_I64 = 1 } spl_index_type;

/* How the leaf iteration space is cut into tiles (Sec. II-B, II-D, IV-C). */
typedef enum spl_sched_kind {
    SPL_SCHED_DEFAULT = 0, /* library choice (merge split)                    */
    SPL_ROW = 1,   /* universe partition of rows, image to positions          */
    SPL_NNZ = 2,   /* non-zero partition of fused positions, rows by preimage */
    SPL_MERGE = 3, /* equal split of the merged (row ends + positions) list   */
    /* SpMV and SpMM only (see spl_mlp_predict and spl_autotune): */
    SPL_SCHED_LEARNED = 4,  /* the context's selector picks one of its
                               candidates from the matrix's features          */
    SPL_SCHED_AUTOTUNE = 5  /* every candidate is timed on this call's
                               operands and the fastest one runs              */
} spl_sched_kind;

typedef enum spl_op {
    SPL_OP_SPMV = 0,   /* a(i) = B(i,j) * c(j)                                */
    SPL_OP_SPMM = 1,   /* A(i,j) = B(i,k) * C(k,j)                            */
    SPL_OP_SPADD3 = 2, /* A(i,j) = B(i,j) + C(i,j) + D(i,j)                   */
    SPL_OP_SDDMM = 3,  /* A(i,j) = B(i,j) * C(i,k) * D(j,k)                   */
    SPL_OP_SPTTV = 4,  /* A(i,j) = B(i,j,k) * c(k)                            */
    SPL_OP_MTTKRP = 5, /* A(i,l) = B(i,j,k) * C(j,l) * D(k,l)                 */
    SPL_OP_INNER = 6   /* a = B(i,j,k) * C(i,j,k)                             */
} spl_op;

typedef struct spl_context spl_context;
typedef void *spl_stream; /* a hipStream_t; NULL is the null stream */

/* A sparse operand (Sec. III-B).  level[0] must be SPL_DENSE and the others
 * SPL_COMPRESSED, except that a 3-tensor's middle level may be SPL_DENSE
 * too: (Dense, Dense, Compressed), the format of the paper's "patents"
 * tensor (Sec. VI).  pos[l]/crd[l] are used for Compressed levels l >= 1 and
 * ignored for Dense ones.  nnz must equal pos[order-1][last] (the caller
 * knows it; the library does not read it back).  For CSF, F = pos[1][dims[0]]
 * fibers is passed in nfibers; for (Dense, Dense, Compressed), nfibers must
 * be dims[0] * dims[1] and fiber f = i * dims[1] + j owns positions
 * [pos[2][f], pos[2][f+1]).  pos_type SPL_I64: pos[l] holds the address of
 * an int64 array (cast to the declared pointer type), so nnz may exceed
 * 2^31 - 1 (a matrix that fills a large part of one GPU's memory); crd
 * stays int32 (every dimension is below 2^31).  SPL_I64 is accepted by
 * spl_spmv (CSR, MERGE schedule, variant 0), spl_spmm (CSR, MERGE schedule,
 * 16-byte vector lanes), spl_spttv (MERGE schedule, variant 0; only the last
 * level's pos is read, as int64), spl_mttkrp (CSF with a Compressed middle
 * level, MERGE schedule, vector lanes; pos[1] and pos[2] int64, fewer than
 * 2^31 fibers) and their workspace queries; every other call returns
 * SPL_ERR_UNSUPPORTED for it. */
typedef struct spl_sparse {
    int32_t order;          /* 2 (CSR) or 3 (CSF)                              */
    int32_t vtype;          /* spl_dtype of vals                               */
    int64_t dims[3];        /* coordinate extents (rows, cols[, depth])        */
    int32_t level[3];       /* spl_level_format per stored dimension           */
    const int32_t *pos[3];  /* device, per Compressed level                    */
    const int32_t *crd[3];  /* device, per Compressed level                    */
    const void *vals;       /* device, nnz values of type vtype                */
    int64_t nnz;            /* stored values                                   */
    int64_t nfibers;        /* CSF only: entries of the middle level           */
    int32_t pos_type;       /* spl_index_type of pos[] (0 = SPL_I32)           */
} spl_sparse;

/* A dense operand: vector (ndim 1) or row-major matrix (ndim 2). */
typedef struct spl_dense {
    void *data;       /* device                                               */
    int32_t dtype;    /* spl_dtype                                            */
    int32_t ndim;     /* 1 or 2                                               */
    int64_t dims[2];  /* extents; dims[1] ignored for ndim 1                  */
    int64_t ld;       /* leading dimension in elements (>= dims[1]); 1 for vectors */
} spl_dense;

/* Tiling of one call.  Zero fields mean "library default". */
typedef struct spl_schedule {
    int32_t kind;           /* spl_sched_kind                                 */
    int32_t lanes_per_row;  /* SPL_ROW: lanes sharing one row: 1,2,..,64      */
    int32_t tile;           /* SPL_NNZ: positions per tile; SPL_MERGE: merged
                               items per tile                                 */
    int32_t items_per_lane; /* merged items one lane (SpMV) or lane group
                               (SpMM, MTTKRP) walks per chunk: 4, 8 or 16
                               (MTTKRP also 3 and 5); 0 = the op's default  */
    int32_t col_tile;       /* SpMM: dense columns per lane group: 8,16,32,64 */
    int32_t variant;        /* op-specific kernel variant, 0 = default        */
} spl_schedule;

/* ---------------------------------------------------------------- context */

/* Create a context bound to HIP device `device`.  *out receives the handle. */
spl_status spl_context_create(int device, spl_context **out);
/* Destroy a context and free its own workspace.  NULL is accepted. */
spl_status spl_context_destroy(spl_context *ctx);
/* Detail of the last error on this context (static storage inside ctx). */
const char *spl_last_error(const spl_context *ctx);
/* Name of a status code. */
const char *spl_status_string(spl_status s);
/* Wait for all work on `stream`; reports asynchronous HIP errors. */
spl_status spl_sync(spl_context *ctx, spl_stream stream);

/* ------------------------------------------------------ index notation */

/* The index-notation statement an op evaluates (Sec. II-A, VI-A). */
const char *spl_op_tin(spl_op op);
/* Parse one of the seven statements (up to renaming of index variables and
 * tensors' case-preserving names B, C, D, and white space); any other
 * statement gives SPL_ERR_UNSUPPORTED.  `tin` is a host string. */
spl_status spl_op_parse(const char *tin, spl_op *out);

/* ------------------------------------------------------------ helpers */

/* Device bytes of workspace that `op` needs for operand B, `ncols` dense
 * columns (SpMM N, MTTKRP R; 1 otherwise) and schedule `sched`.  *bytes is
 * host memory. */
spl_status spl_workspace_query(spl_context *ctx, spl_op op, const spl_sparse *B,
                               int64_t ncols, const spl_schedule *sched,
                               size_t *bytes);

/* The level partition of the leaf iteration space (Sec. IV-B, Table I;
 * Sec. III-A image and preimage), as used by the kernels: for tile t,
 * tile_row[t] is the first row the tile finishes and tile_pos[t] its first
 * position; tile t covers positions [tile_pos[t], tile_pos[t+1]) and
 * finishes rows [tile_row[t], tile_row[t+1]); the last entry is (n, nnz).
 * Row r counts as finished at position p when pos[r+1] <= p, so a tile that
 * begins at position p > 0 begins after every row ending at or before p.
 *   SPL_ROW   : tile t = rows [t*R, (t+1)*R), R = sched->tile (image).
 *   SPL_NNZ   : tile t = positions [t*T, (t+1)*T), T = sched->tile (preimage).
 *   SPL_MERGE : tile t = merged items [t*M, (t+1)*M), M = sched->tile.
 * For CSF operands the split applies to the last level (fibers as rows).
 * `capacity` is the length of both device arrays; *ntiles (host) receives
 * the tile count (capacity must be >= ntiles+1, else SPL_ERR_ARG). */
spl_status spl_tile_bounds(spl_context *ctx, const spl_sparse *B,
                           const spl_schedule *sched, int32_t *tile_row,
                           int32_t *tile_pos, int64_t capacity,
                           int64_t *ntiles, spl_stream stream);

/* The fused non-zero partition of a CSF tensor (Dense, Compressed,
 * Compressed) that SpMTTKRP's SPL_NNZ schedule runs on: the (i,j,k)
 * positions are fused and cut into blocks of T positions (Sec. II-B,
 * coordinate fusion and the non-zero partition), each block boundary is
 * moved back to the start of the fiber that holds it so that every fiber
 * lies in one tile, and slices follow by preimage through pos[1]
 * (Sec. III-A; Table I).  For tile t (0 < t < ntiles), tile_fiber[t] is the
 * fiber holding position t*T and tile_slice[t] the slice holding that
 * fiber; tile t covers the fibers [tile_fiber[t], tile_fiber[t+1]), that
 * is the positions [pos[2][tile_fiber[t]], pos[2][tile_fiber[t+1]]), and
 * finishes the slices [tile_slice[t], tile_slice[t+1]).  Entry 0 is
 * (0, 0) and entry ntiles is (dims[0], nfibers).  ntiles = ceil(nnz / T),
 * at least 1.  tile_slice and tile_fiber: device int32 arrays of `capacity`
 * entries (capacity >= ntiles + 1, else SPL_ERR_ARG; *ntiles, host, is
 * written first either way).  A Dense middle level gives SPL_ERR_FORMAT. */
spl_status spl_csf_tile_bounds(spl_context *ctx, const spl_sparse *B, int64_t T,
                               int32_t *tile_slice, int32_t *tile_fiber, int64_t capacity,
                               int64_t *ntiles, spl_stream stream);

/* Check pos/crd contents on the device: pos[0] = 0, non-decreasing pos,
 * last pos = child count (nnz or nfibers), every crd in [0, extent),
 * strictly increasing within each segment.  Returns SPL_OK or
 * SPL_ERR_INVALID with the first failing condition in spl_last_error.
 * Synchronizes on `stream`. */
spl_status spl_validate(spl_context *ctx, const spl_sparse *B, spl_stream stream);

/* ---------------------------------------------------------- measurement */

/* Kernel timing for roofline reports.  While enabled (enable != 0), every
 * subsequent call brackets its leaf kernel -- the one that streams the
 * sparse operand, not the tile-bound or carry fix-up kernels -- with a pair
 * of hipEvents recorded on the call's own stream.  Disabling keeps the
 * recorded pairs for spl_timing_read. */
spl_status spl_timing_enable(spl_context *ctx, int enable);
/* Wait for the recorded events of `op`, return how many leaf launches were
 * recorded (*launches, host) and their summed duration in milliseconds
 * (*total_ms, host), and forget them. */
spl_status spl_timing_read(spl_context *ctx, spl_op op, int64_t *launches, double *total_ms);

/* Memory-system probes that bound the leaf kernels from above.
 *   kind 0: stream-read `bytes` of `buf` once (16-byte loads; `bytes` a
 *           multiple of 16): the HBM read ceiling for streamed arrays.
 *   kind 1: read `count` rows of `row_bytes` (4, 8, 32, 64, 128 or 256) at
 *           pseudo-random row indices of the table `buf` of `bytes` bytes:
 *           the ceiling for random dense-operand gathers.
 *   kind 2: as kind 1 with 16-byte loads per lane (row_bytes 16, 64, 128
 *           or 256).
 * `out` (device) receives one double per workgroup (`blocks` of them, at
 * least 1); `buf` must be 16-byte aligned. */
spl_status spl_probe(spl_context *ctx, int kind, const void *buf, int64_t bytes,
                     int64_t row_bytes, int64_t count, double *out, int64_t blocks,
                     spl_stream stream);

/* ------------------------------------------------------------ kernels */

/* SpMV  a(i) = B(i,j) * c(j)   (Sec. VI-A; the leaf of Fig. 8b).
 * B CSR n x m; c vector m; a vector n.  dtypes: vals, c, a all F64, or all
 * F32 (products and sums in F64; an F32 output is rounded from the F64
 * sum once, except a row that spans tiles of the NNZ or MERGE split: the
 * tile that finishes it stores its rounded partial, and the carry fix-up
 * adds the other tiles' F64 carries to that value and rounds a second
 * time).  Schedules: ROW,
 * NNZ, MERGE (default MERGE), and SPL_SCHED_LEARNED / SPL_SCHED_AUTOTUNE
 * (below).  sched->variant (MERGE only; all walk chunks of
 * 256 * items_per_lane merged items): 0 = the row ends are staged as flags
 * in the merged sequence and each lane's start comes from a count (default);
 * 1 = each lane finds its start by a merge-path search over the row ends;
 * 2 = each lane sums whole rows of the chunk from its staged products (rows
 * of more than 32 positions in the chunk by a wave each), the open row by
 * the workgroup -- for short rows such as CSF fibers (int32 positions only).
 * Kinds
 * SPL_SCHED_LEARNED / SPL_SCHED_AUTOTUNE are resolved first to one of the
 * candidates (which synchronizes on
 * `stream`; a caller workspace must then fit every candidate, as
 * spl_workspace_query returns for those kinds). */
spl_status spl_spmv(spl_context *ctx, const spl_sparse *B, const spl_dense *c,
                    spl_dense *a, const spl_schedule *sched, void *workspace,
                    size_t workspace_bytes, spl_stream stream);

/* SpMV that allocates nothing, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same operation, dtypes, schedules (ROW, NNZ, MERGE and
 * their fields) and kernels as spl_spmv, with the same results bit for bit;
 * the tile bounds and carries live in a static device array of 16 MiB
 * (each GPU the library runs on holds one until the process ends; its
 * address is looked up once per device by spl_context_create), so the call
 * calls no hipMalloc/hipFree and takes no workspace.  Limits and errors:
 * SPL_ERR_WORKSPACE when spl_workspace_query reports more than 16 MiB for
 * this matrix and schedule (with the default MERGE schedule that is
 * n + nnz beyond about 2e9 merged items; a longer tile needs less);
 * SPL_ERR_UNSUPPORTED for SPL_SCHED_LEARNED / SPL_SCHED_AUTOTUNE (they use
 * the context's workspace); SPL_ERR_HIP when the scratch lookup failed on
 * this device.  Leaf timing (spl_timing_enable) does not record this call.
 * Every call on one GPU shares that GPU's scratch and leaves its contents
 * behind (every entry the kernels read is written first in the same call,
 * so nothing needs clearing): calls that overlap on one GPU -- on two
 * streams, or from two host threads -- race and give undefined results. */
spl_status spl_spmv_noalloc(spl_context *ctx, const spl_sparse *B, const spl_dense *c,
                            spl_dense *a, const spl_schedule *sched, spl_stream stream);

/* Universe partition of B's Compressed level by coordinate value ranges,
 * carried to the rows by a preimage (Sec. III-A; Table I: a Compressed
 * level's universe partition colors each stored coordinate by the value
 * range that holds it, and the preimage through pos gives each row the
 * positions of each color).  B CSR n x m.  bounds: device int32[ncolors+1],
 * non-decreasing (color c holds coordinates in [bounds[c], bounds[c+1]);
 * bounds[0] <= 0 and bounds[ncolors] >= m make the colors cover every
 * column).  out: device int32[(ncolors+1) * n], written: out[c*n + i] is
 * the first position of row i whose coordinate is >= bounds[c]
 * (pos[i+1] if none), so color c of row i is the positions
 * [out[c*n+i], out[(c+1)*n+i]).  Coordinates must be sorted within rows
 * (spl_validate).  The rows of a color are the windows spl_spmv_window
 * takes. */
spl_status spl_coord_partition(spl_context *ctx, const spl_sparse *B, int32_t ncolors,
                               const int32_t *bounds, int32_t *out, spl_stream stream);

/* SpMV over position windows: a(i) = sum over p in [begin[i], end[i]) of
 * B.vals[p] * c(B.crd[p]) — for one color of spl_coord_partition, the
 * product of B's column block with c.  B CSR n x m; begin, end: device
 * int32[n] with pos[i] <= begin[i] <= end[i] <= pos[i+1] (not checked: they
 * are read as row bounds; a window with end < begin counts as empty); c
 * vector m; a vector n, every entry written.  dtypes as spl_spmv.
 * Schedules: MERGE (default; tile, items_per_lane 4 or 8, variant 0): the
 * window lengths are scanned into the positions of a virtual CSR on the
 * device, split by the merge path and summed with the flag leaf's walk and
 * carries, so long windows cost no more than short ones; its workspace
 * (n + 1 int32, scan and tile bounds, sized for B->nnz positions) comes from
 * the context's pool.  ROW (lanes_per_row; default by the mean row length of
 * B): no workspace.  NNZ gives SPL_ERR_ARG. */
spl_status spl_spmv_window(spl_context *ctx, const spl_sparse *B, const int32_t *begin,
                           const int32_t *end, const spl_dense *c, spl_dense *a,
                           const spl_schedule *sched, spl_stream stream);

/* SpMM  A(i,j) = B(i,k) * C(k,j)   (Sec. VI-A).
 * B CSR n x m; C dense m x N; A dense n x N.  dtypes (vals, C, A): all F64;
 * all F32; or vals and C BF16 with A F32 (F32 accumulation; under the
 * NNZ and MERGE splits a row that spans tiles is the finishing tile's
 * partial plus the other tiles' carries, added by the fix-up).  Schedules:
 * ROW, NNZ, MERGE (default MERGE); col_tile 8..64 columns per lane group.
 * sched->variant (MERGE): 0 = each lane reads and writes 4 F32, 2 F64 or 8
 * BF16 consecutive columns (16 bytes of C) with one vector access when N,
 * C->ld, A->ld and the C and A pointers are multiples of that, col_tile
 * leaves 4 to 32 lanes per group and items_per_lane is 8 or 16 (otherwise
 * one column per lane); 1 = one column per lane; 2 (BF16 only) = as 0 with
 * 4 BF16 columns (8 bytes) per lane.
 * The workspace query returns the one-column-per-lane size, enough for
 * both.  SPL_SCHED_LEARNED / SPL_SCHED_AUTOTUNE as for spl_spmv. */
spl_status spl_spmm(spl_context *ctx, const spl_sparse *B, const spl_dense *C,
                    spl_dense *A, const spl_schedule *sched, void *workspace,
                    size_t workspace_bytes, spl_stream stream);

/* SpTTV  A(i,j) = B(i,j,k) * c(k)   (Sec. VI-A).
 * B CSF I x J x K; c vector K.  The output keeps B's (i,j) pattern
 * (pattern-preserving output, Sec. V-B): A shares B's first two levels
 * (A.pos = B.pos[1], A.crd = B.crd[1]) and only its values are written,
 * one per fiber, into the vector A of length B->nfibers.  dtypes: vals, c, A
 * all F64, or all F32 (F64 sums, rounded as for spl_spmv: twice for a
 * fiber that spans tiles).  The schedule applies to the fiber level
 * (fibers play the role of SpMV rows): ROW, NNZ or MERGE (default), with
 * sched->variant as for spl_spmv.  For a (Dense, Dense, Compressed) B the
 * fibers are all I * J pairs (i,j), so A is the dense I x J matrix, row-major
 * (an empty fiber gives 0). */
spl_status spl_spttv(spl_context *ctx, const spl_sparse *B, const spl_dense *c,
                     spl_dense *A, const spl_schedule *sched, void *workspace,
                     size_t workspace_bytes, spl_stream stream);

/* SpMTTKRP  A(i,l) = B(i,j,k) * C(j,l) * D(k,l)   (Sec. VI-A).
 * B CSF I x J x K; C dense J x R; D dense K x R; A dense I x R, F32.
 * dtypes (vals, C, D, A): (F32,F32,F32,F32) or (BF16,BF16,BF16,F32) with F32
 * accumulation.  Schedules: MERGE (default; equal runs of the merged slice
 * ends and fibers), NNZ (blocks of `tile` positions snapped to fiber starts:
 * the fused non-zero partition), ROW (blocks of `tile` slices); col_tile 16,
 * 32 or 64 rank columns per lane group.  sched->variant: 0 = each lane reads
 * and writes 4 consecutive rank columns with one vector access when R,
 * C->ld, D->ld and A->ld are multiples of 4, C and D are aligned to 4
 * elements, A to 16 bytes, col_tile is 32 or 64 and items_per_lane is not
 * 16 (otherwise one column per lane) -- with BF16 factors 8 rank columns
 * (16 bytes) per lane instead when R and every ld are multiples of 8, C and
 * D 16-byte aligned and (col_tile, items_per_lane) is (32, 0), (32, 3),
 * (32, 4), (64, 0), (64, 4) or (64, 8); 1 = one column per lane; 2 (BF16 only, else SPL_ERR_ARG) = 4
 * BF16 rank columns (8 bytes) per lane; 3 (F32 with items_per_lane 4, else
 * SPL_ERR_ARG) = as 0 with each chunk's leading positions staged in LDS, as
 * the BF16 leaf does.
 * items_per_lane: 8 or 16 for either leaf; 4 only with vector lanes, 5
 * only with 4-column lanes at col_tile 32, 3 only with 8-column BF16 lanes
 * at col_tile 32 (SPL_ERR_ARG when they do not apply): fewer registers and
 * LDS than 8, so more waves per SIMD.  0 (default) takes 5 for 4-column
 * lanes at col_tile 32 (4 with int64 positions or variant 3), 3 for
 * 8-column BF16 lanes at col_tile 32, 4 for the other vector lanes and 8
 * for one column per lane; tile 0 (default) takes 512 merged items with
 * vector lanes.  The workspace query returns the largest size over the
 * lane widths the call may take.  A
 * (Dense, Dense, Compressed) B is accepted: its middle level's pos/crd
 * (I + 1 and I * J int32) are written into the workspace, counted by the
 * query, and the leaf runs as for CSF. */
spl_status spl_mttkrp(spl_context *ctx, const spl_sparse *B, const spl_dense *C,
                      const spl_dense *D, spl_dense *A, const spl_schedule *sched,
                      void *workspace, size_t workspace_bytes, spl_stream stream);

/* Inner product  a = B(i,j,k) * C(i,j,k)  (every index summed, the TIN
 * statement with no free index, Sec. II-A; order-2 operands are accepted
 * too).  When B and C share one pattern (identical pos and crd pointers and
 * equal nnz) the aligned values are multiplied; otherwise the two patterns
 * are co-iterated (Sec. IV-C): each coordinate of B's last-but-one level is
 * looked up in C's segment of the same parent, and for CSF the two sorted
 * last-level lists are merged, so only coordinates both store contribute.
 * Same dimensions required.  Values both F64 or both F32, summed in F64
 * with a fixed reduction order; the result is one double written to `out`
 * (device).  Either operand may be (Dense, Dense, Compressed): unless the
 * two share one pattern, a Dense middle level is written out as pos/crd in
 * the workspace first.  The workspace query covers B; when C's middle level
 * is Dense, a caller workspace must also hold the query for C. */
spl_status spl_inner(spl_context *ctx, const spl_sparse *B, const spl_sparse *C, double *out,
                     const spl_schedule *sched, void *workspace, size_t workspace_bytes,
                     spl_stream stream);

/* SDDMM  A(i,j) = B(i,j) * C(i,k) * D(j,k)   (Sec. VI-A; the paper's last
 * factor D(k,j) is stored here transposed, one row per column coordinate j).
 * B CSR n x m; C dense n x K; D dense m x K.  The output keeps B's pattern
 * (Sec. V-B): A is the vector of B->nnz output values (A.pos = B.pos,
 * A.crd = B.crd).  dtypes (vals, C, D, A): all F64; all F32; or
 * (F32, BF16, BF16, F32) with F32 accumulation.  sched->variant: 0 = vector
 * ALU dot products (default; 16-byte factor accesses when K and both ld are
 * multiples of 2 F64, 4 F32 or 8 BF16 and the factors are 16-byte aligned),
 * 1 = matrix cores (BF16 factors only, K a multiple of 32, ld a multiple of
 * 8, 16-byte aligned factors).  Schedules: MERGE (default), NNZ, ROW. */
spl_status spl_sddmm(spl_context *ctx, const spl_sparse *B, const spl_dense *C,
                     const spl_dense *D, spl_dense *A, const spl_schedule *sched,
                     void *workspace, size_t workspace_bytes, spl_stream stream);

/* SpAdd3  A(i,j) = B(i,j) + C(i,j) + D(i,j)   (Sec. VI-A), assembled in
 * two phases (Sec. V-B).  B, C, D CSR with equal dimensions.
 * Symbolic phase: writes A_pos (n+1 entries, device) for the union of the
 * three patterns and the output nonzero count to *nnz_out (host); it
 * synchronizes on `stream` to read that count back.  Values are not read.
 * Only the row split is accepted: sched kind NNZ or MERGE gives
 * SPL_ERR_UNSUPPORTED (a non-zero split of a sum of CSR operands does not
 * align their positions).  sched->variant is checked as for the numeric
 * phase (0..4, else SPL_ERR_ARG); the count is the same for every variant
 * (a three-way merge a lane per row over coordinates staged in LDS). */
spl_status spl_spadd3_symbolic(spl_context *ctx, const spl_sparse *B, const spl_sparse *C,
                               const spl_sparse *D, int32_t *A_pos, int64_t *nnz_out,
                               const spl_schedule *sched, void *workspace,
                               size_t workspace_bytes, spl_stream stream);
/* Numeric phase: with A_pos from the symbolic phase, writes A_crd (strictly
 * increasing per row, *nnz_out entries) and A_vals (same dtype as the
 * operands, F64 or F32): each value sums the operands present at that
 * coordinate in the order B, C, D; a sum that cancels to zero keeps its
 * coordinate.  sched->variant picks the form: 1 a lane per row merging its
 * inputs read directly from memory, 2 the same with the workgroup's
 * coordinate runs staged in LDS, 3 with coordinates and values staged,
 * 4 by ranks (coordinates staged, a lane per input entry computing its
 * output slot by binary search in the other operands' rows); 0 the library
 * default (4).  Workgroups whose runs exceed the
 * stage fall back to direct reads; every variant gives the same bits, and
 * anything else is SPL_ERR_ARG. */
spl_status spl_spadd3_numeric(spl_context *ctx, const spl_sparse *B, const spl_sparse *C,
                              const spl_sparse *D, const int32_t *A_pos, int32_t *A_crd,
                              void *A_vals, const spl_schedule *sched, spl_stream stream);

/* ------------------------------------------------------ transposition */

/* The CSR arrays of B^T from those of B (B CSR n x m, int32 positions; values
 * F64, F32 or BF16, moved bit for bit).  The format language stores a CSC
 * matrix as (Dense, Compressed) over the reversed dimension order
 * (Sec. II-B), i.e. as the CSR arrays of its transpose: passing a CSC
 * matrix A as the n x m CSR of A^T gives A's CSR (m x n), which every CSR
 * leaf takes.  Outputs (device, caller-owned): T_pos m + 1 entries, T_crd
 * and T_vals nnz entries, rows of B^T with strictly increasing coordinates.
 * A stable LSD radix sort of the entries by column (8-bit digits, integer
 * counts and ranks only): deterministic and exact.  Workspace: NULL for the
 * context's pool, else at least spl_transpose_workspace_query bytes (about
 * 16 bytes per nonzero). */
spl_status spl_transpose_workspace_query(spl_context *ctx, const spl_sparse *B, size_t *bytes);
spl_status spl_transpose(spl_context *ctx, const spl_sparse *B, int32_t *T_pos, int32_t *T_crd,
                         void *T_vals, void *workspace, size_t workspace_bytes,
                         spl_stream stream);

/* ------------------------------------------- general index-notation leaves */

/* One tensor of an index-notation statement, bound by name: exactly one of
 * `sparse` (formats (D,C), (D,C,C) or (D,D,C), int32 positions) and `dense`
 * (a vector or row-major matrix) is set.  All pointers inside are device
 * pointers owned by the caller; `name` is a host string. */
typedef struct spl_tin_operand {
    const char *name;
    const spl_sparse *sparse;
    const spl_dense *dense;
} spl_tin_operand;

/* General statements of tensor index notation (Sec. II-A), beyond the seven
 * fixed ones, evaluated by leaves the library generates (Sec. IV-C) and
 * compiles at run time for gfx950 (hiprtc; the first call for a statement
 * and set of operand formats compiles, later calls reuse the context's
 * cache).
 *
 * Statement form: `Out(i,j) = T1 + T2 - ...` (or `Out(i) = ...`, or a scalar
 * `out = ...`), each term a product of tensor accesses such as B(i,j,k) or
 * c(k); every term uses the same index variables; variables not on the
 * left are summed.  Semantics: Out = sum over the summed variables of the
 * signed sum of the terms' products, an absent sparse entry counting as 0.
 * Loop nest: one thread per coordinate of the outermost index, which must
 * index every sparse operand first (their Dense first level) and be the
 * output's first index; the other variables follow in an order concordant
 * with every sparse operand's levels (Sec. IV-C), sparse-level variables
 * before dense-only ones.  A variable indexed by Compressed levels is
 * iterated by merging their sorted coordinates: the intersection within a
 * product, the union across a sum (co-iteration); a variable some term
 * reaches through no Compressed level is iterated over its whole extent.
 * Sums run in F64 in a fixed order (deterministic).  Values: every operand
 * and the output F64, or every one F32 (a scalar output is always F64).
 *
 * Outputs (`out`, named as the statement's left side):
 *   dense vector or matrix: every entry written (assignment semantics);
 *   scalar: a dense F64 vector of one entry;
 *   CSR matrix (Dense, Compressed): assembled in two phases (Sec. V-B):
 *     spl_tin_symbolic writes out->pos (A_pos, n+1 entries) and the count
 *     of stored entries (the coordinates where the statement's
 *     intersection/union structure holds, kept even when the value is 0),
 *     then spl_tin_eval with out->sparse->pos[1] = A_pos writes crd (sorted
 *     per row) and vals.
 * Errors: SPL_ERR_ARG (syntax, unbound or misnamed tensors), SPL_ERR_SHAPE
 * (extents disagree), SPL_ERR_FORMAT / SPL_ERR_DTYPE (operand formats or
 * value types), SPL_ERR_UNSUPPORTED (a statement outside this form: an
 * output whose first index is not the sparse operands' first, level orders
 * with no common loop order, terms over different variables, repeated
 * variables in one access), SPL_ERR_HIP (compilation or launch).
 * Workspace: NULL for the context's pool, else at least
 * spl_tin_workspace_query bytes. */
spl_status spl_tin_workspace_query(spl_context *ctx, const char *tin, int nops,
                                   const spl_tin_operand *ops, const spl_tin_operand *out,
                                   size_t *bytes);
spl_status spl_tin_symbolic(spl_context *ctx, const char *tin, int nops, const spl_tin_operand *ops,
                            const spl_tin_operand *out, int32_t *A_pos, int64_t *nnz_out,
                            void *workspace, size_t workspace_bytes, spl_stream stream);
spl_status spl_tin_eval(spl_context *ctx, const char *tin, int nops, const spl_tin_operand *ops,
                        const spl_tin_operand *out, void *workspace, size_t workspace_bytes,
                        spl_stream stream);
/* The HIP source generated for a statement and these operand formats
 * (host buffer `buf` of `cap` bytes, NUL-terminated, truncated if short;
 * *len receives the full length).  Compiles nothing and touches no GPU;
 * ctx may be NULL (errors then carry no detail). */
spl_status spl_tin_source(spl_context *ctx, const char *tin, int nops, const spl_tin_operand *ops,
                          const spl_tin_operand *out, char *buf, size_t cap, size_t *len);

/* ------------------------------------------------- learned schedule choice */

/* Seven sparsity features of a CSR matrix, computed in one pass over pos and
 * the first and last coordinate of every row, written as 7 floats to `feat`
 * (device): log2(rows), log2(nnz + 1), mean row degree, log2(1 + degree
 * variance), log2(1 + max degree), log2(1 + bandwidth) where bandwidth is
 * max |col - row| over the first and last entry of each row, and the mean
 * column span of a non-empty row divided by the column count. */
spl_status spl_features(spl_context *ctx, const spl_sparse *B, float *feat, void *workspace,
                        size_t workspace_bytes, spl_stream stream);

/* Parameter count of the schedule-selection network with K outputs
 * (7 -> 64 -> 64 -> K, ReLU; flat FP32 layout W1[64][7], b1[64], W2[64][64],
 * b2[64], W3[K][64], b3[K]); 0 for K outside 1..256. */
int64_t spl_mlp_param_count(int K);

/* Forward pass for `batch` feature rows X (batch x 7, device): Y (batch x K,
 * device) = network(standardize(X)).  `norm` (device, may be NULL) holds 7
 * means then 7 inverse standard deviations.  `act` (device, may be NULL)
 * receives the activations the backward pass needs: 2*64*batch + 7*batch
 * floats. */
spl_status spl_mlp_forward(spl_context *ctx, int K, const float *params, const float *X,
                           const float *norm, int64_t batch, float *Y, float *act,
                           spl_stream stream);

/* Backward pass of the mean squared error mean((Y - T)^2) over the batch
 * and the K outputs: gradient w.r.t. every parameter into `grad`
 * (param_count floats, device) and the loss into `loss` (1 float, device,
 * may be NULL).  Y and act come from spl_mlp_forward on the same batch; T is
 * batch x K (device).  Workspace: (128 + K + 1) * batch floats. */
spl_status spl_mlp_backward(spl_context *ctx, int K, const float *params, int64_t batch,
                            const float *Y, const float *T, const float *act, float *grad,
                            float *loss, void *workspace, size_t workspace_bytes,
                            spl_stream stream);

/* One Adam step (Kingma and Ba, 2015) on n parameters, in place: m and v
 * are the moment buffers (device, zero before step 1), `step` counts from 1
 * and sets the bias corrections. */
spl_status spl_adam_step(spl_context *ctx, int64_t n, float *params, float *m, float *v,
                         const float *grad, float lr, float beta1, float beta2, float eps,
                         int step, spl_stream stream);

/* ------------------------------------------------- schedule selection */

/* Exhaustive autotuning, the selector's fallback and its ground truth.
 * Times every candidate schedule of `op` (SPL_OP_SPMV: X = c, Y = a;
 * SPL_OP_SPMM: X = C, Y = A; operands as for spl_spmv / spl_spmm) on
 * `stream` with HIP events: one untimed call, then `reps` (1..100) timed
 * calls, median.  `candidates` (host, `ncand` of them, kinds SPL_ROW,
 * SPL_NNZ or SPL_MERGE) may be NULL with ncand = 0 for the library's list
 * (12 SpMV, 9 SpMM schedules).  Writes the fastest candidate to *best (host)
 * and, if times_ms is not NULL, every median in milliseconds (host, one per
 * candidate).  Y is overwritten.  Synchronizes on `stream`.  The calls use
 * the context's own workspace. */
spl_status spl_autotune(spl_context *ctx, spl_op op, const spl_sparse *B, const spl_dense *X,
                        spl_dense *Y, const spl_schedule *candidates, int ncand, int reps,
                        spl_schedule *best, float *times_ms, spl_stream stream);

/* Install a trained schedule selector for `op` (SPL_OP_SPMV or SPL_OP_SPMM)
 * in the context, which keeps its own device copy: K candidate schedules
 * (host; kinds SPL_ROW, SPL_NNZ, SPL_MERGE), the network parameters (host,
 * spl_mlp_param_count(K) floats, layout of spl_mlp_forward) and the feature
 * standardization (host, 7 means then 7 inverse standard deviations; NULL
 * for none).  Resets the training state of spl_mlp_train_step.  Replaces
 * any selector installed for `op`. */
spl_status spl_mlp_load(spl_context *ctx, spl_op op, int K, const spl_schedule *candidates,
                        const float *params, const float *norm);

/* Copy the selector installed for `op` out of the context (after all work
 * on the device has finished): *K always; then, where not NULL and cap >= K,
 * the candidates, the parameters and the standardization (host buffers of
 * cap schedules, spl_mlp_param_count(K) floats and 14 floats).
 * SPL_ERR_UNSUPPORTED if none is installed. */
spl_status spl_mlp_save(spl_context *ctx, spl_op op, int *K, int cap, spl_schedule *candidates,
                        float *params, float *norm);

/* The installed selector's choice for B: the 7 features (spl_features) and
 * the network's K predictions on the device, the candidate with the
 * smallest prediction (first on ties) to *out (host).  Synchronizes on
 * `stream`.  SPL_ERR_UNSUPPORTED if no selector is installed for `op`.
 * This is what SPL_SCHED_LEARNED runs. */
spl_status spl_mlp_predict(spl_context *ctx, spl_op op, const spl_sparse *B, spl_schedule *out,
                           spl_stream stream);

/* One training step of the installed selector on a batch: X (device,
 * batch x 7 raw features), T (device, batch x K targets); forward, mean
 * squared error backward and one Adam step (beta1 0.9, beta2 0.999, eps
 * 1e-8, learning rate lr) on the context's parameters and moments, all on
 * `stream`; the batch loss before the step to *loss (device, may be NULL).
 * Uses the context's workspace. */
spl_status spl_mlp_train_step(spl_context *ctx, spl_op op, const float *X, const float *T,
                              int64_t batch, float lr, float *loss, spl_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* SPLEAF_H */
