// Host-side declarations shared by the spleaf translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "spleaf.h"

namespace spl {

// Largest span in bytes that the leaves read through one buffer descriptor
// (device.hpp: branch-free gathers): every in-bounds offset then fits 32
// bits and stays below the out-of-range offset the descriptor loads use.
constexpr uint32_t kBufRange = 0xFFFFFF00u;

// Tile bounds of one split, in device memory: ntiles + 1 (row, position)
// pairs, the last one being (rows, nnz).
struct Tiles {
    int32_t *row;
    int32_t *pos;
    int64_t ntiles;
    int64_t *pos64 = nullptr;  // in place of pos when the positions are int64
};

// ---- partition.hip -------------------------------------------------------
// Number of tiles a split produces (at least 1).
int64_t tile_count(int kind, int64_t rows, int64_t nnz, int64_t size);
// Fill `t` (row/pos arrays sized ntiles+1) for the split `kind` of the
// Compressed level (rows, pos) with tile size `size`.
// Merge split of a CSR with int64 positions: t.row and t.pos64.
hipError_t launch_merge_bounds64(int64_t rows, const int64_t *pos, int64_t nnz, int64_t size,
                                 const Tiles &t, hipStream_t s);
// Merge split of a level with int64 pos whose child count is below 2^31 (a
// CSF slice level over fibers): tile positions in t.pos (int32).
hipError_t launch_merge_bounds64_32(int64_t rows, const int64_t *pos, int64_t nnz, int64_t size,
                                    const Tiles &t, hipStream_t s);
hipError_t launch_tile_bounds(int kind, int64_t rows, const int32_t *pos, int64_t nnz,
                              int64_t size, const Tiles &t, hipStream_t s);

// ---- spmv.hip ------------------------------------------------------------
// Row split: row i covers positions [pos_b[i], pos_e[i]); pos_e == nullptr
// means CSR (pos_e = pos_b + 1).
hipError_t launch_spmv_row(int dtype, int lanes, int64_t n, const int32_t *pos_b,
                           const int32_t *pos_e, const int32_t *crd, const void *vals,
                           const void *x, void *y, hipStream_t s);
// Tiled leaves: one workgroup per `stride` consecutive partition pieces of
// `t`; carries are one per workgroup.
// exact_chunks: every piece of `t` is at most one chunk of 256 * items merged
// items (merge split): the row-end flag leaf k_spmv_flag (variant 0) or the
// row-end search leaf k_spmv_pipe (variant 1).
// The row-end flag leaf over exact merge chunks of a CSR with int64
// positions (tile bounds in t.row / t.pos64).
hipError_t launch_spmv_flag64(int dtype, int items, int64_t n, const int64_t *pos,
                              const int32_t *crd, const void *vals, const void *x, void *y,
                              const Tiles &t, int64_t stride, double *carry, hipStream_t s);
hipError_t launch_spmv_tiles(int dtype, int items, int64_t n, const int32_t *pos,
                             const int32_t *crd, const void *vals, const void *x, void *y,
                             const Tiles &t, int64_t stride, bool exact_chunks, int variant,
                             double *carry, hipStream_t s);
// Adds workgroup carries into the rows left open (after the leaf).
// Merge split over position windows [begin[i], end[i]): vpos holds the
// scanned window lengths (n + 1 entries, from launch_window_offsets).
hipError_t launch_spmv_window_merge(int dtype, int items, int64_t n, const int32_t *vpos,
                                    const int32_t *begin, const int32_t *crd, const void *vals,
                                    const void *x, void *y, const Tiles &t, int64_t stride,
                                    double *carry, hipStream_t s);
hipError_t launch_spmv_fixup(int dtype, int64_t n, const Tiles &t, int64_t stride,
                             const double *carry, void *y, hipStream_t s);

// ---- spmm.hip ------------------------------------------------------------
hipError_t launch_spmm_row(int vtype, int otype, int col_tile, int64_t n, int64_t N,
                           const int32_t *pos, const int32_t *crd, const void *vals,
                           const void *B, int64_t ldb, void *C, int64_t ldc, hipStream_t s);
// exact_chunks: every piece of `t` holds at most one leaf chunk
// ((256 / lanes) * items merged items, lanes = col_tile / vec), as the merge
// split is cut here; the leaf then pipelines its staging loads (k_spmm_pipe).
// vec: 1, or spmm_vec_width(vtype) columns per lane (merge split only; N,
// the leading dimensions and both dense pointers aligned to it, and
// col_tile / vec in {8, 16, 32}).
int spmm_vec_width(int vtype);
// buf: the pipelined leaf's 16-byte row gathers go through a buffer
// descriptor (B's rows * ldb span at most kBufRange bytes).
hipError_t launch_spmm_tiles(int vtype, int col_tile, int items, int vec, int64_t n, int64_t N,
                             const int32_t *pos, const int32_t *crd, const void *vals,
                             const void *B, int64_t ldb, void *C, int64_t ldc, const Tiles &t,
                             int64_t stride, bool exact_chunks, bool buf, void *carry,
                             hipStream_t s);
// The same over a CSR with int64 positions: merge split and vector lanes
// only (vec == spmm_vec_width(vtype); tile positions in t.pos64).
hipError_t launch_spmm_tiles64(int vtype, int col_tile, int items, int vec, int64_t n, int64_t N,
                               const int64_t *pos, const int32_t *crd, const void *vals,
                               const void *B, int64_t ldb, void *C, int64_t ldc, const Tiles &t,
                               int64_t stride, bool buf, void *carry, hipStream_t s);
hipError_t launch_spmm_fixup(int vtype, int64_t n, int64_t N, const Tiles &t, int64_t stride,
                             const void *carry, void *C, int64_t ldc, hipStream_t s);

// ---- csf.hip -------------------------------------------------------------
// Threads per workgroup of the vector-lane MTTKRP leaf (the one-column
// leaf uses 256): its merged-item chunk is (128 / lanes) * items_per_lane.
constexpr int kMttkrpThreads = 128;
// Value-range partition of a Compressed level: out[c * rows + i] = first
// position of parent i whose coordinate is >= bounds[c], c < nbounds.
hipError_t launch_coord_split(int64_t rows, const int32_t *pos, const int32_t *crd, int64_t nbounds,
                              const int32_t *bounds, int32_t *out, hipStream_t s);
// pos (I + 1 entries) and crd (I * J entries) of a Dense level of extent J
// under I parents, written out as a Compressed level would store them.
hipError_t launch_dense_level(int64_t I, int64_t J, int32_t *pos, int32_t *crd, hipStream_t s);
// Fiber-aligned non-zero split of a CSF tensor: t.row = slice, t.pos = fiber.
hipError_t launch_csf_nnz_bounds(int64_t I, const int32_t *pos1, int64_t F, const int32_t *pos2,
                                 int64_t nnz, int64_t T, const Tiles &t, hipStream_t s);
// vec: 1, or 4 (8 for BF16) rank columns per lane (R, ldc, ldd, lda
// multiples of vec, aligned factors, col_tile 32 or 64).
// buf: the vector-lane leaf loads through buffer descriptors (mttkrp_buf
// says when the spans allow it).
// stage: FP32 vector lanes with 4 items stage the chunk's leading positions
// in LDS as the BF16 leaf always does.
// Whether every position and factor span fits a buffer descriptor's range
// (the vector-lane leaf's branch-free loads).
bool mttkrp_buf(int64_t nnz, size_t val_bytes, int64_t J, int64_t ldc, int64_t K, int64_t ldd,
                size_t factor_bytes);
hipError_t launch_mttkrp_tiles(int vtype, bool buf, bool stage, int col_tile, int items, int vec, int64_t I,
                               int64_t R, const int32_t *pos1, const int32_t *crd1,
                               const int32_t *pos2, const int32_t *crd2, const void *vals,
                               const void *C, int64_t ldc, const void *D, int64_t ldd, float *A,
                               int64_t lda, const Tiles &t, int64_t stride, float *carry,
                               hipStream_t s);
// The vector-lane MTTKRP leaf over a CSF with int64 pos1/pos2 (fiber count
// below 2^31; merge split over slices and fibers, tiles in t.row / t.pos).
hipError_t launch_mttkrp_tiles64(int vtype, bool buf, int col_tile, int items, int vec, int64_t I,
                                 int64_t R, const int64_t *pos1, const int32_t *crd1,
                                 const int64_t *pos2, const int32_t *crd2, const void *vals,
                                 const void *C, int64_t ldc, const void *D, int64_t ldd, float *A,
                                 int64_t lda, const Tiles &t, int64_t stride, float *carry,
                                 hipStream_t s);
hipError_t launch_mttkrp_fixup(int64_t I, int64_t R, const Tiles &t, int64_t stride,
                               const float *carry, float *A, int64_t lda, hipStream_t s);
hipError_t launch_inner(int vtype, int64_t nnz, const void *a, const void *b, double *part,
                        int64_t nparts, double *out, hipStream_t s);
hipError_t launch_inner_final(int64_t nparts, const double *part, double *out, hipStream_t s);

// ---- inner.hip -----------------------------------------------------------
// Inner product of operands with different patterns (order 2: units are B's
// positions, n rows; order 3: units are B's fibers, n slices); the workspace
// `ws` holds inner_general_ws(units) bytes (per-workgroup partials and range
// bounds).
int64_t inner_general_parts(int64_t units);
size_t inner_general_ws(int64_t units);
hipError_t launch_inner_general(int vtype, int order, int64_t n, int64_t units,
                                const int32_t *bpos, const int32_t *bcrd, const int32_t *bpos2,
                                const int32_t *bcrd2, const void *bv, const int32_t *cpos,
                                const int32_t *ccrd, const int32_t *cpos2, const int32_t *ccrd2,
                                const void *cv, int64_t nnzb, int64_t nnzc, int64_t cunits,
                                void *ws, double *out, hipStream_t s);

// ---- sddmm.hip -----------------------------------------------------------
int64_t sddmm_chunk();
// Factor elements per 16-byte access (2 F64, 4 F32, 8 BF16).
int sddmm_vec_width(int ftype);
// vec_lanes (variant 0): 0 = one element per lane access; 8, 16 or 32 =
// lanes per position reading sddmm_vec_width(ftype) elements each (K, ldc,
// ldd multiples of it, factors 16-byte aligned).
hipError_t launch_sddmm(int vtype, int ftype, int variant, int vec_lanes, int64_t K,
                        const int32_t *pos, const int32_t *crd, const void *bv, const void *C,
                        int64_t ldc, const void *D, int64_t ldd, void *out, const Tiles &t,
                        int64_t stride, hipStream_t s);

// ---- spadd3.hip ----------------------------------------------------------
int64_t spadd3_scan_tiles(int64_t n);
// vpos[0] = 0, vpos[i + 1] = sum over r <= i of max(end[r] - begin[r], 0);
// tile_sum holds spadd3_scan_tiles(n) entries; the sum goes to *total.
hipError_t launch_window_offsets(int64_t n, const int32_t *begin, const int32_t *end,
                                 int32_t *vpos, int64_t *tile_sum, int64_t *total, hipStream_t s);
// In-place scan of per-row counts apos[1..n] into a pos array (apos[0] = 0);
// tile_sum holds spadd3_scan_tiles(n) entries, the total goes to *total.
hipError_t launch_pos_scan(int64_t n, int32_t *apos, int64_t *tile_sum, int64_t *total,
                           hipStream_t s);
hipError_t launch_spadd3_symbolic(int64_t n, const int32_t *bp, const int32_t *bc,
                                  const int32_t *cp, const int32_t *cc, const int32_t *dp,
                                  const int32_t *dc, int32_t *apos, int64_t *tile_sum,
                                  int64_t *total, hipStream_t s);
hipError_t launch_spadd3_numeric(int vtype, int64_t n, const int32_t *bp, const int32_t *bc,
                                 const void *bv, const int32_t *cp, const int32_t *cc,
                                 const void *cv, const int32_t *dp, const int32_t *dc,
                                 const void *dv, const int32_t *apos, int32_t *acrd, void *aval,
                                 int stage, hipStream_t s);

// ---- mlp.hip -------------------------------------------------------------
int64_t mlp_param_count(int K);
int64_t feature_ws_bytes();
hipError_t launch_features(int64_t n, int64_t m, const int32_t *pos, const int32_t *crd,
                           double *part, float *feat, hipStream_t s);
hipError_t launch_mlp_forward(int K, const float *P, const float *X, const float *norm,
                              int64_t B, float *Y, float *act, hipStream_t s);
hipError_t launch_mlp_backward(int K, const float *P, int64_t B, const float *Y, const float *T,
                               const float *act, float *dZ, float *loss_b, float *grad,
                               float *loss, hipStream_t s);
hipError_t launch_adam(int64_t n, float *P, float *m, float *v, const float *g, float lr, float b1,
                       float b2, float eps, int step, hipStream_t s);

// ---- probe.hip -----------------------------------------------------------
hipError_t launch_probe(int kind, const void *buf, int64_t bytes, int64_t row_bytes,
                        int64_t count, double *out, int64_t blocks, hipStream_t s);

// ---- validate.hip --------------------------------------------------------
// Writes a failure code (0 = valid) and the first failing index to flags[0..1].
hipError_t launch_validate_level(int64_t parents, const int32_t *pos, const int32_t *crd,
                                 int64_t children, int64_t extent, int64_t *flags,
                                 hipStream_t s);

// ---- transpose.hip -------------------------------------------------------
// Radix passes for column indices below m (8 bits each).
int transpose_passes(int64_t m);
// Workspace of launch_transpose for nnz entries and m columns.
size_t transpose_ws_bytes(int64_t nnz, int64_t m);
// CSR arrays of B^T (m + 1 pos, nnz crd and vals) from B's (n x m).
hipError_t launch_transpose(int vtype, int64_t n, int64_t m, int64_t nnz, const int32_t *pos,
                            const int32_t *crd, const void *vals, int32_t *tpos, int32_t *tcrd,
                            void *tvals, void *ws, hipStream_t s);

// ---- scratch.hip ---------------------------------------------------------
// Bytes of the static device scratch behind spl_spmv_noalloc.
constexpr size_t kScratchBytes = static_cast<size_t>(16) << 20;
// Look up the scratch's device address on `device` (which must be current)
// once; later calls return the first call's status.
hipError_t scratch_init(int device);
// The address scratch_init found for `device`, or nullptr.
void *scratch_ptr(int device);

}  // namespace spl
