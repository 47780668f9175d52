// Host-side declarations shared by the spleaf translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "spleaf.h"

namespace spl {

// Tile bounds of one split, in device memory: ntiles + 1 (row, position)
// pairs, the last one being (rows, nnz).
struct Tiles {
    int32_t *row;
    int32_t *pos;
    int64_t ntiles;
};

// ---- partition.hip -------------------------------------------------------
// Number of tiles a split produces (at least 1).
int64_t tile_count(int kind, int64_t rows, int64_t nnz, int64_t size);
// Fill `t` (row/pos arrays sized ntiles+1) for the split `kind` of the
// Compressed level (rows, pos) with tile size `size`.
hipError_t launch_tile_bounds(int kind, int64_t rows, const int32_t *pos, int64_t nnz,
                              int64_t size, const Tiles &t, hipStream_t s);

// ---- spmv.hip ------------------------------------------------------------
hipError_t launch_spmv_row(int dtype, int lanes, int64_t n, const int32_t *pos,
                           const int32_t *crd, const void *vals, const void *x, void *y,
                           hipStream_t s);
hipError_t launch_spmv_tiles(int dtype, int items, int64_t n, const int32_t *pos,
                             const int32_t *crd, const void *vals, const void *x, void *y,
                             const Tiles &t, double *carry, hipStream_t s);

// ---- spmm.hip ------------------------------------------------------------
hipError_t launch_spmm_row(int vtype, int otype, int col_tile, int64_t n, int64_t N,
                           const int32_t *pos, const int32_t *crd, const void *vals,
                           const void *B, int64_t ldb, void *C, int64_t ldc, hipStream_t s);
hipError_t launch_spmm_tiles(int vtype, int otype, int col_tile, int items, int64_t n,
                             int64_t N, const int32_t *pos, const int32_t *crd,
                             const void *vals, const void *B, int64_t ldb, void *C,
                             int64_t ldc, const Tiles &t, void *carry, hipStream_t s);

// ---- validate.hip --------------------------------------------------------
// Writes a failure code (0 = valid) and the first failing index to flags[0..1].
hipError_t launch_validate_level(int64_t parents, const int32_t *pos, const int32_t *crd,
                                 int64_t children, int64_t extent, int64_t *flags,
                                 hipStream_t s);

}  // namespace spl
