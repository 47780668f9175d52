// Level partitions of a Compressed level (paper Sec. III-A image/preimage,
// Sec. IV-B Table I level functions), computed on the GPU.
//
// A tile is described by the point at which it starts on the merged
// sequence of row ends and positions: (first row it finishes, first
// position it covers).  Row r is finished once position pos[r+1]-1 has been
// covered, i.e. at any point (i, p) with pos[r+1] <= p; an empty row is
// finished as soon as the position walk reaches its start.
//
//  - Row split (universe partition of the Dense level in blocks of R rows,
//    carried down by an image through pos): tile t starts at
//    (t*R, pos[t*R]).
//  - Non-zero split (non-zero partition of the fused coordinates in blocks of
//    T positions, rows recovered by a preimage through pos): tile t starts at
//    (number of rows finished at position t*T, t*T); tile 0 starts at (0, 0)
//    so that leading empty rows belong to it.
//  - Merge split: tile t starts at the point t*M of the merged sequence
//    (a search per tile, or one sweep over the rows when they are few).
//    A negative nnz means the position total is read from pos[rows] on the
//    device (positions scanned on the device; the tile count passed in is
//    then an upper bound, and every tile past the end starts at the end).
#include <algorithm>

#include "device.hpp"
#include "internal.hpp"

namespace spl {
namespace {

// Number of rows r in [0, rows) with pos[r+1] <= p (binary search; pos is
// non-decreasing).
__device__ __forceinline__ int64_t rows_finished(const int32_t *pos, int64_t rows, int64_t p) {
    int64_t lo = 0, hi = rows;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (static_cast<int64_t>(pos[mid + 1]) <= p)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kBlock) void k_row_bounds(int64_t rows, const int32_t *pos,
                                                       int64_t R, int64_t ntiles,
                                                       int32_t *trow, int32_t *tpos) {
    int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (t > ntiles) return;
    int64_t r = t * R < rows ? t * R : rows;
    trow[t] = static_cast<int32_t>(r);
    tpos[t] = pos[r];
}

__global__ __launch_bounds__(kBlock) void k_nnz_bounds(int64_t rows, const int32_t *pos,
                                                       int64_t nnz, int64_t T, int64_t ntiles,
                                                       int32_t *trow, int32_t *tpos) {
    int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (t > ntiles) return;
    int64_t p = (t == ntiles || t * T > nnz) ? nnz : t * T;
    tpos[t] = static_cast<int32_t>(p);
    trow[t] = static_cast<int32_t>(t == 0 ? 0 : rows_finished(pos, rows, p));
}

template <typename P, typename TP>
__global__ __launch_bounds__(kBlock) void k_merge_bounds(int64_t rows, const P *pos,
                                                         int64_t nnz, int64_t M, int64_t ntiles,
                                                         int32_t *trow, TP *tpos) {
    int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (t > ntiles) return;
    if (nnz < 0) nnz = static_cast<int64_t>(pos[rows]);  // the total is on the device
    int64_t total = rows + nnz;
    int64_t d = (t == ntiles || t * M > total) ? total : t * M;
    int64_t i = merge_search(d, rows, nnz, 0, [&](int64_t k) { return pos[k + 1]; });
    trow[t] = static_cast<int32_t>(i);
    tpos[t] = static_cast<TP>(d - i);
}

// The merge split by a sweep over the rows instead of a search per tile:
// row i (i < rows) owns the merged indices i + pos[i] .. i + pos[i+1] (its
// positions, then its end), so every tile start d = t M in that range has
// trow = i and tpos = d - i (the merge-path search gives the same i: the row
// ends before index d are those of rows 0 .. i-1).  The bounds at or past
// the end are (rows, nnz).  One lane per row; reading pos once costs less
// than a 20-step dependent search per tile when rows are few.
// (log2M >= 0: M is 2^log2M, and the divisions by M are shifts; a 64-bit
// division per lane costs more than the lane's reads.)
template <typename P, typename TP>
__global__ __launch_bounds__(kBlock) void k_merge_sweep(int64_t rows, const P *pos,
                                                        int64_t nnz, int64_t M, int log2M,
                                                        int64_t ntiles, int32_t *trow, TP *tpos) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (nnz < 0) nnz = static_cast<int64_t>(pos[rows]);  // the total is on the device
    auto tiles_to = [&](int64_t d) {  // first tile starting at or after merged index d
        return log2M >= 0 ? (d + M - 1) >> log2M : (d + M - 1) / M;
    };
    // every bound at or past the end (the last one, all of them when there
    // are no items, many when the tile count is an upper bound), spread over
    // all threads
    const int64_t nthreads = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t t = tiles_to(rows + nnz) + i; t <= ntiles; t += nthreads) {
        trow[t] = static_cast<int32_t>(rows);
        tpos[t] = static_cast<TP>(nnz);
    }
    if (i >= rows) return;
    const int64_t lo = i + static_cast<int64_t>(pos[i]), hi = i + static_cast<int64_t>(pos[i + 1]);
    for (int64_t t = tiles_to(lo); t * M <= hi; ++t) {
        trow[t] = static_cast<int32_t>(i);
        tpos[t] = static_cast<TP>(t * M - i);
    }
}

// Universe partition of a Compressed level by coordinate value ranges,
// carried up to the parent level by a preimage (Sec. III-A; Table I, the
// Compressed level's value-range partition): parent i's positions whose
// coordinate lies in [bounds[c], bounds[c+1]) are [out[c][i], out[c+1][i]),
// where out[c][i] is the first position of parent i with coordinate at
// least bounds[c] (coordinates are sorted within a parent).  One lane per
// parent runs the binary searches of up to kSplitBatch bounds in lockstep
// inside its segment, so their loads are in flight together; the writes of
// one bound are coalesced over the lanes.
constexpr int kSplitBatch = 16;

__global__ __launch_bounds__(kBlock) void k_coord_split(int64_t rows, const int32_t *__restrict__ pos,
                                                        const int32_t *__restrict__ crd,
                                                        int64_t nbounds,
                                                        const int32_t *__restrict__ bounds,
                                                        int32_t *__restrict__ out) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= rows) return;
    const int32_t lo0 = pos[i], hi0 = pos[i + 1];
    for (int64_t c0 = 0; c0 < nbounds; c0 += kSplitBatch) {
        int32_t lo[kSplitBatch], hi[kSplitBatch], b[kSplitBatch];
#pragma unroll
        for (int k = 0; k < kSplitBatch; ++k) {
            const bool live = c0 + k < nbounds;
            b[k] = live ? bounds[c0 + k] : 0;
            lo[k] = lo0;
            hi[k] = live ? hi0 : lo0;
        }
        for (int32_t len = hi0 - lo0; len > 0; len >>= 1) {  // one halving per step
#pragma unroll
            for (int k = 0; k < kSplitBatch; ++k) {
                if (lo[k] < hi[k]) {
                    const int32_t mid = lo[k] + ((hi[k] - lo[k]) >> 1);
                    if (crd[mid] < b[k])
                        lo[k] = mid + 1;
                    else
                        hi[k] = mid;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < kSplitBatch; ++k)
            if (c0 + k < nbounds) out[(c0 + k) * rows + i] = lo[k];
    }
}

// The pos and crd arrays a Dense level of extent J under I parents would
// have if it were stored compressed (the Dense level functions, Sec. III-B
// and Table I): parent i owns positions [i J, (i + 1) J) and position f holds
// coordinate f mod J.
__global__ __launch_bounds__(kBlock) void k_dense_level(int64_t I, int64_t J,
                                                        int32_t *__restrict__ pos,
                                                        int32_t *__restrict__ crd) {
    const int64_t F = I * J;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t f = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; f < F; f += stride)
        crd[f] = static_cast<int32_t>(f % J);
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i <= I; i += stride)
        pos[i] = static_cast<int32_t>(i * J);
}

}  // namespace

hipError_t launch_coord_split(int64_t rows, const int32_t *pos, const int32_t *crd, int64_t nbounds,
                              const int32_t *bounds, int32_t *out, hipStream_t s) {
    if (nbounds == 0 || rows == 0) return hipSuccess;
    k_coord_split<<<dim3(static_cast<unsigned>(ceil_div(rows, kBlock))), kBlock, 0, s>>>(
        rows, pos, crd, nbounds, bounds, out);
    return hipGetLastError();
}

hipError_t launch_dense_level(int64_t I, int64_t J, int32_t *pos, int32_t *crd, hipStream_t s) {
    const int64_t F = I * J;
    const int64_t work = (F > I + 1 ? F : I + 1);
    const int64_t blocks = std::min<int64_t>(ceil_div(work, kBlock), 8192);
    k_dense_level<<<dim3(static_cast<unsigned>(blocks)), kBlock, 0, s>>>(I, J, pos, crd);
    return hipGetLastError();
}

int64_t tile_count(int kind, int64_t rows, int64_t nnz, int64_t size) {
    int64_t items = kind == SPL_ROW ? rows : kind == SPL_NNZ ? nnz : rows + nnz;
    int64_t nt = (items + size - 1) / size;
    return nt > 0 ? nt : 1;
}

// Up to this many rows, and while there are fewer tiles than rows, the
// merge split is computed by the sweep (a read of 4 (rows + 1) bytes);
// otherwise by one merge-path search per tile.  With more tiles than rows
// the sweep's lanes would write many bounds each, one after another: the
// 200,000 power-law slices of a 1e8-nonzero CSF cut into 990,000 chunks of
// 64 merged items took 253 us by the sweep, its longest slice writing about
// 3,000 bounds.
constexpr int64_t kMergeSweepRows = 8000000;

template <typename P, typename TP>
hipError_t merge_bounds(int64_t rows, const P *pos, int64_t nnz, int64_t size, int64_t ntiles,
                        int32_t *trow, TP *tpos, hipStream_t s) {
    if (rows <= kMergeSweepRows && ntiles < rows) {
        int log2M = -1;  // the tile size is 2^log2M, or -1
        if (size > 0 && (size & (size - 1)) == 0) log2M = __builtin_ctzll(static_cast<uint64_t>(size));
        k_merge_sweep<P, TP><<<dim3(static_cast<unsigned>(ceil_div(rows + 1, kBlock))), kBlock, 0,
                               s>>>(rows, pos, nnz, size, log2M, ntiles, trow, tpos);
    } else {
        k_merge_bounds<P, TP><<<dim3(static_cast<unsigned>(ceil_div(ntiles + 1, kBlock))), kBlock,
                                0, s>>>(rows, pos, nnz, size, ntiles, trow, tpos);
    }
    return hipGetLastError();
}

hipError_t launch_tile_bounds(int kind, int64_t rows, const int32_t *pos, int64_t nnz,
                              int64_t size, const Tiles &t, hipStream_t s) {
    dim3 grid(static_cast<unsigned>((t.ntiles + 1 + kBlock - 1) / kBlock));
    switch (kind) {
    case SPL_ROW:
        k_row_bounds<<<grid, kBlock, 0, s>>>(rows, pos, size, t.ntiles, t.row, t.pos);
        break;
    case SPL_NNZ:
        k_nnz_bounds<<<grid, kBlock, 0, s>>>(rows, pos, nnz, size, t.ntiles, t.row, t.pos);
        break;
    default:
        return merge_bounds(rows, pos, nnz, size, t.ntiles, t.row, t.pos, s);
    }
    return hipGetLastError();
}

hipError_t launch_merge_bounds64(int64_t rows, const int64_t *pos, int64_t nnz, int64_t size,
                                 const Tiles &t, hipStream_t s) {
    return merge_bounds(rows, pos, nnz, size, t.ntiles, t.row, t.pos64, s);
}

hipError_t launch_merge_bounds64_32(int64_t rows, const int64_t *pos, int64_t nnz, int64_t size,
                                    const Tiles &t, hipStream_t s) {
    return merge_bounds(rows, pos, nnz, size, t.ntiles, t.row, t.pos, s);
}

}  // namespace spl
