// Carry fix-up shared by the non-zero / merge split leaves.
//
// A leaf workgroup ("tile") covers `stride` consecutive pieces of the level
// partition (pieces [u*stride, (u+1)*stride), capped at npieces).  The row
// (or fiber, or slice) still open at its end is
//     R(u) = trow[min((u+1)*stride, npieces)],
// and its partial sum is the tile's carry: `ncols` accumulators.  Several
// consecutive tiles can be open on one long row.  Tile u is the first of its
// run when u == 0 or R(u-1) != R(u).
//
// k_carry_fixup runs one wave per tile; only first-of-run waves work.  The
// run's end is found 64 tiles at a time with a wave ballot, then the run's
// carries are summed with a fixed assignment of tiles to lanes and a fixed
// reduction order and added to the output row (which the tile finishing the
// row wrote in the leaf kernel).  Every load of the run is independent, so
// a row spanning hundreds of tiles costs a few memory latencies, and the
// result is bitwise reproducible.
#pragma once

#include "device.hpp"

namespace spl {

constexpr int kFixBlock = 64;  // one wave per tile

template <typename OT, typename Acc>
__global__ __launch_bounds__(kFixBlock) void k_carry_fixup(int64_t rows, int64_t ncols,
                                                           const int32_t *__restrict__ trow,
                                                           int64_t npieces, int64_t stride,
                                                           int64_t ntiles,
                                                           const Acc *__restrict__ carry,
                                                           OT *__restrict__ out, int64_t ldo) {
    const int64_t u = blockIdx.x;
    const int lane = threadIdx.x;
    auto open_row = [&](int64_t v) {  // R(v)
        const int64_t piece = (v + 1) * stride;
        return trow[piece < npieces ? piece : npieces];
    };
    const int32_t r = open_row(u);
    if (r >= rows) return;
    if (u > 0 && open_row(u - 1) == r) return;  // not the first tile open on row r

    // Run end: the first v > u whose open row differs from r.
    int64_t end = u;
    for (int64_t v0 = u;; v0 += kFixBlock) {
        const int64_t v = v0 + lane;
        const bool same = v < ntiles && open_row(v) == r;
        const uint64_t mask = __ballot(same);
        const int cnt = __popcll(mask);
        if (cnt < kFixBlock) {
            end = v0 + cnt;
            break;
        }
    }

    OT *orow = out + static_cast<int64_t>(r) * ldo;
    if (ncols == 1) {
        Acc part = 0;
        for (int64_t v = u + lane; v < end; v += kFixBlock) part += carry[v];
        // fixed butterfly order over the wave
#pragma unroll
        for (int off = kFixBlock / 2; off > 0; off >>= 1) part += __shfl_xor(part, off);
        if (lane == 0) orow[0] = narrow<OT>(static_cast<Acc>(orow[0]) + part);
        return;
    }
    // vectors: two slices of 32 columns
    const int slice = lane / 32, c = lane % 32;
    for (int64_t c0 = 0; c0 < ncols; c0 += 32) {
        const int64_t col = c0 + c;
        Acc part = 0;
        if (col < ncols)
            for (int64_t v = u + slice; v < end; v += 2) part += carry[v * ncols + col];
        part += __shfl_xor(part, 32);
        if (slice == 0 && col < ncols) orow[col] = narrow<OT>(static_cast<Acc>(orow[col]) + part);
    }
}

template <typename OT, typename Acc>
hipError_t launch_carry_fixup(int64_t rows, int64_t ncols, const int32_t *trow, int64_t npieces,
                              int64_t stride, int64_t ntiles, const Acc *carry, OT *out,
                              int64_t ldo, hipStream_t s) {
    if (ntiles == 0 || ncols == 0) return hipSuccess;
    k_carry_fixup<OT, Acc><<<dim3(static_cast<unsigned>(ntiles)), kFixBlock, 0, s>>>(
        rows, ncols, trow, npieces, stride, ntiles, carry, out, ldo);
    return hipGetLastError();
}

}  // namespace spl
