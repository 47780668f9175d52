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
// k_carry_fixup gives each tile a lane (one column) or 8 lanes (lane c
// takes columns c, c + 8, ...: a wave covers 8 tiles, so a wave's chain of
// dependent loads serves 8 rows).  The lanes of the first tile of a run
// follow the run for up to kFixShort tiles and, if it ends there, add the
// run's carries to the output row themselves, in tile order (the row was
// written by the tile that finished it, in the leaf kernel).  Longer runs
// (rows spanning many tiles) are taken by the whole wave, one after
// another: the run's end is found 64 tiles at a time with a ballot, and the
// carries are summed with a fixed assignment of tiles to lanes and a fixed
// reduction order.  Every order is fixed, so the result is bitwise
// reproducible.
#pragma once

#include "device.hpp"

namespace spl {

constexpr int kFixBlock = 256;  // tiles per workgroup, one per lane
constexpr int kFixShort = 8;    // longest run a lane sums alone
static_assert(kFixShort >= 2, "the first step of a run is taken before the loop");
constexpr int kFixLanes = 8;    // lanes per tile for vector carries
constexpr int kFixBatch = 8;    // carries one lane loads before adding them

template <typename OT, typename Acc>
__global__ __launch_bounds__(kFixBlock) void k_carry_fixup(int64_t rows, int64_t ncols,
                                                           const int32_t *__restrict__ trow,
                                                           int64_t npieces, int64_t stride,
                                                           int64_t ntiles,
                                                           const Acc *__restrict__ carry,
                                                           OT *__restrict__ out, int64_t ldo) {
    const int lane = threadIdx.x % kWave;
    // lanes per tile: 1 for a single column, else 8 (lane c takes columns c, c + 8, ...)
    const int per = ncols == 1 ? 1 : kFixLanes;
    const int c = lane % per;
    const int64_t u = (static_cast<int64_t>(blockIdx.x) * kFixBlock + threadIdx.x) / per;
    auto open_row = [&](int64_t v) {  // R(v)
        const int64_t piece = (v + 1) * stride;
        return trow[piece < npieces ? piece : npieces];
    };
    // the open rows of tiles u - 1, u and u + 1 loaded together (indices
    // clamped into [0, ntiles)), so the common case -- a run of one tile --
    // needs one round of these loads, not three
    const int64_t uc = u < ntiles ? u : ntiles - 1;
    const int32_t r_here = open_row(uc);
    const int32_t r_prev = open_row(uc > 0 ? uc - 1 : 0);
    const int32_t r_next = open_row(uc + 1 < ntiles ? uc + 1 : uc);
    const int32_t r = u < ntiles ? r_here : static_cast<int32_t>(rows);
    const bool first = r < rows && (u == 0 || r_prev != r);
    int64_t end = u + 1;
    bool longrun = false;
    if (first && end < ntiles && r_next == r) {
        ++end;  // (kFixShort >= 2)
        while (end < ntiles && open_row(end) == r) {
            if (++end - u > kFixShort) {
                longrun = true;
                break;
            }
        }
    }
    if (first) {
        if (!longrun) {
            OT *orow = out + static_cast<int64_t>(r) * ldo;
            for (int64_t col = c; col < ncols; col += per) {
                Acc part = 0;
                for (int64_t v = u; v < end; ++v) part += carry[v * ncols + col];
                orow[col] = narrow<OT>(static_cast<Acc>(orow[col]) + part);
            }
        }
    }

    // long runs: the whole wave on each in turn (the mask is wave-uniform)
    uint64_t pending = __ballot(first && longrun && c == 0);
    while (pending) {
        const int src = __ffsll(static_cast<unsigned long long>(pending)) - 1;
        pending &= pending - 1;
        const int64_t us = __shfl(u, src);
        const int32_t rr = __shfl(r, src);
        int64_t e = us;
        for (int64_t v0 = us;; v0 += kWave) {
            const int64_t v = v0 + lane;
            const bool same = v < ntiles && open_row(v) == rr;
            const int cnt = __popcll(__ballot(same));
            if (cnt < kWave) {
                e = v0 + cnt;
                break;
            }
        }
        OT *orow = out + static_cast<int64_t>(rr) * ldo;
        if (ncols == 1) {
            Acc part = 0;
            int64_t v = us + lane;
            for (; v + 7 * kWave < e; v += 8 * kWave) {
                Acc t[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) t[k] = carry[v + k * kWave];
#pragma unroll
                for (int k = 0; k < 8; ++k) part += t[k];
            }
            for (; v < e; v += kWave) part += carry[v];
#pragma unroll
            for (int off = kWave / 2; off > 0; off >>= 1) part += __shfl_xor(part, off);
            if (lane == 0) orow[0] = narrow<OT>(static_cast<Acc>(orow[0]) + part);
            continue;
        }
        // vectors: two slices of 32 columns; each lane's tiles are loaded
        // kFixBatch at a time before they are added (in tile order)
        const int slice = lane / 32, cc = lane % 32;
        for (int64_t c0 = 0; c0 < ncols; c0 += 32) {
            const int64_t col = c0 + cc;
            Acc part = 0;
            if (col < ncols) {
                int64_t v = us + slice;
                for (; v + 2 * (kFixBatch - 1) < e; v += 2 * kFixBatch) {
                    Acc t[kFixBatch];
#pragma unroll
                    for (int k = 0; k < kFixBatch; ++k) t[k] = carry[(v + 2 * k) * ncols + col];
#pragma unroll
                    for (int k = 0; k < kFixBatch; ++k) part += t[k];
                }
                for (; v < e; v += 2) part += carry[v * ncols + col];
            }
            part += __shfl_xor(part, 32);
            if (slice == 0 && col < ncols) orow[col] = narrow<OT>(static_cast<Acc>(orow[col]) + part);
        }
    }
}

template <typename OT, typename Acc>
hipError_t launch_carry_fixup(int64_t rows, int64_t ncols, const int32_t *trow, int64_t npieces,
                              int64_t stride, int64_t ntiles, const Acc *carry, OT *out,
                              int64_t ldo, hipStream_t s) {
    if (ntiles == 0 || ncols == 0) return hipSuccess;
    const int64_t lanes = ntiles * (ncols == 1 ? 1 : kFixLanes);
    k_carry_fixup<OT, Acc><<<dim3(static_cast<unsigned>(ceil_div(lanes, kFixBlock))), kFixBlock,
                             0, s>>>(rows, ncols, trow, npieces, stride, ntiles, carry, out, ldo);
    return hipGetLastError();
}

}  // namespace spl
