// SDDMM leaf  A(i,j) = B(i,j) * C(i,k) * D(j,k)  (paper Sec. VI-A; D stored
// with one row per column coordinate j).  The output keeps B's pattern, so
// only A's values are produced (Sec. V-B): no output reduction, no carries.
//
// Work split: the merge split of B's rows and positions (pieces of one
// chunk each, from partition.hip), one chunk per workgroup iteration.  The
// chunk's row ends are staged in LDS and each position's row is found by a
// binary search there, so a row's positions may straddle chunks freely.
//
//  * k_sddmm_valu: a half-wave (32 lanes) per position; lane l accumulates
//    C(i,k) D(j,k) for k = l, l+32, ... (every row access is coalesced), then
//    a 32-lane butterfly.  FP64, FP32, or BF16 factors with FP32
//    accumulation.
//  * k_sddmm_vec: the same with vector lanes (16-byte factor accesses) and
//    8, 16 or 32 lanes per position, two positions per lane group in
//    flight.
//  * k_sddmm_mfma: BF16 factors on the matrix cores.  A wave takes 16
//    positions; v_mfma_f32_16x16x32_bf16 multiplies the 16 gathered C rows
//    (as A, 16 x 32 per step) by the 16 gathered D rows (as B, 32 x 16) and
//    the diagonal of the 16 x 16 FP32 result holds the 16 dot products.
//    Only 1/16 of the MFMA work is kept, but the operation is bound by the
//    D-row gathers, not by arithmetic.
#include "device.hpp"
#include "internal.hpp"

namespace spl {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Row of every position of the chunk: s_row[k] = ci + #(row ends <= cp + k).
__device__ __forceinline__ void chunk_rows(const int32_t *__restrict__ pos, int64_t ci,
                                           int64_t cp, int nr, int np, int32_t *s_end,
                                           int32_t *s_row) {
    for (int k = threadIdx.x; k < nr; k += kBlock) s_end[k] = pos[ci + 1 + k];
    __syncthreads();
    for (int k = threadIdx.x; k < np; k += kBlock) {
        const int64_t p = cp + k;
        int lo = 0, hi = nr;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (s_end[mid] <= p)
                lo = mid + 1;
            else
                hi = mid;
        }
        s_row[k] = static_cast<int32_t>(ci + lo);
    }
    __syncthreads();
}

template <typename V, typename FT, typename Acc, int CHUNK>
__global__ __launch_bounds__(kBlock) void k_sddmm_valu(
    int64_t K, const int32_t *__restrict__ pos, const int32_t *__restrict__ crd,
    const V *__restrict__ bv, const FT *__restrict__ C, int64_t ldc, const FT *__restrict__ D,
    int64_t ldd, V *__restrict__ out, const int32_t *__restrict__ trow,
    const int32_t *__restrict__ tpos, int64_t npieces, int64_t stride) {
    __shared__ int32_t s_end[CHUNK];
    __shared__ int32_t s_row[CHUNK];
    __shared__ int64_t s_next[2];
    constexpr int kHalves = kBlock / 32;
    const int h = threadIdx.x / 32, lane = threadIdx.x % 32;
    int64_t piece = static_cast<int64_t>(blockIdx.x) * stride;
    const int64_t piece_end = piece + stride < npieces ? piece + stride : npieces;
    int64_t ci = trow[piece], cp = tpos[piece];
    while (piece < piece_end) {
        piece = chunk_end(pos, trow, tpos, piece, ci, cp, CHUNK, s_next);
        const int64_t ei = s_next[0], ep = s_next[1];
        const int nr = static_cast<int>(ei - ci), np = static_cast<int>(ep - cp);
        chunk_rows(pos, ci, cp, nr, np, s_end, s_row);
        // two positions in flight per half-wave
        for (int k = h; k < np; k += 2 * kHalves) {
            const int k2 = k + kHalves;
            const bool has2 = k2 < np;
            const int64_t p = cp + k, p2 = cp + k2;
            const FT *crow = C + static_cast<int64_t>(s_row[k]) * ldc;
            const FT *drow = D + static_cast<int64_t>(crd[p]) * ldd;
            const FT *crow2 = C + static_cast<int64_t>(s_row[has2 ? k2 : k]) * ldc;
            const FT *drow2 = D + static_cast<int64_t>(crd[has2 ? p2 : p]) * ldd;
            Acc a1 = 0, a2 = 0;
            for (int64_t kk = lane; kk < K; kk += 32) {
                a1 += widen<Acc>(crow[kk]) * widen<Acc>(drow[kk]);
                a2 += widen<Acc>(crow2[kk]) * widen<Acc>(drow2[kk]);
            }
            a1 = group_sum<32>(a1);
            a2 = group_sum<32>(a2);
            if (lane == 0) {
                store_stream(out + p, static_cast<V>(widen<Acc>(load_stream(bv + p)) * a1));
                if (has2) store_stream(out + p2, static_cast<V>(widen<Acc>(load_stream(bv + p2)) * a2));
            }
        }
        ci = ei;
        cp = ep;
        __syncthreads();
    }
}

// k_sddmm_valu with vector lanes: a group of L lanes per position, each lane
// reading VEC consecutive k of the C and D rows with one vector access
// (K, ldc, ldd multiples of VEC, factors aligned), P positions per group in
// flight; then an L-lane butterfly.
template <typename V, typename FT, typename Acc, int CHUNK, int L, int VEC, int P>
__global__ __launch_bounds__(kBlock) void k_sddmm_vec(
    int64_t K, const int32_t *__restrict__ pos, const int32_t *__restrict__ crd,
    const V *__restrict__ bv, const FT *__restrict__ C, int64_t ldc, const FT *__restrict__ D,
    int64_t ldd, V *__restrict__ out, const int32_t *__restrict__ trow,
    const int32_t *__restrict__ tpos, int64_t npieces, int64_t stride) {
    __shared__ int32_t s_end[CHUNK];
    __shared__ int32_t s_row[CHUNK];
    __shared__ int64_t s_next[2];
    constexpr int kGroups = kBlock / L;
    const int grp = threadIdx.x / L, lane = threadIdx.x % L;
    int64_t piece = static_cast<int64_t>(blockIdx.x) * stride;
    const int64_t piece_end = piece + stride < npieces ? piece + stride : npieces;
    int64_t ci = trow[piece], cp = tpos[piece];
    while (piece < piece_end) {
        piece = chunk_end(pos, trow, tpos, piece, ci, cp, CHUNK, s_next);
        const int64_t ei = s_next[0], ep = s_next[1];
        const int nr = static_cast<int>(ei - ci), np = static_cast<int>(ep - cp);
        chunk_rows(pos, ci, cp, nr, np, s_end, s_row);
        for (int k = grp; k < np; k += P * kGroups) {
            const FT *crow[P];
            const FT *drow[P];
            bool live[P];
#pragma unroll
            for (int u = 0; u < P; ++u) {
                const int ku = k + u * kGroups;
                live[u] = ku < np;
                const int kk = live[u] ? ku : k;  // dead slots reread a live position
                crow[u] = C + static_cast<int64_t>(s_row[kk]) * ldc;
                // (the default cache policy: the next iteration's positions
                // share these lines)
                drow[u] = D + static_cast<int64_t>(crd[cp + kk]) * ldd;
            }
            Acc a[P];
#pragma unroll
            for (int u = 0; u < P; ++u) a[u] = 0;
            for (int64_t k0 = static_cast<int64_t>(lane) * VEC; k0 < K; k0 += L * VEC) {
                Acc cr[P][VEC], dr[P][VEC];
#pragma unroll
                for (int u = 0; u < P; ++u) {
                    load_row<VEC>(crow[u] + k0, cr[u]);
                    load_row<VEC>(drow[u] + k0, dr[u]);
                }
#pragma unroll
                for (int u = 0; u < P; ++u) {
#pragma unroll
                    for (int v = 0; v < VEC; ++v) a[u] += cr[u][v] * dr[u][v];
                }
            }
#pragma unroll
            for (int u = 0; u < P; ++u) a[u] = group_sum<L>(a[u]);
            if (lane == 0) {
#pragma unroll
                for (int u = 0; u < P; ++u) {
                    if (live[u]) {
                        const int64_t p = cp + k + u * kGroups;
                        store_stream(out + p, static_cast<V>(widen<Acc>(load_stream(bv + p)) * a[u]));
                    }
                }
            }
        }
        ci = ei;
        cp = ep;
        __syncthreads();
    }
}

// BF16 factors, FP32 values and output, K a multiple of 32.
template <int CHUNK>
__global__ __launch_bounds__(kBlock) void k_sddmm_mfma(
    int64_t K, const int32_t *__restrict__ pos, const int32_t *__restrict__ crd,
    const float *__restrict__ bv, const bf16 *__restrict__ C, int64_t ldc,
    const bf16 *__restrict__ D, int64_t ldd, float *__restrict__ out,
    const int32_t *__restrict__ trow, const int32_t *__restrict__ tpos, int64_t npieces,
    int64_t stride) {
    __shared__ int32_t s_end[CHUNK];
    __shared__ int32_t s_row[CHUNK];
    __shared__ int64_t s_next[2];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int r = lane % 16, kg = lane / 16;  // operand row/column and k-group of this lane
    int64_t piece = static_cast<int64_t>(blockIdx.x) * stride;
    const int64_t piece_end = piece + stride < npieces ? piece + stride : npieces;
    int64_t ci = trow[piece], cp = tpos[piece];
    while (piece < piece_end) {
        piece = chunk_end(pos, trow, tpos, piece, ci, cp, CHUNK, s_next);
        const int64_t ei = s_next[0], ep = s_next[1];
        const int nr = static_cast<int>(ei - ci), np = static_cast<int>(ep - cp);
        chunk_rows(pos, ci, cp, nr, np, s_end, s_row);
        for (int base = wave * 16; base < np; base += 16 * (kBlock / kWave)) {
            const int k = base + r;
            const bool live = k < np;
            const int kk = live ? k : base;  // dead lanes read a live position
            const int64_t p = cp + kk;
            const bf16 *crow = C + static_cast<int64_t>(s_row[kk]) * ldc + kg * 8;
            const bf16 *drow = D + static_cast<int64_t>(crd[p]) * ldd + kg * 8;
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            for (int64_t k0 = 0; k0 < K; k0 += 32) {
                const u32x4 ca = *reinterpret_cast<const u32x4 *>(crow + k0);
                const u32x4 db = *reinterpret_cast<const u32x4 *>(drow + k0);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, ca),
                                                              __builtin_bit_cast(bf16x8, db), acc,
                                                              0, 0, 0);
            }
            // result (row 4*kg + e, column r) sits in acc[e] of this lane; the
            // diagonal element of position r is in the lane with kg == r / 4
            if (live && kg == r / 4) {
                const int e = r % 4;
                const float d = e == 0 ? acc[0] : e == 1 ? acc[1] : e == 2 ? acc[2] : acc[3];
                store_stream(out + cp + k, load_stream(bv + cp + k) * d);
            }
        }
        ci = ei;
        cp = ep;
        __syncthreads();
    }
}

constexpr int kSddmmChunk = 512;

}  // namespace

int64_t sddmm_chunk() { return kSddmmChunk; }

int sddmm_vec_width(int ftype) { return ftype == SPL_F64 ? 2 : ftype == SPL_F32 ? 4 : 8; }

namespace {
template <typename V, typename FT, int VEC>
hipError_t sddmm_vec(int lanes, dim3 grid, int64_t K, const int32_t *pos, const int32_t *crd,
                     const void *bv, const void *C, int64_t ldc, const void *D, int64_t ldd,
                     void *out, const Tiles &t, int64_t stride, hipStream_t s) {
    auto go = [&](auto kern) {
        kern<<<grid, kBlock, 0, s>>>(K, pos, crd, static_cast<const V *>(bv),
                                     static_cast<const FT *>(C), ldc, static_cast<const FT *>(D),
                                     ldd, static_cast<V *>(out), t.row, t.pos, t.ntiles, stride);
        return hipGetLastError();
    };
    using Acc = V;  // FP64 or FP32 accumulation, as the values
    // positions per lane group in flight: 2 (fewer registers, more waves per
    // SIMD) measured best at K = 128 on 8e6 positions: FP32 0.874 ms, BF16
    // 0.433 ms, against 0.928 / 0.529 with 4, 1.08 / 0.51 with 1 and 1.28
    // (FP32) with 8
    constexpr int kP = 2;
    if (lanes == 32) return go(k_sddmm_vec<V, FT, Acc, kSddmmChunk, 32, VEC, kP>);
    if (lanes == 16) return go(k_sddmm_vec<V, FT, Acc, kSddmmChunk, 16, VEC, kP>);
    if (lanes == 8) return go(k_sddmm_vec<V, FT, Acc, kSddmmChunk, 8, VEC, kP>);
    return hipErrorInvalidValue;
}
}  // namespace

hipError_t launch_sddmm(int vtype, int ftype, int variant, int vec_lanes, int64_t K,
                        const int32_t *pos, const int32_t *crd, const void *bv, const void *C,
                        int64_t ldc, const void *D, int64_t ldd, void *out, const Tiles &t,
                        int64_t stride, hipStream_t s) {
    dim3 grid(static_cast<unsigned>(ceil_div(t.ntiles, stride)));
    if (variant == 0 && vec_lanes > 0) {
        if (ftype == SPL_BF16)
            return sddmm_vec<float, bf16, 8>(vec_lanes, grid, K, pos, crd, bv, C, ldc, D, ldd,
                                             out, t, stride, s);
        if (vtype == SPL_F64)
            return sddmm_vec<double, double, 2>(vec_lanes, grid, K, pos, crd, bv, C, ldc, D, ldd,
                                                out, t, stride, s);
        return sddmm_vec<float, float, 4>(vec_lanes, grid, K, pos, crd, bv, C, ldc, D, ldd, out,
                                          t, stride, s);
    }
    if (ftype == SPL_BF16 && variant == 1) {
        k_sddmm_mfma<kSddmmChunk><<<grid, kBlock, 0, s>>>(
            K, pos, crd, static_cast<const float *>(bv), static_cast<const bf16 *>(C), ldc,
            static_cast<const bf16 *>(D), ldd, static_cast<float *>(out), t.row, t.pos, t.ntiles,
            stride);
    } else if (ftype == SPL_BF16) {
        k_sddmm_valu<float, bf16, float, kSddmmChunk><<<grid, kBlock, 0, s>>>(
            K, pos, crd, static_cast<const float *>(bv), static_cast<const bf16 *>(C), ldc,
            static_cast<const bf16 *>(D), ldd, static_cast<float *>(out), t.row, t.pos, t.ntiles,
            stride);
    } else if (vtype == SPL_F64) {
        k_sddmm_valu<double, double, double, kSddmmChunk><<<grid, kBlock, 0, s>>>(
            K, pos, crd, static_cast<const double *>(bv), static_cast<const double *>(C), ldc,
            static_cast<const double *>(D), ldd, static_cast<double *>(out), t.row, t.pos,
            t.ntiles, stride);
    } else {
        k_sddmm_valu<float, float, float, kSddmmChunk><<<grid, kBlock, 0, s>>>(
            K, pos, crd, static_cast<const float *>(bv), static_cast<const float *>(C), ldc,
            static_cast<const float *>(D), ldd, static_cast<float *>(out), t.row, t.pos, t.ntiles,
            stride);
    }
    return hipGetLastError();
}

}  // namespace spl
