// Leaves over CSF = (Dense, Compressed, Compressed) 3-tensors (paper
// Sec. VI-A): SpMTTKRP and the inner product.  (SpTTV is the SpMV leaf run on
// the fiber level; see abi.cpp.)
//
// Level partition of a CSF tensor for MTTKRP: pieces are contiguous runs of
// the merged sequence of slice ends (pos1) and fibers, described like the
// CSR pieces by (first slice the piece finishes, first fiber it covers).
//  - merge split: equal numbers of merged items (slices + fibers);
//  - non-zero split: blocks of T positions (the fused xyz -> f non-zero
//    partition, Sec. II-B) snapped back to the first fiber not finished at
//    the block boundary, slices derived by preimage through pos1.
//
// k_mttkrp_tiles: A(i,l) = sum_{f in slice i} C(j_f,l) * sum_{p in f} v_p D(k_p,l).
// As in the SpMM leaf, a lane group of W lanes owns W rank columns and walks
// ITEMS consecutive merged items of a chunk staged in LDS; here the items
// are fibers.  For its fibers the group first issues every C-row gather and
// (up to kPosCap positions) every D-row gather, keeping the scaled D rows in
// a per-group LDS slab so the fiber loop can index them; then it walks the
// fibers: t = sum over the fiber's positions, acc += C(j_f,:) * t, and a
// slice end writes acc (first finished slice and the open one go through
// the cross-group pass and the tile carry exactly as the SpMM rows do).
//
// k_mttkrp_vec: the same leaf with 4 (FP32) or 8 (BF16) rank columns per
// lane, one vector access per row, in 128-thread workgroups: the C rows of
// the group's fibers go to an LDS slab, the D rows of its positions are
// gathered a batch at a time into registers (details below).
#include "carry.hpp"
#include "device.hpp"
#include "internal.hpp"

namespace spl {
namespace {

// Rank columns per lane of k_mttkrp_vec (16-byte FP32, 8-byte BF16 rows).
constexpr int kMttkrpVec = 4;
// rank columns per lane of BF16 factors read 16 bytes at a time
constexpr int kMttkrpVecWide = 8;

__device__ __forceinline__ int64_t finished_at(const int32_t *pos, int64_t rows, int64_t p) {
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

// Fiber-aligned non-zero split bounds (tile t: slice, fiber).
__global__ __launch_bounds__(kBlock) void k_csf_nnz_bounds(int64_t I, const int32_t *pos1,
                                                           int64_t F, const int32_t *pos2,
                                                           int64_t nnz, int64_t T, int64_t ntiles,
                                                           int32_t *tslice, int32_t *tfib) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (t > ntiles) return;
    const int64_t p = (t == ntiles || t * T > nnz) ? nnz : t * T;
    const int64_t f = t == 0 ? 0 : finished_at(pos2, F, p);
    tfib[t] = static_cast<int32_t>(f);
    tslice[t] = static_cast<int32_t>(t == 0 ? 0 : finished_at(pos1, I, f));
}

template <int W, int ITEMS, typename V, typename FT, typename Acc>
__global__ __launch_bounds__(kBlock) void k_mttkrp_tiles(
    int64_t I, int64_t R, const int32_t *__restrict__ pos1, const int32_t *__restrict__ crd1,
    const int32_t *__restrict__ pos2, const int32_t *__restrict__ crd2,
    const V *__restrict__ vals, const FT *__restrict__ C, int64_t ldc,
    const FT *__restrict__ D, int64_t ldd, float *__restrict__ A, int64_t lda,
    const int32_t *__restrict__ tslice, const int32_t *__restrict__ tfib, int64_t npieces,
    int64_t stride, Acc *__restrict__ carry) {
    constexpr int G = kBlock / W;
    constexpr int kChunk = G * ITEMS;
    constexpr int kPosCap = 2 * ITEMS;  // positions per group kept in LDS
    __shared__ int32_t s_end[kChunk];         // slice ends (fiber index)
    __shared__ int32_t s_j[kChunk];           // crd1 of each fiber
    __shared__ int32_t s_fp[kChunk + 1];      // pos2 of each fiber (+ end)
    __shared__ Acc s_dv[G][kPosCap][W];       // v_p * D(k_p, :) per group
    __shared__ Acc s_head[G][W];
    __shared__ Acc s_tail[G][W];
    __shared__ int s_done[G];
    __shared__ int s_a0[G];
    __shared__ int64_t s_next[2];

    const int tid = threadIdx.x;
    const int g = tid / W, lane = tid % W;
    const int64_t col = static_cast<int64_t>(blockIdx.y) * W + lane;
    const bool colok = col < R;
    int64_t piece = static_cast<int64_t>(blockIdx.x) * stride;
    const int64_t piece_end = piece + stride < npieces ? piece + stride : npieces;
    int64_t ci = tslice[piece], cf = tfib[piece];
    Acc open = 0;

    while (piece < piece_end) {
        const int64_t next = chunk_end(pos1, tslice, tfib, piece, ci, cf, kChunk, s_next);
        const int64_t ei = s_next[0], ef = s_next[1];
        piece = next;
        const int nr = static_cast<int>(ei - ci), nf = static_cast<int>(ef - cf);
        for (int k = tid; k < nr; k += kBlock) s_end[k] = pos1[ci + 1 + k];
        for (int k = tid; k < nf; k += kBlock) s_j[k] = crd1[cf + k];
        for (int k = tid; k <= nf; k += kBlock) s_fp[k] = pos2[cf + k];
        __syncthreads();

        const int total = nr + nf;
        const int d0 = min(g * ITEMS, total);
        const int d1 = min(d0 + ITEMS, total);
        auto end_at = [&](int64_t m) { return s_end[m]; };
        const int a0 = static_cast<int>(merge_search(d0, nr, nf, cf, end_at));
        const int a1 = static_cast<int>(merge_search(d1, nr, nf, cf, end_at));
        const int b0 = d0 - a0, b1 = d1 - a1;

        // all C-row gathers of the group's fibers, then all D-row gathers of
        // its first kPosCap positions
        Acc cv[ITEMS];
#pragma unroll
        for (int k = 0; k < ITEMS; ++k)
            cv[k] = (b0 + k < b1 && colok)
                        ? widen<Acc>(C[static_cast<int64_t>(s_j[b0 + k]) * ldc + col])
                        : Acc(0);
        const int64_t P0 = s_fp[b0], P1 = s_fp[b1];
        const int np = static_cast<int>(P1 - P0);
        {
            // every index and value load, then every D-row gather, then the LDS
            // stores: kPosCap independent gathers in flight per lane
            int kq[kPosCap];
            Acc vq[kPosCap], dq[kPosCap];
#pragma unroll
            for (int q = 0; q < kPosCap; ++q) {
                kq[q] = 0;
                vq[q] = 0;
                if (q < np) {  // (default cache policy: the next loads share the lines)
                    kq[q] = crd2[P0 + q];
                    vq[q] = widen<Acc>(vals[P0 + q]);
                }
            }
#pragma unroll
            for (int q = 0; q < kPosCap; ++q)
                dq[q] = (q < np && colok) ? widen<Acc>(D[static_cast<int64_t>(kq[q]) * ldd + col])
                                          : Acc(0);
#pragma unroll
            for (int q = 0; q < kPosCap; ++q) s_dv[g][q][lane] = vq[q] * dq[q];
        }

        Acc acc = 0;
        int a = a0;
        bool first = true;
        auto finish = [&](int r) {
            if (first) {
                s_head[g][lane] = acc;
                first = false;
            } else if (colok) {
                store_stream(A + (ci + r) * lda + col, acc);
            }
            acc = 0;
        };
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            if (b0 + k < b1) {
                while (a < a1 && s_end[a] <= cf + b0 + k) finish(a++);
                Acc t = 0;
                const int q0 = static_cast<int>(s_fp[b0 + k] - P0);
                const int q1 = static_cast<int>(s_fp[b0 + k + 1] - P0);
                for (int q = q0; q < q1; ++q) {
                    if (q < kPosCap) {
                        t += s_dv[g][q][lane];
                    } else if (colok) {
                        const int64_t p = P0 + q;
                        t += widen<Acc>(vals[p]) *
                             widen<Acc>(D[static_cast<int64_t>(crd2[p]) * ldd + col]);
                    }
                }
                acc += cv[k] * t;
            }
        }
        while (a < a1) finish(a++);
        s_tail[g][lane] = acc;
        if (lane == 0) {
            s_done[g] = a1 - a0;
            s_a0[g] = a0;
        }
        __syncthreads();

        if (g == 0) {
            Acc c = open;
            for (int gg = 0; gg < G; ++gg) {
                if (s_done[gg] > 0) {
                    const Acc v = c + s_head[gg][lane];
                    if (colok) store_stream(A + (ci + s_a0[gg]) * lda + col, v);
                    c = s_tail[gg][lane];
                } else {
                    c += s_tail[gg][lane];
                }
            }
            open = c;
        }
        ci = ei;
        cf = ef;
        __syncthreads();
    }
    if (g == 0 && colok) carry[static_cast<int64_t>(blockIdx.x) * R + col] = open;
}

// k_mttkrp_vec: k_mttkrp_tiles with VEC rank columns per lane, so that one
// lane group of W = col_tile / VEC lanes reads a C or D row with W vector
// accesses.  The D rows of the group's positions are gathered kPosCap at a
// time into the same registers (every position load of a batch, then every
// gather, then the walk: a group with more positions than one batch pays
// two dependent rounds per batch, not per position -- 4.56 -> 3.85 ms FP32
// on the 1e8-nonzero tensor) and the C rows of its fibers go to a per-group LDS slab (each
// lane reads back only what it wrote, so no barrier): the group walks its
// positions in order, closing a fiber when the walk passes the fiber's end
// (acc += C(j_f, :) * t, the C row read from the slab) and finishing every
// slice that ends before the fiber it is about to close.  The next chunk's
// slice ends, fiber coordinates and fiber starts (one of each per thread)
// are loaded right after this chunk's gathers are issued, and the groups'
// heads and tails are combined by all threads at once (a column of a part
// each), so a chunk costs one barrier-separated round of gathers.  With
// BF16 factors the chunk's first 2 * NT positions (k and value) are staged
// in LDS with the chunk, so the D-row gathers wait on LDS rather than on a
// load from HBM (7.2 -> 6.4 ms on the 1e8-nonzero tensor); with FP32 the
// registers this needs cost more than it saves (4.08 against 3.69 ms), so
// FP32 keeps the direct loads.  ITEMS 4 halves the C-row slab and the
// per-group registers (116 VGPRs against 161): 4 waves per SIMD instead of
// 3, more gathers in flight (4.93 -> 4.56 ms FP32, 6.40 -> 5.32 ms BF16).
// Workgroups of NT = 128 threads (two waves): a barrier waits for one
// other wave instead of three, and the 16-byte BF16 leaf's LDS (41 KB per
// 256 threads) no longer caps it at 3 workgroups of 4 waves per CU
// (FP32 3.85 -> 3.69 ms, BF16 3.76 -> 3.25 ms; 64 threads: 3.78 and 3.33).
//
// int64 positions (PosT): pos1's entries are fiber indices (below 2^31) and
// are staged as they are; pos2's are staged relative to the chunk's first
// position (the low 32 bits of the difference), and the global loads add
// that base back.  With int32 positions the base is 0.
template <typename PosT>
__device__ __forceinline__ int32_t rel_pos(PosT p, int64_t base) {
    if constexpr (sizeof(PosT) == 4) return p;
    return static_cast<int32_t>(static_cast<uint32_t>(p) - static_cast<uint32_t>(base));
}

template <int W, int ITEMS, int VEC, typename V, typename FT, typename Acc,
          typename PosT = int32_t, bool STAGE = sizeof(FT) == 2, int NT = kMttkrpThreads,
          bool BUF = true>
__global__ __launch_bounds__(NT) void k_mttkrp_vec(
    int64_t I, int64_t R, const PosT *__restrict__ pos1, const int32_t *__restrict__ crd1,
    const PosT *__restrict__ pos2, const int32_t *__restrict__ crd2,
    const V *__restrict__ vals, const FT *__restrict__ C, int64_t ldc,
    const FT *__restrict__ D, int64_t ldd, float *__restrict__ A, int64_t lda,
    const int32_t *__restrict__ tslice, const int32_t *__restrict__ tfib, int64_t npieces,
    int64_t stride, Acc *__restrict__ carry) {
    constexpr int G = NT / W;
    constexpr int kChunk = G * ITEMS;
    static_assert(kChunk <= NT, "the chunk is staged one item per thread");
    // BF16 factors stage the chunk's leading positions in LDS (below); FP32
    // keeps more positions per group in registers instead.  Positions per
    // batch, measured on the 1e8-nonzero tensor: FP32 with buffer loads, 5
    // items: 9 (125 VGPRs; 7: 3.01 ms, 8: 2.97, 6: 3.04 against 2.97); with
    // the branching loads 4 items: 7 (122 VGPRs; 6: 3.69, 8: 3.75 against
    // 3.65), 5 items: 7 (128 VGPRs; 6: 3.40, 8: 3.38 against 3.30); BF16
    // 8-column lanes with 3 items: 5 (4: 2.50, 6: 2.84 against 2.48 with
    // buffer loads)
    constexpr bool kStage = STAGE;
    constexpr int kPosCap = kStage           ? (ITEMS == 3 ? 5 : ITEMS + ITEMS / 4)
                            : BUF && ITEMS == 5 ? 9
                            : (ITEMS == 4 || ITEMS == 5) ? 7
                                                         : ITEMS + ITEMS / 2;
    __shared__ int32_t s_end[kChunk];
    __shared__ int32_t s_j[kChunk];
    __shared__ int32_t s_fp[kChunk + 1];
    // C rows of each group's fibers, as loaded (BF16 stays packed)
    __shared__ RowVec<VEC, FT> s_c[G][ITEMS][W];
    __shared__ Acc s_head[G][W * VEC];
    __shared__ Acc s_tail[G][W * VEC];
    __shared__ int s_done[G];
    __shared__ int s_a0[G];
    __shared__ int64_t s_next[2];
    // cross-group combine: the tile's columns split over kParts parts of
    // G / kParts groups each
    constexpr int NC = W * VEC;
    constexpr int kParts = NT / NC;
    constexpr int kGroupsPerPart = G / kParts;
    static_assert(kParts * NC == NT && kGroupsPerPart * kParts == G, "combine layout");
    __shared__ Acc s_open[NC];  // the open row's partial entering the chunk
    // the chunk's first kStagePos positions (k and value), staged with the
    // chunk so that the D-row gathers wait on LDS, not on HBM
    constexpr int kStagePos = kStage ? 2 * NT : 0;
    __shared__ int32_t s_kq[kStage ? kStagePos : 1];
    __shared__ Acc s_vq[kStage ? kStagePos : 1];
    __shared__ Acc s_pb[kParts][NC];
    __shared__ int s_pa[kParts];

    const int tid = threadIdx.x;
    const int g = tid / W, lane = tid % W;
    // this lane's rank columns: col0 .. col0 + VEC - 1 (R is a multiple of VEC)
    const int64_t col0 = (static_cast<int64_t>(blockIdx.y) * W + lane) * VEC;
    const bool colok = col0 < R;
    int64_t piece = static_cast<int64_t>(blockIdx.x) * stride;
    const int64_t piece_end = piece + stride < npieces ? piece + stride : npieces;
    int64_t ci = tslice[piece], cf = tfib[piece];
    if (tid < NC) s_open[tid] = 0;
    // this thread's share of the next chunk's slice ends, fiber coordinates
    // and fiber starts, loaded behind the current chunk's gathers
    int32_t pre_e = 0, pre_j = 0, pre_f = 0, pre_f2 = 0;
    int32_t pre_k[2] = {0, 0};
    V pre_v[2] = {};
    int64_t pre_np = 0;
    int64_t pre_base = 0;  // the next chunk's first position (int64 positions)
    bool have = false;

    while (piece < piece_end) {
        // a piece that ends within this chunk needs no search, so no
        // barrier (every thread sees the same bounds; the loop's closing
        // barrier orders the reuse of the staging arrays)
        int64_t ei = tslice[piece + 1], ef = tfib[piece + 1], next = piece + 1;
        if (ei + ef - ci - cf > kChunk) {
            next = chunk_end(pos1, tslice, tfib, piece, ci, cf, kChunk, s_next);
            ei = s_next[0];
            ef = s_next[1];
        }
        piece = next;
        const int nr = static_cast<int>(ei - ci), nf = static_cast<int>(ef - cf);
        // the base the chunk's staged fiber starts count from (0 for int32)
        int64_t pbase = 0;
        if (have) {
            if constexpr (sizeof(PosT) == 8) pbase = pre_base;
            if (tid < nr) s_end[tid] = pre_e;
            if (tid < nf) s_j[tid] = pre_j;
            if (tid <= nf) s_fp[tid] = pre_f;
            if constexpr (kChunk >= NT)  // nf + 1 entries: one more than lanes
                if (tid == 0 && nf == NT) s_fp[NT] = pre_f2;
            if constexpr (kStage) {
#pragma unroll
                for (int jj = 0; jj < 2; ++jj) {
                    const int k = tid + jj * NT;
                    if (k < pre_np && k < kStagePos) {
                        s_kq[k] = pre_k[jj];
                        s_vq[k] = widen<Acc>(pre_v[jj]);
                    }
                }
            }
        } else {
            if constexpr (sizeof(PosT) == 8) pbase = pos2[cf];
            for (int k = tid; k < nr; k += NT) s_end[k] = static_cast<int32_t>(pos1[ci + 1 + k]);
            for (int k = tid; k < nf; k += NT) s_j[k] = crd1[cf + k];
            for (int k = tid; k <= nf; k += NT) s_fp[k] = rel_pos(pos2[cf + k], pbase);
            if constexpr (kStage) {
                const int64_t p0 = pos2[cf], npb = pos2[ef] - p0;
                for (int k = tid; k < npb && k < kStagePos; k += NT) {
                    s_kq[k] = crd2[p0 + k];
                    s_vq[k] = widen<Acc>(vals[p0 + k]);
                }
            }
        }
        __syncthreads();

        const int total = nr + nf;
        const int d0 = min(g * ITEMS, total);
        const int d1 = min(d0 + ITEMS, total);
        auto end_at = [&](int64_t m) { return s_end[m]; };
        const int a0 = static_cast<int>(merge_search(d0, nr, nf, cf, end_at));
        const int a1 = static_cast<int>(merge_search(d1, nr, nf, cf, end_at));
        const int b0 = d0 - a0, b1 = d1 - a1;
        const int64_t P0 = s_fp[b0];  // relative to pbase
        const int np = static_cast<int>(s_fp[b1] - P0);
        const int32_t *__restrict__ kcrd = crd2 + pbase;
        const V *__restrict__ kval = vals + pbase;

        // every C-row and D-row gather of the group before any is used
        // (BF16 rows stay packed until they are read)
        RowVec<VEC, FT> cv[ITEMS];
        int kq[kPosCap];
        Acc vq[kPosCap];
        RowVec<VEC, FT> dv[kPosCap];
        // the group's first position within the chunk (staged positions)
        const int64_t rel0 = kStage ? P0 - s_fp[0] : 0;
        // BUF: every load below is issued by every lane (buffer descriptors
        // over the chunk's positions, relative to its first one, and over
        // the factors; a lane with nothing to load reads 0 at kBufOut), so a
        // batch's gathers are all in flight at once.  The host takes this
        // form when the positions and both factors span at most kBufRange
        // bytes.
        const int32_t cp0 = BUF ? __builtin_amdgcn_readfirstlane(static_cast<int32_t>(s_fp[0])) : 0;
        const int32_t cpn =
            BUF ? __builtin_amdgcn_readfirstlane(static_cast<int32_t>(s_fp[nf])) - cp0 : 0;
        const auto rK = span_rsrc(kcrd + cp0, static_cast<uint32_t>(cpn) * 4u);
        const auto rV = span_rsrc(kval + cp0, static_cast<uint32_t>(cpn) * static_cast<uint32_t>(sizeof(V)));
        const auto rC = span_rsrc(C, kBufRange);
        const auto rD = span_rsrc(D, kBufRange);
        constexpr uint32_t kFs = sizeof(FT), kVs = sizeof(V);
        // positions q0 .. q0 + kPosCap - 1 of the group: coordinates, values
        // (a staged position from LDS, selected per position: separate
        // arrays for the LDS values cost a wave per SIMD)
        auto load_pos = [&](int q0) {
#pragma unroll
            for (int q = 0; q < kPosCap; ++q) {
                const int qq = q0 + q;
                const bool ok = qq < np;
                const bool staged = kStage && rel0 + qq < kStagePos;
                const uint32_t rel = static_cast<uint32_t>(P0 - cp0 + qq);
                int k = static_cast<int>(buf_u32<0>(rK, ok && !staged ? 4u * rel : kBufOut));
                Acc v = buf_val<0>(kval, rV, ok && !staged ? kVs * rel : kBufOut);
                if constexpr (kStage) {
                    const int si = static_cast<int>(rel0 + qq < kStagePos ? rel0 + qq : kStagePos - 1);
                    const int ksv = s_kq[si];
                    const Acc vsv = s_vq[si];
                    k = ok && staged ? ksv : k;
                    v = ok && staged ? vsv : v;
                }
                kq[q] = k;
                vq[q] = v;
            }
        };
        auto gather_d = [&](int q0) {
#pragma unroll
            for (int q = 0; q < kPosCap; ++q) {
                const bool ok = q0 + q < np && colok;
                dv[q].load_buf(rD, ok ? kFs * (static_cast<uint32_t>(kq[q]) *
                                                   static_cast<uint32_t>(ldd) +
                                               static_cast<uint32_t>(col0))
                                      : kBufOut);
            }
        };
        if constexpr (BUF) {
#pragma unroll
            for (int k = 0; k < ITEMS; ++k) {
                const bool ok = b0 + k < b1 && colok;
                const int jj = s_j[b0 + k < kChunk ? b0 + k : kChunk - 1];
                cv[k].load_buf(rC, ok ? kFs * (static_cast<uint32_t>(jj) *
                                                   static_cast<uint32_t>(ldc) +
                                               static_cast<uint32_t>(col0))
                                      : kBufOut);
            }
            load_pos(0);
            gather_d(0);
        } else {
#pragma unroll
            for (int k = 0; k < ITEMS; ++k) {
                cv[k].zero();
                if (b0 + k < b1 && colok)
                    cv[k].load(C + static_cast<int64_t>(s_j[b0 + k]) * ldc + col0);
            }
#pragma unroll
            for (int q = 0; q < kPosCap; ++q) {
                kq[q] = 0;
                vq[q] = 0;
                if (q < np) {
                    if (kStage && rel0 + q < kStagePos) {
                        kq[q] = s_kq[rel0 + q];
                        vq[q] = s_vq[rel0 + q];
                    } else {
                        kq[q] = kcrd[P0 + q];
                        vq[q] = widen<Acc>(kval[P0 + q]);
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < kPosCap; ++q) {
                dv[q].zero();
                if (q < np && colok) dv[q].load(D + static_cast<int64_t>(kq[q]) * ldd + col0);
            }
        }
        // the next chunk's staging, when it is a whole piece (no search):
        // issued after this chunk's gathers, it lands while they are used
        have = false;
        if (piece < piece_end) {
            const int64_t nei = tslice[piece + 1], nef = tfib[piece + 1];
            if (nei + nef - ei - ef <= kChunk) {
                const int nnr = static_cast<int>(nei - ei), nnf = static_cast<int>(nef - ef);
                if constexpr (sizeof(PosT) == 8) pre_base = pos2[ef];
                if (tid < nnr) pre_e = static_cast<int32_t>(pos1[ei + 1 + tid]);
                if (tid < nnf) pre_j = crd1[ef + tid];
                if (tid <= nnf) pre_f = rel_pos(pos2[ef + tid], pre_base);
                if constexpr (kChunk >= NT)
                    if (tid == 0 && nnf == NT) pre_f2 = rel_pos(pos2[ef + NT], pre_base);
                if constexpr (kStage) {
                    const int64_t pp0 = pos2[ef];
                    pre_np = pos2[nef] - pp0;
#pragma unroll
                    for (int jj = 0; jj < 2; ++jj) {
                        const int kk = tid + jj * NT;
                        if (kk < pre_np && kk < kStagePos) {
                            pre_k[jj] = load_stream(crd2 + pp0 + kk);
                            pre_v[jj] = load_stream(vals + pp0 + kk);
                        }
                    }
                }
                have = true;
            }
        }
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) s_c[g][k][lane] = cv[k];

        Acc acc[VEC], t[VEC];
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[v] = t[v] = 0;
        int a = a0, f = b0;
        bool first = true;
        auto finish = [&](int r) {
            if (first) {
#pragma unroll
                for (int v = 0; v < VEC; ++v) s_head[g][lane * VEC + v] = acc[v];
                first = false;
            } else if (colok) {
                store_row<VEC>(A + (ci + r) * lda + col0, acc);
            }
#pragma unroll
            for (int v = 0; v < VEC; ++v) acc[v] = 0;
        };
        auto close_fiber = [&]() {
            while (a < a1 && s_end[a] <= cf + f) finish(a++);
            const RowVec<VEC, FT> crow = s_c[g][f - b0][lane];
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                acc[v] += static_cast<Acc>(crow.at(v)) * t[v];
                t[v] = 0;
            }
            ++f;
        };
#pragma unroll
        for (int q = 0; q < kPosCap; ++q) {
            if (q < np) {
                while (P0 + q >= s_fp[f + 1]) close_fiber();
#pragma unroll
                for (int v = 0; v < VEC; ++v) t[v] += vq[q] * static_cast<Acc>(dv[q].at(v));
            }
        }
        // positions past the first batch, kPosCap at a time in the same
        // registers: every batch issues all its position loads, then all its
        // D-row gathers, then walks them
        for (int q0 = kPosCap; q0 < np; q0 += kPosCap) {
            if constexpr (BUF) {
                load_pos(q0);
                gather_d(q0);
            } else {
#pragma unroll
                for (int q = 0; q < kPosCap; ++q) {
                    kq[q] = 0;
                    vq[q] = 0;
                    if (q0 + q < np) {
                        const int64_t qq = q0 + q;
                        if (kStage && rel0 + qq < kStagePos) {
                            kq[q] = s_kq[rel0 + qq];
                            vq[q] = s_vq[rel0 + qq];
                        } else {
                            kq[q] = kcrd[P0 + qq];
                            vq[q] = widen<Acc>(kval[P0 + qq]);
                        }
                    }
                }
#pragma unroll
                for (int q = 0; q < kPosCap; ++q) {
                    dv[q].zero();
                    if (q0 + q < np && colok)
                        dv[q].load(D + static_cast<int64_t>(kq[q]) * ldd + col0);
                }
            }
#pragma unroll
            for (int q = 0; q < kPosCap; ++q) {
                if (q0 + q < np) {
                    while (P0 + q0 + q >= s_fp[f + 1]) close_fiber();
#pragma unroll
                    for (int v = 0; v < VEC; ++v) t[v] += vq[q] * static_cast<Acc>(dv[q].at(v));
                }
            }
        }
        while (f < b1) close_fiber();
        while (a < a1) finish(a++);
#pragma unroll
        for (int v = 0; v < VEC; ++v) s_tail[g][lane * VEC + v] = acc[v];
        if (lane == 0) {
            s_done[g] = a1 - a0;
            s_a0[g] = a0;
        }
        __syncthreads();

        // Combine across groups, in group order: a group that finished a
        // slice writes it as (partial entering the group) + its head and
        // restarts the partial from its tail; any other group adds its tail.
        // Each thread takes one column of one part: it composes its part's
        // groups, then starts from the partials of the parts before it.
        {
            const int col = tid % NC, part = tid / NC;
            const int64_t gcol = static_cast<int64_t>(blockIdx.y) * NC + col;
            int pa = 1;
            Acc pb = 0;
            for (int k = 0; k < kGroupsPerPart; ++k) {
                const int gg = part * kGroupsPerPart + k;
                const Acc t = s_tail[gg][col];
                pb = s_done[gg] > 0 ? t : pb + t;
                pa = s_done[gg] > 0 ? 0 : pa;
            }
            s_pb[part][col] = pb;
            if (col == 0) s_pa[part] = pa;
            Acc o = s_open[col];
            __syncthreads();
            for (int q = 0; q < part; ++q) o = s_pa[q] ? o + s_pb[q][col] : s_pb[q][col];
            for (int k = 0; k < kGroupsPerPart; ++k) {
                const int gg = part * kGroupsPerPart + k;
                if (s_done[gg] > 0) {
                    if (gcol < R) A[(ci + s_a0[gg]) * lda + gcol] = o + s_head[gg][col];
                    o = s_tail[gg][col];
                } else {
                    o += s_tail[gg][col];
                }
            }
            if (part == kParts - 1) s_open[col] = o;
        }
        ci = ei;
        cf = ef;
        __syncthreads();
    }
    if (tid < NC) {
        const int64_t gcol = static_cast<int64_t>(blockIdx.y) * NC + tid;
        if (gcol < R) carry[static_cast<int64_t>(blockIdx.x) * R + gcol] = s_open[tid];
    }
}

// Inner product of two value arrays on one pattern: per-workgroup FP64
// partial sums over a fixed grid-stride assignment, then one workgroup adds
// the partials in a fixed tree.  Bitwise reproducible for a fixed grid.
template <typename V>
__global__ __launch_bounds__(kBlock) void k_inner_partial(int64_t nnz, const V *__restrict__ a,
                                                          const V *__restrict__ b,
                                                          double *__restrict__ part) {
    double acc = 0.0, acc2 = 0.0;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    for (; i + stride < nnz; i += 2 * stride) {
        acc += to_f64(load_stream(a + i)) * to_f64(load_stream(b + i));
        acc2 += to_f64(load_stream(a + i + stride)) * to_f64(load_stream(b + i + stride));
    }
    if (i < nnz) acc += to_f64(load_stream(a + i)) * to_f64(load_stream(b + i));
    acc += acc2;
    __shared__ double s[kBlock];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(kBlock) void k_inner_final(int64_t nparts,
                                                        const double *__restrict__ part,
                                                        double *__restrict__ out) {
    // four independent chains per thread (their loads overlap), combined in
    // a fixed order
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int64_t i = threadIdx.x;
    for (; i + 3 * kBlock < nparts; i += 4 * kBlock) {
        a0 += part[i];
        a1 += part[i + kBlock];
        a2 += part[i + 2 * kBlock];
        a3 += part[i + 3 * kBlock];
    }
    for (; i < nparts; i += kBlock) a0 += part[i];
    const double acc = (a0 + a1) + (a2 + a3);
    __shared__ double s[kBlock];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s[0];
}

template <typename V, typename FT, typename PosT, bool BUF>
hipError_t mttkrp_types_b(bool stage, int col_tile, int items, int vec, int64_t I, int64_t R,
                        const PosT *pos1, const int32_t *crd1, const PosT *pos2,
                        const int32_t *crd2, const void *vals, const void *C, int64_t ldc,
                        const void *D, int64_t ldd, float *A, int64_t lda, const Tiles &t,
                        int64_t stride, float *carry, hipStream_t s) {
    const int lanes = col_tile / vec;
    dim3 grid(static_cast<unsigned>(ceil_div(t.ntiles, stride)),
              static_cast<unsigned>(ceil_div(R, col_tile)));
    // every launch names its thread count, which must be the kernel's NT
    // (k_mttkrp_vec) or kBlock (k_mttkrp_tiles)
    auto launch = [&](auto kern, int threads) {
        kern<<<grid, threads, 0, s>>>(I, R, pos1, crd1, pos2, crd2, static_cast<const V *>(vals),
                                     static_cast<const FT *>(C), ldc, static_cast<const FT *>(D),
                                     ldd, A, lda, t.row, t.pos, t.ntiles, stride, carry);
        return hipGetLastError();
    };
    auto go = [&](auto kern) { return launch(kern, kMttkrpThreads); };
    auto go_tiles = [&](auto kern) { return launch(kern, kBlock); };
    if constexpr (sizeof(FT) == 4) {
        // FP32 with the chunk's leading positions staged in LDS as for BF16
        if (stage && vec == kMttkrpVec && items == 4) {
            if (lanes == 8) return go(k_mttkrp_vec<8, 4, kMttkrpVec, V, FT, float, PosT, true, kMttkrpThreads, BUF>);
            if (lanes == 16) return go(k_mttkrp_vec<16, 4, kMttkrpVec, V, FT, float, PosT, true, kMttkrpThreads, BUF>);
            return hipErrorInvalidValue;
        }
    }
    if (vec == kMttkrpVec) {
        if (items == 5)  // col_tile 32 only
            return lanes == 8 ? go(k_mttkrp_vec<8, 5, kMttkrpVec, V, FT, float, PosT, sizeof(FT) == 2, kMttkrpThreads, BUF>)
                              : hipErrorInvalidValue;
        if (items != 8 && items != 4) return hipErrorInvalidValue;
        if (items == 4) {
            if (lanes == 8) return go(k_mttkrp_vec<8, 4, kMttkrpVec, V, FT, float, PosT, sizeof(FT) == 2, kMttkrpThreads, BUF>);
            if (lanes == 16) return go(k_mttkrp_vec<16, 4, kMttkrpVec, V, FT, float, PosT, sizeof(FT) == 2, kMttkrpThreads, BUF>);
            return hipErrorInvalidValue;
        }
        if (lanes == 8) return go(k_mttkrp_vec<8, 8, kMttkrpVec, V, FT, float, PosT, sizeof(FT) == 2, kMttkrpThreads, BUF>);
        if (lanes == 16) return go(k_mttkrp_vec<16, 8, kMttkrpVec, V, FT, float, PosT, sizeof(FT) == 2, kMttkrpThreads, BUF>);
        return hipErrorInvalidValue;
    }
    if constexpr (sizeof(FT) == 2) {
        // 16-byte BF16 lanes: chunks of at most 256 merged items (lanes x
        // items >= 32), as the one-item-per-thread staging needs
        if (vec == kMttkrpVecWide) {
            if (lanes == 4 && items == 3)
                return go(k_mttkrp_vec<4, 3, kMttkrpVecWide, V, FT, float, PosT, sizeof(FT) == 2, kMttkrpThreads, BUF>);
            if (lanes == 4 && items == 4)
                return go(k_mttkrp_vec<4, 4, kMttkrpVecWide, V, FT, float, PosT, sizeof(FT) == 2, kMttkrpThreads, BUF>);
            if (lanes == 8 && items == 4)
                return go(k_mttkrp_vec<8, 4, kMttkrpVecWide, V, FT, float, PosT, sizeof(FT) == 2, kMttkrpThreads, BUF>);
            if (lanes == 8 && items == 8)
                return go(k_mttkrp_vec<8, 8, kMttkrpVecWide, V, FT, float, PosT, sizeof(FT) == 2, kMttkrpThreads, BUF>);
            return hipErrorInvalidValue;
        }
    }
    if constexpr (sizeof(PosT) == 8) {
        return hipErrorInvalidValue;  // int64 positions: vector lanes only
    } else {
    if (vec > 1) return hipErrorInvalidValue;
    if (col_tile == 16) return items <= 8 ? go_tiles(k_mttkrp_tiles<16, 8, V, FT, float>)
                                          : go_tiles(k_mttkrp_tiles<16, 16, V, FT, float>);
    if (col_tile == 64) return items <= 8 ? go_tiles(k_mttkrp_tiles<64, 8, V, FT, float>)
                                          : go_tiles(k_mttkrp_tiles<64, 16, V, FT, float>);
    return items <= 8 ? go_tiles(k_mttkrp_tiles<32, 8, V, FT, float>)
                      : go_tiles(k_mttkrp_tiles<32, 16, V, FT, float>);
    }
}


// BUF (buffer loads, no per-lane branches) when every position and factor
// span fits kBufRange bytes; the branching loads otherwise
template <typename V, typename FT, typename PosT = int32_t>
hipError_t mttkrp_types(bool buf, bool stage, int col_tile, int items, int vec, int64_t I,
                        int64_t R, const PosT *pos1, const int32_t *crd1, const PosT *pos2,
                        const int32_t *crd2, const void *vals, const void *C, int64_t ldc,
                        const void *D, int64_t ldd, float *A, int64_t lda, const Tiles &t,
                        int64_t stride, float *carry, hipStream_t s) {
    if (buf)
        return mttkrp_types_b<V, FT, PosT, true>(stage, col_tile, items, vec, I, R, pos1, crd1,
                                                 pos2, crd2, vals, C, ldc, D, ldd, A, lda, t,
                                                 stride, carry, s);
    return mttkrp_types_b<V, FT, PosT, false>(stage, col_tile, items, vec, I, R, pos1, crd1, pos2,
                                              crd2, vals, C, ldc, D, ldd, A, lda, t, stride, carry,
                                              s);
}

}  // namespace

bool mttkrp_buf(int64_t nnz, size_t val_bytes, int64_t J, int64_t ldc, int64_t K, int64_t ldd,
                size_t factor_bytes) {
    auto fits = [](int64_t count, size_t elem) {
        return count >= 0 && static_cast<double>(count) * static_cast<double>(elem) <= kBufRange;
    };
    return fits(nnz, 4) && fits(nnz, val_bytes) && fits(J * ldc, factor_bytes) &&
           fits(K * ldd, factor_bytes);
}

hipError_t launch_csf_nnz_bounds(int64_t I, const int32_t *pos1, int64_t F, const int32_t *pos2,
                                 int64_t nnz, int64_t T, const Tiles &t, hipStream_t s) {
    dim3 grid(static_cast<unsigned>((t.ntiles + 1 + kBlock - 1) / kBlock));
    k_csf_nnz_bounds<<<grid, kBlock, 0, s>>>(I, pos1, F, pos2, nnz, T, t.ntiles, t.row, t.pos);
    return hipGetLastError();
}

hipError_t launch_mttkrp_tiles(int vtype, bool buf, bool stage, int col_tile, int items, int vec, int64_t I,
                               int64_t R, const int32_t *pos1, const int32_t *crd1,
                               const int32_t *pos2, const int32_t *crd2, const void *vals,
                               const void *C, int64_t ldc, const void *D, int64_t ldd, float *A,
                               int64_t lda, const Tiles &t, int64_t stride, float *carry,
                               hipStream_t s) {
    if (vtype == SPL_F32)
        return mttkrp_types<float, float>(buf, stage, col_tile, items, vec, I, R, pos1, crd1, pos2,
                                          crd2, vals, C, ldc, D, ldd, A, lda, t, stride, carry, s);
    return mttkrp_types<bf16, bf16>(buf, stage, col_tile, items, vec, I, R, pos1, crd1, pos2, crd2,
                                    vals, C, ldc, D, ldd, A, lda, t, stride, carry, s);
}

hipError_t launch_mttkrp_tiles64(int vtype, bool buf, int col_tile, int items, int vec, int64_t I,
                                 int64_t R, const int64_t *pos1, const int32_t *crd1,
                                 const int64_t *pos2, const int32_t *crd2, const void *vals,
                                 const void *C, int64_t ldc, const void *D, int64_t ldd, float *A,
                                 int64_t lda, const Tiles &t, int64_t stride, float *carry,
                                 hipStream_t s) {
    if (vtype == SPL_F32)
        return mttkrp_types<float, float, int64_t>(buf, false, col_tile, items, vec, I, R, pos1, crd1, pos2,
                                                   crd2, vals, C, ldc, D, ldd, A, lda, t, stride,
                                                   carry, s);
    return mttkrp_types<bf16, bf16, int64_t>(buf, false, col_tile, items, vec, I, R, pos1, crd1, pos2, crd2,
                                             vals, C, ldc, D, ldd, A, lda, t, stride, carry, s);
}

hipError_t launch_mttkrp_fixup(int64_t I, int64_t R, const Tiles &t, int64_t stride,
                               const float *carry, float *A, int64_t lda, hipStream_t s) {
    return launch_carry_fixup<float, float>(I, R, t.row, t.ntiles, stride,
                                            ceil_div(t.ntiles, stride), carry, A, lda, s);
}

hipError_t launch_inner_final(int64_t nparts, const double *part, double *out, hipStream_t s) {
    k_inner_final<<<1, kBlock, 0, s>>>(nparts, part, out);
    return hipGetLastError();
}

hipError_t launch_inner(int vtype, int64_t nnz, const void *a, const void *b, double *part,
                        int64_t nparts, double *out, hipStream_t s) {
    dim3 grid(static_cast<unsigned>(nparts));
    if (vtype == SPL_F64)
        k_inner_partial<double><<<grid, kBlock, 0, s>>>(nnz, static_cast<const double *>(a),
                                                         static_cast<const double *>(b), part);
    else
        k_inner_partial<float><<<grid, kBlock, 0, s>>>(nnz, static_cast<const float *>(a),
                                                        static_cast<const float *>(b), part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_inner_final<<<1, kBlock, 0, s>>>(nparts, part, out);
    return hipGetLastError();
}

}  // namespace spl
