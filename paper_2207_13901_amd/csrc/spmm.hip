// SpMM leaf  A(i,j) = B(i,k) * C(k,j)  for CSR B and row-major dense C
// (paper Sec. VI-A).  The dense operand is named `Bd` here and the output
// `Out` to keep the sparse operand's name B.
//
// A lane group of W lanes (W = col_tile) owns W consecutive dense columns:
// lane l accumulates column blockIdx.y*W + l, so every gathered row of Bd is
// one coalesced W-element read (128 bytes for W = 32 FP32 columns).
//
//  * k_spmm_row: row split; group g of the workgroup owns one row.  The
//    row's crd/vals are read W at a time by the group's lanes (coalesced) and
//    broadcast with shuffles, then one Bd row is gathered per position.
//
//  * k_spmm_tiles: non-zero or merge split (the load-balanced GPU SpMM
//    schedule of Sec. VI-A, GPU results).  A workgroup owns `stride`
//    consecutive pieces of the level partition (merge split: pieces of
//    exactly one chunk; non-zero split: pieces of T positions cut into chunks
//    by a merge-path search) and processes them in chunks of G*ITEMS merged
//    items (G = 256/W groups).  The chunk's row ends, crd and vals are
//    staged in LDS; each group walks ITEMS consecutive merged items, first
//    issuing all of its Bd gathers (up to ITEMS rows in flight per group) and
//    then consuming them in order.  Rows a group finishes after its first
//    are written directly; the first finished row and the row left open are
//    combined across groups in order by group 0 (G steps), and the row open
//    at the tile end is written to the tile's carry vector.  k_carry_fixup
//    (carry.hpp) adds carries into their rows in a fixed order.  Deterministic, no atomics.
//
//  * k_spmm_pipe: the merge-split form of k_spmm_tiles, with the staging
//    loads of the next chunk software-pipelined behind the current walk.
#include "carry.hpp"
#include "device.hpp"
#include "internal.hpp"

namespace spl {
namespace {

template <int W, typename V, typename BT, typename OT, typename Acc>
__global__ __launch_bounds__(kBlock) void k_spmm_row(int64_t n, int64_t N,
                                                     const int32_t *__restrict__ pos,
                                                     const int32_t *__restrict__ crd,
                                                     const V *__restrict__ vals,
                                                     const BT *__restrict__ Bd, int64_t ldb,
                                                     OT *__restrict__ Out, int64_t ldo) {
    constexpr int G = kBlock / W;
    const int g = threadIdx.x / W, lane = threadIdx.x % W;
    const int64_t row = static_cast<int64_t>(blockIdx.x) * G + g;
    const int64_t col = static_cast<int64_t>(blockIdx.y) * W + lane;
    const bool colok = col < N;
    Acc acc = 0;
    if (row < n) {
        const int p0 = pos[row], p1 = pos[row + 1];
        for (int base = p0; base < p1; base += W) {
            const int cnt = min(W, p1 - base);
            int my_c = 0;
            Acc my_v = 0;
            if (lane < cnt) {
                my_c = load_stream(crd + base + lane);
                my_v = widen<Acc>(load_stream(vals + base + lane));
            }
            // eight gathers in flight per lane, then eight FMAs
            for (int k0 = 0; k0 < cnt; k0 += 8) {
                Acc bv[8], vv[8];
#pragma unroll
                for (int kk = 0; kk < 8; ++kk) {
                    const int k = (k0 + kk) & (W - 1);
                    const int c = __shfl(my_c, k, W);
                    vv[kk] = __shfl(my_v, k, W);
                    bv[kk] = (k0 + kk < cnt && colok)
                                 ? widen<Acc>(Bd[static_cast<int64_t>(c) * ldb + col])
                                 : Acc(0);
                }
#pragma unroll
                for (int kk = 0; kk < 8; ++kk) acc += vv[kk] * bv[kk];
            }
        }
        if (colok) store_stream(Out + row * ldo + col, narrow<OT>(acc));
    }
}

template <int W, int ITEMS, typename V, typename BT, typename OT, typename Acc>
__global__ __launch_bounds__(kBlock) void k_spmm_tiles(
    int64_t n, int64_t N, const int32_t *__restrict__ pos, const int32_t *__restrict__ crd,
    const V *__restrict__ vals, const BT *__restrict__ Bd, int64_t ldb, OT *__restrict__ Out,
    int64_t ldo, const int32_t *__restrict__ trow, const int32_t *__restrict__ tpos,
    int64_t npieces, int64_t stride, Acc *__restrict__ carry) {
    constexpr int G = kBlock / W;
    constexpr int kChunk = G * ITEMS;
    __shared__ int32_t s_end[kChunk];
    __shared__ int32_t s_crd[kChunk];
    __shared__ Acc s_val[kChunk];
    __shared__ Acc s_head[G][W];
    __shared__ Acc s_tail[G][W];
    __shared__ int s_done[G];
    __shared__ int s_a0[G];
    __shared__ int64_t s_next[2];

    const int tid = threadIdx.x;
    const int g = tid / W, lane = tid % W;
    const int64_t col = static_cast<int64_t>(blockIdx.y) * W + lane;
    const bool colok = col < N;
    // this workgroup walks partition pieces [piece, piece_end)
    int64_t piece = static_cast<int64_t>(blockIdx.x) * stride;
    const int64_t piece_end = piece + stride < npieces ? piece + stride : npieces;
    int64_t ci = trow[piece], cp = tpos[piece];
    Acc open = 0;  // group 0: partial of row ci carried between chunks

    while (piece < piece_end) {
        const int64_t next = chunk_end(pos, trow, tpos, piece, ci, cp, kChunk, s_next);
        const int64_t ei = s_next[0], ep = s_next[1];
        piece = next;
        const int nr = static_cast<int>(ei - ci), np = static_cast<int>(ep - cp);
        for (int k = tid; k < nr; k += kBlock) s_end[k] = pos[ci + 1 + k];
        for (int k = tid; k < np; k += kBlock) {
            s_crd[k] = load_stream(crd + cp + k);
            s_val[k] = widen<Acc>(load_stream(vals + cp + k));
        }
        __syncthreads();

        const int total = nr + np;
        const int d0 = min(g * ITEMS, total);
        const int d1 = min(d0 + ITEMS, total);
        auto end_at = [&](int64_t m) { return s_end[m]; };
        const int a0 = static_cast<int>(merge_search(d0, nr, np, cp, end_at));
        const int a1 = static_cast<int>(merge_search(d1, nr, np, cp, end_at));
        const int b0 = d0 - a0, b1 = d1 - a1;

        // Issue every gather of this group's positions before consuming any.
        Acc pv[ITEMS];
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            pv[k] = 0;
            if (b0 + k < b1 && colok)
                pv[k] = s_val[b0 + k] *
                        widen<Acc>(Bd[static_cast<int64_t>(s_crd[b0 + k]) * ldb + col]);
        }
        Acc acc = 0;
        int a = a0;
        bool first = true;
        auto finish = [&](int r) {
            if (first) {
                s_head[g][lane] = acc;
                first = false;
            } else if (colok) {
                store_stream(Out + (ci + r) * ldo + col, narrow<OT>(acc));
            }
            acc = 0;
        };
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            if (b0 + k < b1) {
                while (a < a1 && s_end[a] <= cp + b0 + k) finish(a++);
                acc += pv[k];
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
                    if (colok) store_stream(Out + (ci + s_a0[gg]) * ldo + col, narrow<OT>(v));
                    c = s_tail[gg][lane];
                } else {
                    c += s_tail[gg][lane];
                }
            }
            open = c;
        }
        ci = ei;
        cp = ep;
        __syncthreads();
    }
    if (g == 0 && colok) carry[static_cast<int64_t>(blockIdx.x) * N + col] = open;
}

// Merge-split pieces are exactly one chunk each, so every chunk's bounds
// are known in advance and the staging can be software-pipelined: while a
// workgroup gathers and walks chunk c (LDS buffer c % 2), its lanes already
// hold in registers the row ends, coordinates and values of chunk c + 1,
// loaded before chunk c's gathers were issued, and the bounds of chunk c + 2
// one iteration earlier still.  After the walk they are stored to the other
// LDS buffer, so the loads of the next chunk never sit on the critical path.
// The walk, the cross-group pass and the carries are those of k_spmm_tiles.
// With int64 positions (PosT) the row ends are staged relative to the
// chunk's first position (they lie in [0, chunk]), so the walk and the
// searches stay 32-bit; int32 positions are staged as they are.
template <int W, int ITEMS, int VEC, typename V, typename BT, typename OT, typename Acc,
          typename PosT = int32_t, bool BUF = false>
__global__ __launch_bounds__(kBlock) void k_spmm_pipe(
    int64_t n, int64_t N, const PosT *__restrict__ pos, const int32_t *__restrict__ crd,
    const V *__restrict__ vals, const BT *__restrict__ Bd, int64_t ldb, OT *__restrict__ Out,
    int64_t ldo, const int32_t *__restrict__ trow, const PosT *__restrict__ tpos,
    int64_t npieces, int64_t stride, Acc *__restrict__ carry) {
    constexpr int G = kBlock / W;
    constexpr int kChunk = G * ITEMS;
    constexpr int kPer = (kChunk + kBlock - 1) / kBlock;
    __shared__ int32_t s_end[2][kChunk];
    __shared__ int32_t s_crd[2][kChunk];
    __shared__ Acc s_val[2][kChunk];
    __shared__ Acc s_head[G][W * VEC];
    __shared__ Acc s_tail[G][W * VEC];
    __shared__ int s_done[G];
    __shared__ int s_a0[G];
    // cross-group combine: the tile's columns split over kParts parts of
    // G / kParts groups each
    constexpr int NC = W * VEC;
    constexpr int kParts = kBlock / NC;
    constexpr int kGroupsPerPart = G / kParts;
    static_assert(kParts * NC == kBlock && kGroupsPerPart * kParts == G, "combine layout");
    __shared__ Acc s_open[NC];  // the open row's partial entering the chunk
    __shared__ Acc s_pb[kParts][NC];
    __shared__ int s_pa[kParts];

    const int tid = threadIdx.x;
    const int g = tid / W, lane = tid % W;
    // this lane's columns: col0 .. col0 + VEC - 1 (N is a multiple of VEC)
    const int64_t col0 = (static_cast<int64_t>(blockIdx.y) * W + lane) * VEC;
    const bool colok = col0 < N;
    const int64_t p0 = static_cast<int64_t>(blockIdx.x) * stride;
    const int64_t pend = p0 + stride < npieces ? p0 + stride : npieces;
    auto bound_i = [&](int64_t c) { return static_cast<int64_t>(trow[c < pend ? c : pend]); };
    auto bound_p = [&](int64_t c) { return static_cast<int64_t>(tpos[c < pend ? c : pend]); };

    int r_end[kPer], r_crd[kPer];
    Acc r_val[kPer];
    // issue the loads of the chunk [(fi, fp), (ei, ep)) into registers
    auto fetch = [&](int64_t fi, int64_t fp, int nr, int np) {
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int k = tid + j * kBlock;
            if (k < nr) {
                if constexpr (sizeof(PosT) == 4)
                    r_end[j] = pos[fi + 1 + k];
                else  // the difference fits 32 bits: subtract the low words
                    r_end[j] = static_cast<int>(static_cast<uint32_t>(pos[fi + 1 + k]) -
                                                static_cast<uint32_t>(fp));
            }
            if (k < np) {
                r_crd[j] = load_stream(crd + fp + k);
                r_val[j] = widen<Acc>(load_stream(vals + fp + k));
            }
        }
    };
    auto stash = [&](int buf, int nr, int np) {
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int k = tid + j * kBlock;
            if (k < nr) s_end[buf][k] = r_end[j];
            if (k < np) {
                s_crd[buf][k] = r_crd[j];
                s_val[buf][k] = r_val[j];
            }
        }
    };

    // bounds of the current chunk (ci, cp)-(ei, ep) and of the one after it
    int64_t ci = bound_i(p0), cp = bound_p(p0);
    int64_t ei = bound_i(p0 + 1), ep = bound_p(p0 + 1);
    int64_t ni = bound_i(p0 + 2), np2 = bound_p(p0 + 2);
    int nr = static_cast<int>(ei - ci), np = static_cast<int>(ep - cp);
    fetch(ci, cp, nr, np);
    stash(0, nr, np);
    if (tid < NC) s_open[tid] = 0;
    int buf = 0;
    for (int64_t c = p0; c < pend; ++c) {
        __syncthreads();  // buffer `buf` holds chunk c; the previous pass is done
        const bool more = c + 1 < pend;
        const int nnr = static_cast<int>(ni - ei), nnp = static_cast<int>(np2 - ep);
        const int64_t fi = bound_i(c + 3), fp = bound_p(c + 3);  // for the next iteration
        if (more) fetch(ei, ep, nnr, nnp);

        const int total = nr + np;
        const int d0 = min(g * ITEMS, total);
        const int d1 = min(d0 + ITEMS, total);
        const int32_t *send = s_end[buf];
        auto end_at = [&](int64_t m) { return send[m]; };
        const int64_t ebase = sizeof(PosT) == 4 ? cp : 0;  // what the staged ends count from
        const int a0 = static_cast<int>(merge_search(d0, nr, np, ebase, end_at));
        const int a1 = static_cast<int>(merge_search(d1, nr, np, ebase, end_at));
        const int b0 = d0 - a0, b1 = d1 - a1;
        // every gather of the group's positions is issued before any is used
        // (BF16 rows stay packed until they are read)
        RowVec<VEC, BT> pv[ITEMS];
        if constexpr (BUF) {
            // every lane issues every gather (a lane with no row reads 0 at
            // kBufOut): the walk then waits for each row as it reaches it
            // rather than for all of them (FP32 0.691 -> 0.678 ms, FP64
            // 1.276 -> 1.253 on the 2e6-row power-law matrix)
            static_assert(VEC * sizeof(BT) == 16, "16-byte lanes");
            const auto rB = span_rsrc(Bd, kBufRange);
#pragma unroll
            for (int k = 0; k < ITEMS; ++k) {
                const bool ok = b0 + k < b1 && colok;
                const int jj = s_crd[buf][b0 + k < kChunk ? b0 + k : kChunk - 1];
                pv[k].load_buf(rB, ok ? static_cast<uint32_t>(sizeof(BT)) *
                                            (static_cast<uint32_t>(jj) * static_cast<uint32_t>(ldb) +
                                             static_cast<uint32_t>(col0))
                                      : kBufOut);
            }
        } else {
#pragma unroll
            for (int k = 0; k < ITEMS; ++k) {
                pv[k].zero();
                if (b0 + k < b1 && colok)
                    pv[k].load(Bd + static_cast<int64_t>(s_crd[buf][b0 + k]) * ldb + col0);
            }
        }
        Acc acc[VEC];
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[v] = 0;
        int a = a0;
        bool first = true;
        auto finish = [&](int r) {
            if (first) {
#pragma unroll
                for (int v = 0; v < VEC; ++v) s_head[g][lane * VEC + v] = acc[v];
                first = false;
            } else if (colok) {
                store_row<VEC>(Out + (ci + r) * ldo + col0, acc);
            }
#pragma unroll
            for (int v = 0; v < VEC; ++v) acc[v] = 0;
        };
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            if (b0 + k < b1) {
                while (a < a1 && send[a] <= ebase + b0 + k) finish(a++);
                const Acc sv = s_val[buf][b0 + k];
#pragma unroll
                for (int v = 0; v < VEC; ++v) acc[v] += sv * static_cast<Acc>(pv[k].at(v));
            }
        }
        while (a < a1) finish(a++);
#pragma unroll
        for (int v = 0; v < VEC; ++v) s_tail[g][lane * VEC + v] = acc[v];
        if (lane == 0) {
            s_done[g] = a1 - a0;
            s_a0[g] = a0;
        }
        __syncthreads();
        // Combine across groups, in group order: a group that finished a row
        // writes it as (partial entering the group) + its head and restarts
        // the partial from its tail; any other group adds its tail.  Each
        // thread takes one column of one part: it composes its part's
        // groups, then starts from the partials of the parts before it.
        {
            const int cc = tid % NC, part = tid / NC;
            const int64_t gcol = static_cast<int64_t>(blockIdx.y) * NC + cc;
            int pa = 1;
            Acc pb = 0;
            for (int k = 0; k < kGroupsPerPart; ++k) {
                const int gg = part * kGroupsPerPart + k;
                const Acc t = s_tail[gg][cc];
                pb = s_done[gg] > 0 ? t : pb + t;
                pa = s_done[gg] > 0 ? 0 : pa;
            }
            s_pb[part][cc] = pb;
            if (cc == 0) s_pa[part] = pa;
            Acc o = s_open[cc];
            __syncthreads();
            for (int q = 0; q < part; ++q) o = s_pa[q] ? o + s_pb[q][cc] : s_pb[q][cc];
            for (int k = 0; k < kGroupsPerPart; ++k) {
                const int gg = part * kGroupsPerPart + k;
                if (s_done[gg] > 0) {
                    if (gcol < N)
                        store_stream(Out + (ci + s_a0[gg]) * ldo + gcol, narrow<OT>(o + s_head[gg][cc]));
                    o = s_tail[gg][cc];
                } else {
                    o += s_tail[gg][cc];
                }
            }
            if (part == kParts - 1) s_open[cc] = o;
        }
        if (more) stash(buf ^ 1, nnr, nnp);
        ci = ei;
        cp = ep;
        ei = ni;
        ep = np2;
        ni = fi;
        np2 = fp;
        nr = nnr;
        np = nnp;
        buf ^= 1;
    }
    __syncthreads();  // the last part's s_open
    if (tid < NC) {
        const int64_t gcol = static_cast<int64_t>(blockIdx.y) * NC + tid;
        if (gcol < N) carry[static_cast<int64_t>(blockIdx.x) * N + gcol] = s_open[tid];
    }
}


// Columns per lane of the vector-lane leaf: one 16-byte access (4 FP32, 2
// FP64 or 8 BF16 columns), so a 32-column BF16 row takes a group of 4 lanes
// and half the gather instructions of FP32.  BF16 rows can also be read 4
// columns (8 bytes) per lane (kSpmmVecNarrow).
template <typename BT>
constexpr int kSpmmVec = 16 / static_cast<int>(sizeof(BT));
constexpr int kSpmmVecNarrow = 4;

#define SPL_SPMM_ARGS n, N, pos, crd, vals, Bd, ldb, Out, ldo, t, stride, exact, buf, carry, s
template <typename V, typename BT, typename OT, typename Acc>
struct SpmmTypes {
    static hipError_t row(int W, int64_t n, int64_t N, const int32_t *pos, const int32_t *crd,
                          const void *vals, const void *Bd, int64_t ldb, void *Out, int64_t ldo,
                          hipStream_t s) {
        auto go = [&](auto kern, int w) {
            const int64_t G = kBlock / w;
            dim3 grid(static_cast<unsigned>((n + G - 1) / G), static_cast<unsigned>((N + w - 1) / w));
            if (grid.x == 0 || grid.y == 0) return hipSuccess;
            kern<<<grid, kBlock, 0, s>>>(n, N, pos, crd, static_cast<const V *>(vals),
                                         static_cast<const BT *>(Bd), ldb, static_cast<OT *>(Out), ldo);
            return hipGetLastError();
        };
        switch (W) {
        case 8: return go(k_spmm_row<8, V, BT, OT, Acc>, 8);
        case 16: return go(k_spmm_row<16, V, BT, OT, Acc>, 16);
        case 64: return go(k_spmm_row<64, V, BT, OT, Acc>, 64);
        default: return go(k_spmm_row<32, V, BT, OT, Acc>, 32);
        }
    }

    template <int W, int ITEMS, int VEC, typename PosT>
    static hipError_t tiles_w(int64_t n, int64_t N, const PosT *pos, const int32_t *crd,
                              const void *vals, const void *Bd, int64_t ldb, void *Out,
                              int64_t ldo, const Tiles &t, int64_t stride, bool exact,
                              bool buf, void *carry, hipStream_t s) {
        const int64_t tiles = ceil_div(t.ntiles, stride);
        dim3 grid(static_cast<unsigned>(tiles), static_cast<unsigned>(ceil_div(N, W * VEC)));
        if (grid.y == 0) return hipSuccess;
        // the buffer-descriptor gathers need 16-byte lanes
        constexpr bool kCanBuf = VEC * sizeof(BT) == 16;
        if constexpr (sizeof(PosT) == 8) {
            // int64 positions: merge pieces only (tile positions in t.pos64)
            if (!exact) return hipErrorInvalidValue;
            auto kern = buf && kCanBuf ? k_spmm_pipe<W, ITEMS, VEC, V, BT, OT, Acc, int64_t, kCanBuf>
                                       : k_spmm_pipe<W, ITEMS, VEC, V, BT, OT, Acc, int64_t, false>;
            kern<<<grid, kBlock, 0, s>>>(
                n, N, pos, crd, static_cast<const V *>(vals), static_cast<const BT *>(Bd), ldb,
                static_cast<OT *>(Out), ldo, t.row, t.pos64, t.ntiles, stride,
                static_cast<Acc *>(carry));
        } else {
            // pieces of exactly one chunk (merge split): the pipelined leaf
            auto kern = !exact ? k_spmm_tiles<W, ITEMS, V, BT, OT, Acc>
                        : buf && kCanBuf
                            ? k_spmm_pipe<W, ITEMS, VEC, V, BT, OT, Acc, int32_t, kCanBuf>
                            : k_spmm_pipe<W, ITEMS, VEC, V, BT, OT, Acc, int32_t, false>;
            kern<<<grid, kBlock, 0, s>>>(n, N, pos, crd, static_cast<const V *>(vals),
                                         static_cast<const BT *>(Bd), ldb, static_cast<OT *>(Out),
                                         ldo, t.row, t.pos, t.ntiles, stride,
                                         static_cast<Acc *>(carry));
        }
        return hipGetLastError();
    }

    static hipError_t fixup(int64_t n, int64_t N, const Tiles &t, int64_t stride,
                            const void *carry, void *Out, int64_t ldo, hipStream_t s) {
        return launch_carry_fixup<OT, Acc>(n, N, t.row, t.ntiles, stride,
                                           ceil_div(t.ntiles, stride),
                                           static_cast<const Acc *>(carry),
                                           static_cast<OT *>(Out), ldo, s);
    }

    // vector lanes of VEC columns each: col_tile / VEC lanes per group
    template <int VEC, typename PosT>
    static hipError_t tiles_vec(int col_tile, int items, int64_t n, int64_t N,
                                const PosT *pos, const int32_t *crd, const void *vals,
                                const void *Bd, int64_t ldb, void *Out, int64_t ldo,
                                const Tiles &t, int64_t stride, bool exact, bool buf, void *carry,
                                hipStream_t s) {
        switch (col_tile / VEC) {
        case 4: return items <= 8 ? tiles_w<4, 8, VEC, PosT>(SPL_SPMM_ARGS)
                                  : tiles_w<4, 16, VEC, PosT>(SPL_SPMM_ARGS);
        case 8: return items <= 8 ? tiles_w<8, 8, VEC, PosT>(SPL_SPMM_ARGS)
                                  : tiles_w<8, 16, VEC, PosT>(SPL_SPMM_ARGS);
        case 16: return items <= 8 ? tiles_w<16, 8, VEC, PosT>(SPL_SPMM_ARGS)
                                   : tiles_w<16, 16, VEC, PosT>(SPL_SPMM_ARGS);
        case 32: return items <= 8 ? tiles_w<32, 8, VEC, PosT>(SPL_SPMM_ARGS)
                                   : tiles_w<32, 16, VEC, PosT>(SPL_SPMM_ARGS);
        default: return hipErrorInvalidValue;
        }
    }

    // col_tile columns per lane group; vec > 1 (merge split only): vec
    // columns per lane, so col_tile / vec lanes per group
    // int64 positions: vector lanes and the merge split only
    static hipError_t tiles64(int col_tile, int items, int vec, int64_t n, int64_t N,
                              const int64_t *pos, const int32_t *crd, const void *vals,
                              const void *Bd, int64_t ldb, void *Out, int64_t ldo, const Tiles &t,
                              int64_t stride, bool exact, bool buf, void *carry, hipStream_t s) {
        if (vec != kSpmmVec<BT> || !exact || (items != 8 && items != 16))
            return hipErrorInvalidValue;
        return tiles_vec<kSpmmVec<BT>>(col_tile, items, SPL_SPMM_ARGS);
    }

    static hipError_t tiles(int col_tile, int items, int vec, int64_t n, int64_t N,
                            const int32_t *pos, const int32_t *crd, const void *vals,
                            const void *Bd, int64_t ldb, void *Out, int64_t ldo, const Tiles &t,
                            int64_t stride, bool exact, bool buf, void *carry, hipStream_t s) {
        if (vec > 1) {
            if (!exact || (items != 8 && items != 16)) return hipErrorInvalidValue;
            if (vec == kSpmmVec<BT>) return tiles_vec<kSpmmVec<BT>>(col_tile, items, SPL_SPMM_ARGS);
            if constexpr (sizeof(BT) == 2) {
                if (vec == kSpmmVecNarrow)
                    return tiles_vec<kSpmmVecNarrow>(col_tile, items, SPL_SPMM_ARGS);
            }
            return hipErrorInvalidValue;
        }
#define SPL_SPMM_ITEMS(Wv)                                                                    \
    if (items <= 8) return tiles_w<Wv, 8, 1, int32_t>(SPL_SPMM_ARGS);                         \
    if (items <= 16) return tiles_w<Wv, 16, 1, int32_t>(SPL_SPMM_ARGS);                       \
    return tiles_w<Wv, 32, 1, int32_t>(SPL_SPMM_ARGS);
        switch (col_tile) {
        case 8: SPL_SPMM_ITEMS(8)
        case 16: SPL_SPMM_ITEMS(16)
        case 64: SPL_SPMM_ITEMS(64)
        default: SPL_SPMM_ITEMS(32)
        }
#undef SPL_SPMM_ITEMS
    }
};
#undef SPL_SPMM_ARGS

}  // namespace

hipError_t launch_spmm_fixup(int vtype, int64_t n, int64_t N, const Tiles &t, int64_t stride,
                             const void *carry, void *Out, int64_t ldo, hipStream_t s) {
    if (vtype == SPL_F64)
        return SpmmTypes<double, double, double, double>::fixup(n, N, t, stride, carry, Out, ldo, s);
    return SpmmTypes<float, float, float, float>::fixup(n, N, t, stride, carry, Out, ldo, s);
}

hipError_t launch_spmm_row(int vtype, int otype, int col_tile, int64_t n, int64_t N,
                           const int32_t *pos, const int32_t *crd, const void *vals,
                           const void *Bd, int64_t ldb, void *Out, int64_t ldo, hipStream_t s) {
    (void)otype;
    if (vtype == SPL_F64)
        return SpmmTypes<double, double, double, double>::row(col_tile, n, N, pos, crd, vals, Bd,
                                                              ldb, Out, ldo, s);
    if (vtype == SPL_F32)
        return SpmmTypes<float, float, float, float>::row(col_tile, n, N, pos, crd, vals, Bd, ldb,
                                                          Out, ldo, s);
    return SpmmTypes<bf16, bf16, float, float>::row(col_tile, n, N, pos, crd, vals, Bd, ldb, Out,
                                                    ldo, s);
}

int spmm_vec_width(int vtype) {
    return vtype == SPL_F64 ? kSpmmVec<double> : vtype == SPL_F32 ? kSpmmVec<float>
                                                                  : kSpmmVec<bf16>;
}

hipError_t launch_spmm_tiles64(int vtype, int col_tile, int items, int vec, int64_t n, int64_t N,
                               const int64_t *pos, const int32_t *crd, const void *vals,
                               const void *Bd, int64_t ldb, void *Out, int64_t ldo,
                               const Tiles &t, int64_t stride, bool buf, void *carry,
                               hipStream_t s) {
    if (vtype == SPL_F64)
        return SpmmTypes<double, double, double, double>::tiles64(col_tile, items, vec, n, N, pos,
                                                                  crd, vals, Bd, ldb, Out, ldo, t,
                                                                  stride, true, buf, carry, s);
    if (vtype == SPL_F32)
        return SpmmTypes<float, float, float, float>::tiles64(col_tile, items, vec, n, N, pos, crd,
                                                              vals, Bd, ldb, Out, ldo, t, stride,
                                                              true, buf, carry, s);
    return SpmmTypes<bf16, bf16, float, float>::tiles64(col_tile, items, vec, n, N, pos, crd, vals,
                                                        Bd, ldb, Out, ldo, t, stride, true, buf,
                                                        carry, s);
}

hipError_t launch_spmm_tiles(int vtype, int col_tile, int items, int vec, int64_t n, int64_t N,
                             const int32_t *pos, const int32_t *crd, const void *vals,
                             const void *Bd, int64_t ldb, void *Out, int64_t ldo, const Tiles &t,
                             int64_t stride, bool exact_chunks, bool buf, void *carry,
                             hipStream_t s) {
    if (vtype == SPL_F64)
        return SpmmTypes<double, double, double, double>::tiles(col_tile, items, vec, n, N, pos,
                                                                crd, vals, Bd, ldb, Out, ldo, t,
                                                                stride, exact_chunks, buf, carry, s);
    if (vtype == SPL_F32)
        return SpmmTypes<float, float, float, float>::tiles(col_tile, items, vec, n, N, pos, crd,
                                                            vals, Bd, ldb, Out, ldo, t, stride,
                                                            exact_chunks, buf, carry, s);
    return SpmmTypes<bf16, bf16, float, float>::tiles(col_tile, items, vec, n, N, pos, crd, vals,
                                                      Bd, ldb, Out, ldo, t, stride, exact_chunks,
                                                      buf, carry, s);
}

}  // namespace spl
