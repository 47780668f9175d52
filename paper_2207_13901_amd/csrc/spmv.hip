// SpMV leaf  a(i) = B(i,j) * c(j)  for CSR B (paper Sec. VI-A, leaf loop of
// Fig. 8b), on one GPU.
//
// The kernels, by partition kind:
//
//  * k_spmv_row<L>: row split.  A group of L lanes owns one row (a universe
//    partition of the rows into blocks of 256/L per workgroup, image to the
//    positions).  No carries: every row is finished by the group that owns
//    it.  Good for short, even rows; a long row serializes on its group.
//    Rows are given by begin and end arrays, so the same leaf runs over the
//    position windows of one color of a coordinate-value partition.
//
//  * k_spmv_tiles: non-zero or merge split.  A workgroup owns `stride`
//    consecutive pieces of the level partition computed by partition.hip
//    (for the merge split, pieces of exactly one chunk, so no search is
//    needed; for the non-zero split, pieces of T positions, cut into chunks
//    by a merge-path search).  Each chunk has at most 256*ITEMS merged
//    items: the chunk's products vals[p]*c[crd[p]] and row ends are staged in
//    LDS with coalesced loads, every lane walks ITEMS consecutive merged
//    items (a merge-path split inside the chunk, so empty and long rows cost
//    the same as positions), and the partial sum a lane holds for the row it
//    is inside when its items run out is combined with its neighbours' by a
//    wavefront segmented scan (xor/up shuffles) plus a 4-entry cross-wave
//    pass through LDS.  The sum of the row still open at the end of the tile
//    is the tile's carry; k_carry_fixup (carry.hpp) adds carries into their
//    rows in a fixed order after the leaf kernel, the reduction into boundary rows that the
//    non-zero algorithm of Sec. II-D requires.  No floating-point atomics,
//    so results are bitwise reproducible.
//
//  * k_spmv_pipe (schedule variant 1): the merge-split form of
//    k_spmv_tiles with its staging software-pipelined two chunks deep.
//
//  * k_spmv_flag (merge split, default): the same pipeline with the row
//    ends staged as flags in the merged sequence, so that no lane searches
//    or reads row ends (see below).
//
//  * k_spmv_window_flag: the flag leaf over position windows (one color of
//    a coordinate-value partition), whose lengths are scanned into the
//    positions of a virtual CSR; each position maps back to its stored
//    position through the chunk's row offsets staged in LDS.
//
// Accumulation is in double for both double and float data (a float output
// is rounded once from the double sum, then once more if a carry lands on it).
#include <type_traits>

#include "carry.hpp"
#include "device.hpp"
#include "internal.hpp"

namespace spl {
namespace {

template <int L, typename V>
__global__ __launch_bounds__(kBlock) void k_spmv_row(int64_t n, const int32_t *__restrict__ pos_b,
                                                     const int32_t *__restrict__ pos_e,
                                                     const int32_t *__restrict__ crd,
                                                     const V *__restrict__ vals,
                                                     const V *__restrict__ x, V *__restrict__ y) {
    constexpr int kRows = kBlock / L;
    const int64_t row = static_cast<int64_t>(blockIdx.x) * kRows + threadIdx.x / L;
    const int lane = threadIdx.x % L;
    double acc = 0.0;
    if (row < n) {
        const int p0 = pos_b[row], p1 = pos_e[row];
        int p = p0 + lane;
        // two independent partial sums keep two gathers in flight per lane
        double acc2 = 0.0;
        for (; p + L < p1; p += 2 * L) {
            acc += to_f64(load_stream(vals + p)) * to_f64(x[load_stream(crd + p)]);
            acc2 += to_f64(load_stream(vals + p + L)) * to_f64(x[load_stream(crd + p + L)]);
        }
        if (p < p1) acc += to_f64(load_stream(vals + p)) * to_f64(x[load_stream(crd + p)]);
        acc += acc2;
    }
    acc = group_sum<L>(acc);
    if (row < n && lane == 0) store_stream(y + row, static_cast<V>(acc));
}

// Row split with one lane per row and kRows rows per lane (rows
// r0 + lane + 256 k): every step issues the next position of all of the
// lane's rows at once, so short rows (fibers of a CSF tensor) keep kRows
// independent gathers in flight instead of one.
template <typename V, int kRows>
__global__ __launch_bounds__(kBlock) void k_spmv_row_multi(int64_t n,
                                                           const int32_t *__restrict__ pos_b,
                                                           const int32_t *__restrict__ pos_e,
                                                           const int32_t *__restrict__ crd,
                                                           const V *__restrict__ vals,
                                                           const V *__restrict__ x,
                                                           V *__restrict__ y) {
    const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kBlock * kRows + threadIdx.x;
    int p[kRows], e[kRows];
    double acc[kRows];
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
        const int64_t r = r0 + static_cast<int64_t>(k) * kBlock;
        p[k] = r < n ? pos_b[r] : 0;
        e[k] = r < n ? pos_e[r] : 0;
        acc[k] = 0.0;
    }
    for (;;) {
        bool any = false;
        int c[kRows];
        V v[kRows], xv[kRows];
#pragma unroll
        for (int k = 0; k < kRows; ++k) {
            if (p[k] < e[k]) {
                any = true;
                c[k] = load_stream(crd + p[k]);
                v[k] = load_stream(vals + p[k]);
            }
        }
        if (!any) break;
#pragma unroll
        for (int k = 0; k < kRows; ++k)
            if (p[k] < e[k]) xv[k] = x[c[k]];
#pragma unroll
        for (int k = 0; k < kRows; ++k) {
            if (p[k] < e[k]) {
                acc[k] += to_f64(v[k]) * to_f64(xv[k]);
                ++p[k];
            }
        }
    }
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
        const int64_t r = r0 + static_cast<int64_t>(k) * kBlock;
        if (r < n) store_stream(y + r, static_cast<V>(acc[k]));
    }
}

// Inclusive segmented sum across the 256 lanes of a workgroup.  Lanes are
// ordered by key (non-decreasing); each lane ends with the sum of `v` over
// all lanes up to itself that share its key.
__device__ __forceinline__ double block_segmented_scan(double v, int key, int *s_first_key,
                                                      int *s_last_key, double *s_last_val) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        double vu = __shfl_up(v, off);
        int ku = __shfl_up(key, off);
        if (lane >= off && ku == key) v += vu;
    }
    if (lane == 0) s_first_key[wave] = key;
    if (lane == kWave - 1) {
        s_last_key[wave] = key;
        s_last_val[wave] = v;
    }
    __syncthreads();
    for (int w = wave - 1; w >= 0; --w) {
        if (s_last_key[w] != key) break;
        v += s_last_val[w];
        if (s_first_key[w] != key) break;
    }
    return v;
}

template <typename V, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_spmv_tiles(
    int64_t n, const int32_t *__restrict__ pos, const int32_t *__restrict__ crd,
    const V *__restrict__ vals, const V *__restrict__ x, V *__restrict__ y,
    const int32_t *__restrict__ trow, const int32_t *__restrict__ tpos, int64_t npieces,
    int64_t stride, double *__restrict__ carry) {
    constexpr int kChunk = kBlock * ITEMS;
    __shared__ double s_prod[kChunk];
    __shared__ double s_out[kChunk];
    __shared__ int32_t s_end[kChunk];
    __shared__ int s_first_key[kBlock / kWave], s_last_key[kBlock / kWave];
    __shared__ double s_last_val[kBlock / kWave];
    __shared__ int64_t s_next[2];
    __shared__ double s_open;

    const int tid = threadIdx.x;
    // this workgroup walks partition pieces [piece, piece_end)
    int64_t piece = static_cast<int64_t>(blockIdx.x) * stride;
    const int64_t piece_end = piece + stride < npieces ? piece + stride : npieces;
    int64_t ci = trow[piece], cp = tpos[piece];
    double open = 0.0;  // partial sum of row ci carried between chunks

    while (piece < piece_end) {
        const int64_t next = chunk_end(pos, trow, tpos, piece, ci, cp, kChunk, s_next);
        const int64_t ei = s_next[0], ep = s_next[1];
        piece = next;
        const int nr = static_cast<int>(ei - ci), np = static_cast<int>(ep - cp);

        for (int k = tid; k < nr; k += kBlock) s_end[k] = pos[ci + 1 + k];
        {
            // all ITEMS index loads, then all ITEMS gathers, then the products:
            // ITEMS independent gathers in flight per lane
            int c[ITEMS];
            V v[ITEMS], xv[ITEMS];
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) {
                const int k = tid + j * kBlock;
                if (k < np) {
                    c[j] = load_stream(crd + cp + k);
                    v[j] = load_stream(vals + cp + k);
                }
            }
#pragma unroll
            for (int j = 0; j < ITEMS; ++j)
                if (tid + j * kBlock < np) xv[j] = x[c[j]];
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) {
                const int k = tid + j * kBlock;
                if (k < np) s_prod[k] = to_f64(v[j]) * to_f64(xv[j]);
            }
        }
        __syncthreads();

        // This lane's share of the chunk's merged items.
        const int total = nr + np;
        const int d0 = min(tid * ITEMS, total);
        const int d1 = min(d0 + ITEMS, total);
        int a = static_cast<int>(merge_search(d0, nr, np, cp, [&](int64_t m) { return s_end[m]; }));
        int b = d0 - a;
        double acc = tid == 0 ? open : 0.0;
#pragma unroll
        for (int s = 0; s < ITEMS; ++s) {
            if (d0 + s < d1) {
                if (a < nr && s_end[a] <= cp + b) {
                    s_out[a] = acc;  // row a finished by this lane
                    acc = 0.0;
                    ++a;
                } else {
                    acc += s_prod[b];
                    ++b;
                }
            }
        }
        // `acc` belongs to row a (a == nr: the row still open at chunk end).
        double v = block_segmented_scan(acc, a, s_first_key, s_last_key, s_last_val);
        // The last lane of each run of equal keys holds the run total; the
        // key of the next lane comes from a shuffle inside the wave and from
        // the next wave's first key (stored by the scan) at a wave edge.
        int next_key = __shfl_down(a, 1);
        const int lane = tid & (kWave - 1), wave = tid / kWave;
        if (lane == kWave - 1) next_key = wave + 1 < kBlock / kWave ? s_first_key[wave + 1] : -1;
        if (next_key != a) {
            if (a < nr)
                s_out[a] += v;
            else
                s_open = v;
        }
        __syncthreads();
        for (int k = tid; k < nr; k += kBlock) store_stream(y + ci + k, static_cast<V>(s_out[k]));
        open = s_open;
        ci = ei;
        cp = ep;
        __syncthreads();
    }
    if (tid == 0) carry[blockIdx.x] = open;
}

// Merge-split pieces are exactly one chunk each, so the chunk bounds are
// known ahead and the staging is software-pipelined two chunks deep: while
// a workgroup walks chunk c (LDS buffer c % 2), the x gathers of chunk c + 1
// and the crd/vals/row-end loads of chunk c + 2 are in flight in registers;
// after the walk, chunk c + 1's products go to the other buffer, its gathers
// having had a whole iteration to land.  The walk, the segmented scan and
// the carry are those of k_spmv_tiles.
template <typename V, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_spmv_pipe(
    int64_t n, const int32_t *__restrict__ pos, const int32_t *__restrict__ crd,
    const V *__restrict__ vals, const V *__restrict__ x, V *__restrict__ y,
    const int32_t *__restrict__ trow, const int32_t *__restrict__ tpos, int64_t npieces,
    int64_t stride, double *__restrict__ carry) {
    constexpr int kChunk = kBlock * ITEMS;
    __shared__ double s_prod[2][kChunk + 1];  // + a spare slot for the walk
    __shared__ int32_t s_end[2][kChunk];
    __shared__ int s_first_key[kBlock / kWave], s_last_key[kBlock / kWave];
    __shared__ double s_last_val[kBlock / kWave];
    __shared__ double s_open;

    const int tid = threadIdx.x;
    const int64_t p0 = static_cast<int64_t>(blockIdx.x) * stride;
    const int64_t pend = p0 + stride < npieces ? p0 + stride : npieces;
    auto bound_i = [&](int64_t c) { return static_cast<int64_t>(trow[c < pend ? c : pend]); };
    auto bound_p = [&](int64_t c) { return static_cast<int64_t>(tpos[c < pend ? c : pend]); };

    // stage 2: loads of a chunk; stage 1: its x gathers
    int e2[ITEMS], k2[ITEMS], e1[ITEMS];
    V v2[ITEMS], v1[ITEMS], x1[ITEMS];
    auto load = [&](int64_t bi, int64_t bp, int nr, int np) {
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const int k = tid + j * kBlock;
            if (k < nr) e2[j] = pos[bi + 1 + k];
            if (k < np) {
                k2[j] = load_stream(crd + bp + k);
                v2[j] = load_stream(vals + bp + k);
            }
        }
    };
    auto gather = [&](int np) {
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            e1[j] = e2[j];
            v1[j] = v2[j];
            if (tid + j * kBlock < np) x1[j] = x[k2[j]];
        }
    };
    auto stash = [&](int buf, int nr, int np) {
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const int k = tid + j * kBlock;
            if (k < nr) s_end[buf][k] = e1[j];
            if (k < np) s_prod[buf][k] = to_f64(v1[j]) * to_f64(x1[j]);
        }
    };

    // bounds of chunks c .. c + 3 as (b*0 .. b*3)
    int64_t bi0 = bound_i(p0), bp0 = bound_p(p0);
    int64_t bi1 = bound_i(p0 + 1), bp1 = bound_p(p0 + 1);
    int64_t bi2 = bound_i(p0 + 2), bp2 = bound_p(p0 + 2);
    int64_t bi3 = bound_i(p0 + 3), bp3 = bound_p(p0 + 3);
    // prologue: chunk p0 into buffer 0, chunk p0 + 1 gathering, p0 + 2 loading
    load(bi0, bp0, static_cast<int>(bi1 - bi0), static_cast<int>(bp1 - bp0));
    gather(static_cast<int>(bp1 - bp0));
    stash(0, static_cast<int>(bi1 - bi0), static_cast<int>(bp1 - bp0));
    load(bi1, bp1, static_cast<int>(bi2 - bi1), static_cast<int>(bp2 - bp1));
    gather(static_cast<int>(bp2 - bp1));
    load(bi2, bp2, static_cast<int>(bi3 - bi2), static_cast<int>(bp3 - bp2));

    double open = 0.0;  // partial sum of the row open at the chunk start
    int buf = 0;
    for (int64_t c = p0; c < pend; ++c) {
        const int64_t bi4 = bound_i(c + 4), bp4 = bound_p(c + 4);
        __syncthreads();  // buffer `buf` holds chunk c
        const int nr = static_cast<int>(bi1 - bi0), np = static_cast<int>(bp1 - bp0);
        const int total = nr + np;
        const int d0 = min(tid * ITEMS, total);
        const int d1 = min(d0 + ITEMS, total);
        const int32_t *send = s_end[buf];
        const double *sprod = s_prod[buf];
        // finished rows' sums go to the idle product buffer until written out
        double *s_out = s_prod[buf ^ 1];
        int a = static_cast<int>(merge_search(d0, nr, np, bp0, [&](int64_t m) { return send[m]; }));
        int b = d0 - a;
        double acc = tid == 0 ? open : 0.0;
        // Branch-free walk (selects instead of divergent branches, whose
        // exec-mask bookkeeping dominated the instruction count for short
        // rows): each step reads the next row end and product at clamped
        // indices and either finishes row a (its sum to s_out[a], else to the
        // spare slot) or adds position b.
#pragma unroll
        for (int s = 0; s < ITEMS; ++s) {
            const bool in = d0 + s < d1;
            const int32_t e = send[a < kChunk ? a : kChunk - 1];
            const double pv = sprod[b < kChunk ? b : kChunk - 1];
            const bool fin = in && a < nr && e <= bp0 + b;
            const bool add = in && !fin;
            s_out[fin ? a : kChunk] = acc;
            acc = fin ? 0.0 : (add ? acc + pv : acc);
            a += fin ? 1 : 0;
            b += add ? 1 : 0;
        }
        double v = block_segmented_scan(acc, a, s_first_key, s_last_key, s_last_val);
        int next_key = __shfl_down(a, 1);
        const int lane = tid & (kWave - 1), wave = tid / kWave;
        if (lane == kWave - 1) next_key = wave + 1 < kBlock / kWave ? s_first_key[wave + 1] : -1;
        if (next_key != a) {
            if (a < nr)
                s_out[a] += v;
            else
                s_open = v;
        }
        __syncthreads();
        for (int k = tid; k < nr; k += kBlock) store_stream(y + bi0 + k, static_cast<V>(s_out[k]));
        open = s_open;
        __syncthreads();  // the row sums are out of the buffer the stash refills
        // chunk c + 1 to the other buffer; c + 2 starts gathering, c + 3 loading
        if (c + 1 < pend) {
            stash(buf ^ 1, static_cast<int>(bi2 - bi1), static_cast<int>(bp2 - bp1));
            gather(static_cast<int>(bp3 - bp2));
            if (c + 3 < pend) load(bi3, bp3, static_cast<int>(bi4 - bi3), static_cast<int>(bp4 - bp3));
        }
        bi0 = bi1; bp0 = bp1;
        bi1 = bi2; bp1 = bp2;
        bi2 = bi3; bp2 = bp3;
        bi3 = bi4; bp3 = bp4;
        buf ^= 1;
    }
    if (tid == 0) carry[blockIdx.x] = open;
}

// A raw buffer descriptor over `bytes` bytes at `base` (data format word of
// gfx9): lane offsets at or past `bytes` read 0 without touching memory.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t chunk_rsrc(const void *base, int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, bytes, 0x00020000);
}
constexpr int kNtAux = 2;  // non-temporal cache policy for streamed arrays

template <typename V>
__device__ __forceinline__ V chunk_load(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <>
__device__ __forceinline__ float chunk_load<float>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, kNtAux));
}
template <>
__device__ __forceinline__ double chunk_load<double>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, kNtAux));
}

// Wave-wide inclusive scans with DPP (GFX9 data-parallel primitives): four
// shifts inside each row of 16 lanes, then lane 15 of rows 0 and 2 is added
// to rows 1 and 3, and lane 31 to rows 2 and 3.  A lane whose source is out
// of its row, or whose row is masked off, receives the `old` operand.
template <int CTL, int ROWS>
__device__ __forceinline__ int dpp_i32(int old, int v) {
    return __builtin_amdgcn_update_dpp(old, v, CTL, ROWS, 0xf, false);
}
template <int CTL, int ROWS>
__device__ __forceinline__ double dpp_f64(double old, double v) {
    return __builtin_amdgcn_update_dpp(old, v, CTL, ROWS, 0xf, false);
}

__device__ __forceinline__ int wave_inclusive_sum(int s) {
    s += dpp_i32<0x111, 0xf>(0, s);  // row_shr:1
    s += dpp_i32<0x112, 0xf>(0, s);  // row_shr:2
    s += dpp_i32<0x114, 0xf>(0, s);  // row_shr:4
    s += dpp_i32<0x118, 0xf>(0, s);  // row_shr:8
    s += dpp_i32<0x142, 0xa>(0, s);  // row_bcast:15 into rows 1, 3
    s += dpp_i32<0x143, 0xc>(0, s);  // row_bcast:31 into rows 2, 3
    return s;
}

// One step of the segmented scan: add the source lane's sum when it holds
// the same key (key -1 from a lane without a source never matches).
template <int CTL, int ROWS>
__device__ __forceinline__ void seg_step(double &v, int key) {
    const int k = dpp_i32<CTL, ROWS>(-1, key);
    const double t = dpp_f64<CTL, ROWS>(0.0, v);
    if (k == key) v += t;
}

// Inclusive sum of `v` over the lanes of the wave up to this one that share
// its key (keys non-decreasing over the lanes).
__device__ __forceinline__ double wave_segmented_sum(double v, int key) {
    seg_step<0x111, 0xf>(v, key);
    seg_step<0x112, 0xf>(v, key);
    seg_step<0x114, 0xf>(v, key);
    seg_step<0x118, 0xf>(v, key);
    seg_step<0x142, 0xa>(v, key);
    seg_step<0x143, 0xc>(v, key);
    return v;
}

// Exclusive sum of `v` over the lanes of the workgroup before this one.
__device__ __forceinline__ int block_exclusive_sum(int v, int *s_wave_total) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int inc = wave_inclusive_sum(v);
    if (lane == kWave - 1) s_wave_total[wave] = inc;
    __syncthreads();
    static_assert(kBlock / kWave == 4, "four waves per workgroup");
    const int4 t = *reinterpret_cast<const int4 *>(s_wave_total);
    const int before = (wave > 0 ? t.x : 0) + (wave > 1 ? t.y : 0) + (wave > 2 ? t.z : 0);
    return before + inc - v;
}

// block_segmented_scan with the wave part done by DPP.
__device__ __forceinline__ double block_segmented_scan_dpp(double v, int key, int *s_first_key,
                                                          int *s_last_key, double *s_last_val) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    v = wave_segmented_sum(v, key);
    if (lane == 0) s_first_key[wave] = key;
    if (lane == kWave - 1) {
        s_last_key[wave] = key;
        s_last_val[wave] = v;
    }
    __syncthreads();
    for (int w = wave - 1; w >= 0; --w) {
        if (s_last_key[w] != key) break;
        v += s_last_val[w];
        if (s_first_key[w] != key) break;
    }
    return v;
}

// Merge-split leaf with row-end flags (the default; k_spmv_pipe is schedule
// variant 1).  The same pieces, pipeline and carries as k_spmv_pipe, but
// instead of the row ends
// the staging writes a flag byte at each row end's place in the chunk's
// merged sequence (row end r of the chunk sits at r + pos[r+1] - chunk
// start).  A lane reads its ITEMS flags with one LDS load, counts them, and
// an exclusive sum over the workgroup gives the rows finished before its
// first item; its walk then needs no search and no row-end reads: a flagged
// item finishes the open row, any other adds the next product.
//
// P is the element type of pos and TP that of the tile positions (int32 or
// int64).  Only the low 32 bits of a row end are loaded: its offset from the
// chunk start is below 2^31, so the 32-bit difference of the low words is
// exact.
template <typename V, int ITEMS, typename P = int32_t, typename TP = int32_t>
__global__ __launch_bounds__(kBlock) void k_spmv_flag(
    int64_t n, const P *__restrict__ pos, const int32_t *__restrict__ crd,
    const V *__restrict__ vals, const V *__restrict__ x, V *__restrict__ y,
    const int32_t *__restrict__ trow, const TP *__restrict__ tpos, int64_t npieces,
    int64_t stride, double *__restrict__ carry) {
    static_assert(ITEMS == 4 || ITEMS == 8, "flags are read as one 4- or 8-byte word");
    using Flags = typename std::conditional<ITEMS == 4, uint32_t, uint64_t>::type;
    constexpr int kChunk = kBlock * ITEMS;
    __shared__ double s_prod[2][kChunk + 1];  // + a spare slot for the walk
    // byte k: merged item k is a row end; byte kChunk is a spare
    __shared__ __align__(8) uint8_t s_flag[2][kChunk + 8];
    __shared__ __align__(16) int s_wave_total[kBlock / kWave];
    __shared__ int s_first_key[kBlock / kWave], s_last_key[kBlock / kWave];
    __shared__ double s_last_val[kBlock / kWave];
    __shared__ double s_open;

    const int tid = threadIdx.x;
    const int64_t p0 = static_cast<int64_t>(blockIdx.x) * stride;
    const int64_t pend = p0 + stride < npieces ? p0 + stride : npieces;
    auto bound_i = [&](int64_t c) { return static_cast<int64_t>(trow[c < pend ? c : pend]); };
    auto bound_p = [&](int64_t c) { return static_cast<int64_t>(tpos[c < pend ? c : pend]); };
    auto flag_word = [&](int buf) -> Flags & { return reinterpret_cast<Flags *>(s_flag[buf])[tid]; };

    // Loads are not predicated per lane: each goes through a buffer
    // descriptor over the chunk's own rows or positions, so a lane past its
    // end reads 0 (the hardware range check) and the stash sends its flag
    // and product to the spare slots.  The lane offsets do not depend on the
    // chunk.
    int e2[ITEMS], k2[ITEMS], e1[ITEMS];
    V v2[ITEMS], v1[ITEMS], x1[ITEMS];
    auto load = [&](int64_t bi, int64_t bp, int nr, int np) {
        const auto rp = chunk_rsrc(pos + bi + 1, static_cast<int>(sizeof(P)) * nr);
        const auto rc = chunk_rsrc(crd + bp, 4 * np);
        const auto rv = chunk_rsrc(vals + bp, static_cast<int>(sizeof(V)) * np);
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t k = static_cast<uint32_t>(tid + j * kBlock);
            e2[j] = static_cast<int32_t>(__builtin_amdgcn_raw_buffer_load_b32(
                rp, k * static_cast<uint32_t>(sizeof(P)), 0, 0));  // low word
            k2[j] = static_cast<int32_t>(__builtin_amdgcn_raw_buffer_load_b32(rc, k * 4, 0, kNtAux));
            v2[j] = chunk_load<V>(rv, k * static_cast<uint32_t>(sizeof(V)));
        }
    };
    auto gather = [&](int np) {
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            e1[j] = e2[j];
            v1[j] = v2[j];
        }
        if (np > 0) {  // lanes past the positions gather x[0]
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) x1[j] = x[k2[j]];
        }
    };
    // chunk starting at position bp into buffer `buf`: flags and products
    auto stash = [&](int buf, int nr, int np, int64_t bp) {
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const int k = tid + j * kBlock;
            const int rel = static_cast<int>(static_cast<uint32_t>(e1[j]) -
                                             static_cast<uint32_t>(bp));
            s_flag[buf][k < nr ? k + rel : kChunk] = 1;
            s_prod[buf][k < np ? k : kChunk] = to_f64(v1[j]) * to_f64(x1[j]);
        }
    };

    flag_word(0) = 0;
    flag_word(1) = 0;
    int64_t bi0 = bound_i(p0), bp0 = bound_p(p0);
    int64_t bi1 = bound_i(p0 + 1), bp1 = bound_p(p0 + 1);
    int64_t bi2 = bound_i(p0 + 2), bp2 = bound_p(p0 + 2);
    int64_t bi3 = bound_i(p0 + 3), bp3 = bound_p(p0 + 3);
    load(bi0, bp0, static_cast<int>(bi1 - bi0), static_cast<int>(bp1 - bp0));
    gather(static_cast<int>(bp1 - bp0));
    __syncthreads();  // flags cleared
    stash(0, static_cast<int>(bi1 - bi0), static_cast<int>(bp1 - bp0), bp0);
    load(bi1, bp1, static_cast<int>(bi2 - bi1), static_cast<int>(bp2 - bp1));
    gather(static_cast<int>(bp2 - bp1));
    load(bi2, bp2, static_cast<int>(bi3 - bi2), static_cast<int>(bp3 - bp2));

    double open = 0.0;
    int buf = 0;
    for (int64_t c = p0; c < pend; ++c) {
        const int64_t bi4 = bound_i(c + 4), bp4 = bound_p(c + 4);
        __syncthreads();  // buffer `buf` holds chunk c
        const int nr = static_cast<int>(bi1 - bi0), np = static_cast<int>(bp1 - bp0);
        const int total = nr + np;
        const int d0 = min(tid * ITEMS, total);
        const int steps = min(d0 + ITEMS, total) - d0;
        const Flags fl = flag_word(buf);
        flag_word(buf) = 0;  // cleared for the chunk after next
        int a = block_exclusive_sum(static_cast<int>(__builtin_popcountll(fl)), s_wave_total);
        int b = d0 - a;
        const double *sprod = s_prod[buf];
        double *s_out = s_prod[buf ^ 1];  // finished rows until written out
        double acc = tid == 0 ? open : 0.0;
#pragma unroll
        for (int st = 0; st < ITEMS; ++st) {
            const bool fin = (fl >> (8 * st)) & 1;
            const bool add = !fin && st < steps;
            const double pv = sprod[b];  // b <= np; slot kChunk is the spare
            s_out[fin ? a : kChunk] = acc;
            acc = (fin ? 0.0 : acc) + (add ? pv : 0.0);
            a += fin ? 1 : 0;
            b += add ? 1 : 0;
        }
        double v = block_segmented_scan_dpp(acc, a, s_first_key, s_last_key, s_last_val);
        int next_key = __shfl_down(a, 1);
        const int lane = tid & (kWave - 1), wave = tid / kWave;
        if (lane == kWave - 1) next_key = wave + 1 < kBlock / kWave ? s_first_key[wave + 1] : -1;
        if (next_key != a) {
            if (a < nr)
                s_out[a] += v;
            else
                s_open = v;
        }
        __syncthreads();
        for (int k = tid; k < nr; k += kBlock) store_stream(y + bi0 + k, static_cast<V>(s_out[k]));
        open = s_open;
        __syncthreads();  // the row sums are out of the buffer the stash refills
        if (c + 1 < pend) {
            stash(buf ^ 1, static_cast<int>(bi2 - bi1), static_cast<int>(bp2 - bp1), bp1);
            gather(static_cast<int>(bp3 - bp2));
            if (c + 3 < pend) load(bi3, bp3, static_cast<int>(bi4 - bi3), static_cast<int>(bp4 - bp3));
        }
        bi0 = bi1; bp0 = bp1;
        bi1 = bi2; bp1 = bp2;
        bi2 = bi3; bp2 = bp3;
        bi3 = bi4; bp3 = bp4;
        buf ^= 1;
    }
    if (tid == 0) carry[blockIdx.x] = open;
}

// Merge-split leaf that sums whole rows per lane (schedule variant 2).  The
// same pieces and carries as k_spmv_flag, without a scan: per chunk the
// products vals[p] * c[crd[p]] of its positions and the ends of its rows
// (relative to the chunk's first position) are staged in LDS with
// coalesced loads; lane t then sums rows t, t + 256, ... of the chunk from
// LDS in position order and writes them, and the row still open at the end
// of the chunk is summed by the workgroup (lane-strided partials, then a
// fixed tree).  A row with more than kLongRow positions in the chunk is
// queued and summed by one wave (lane-strided partials and a butterfly),
// so one long row does not serialize its lane.  For rows of one or two
// positions (the fibers of a CSF tensor) this costs a fraction of the flag
// walk's instructions: one LDS read and add per position, no segmented
// scan and two barriers per chunk.  Every order is fixed, so the result is
// reproducible; sums are in double as in the other leaves.
constexpr int kLongRow = 32;

template <typename V, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_spmv_rows(
    int64_t n, const int32_t *__restrict__ pos, const int32_t *__restrict__ crd,
    const V *__restrict__ vals, const V *__restrict__ x, V *__restrict__ y,
    const int32_t *__restrict__ trow, const int32_t *__restrict__ tpos, int64_t npieces,
    int64_t stride, double *__restrict__ carry) {
    constexpr int kChunk = kBlock * ITEMS;
    constexpr int kWaves = kBlock / kWave;
    __shared__ double s_prod[kChunk];
    __shared__ int32_t s_end[kChunk];
    __shared__ int32_t s_long[kChunk / (kLongRow + 1) + 1];
    __shared__ int s_nlong;
    __shared__ double s_red[kWaves];
    const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    const int64_t p0 = static_cast<int64_t>(blockIdx.x) * stride;
    const int64_t pend = p0 + stride < npieces ? p0 + stride : npieces;
    double open = 0.0;
    if (tid == 0) s_nlong = 0;
    // two chunks ahead: the coordinates, values and row ends of chunk c + 2
    // are loaded and the c gathers of chunk c + 1 issued while chunk c is
    // summed
    int32_t k2[ITEMS], e2[ITEMS], e1[ITEMS];
    V v2[ITEMS], v1[ITEMS], x1[ITEMS];
    int np2 = 0;  // positions of the loaded chunk
    auto load = [&](int64_t cc) {
        const int64_t li0 = trow[cc], lp0 = tpos[cc];
        const int lnr = static_cast<int>(trow[cc + 1] - li0);
        const int lnp = static_cast<int>(tpos[cc + 1] - lp0);
        np2 = lnp;
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const int k = tid + j * kBlock;
            k2[j] = k < lnp ? load_stream(crd + lp0 + k) : 0;
            v2[j] = k < lnp ? load_stream(vals + lp0 + k) : V(0);
            e2[j] = k < lnr ? pos[li0 + k + 1] : 0;
        }
    };
    auto gather = [&]() {
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            e1[j] = e2[j];
            v1[j] = v2[j];
        }
        if (np2 > 0) {  // lanes past the positions gather c[0]
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) x1[j] = x[k2[j]];
        }
    };
    if (p0 < pend) {
        load(p0);
        gather();
        if (p0 + 1 < pend) load(p0 + 1);
    }
    for (int64_t c = p0; c < pend; ++c) {
        const int64_t bi0 = trow[c], bp0 = tpos[c];
        const int nr = static_cast<int>(trow[c + 1] - bi0);
        const int np = static_cast<int>(tpos[c + 1] - bp0);
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const int k = tid + j * kBlock;
            if (k < np) s_prod[k] = to_f64(v1[j]) * to_f64(x1[j]);
            if (k < nr) s_end[k] = static_cast<int32_t>(e1[j] - bp0);
        }
        if (c + 1 < pend) {
            gather();
            if (c + 2 < pend) load(c + 2);
        }
        __syncthreads();
        for (int k = tid; k < nr; k += kBlock) {
            const int b = k ? s_end[k - 1] : 0, e = s_end[k];
            if (e - b > kLongRow) {
                s_long[atomicAdd(&s_nlong, 1)] = k;
                continue;
            }
            double acc = k ? 0.0 : open;
            for (int q = b; q < e; ++q) acc += s_prod[q];
            store_stream(y + bi0 + k, static_cast<V>(acc));
        }
        // the row open at the chunk's end
        const int t0 = nr ? s_end[nr - 1] : 0;
        double part = 0.0;
        for (int q = t0 + tid; q < np; q += kBlock) part += s_prod[q];
        part = group_sum<kWave>(part);
        if (lane == 0) s_red[wave] = part;
        __syncthreads();  // the tail partials and the long-row queue
        double tail = 0.0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) tail += s_red[w];
        const int nlong = s_nlong;
        for (int u = wave; u < nlong; u += kWaves) {
            const int k = s_long[u];
            const int b = k ? s_end[k - 1] : 0, e = s_end[k];
            double acc = 0.0;
            for (int q = b + lane; q < e; q += kWave) acc += s_prod[q];
            acc = group_sum<kWave>(acc);
            if (lane == 0) store_stream(y + bi0 + k, static_cast<V>(k ? acc : open + acc));
        }
        open = nr ? tail : open + tail;
        __syncthreads();  // the chunk's LDS is read before the next one overwrites it
        if (tid == 0) s_nlong = 0;
    }
    if (tid == 0) carry[blockIdx.x] = open;
}

// Merge-split leaf over position windows: row i contributes its positions
// [begin[i], end[i]) (the windows of one color of a coordinate-value
// partition).  The rows and the window positions are merged as for a CSR
// whose pos is vpos, the scan of the window lengths (virtual positions);
// virtual position q of row r is the stored position q + begin[r] - vpos[r].
// Per chunk the row ends (as flags, as in k_spmv_flag) and the offsets of
// the chunk's rows are staged in LDS; each position finds its row by a
// binary search over the staged row ends, then loads its coordinate and
// value and gathers x.  The walk, the scans and the carries are those of
// k_spmv_flag; no software pipeline.
template <typename V, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_spmv_window_flag(
    int64_t n, const int32_t *__restrict__ vpos, const int32_t *__restrict__ begin,
    const int32_t *__restrict__ crd, const V *__restrict__ vals, const V *__restrict__ x,
    V *__restrict__ y, const int32_t *__restrict__ trow, const int32_t *__restrict__ tpos,
    int64_t npieces, int64_t stride, double *__restrict__ carry) {
    static_assert(ITEMS == 4 || ITEMS == 8, "flags are read as one 4- or 8-byte word");
    using Flags = typename std::conditional<ITEMS == 4, uint32_t, uint64_t>::type;
    constexpr int kChunk = kBlock * ITEMS;
    __shared__ double s_prod[kChunk + 1];
    __shared__ double s_out[kChunk + 1];  // finished rows; slot kChunk is a spare
    __shared__ __align__(8) uint8_t s_flag[kChunk + 8];
    __shared__ int32_t s_vend[kChunk];     // virtual ends of the rows finished in the chunk
    __shared__ int32_t s_off[kChunk + 1];  // begin - vpos of the chunk's rows bi .. bi + nr
    __shared__ __align__(16) int s_wave_total[kBlock / kWave];
    __shared__ int s_first_key[kBlock / kWave], s_last_key[kBlock / kWave];
    __shared__ double s_last_val[kBlock / kWave];
    __shared__ double s_open;

    const int tid = threadIdx.x;
    const int64_t p0 = static_cast<int64_t>(blockIdx.x) * stride;
    const int64_t pend = p0 + stride < npieces ? p0 + stride : npieces;
    Flags &flag_word = reinterpret_cast<Flags *>(s_flag)[tid];
    flag_word = 0;
    double open = 0.0;
    for (int64_t c = p0; c < pend; ++c) {
        const int64_t bi = trow[c], bp = tpos[c];
        const int nr = static_cast<int>(trow[c + 1] - bi), np = static_cast<int>(tpos[c + 1] - bp);
        // chunks past the end (the grid is sized for all positions, the
        // windows hold fewer) are empty: the same for every thread
        if (nr + np == 0) continue;
        __syncthreads();  // the previous chunk is done with every staging array
        for (int k = tid; k < nr; k += kBlock) {
            const int32_t e = vpos[bi + 1 + k];
            s_vend[k] = e;
            s_flag[k + static_cast<int>(e - bp)] = 1;
        }
        for (int k = tid; k <= nr; k += kBlock)
            if (bi + k < n) s_off[k] = begin[bi + k] - vpos[bi + k];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const int k = tid + j * kBlock;
            if (k < np) {
                const int32_t q = static_cast<int32_t>(bp) + k;
                int lo = 0, hi = nr;  // rows of the chunk finished at or before q
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (s_vend[mid] <= q)
                        lo = mid + 1;
                    else
                        hi = mid;
                }
                const int32_t at = q + s_off[lo];
                s_prod[k] = to_f64(vals[at]) * to_f64(x[crd[at]]);
            }
        }
        __syncthreads();
        const int total = nr + np;
        const int d0 = min(tid * ITEMS, total);
        const int steps = min(d0 + ITEMS, total) - d0;
        const Flags fl = flag_word;
        flag_word = 0;  // cleared for the next chunk
        int a = block_exclusive_sum(static_cast<int>(__builtin_popcountll(fl)), s_wave_total);
        int b = d0 - a;
        double acc = tid == 0 ? open : 0.0;
#pragma unroll
        for (int st = 0; st < ITEMS; ++st) {
            const bool fin = (fl >> (8 * st)) & 1;
            const bool add = !fin && st < steps;
            const double pv = s_prod[b];  // b <= np <= kChunk
            s_out[fin ? a : kChunk] = acc;
            acc = (fin ? 0.0 : acc) + (add ? pv : 0.0);
            a += fin ? 1 : 0;
            b += add ? 1 : 0;
        }
        double v = block_segmented_scan_dpp(acc, a, s_first_key, s_last_key, s_last_val);
        int next_key = __shfl_down(a, 1);
        const int lane = tid & (kWave - 1), wave = tid / kWave;
        if (lane == kWave - 1) next_key = wave + 1 < kBlock / kWave ? s_first_key[wave + 1] : -1;
        if (next_key != a) {
            if (a < nr)
                s_out[a] += v;
            else
                s_open = v;
        }
        __syncthreads();
        for (int k = tid; k < nr; k += kBlock) store_stream(y + bi + k, static_cast<V>(s_out[k]));
        open = s_open;
    }
    if (tid == 0) carry[blockIdx.x] = open;
}

template <typename V>
hipError_t spmv_row_dispatch(int lanes, int64_t n, const int32_t *pos_b, const int32_t *pos_e,
                             const int32_t *crd, const V *vals, const V *x, V *y, hipStream_t s) {
    auto go = [&](auto kern, int rows_per_block) {
        int64_t blocks = (n + rows_per_block - 1) / rows_per_block;
        if (blocks == 0) return hipSuccess;
        kern<<<dim3(static_cast<unsigned>(blocks)), kBlock, 0, s>>>(n, pos_b, pos_e, crd, vals, x,
                                                                    y);
        return hipGetLastError();
    };
    switch (lanes) {
    case 1: return go(k_spmv_row_multi<V, 4>, 1024);
    case 2: return go(k_spmv_row<2, V>, 128);
    case 4: return go(k_spmv_row<4, V>, 64);
    case 8: return go(k_spmv_row<8, V>, 32);
    case 16: return go(k_spmv_row<16, V>, 16);
    case 32: return go(k_spmv_row<32, V>, 8);
    default: return go(k_spmv_row<64, V>, 4);
    }
}

template <typename V>
hipError_t spmv_tiles_dispatch(int items, int64_t n, const int32_t *pos, const int32_t *crd,
                               const V *vals, const V *x, V *y, const Tiles &t, int64_t stride,
                               bool exact, int variant, double *carry, hipStream_t s) {
    dim3 grid(static_cast<unsigned>(ceil_div(t.ntiles, stride)));
    if (exact && variant == 2) {
        if (items <= 4)
            k_spmv_rows<V, 4><<<grid, kBlock, 0, s>>>(n, pos, crd, vals, x, y, t.row, t.pos,
                                                       t.ntiles, stride, carry);
        else
            k_spmv_rows<V, 8><<<grid, kBlock, 0, s>>>(n, pos, crd, vals, x, y, t.row, t.pos,
                                                       t.ntiles, stride, carry);
        return hipGetLastError();
    }
    if (exact && variant == 0) {
        if (items <= 4)
            k_spmv_flag<V, 4><<<grid, kBlock, 0, s>>>(n, pos, crd, vals, x, y, t.row, t.pos,
                                                       t.ntiles, stride, carry);
        else
            k_spmv_flag<V, 8><<<grid, kBlock, 0, s>>>(n, pos, crd, vals, x, y, t.row, t.pos,
                                                       t.ntiles, stride, carry);
        return hipGetLastError();
    }
    if (exact) {
        if (items <= 4)
            k_spmv_pipe<V, 4><<<grid, kBlock, 0, s>>>(n, pos, crd, vals, x, y, t.row, t.pos,
                                                       t.ntiles, stride, carry);
        else
            k_spmv_pipe<V, 8><<<grid, kBlock, 0, s>>>(n, pos, crd, vals, x, y, t.row, t.pos,
                                                       t.ntiles, stride, carry);
        return hipGetLastError();
    }
    if (items <= 4)
        k_spmv_tiles<V, 4><<<grid, kBlock, 0, s>>>(n, pos, crd, vals, x, y, t.row, t.pos,
                                                    t.ntiles, stride, carry);
    else
        k_spmv_tiles<V, 8><<<grid, kBlock, 0, s>>>(n, pos, crd, vals, x, y, t.row, t.pos,
                                                    t.ntiles, stride, carry);
    return hipGetLastError();
}

template <typename V>
hipError_t spmv_fixup_dispatch(int64_t n, const Tiles &t, int64_t stride, const double *carry,
                               V *y, hipStream_t s) {
    return launch_carry_fixup<V, double>(n, 1, t.row, t.ntiles, stride, ceil_div(t.ntiles, stride),
                                         carry, y, 1, s);
}

}  // namespace

hipError_t launch_spmv_fixup(int dtype, int64_t n, const Tiles &t, int64_t stride,
                             const double *carry, void *y, hipStream_t s) {
    if (dtype == SPL_F64)
        return spmv_fixup_dispatch<double>(n, t, stride, carry, static_cast<double *>(y), s);
    return spmv_fixup_dispatch<float>(n, t, stride, carry, static_cast<float *>(y), s);
}

hipError_t launch_spmv_row(int dtype, int lanes, int64_t n, const int32_t *pos_b,
                           const int32_t *pos_e, const int32_t *crd, const void *vals,
                           const void *x, void *y, hipStream_t s) {
    if (!pos_e) pos_e = pos_b + 1;  // CSR: row i ends where row i + 1 begins
    if (dtype == SPL_F64)
        return spmv_row_dispatch<double>(lanes, n, pos_b, pos_e, crd,
                                         static_cast<const double *>(vals),
                                         static_cast<const double *>(x), static_cast<double *>(y), s);
    return spmv_row_dispatch<float>(lanes, n, pos_b, pos_e, crd, static_cast<const float *>(vals),
                                    static_cast<const float *>(x), static_cast<float *>(y), s);
}

hipError_t launch_spmv_window_merge(int dtype, int items, int64_t n, const int32_t *vpos,
                                    const int32_t *begin, const int32_t *crd, const void *vals,
                                    const void *x, void *y, const Tiles &t, int64_t stride,
                                    double *carry, hipStream_t s) {
    dim3 grid(static_cast<unsigned>(ceil_div(t.ntiles, stride)));
    auto go = [&](auto *v, auto *xx, auto *yy) {
        using V = std::remove_const_t<std::remove_pointer_t<decltype(v)>>;
        if (items <= 4)
            k_spmv_window_flag<V, 4><<<grid, kBlock, 0, s>>>(n, vpos, begin, crd, v, xx, yy, t.row,
                                                             t.pos, t.ntiles, stride, carry);
        else
            k_spmv_window_flag<V, 8><<<grid, kBlock, 0, s>>>(n, vpos, begin, crd, v, xx, yy, t.row,
                                                             t.pos, t.ntiles, stride, carry);
        return hipGetLastError();
    };
    if (dtype == SPL_F64)
        return go(static_cast<const double *>(vals), static_cast<const double *>(x),
                  static_cast<double *>(y));
    return go(static_cast<const float *>(vals), static_cast<const float *>(x),
              static_cast<float *>(y));
}

hipError_t launch_spmv_flag64(int dtype, int items, int64_t n, const int64_t *pos,
                              const int32_t *crd, const void *vals, const void *x, void *y,
                              const Tiles &t, int64_t stride, double *carry, hipStream_t s) {
    dim3 grid(static_cast<unsigned>(ceil_div(t.ntiles, stride)));
    auto go = [&](auto *v, auto *xx, auto *yy) {
        using V = std::remove_const_t<std::remove_pointer_t<decltype(v)>>;
        if (items <= 4)
            k_spmv_flag<V, 4, int64_t, int64_t><<<grid, kBlock, 0, s>>>(
                n, pos, crd, v, xx, yy, t.row, t.pos64, t.ntiles, stride, carry);
        else
            k_spmv_flag<V, 8, int64_t, int64_t><<<grid, kBlock, 0, s>>>(
                n, pos, crd, v, xx, yy, t.row, t.pos64, t.ntiles, stride, carry);
        return hipGetLastError();
    };
    if (dtype == SPL_F64)
        return go(static_cast<const double *>(vals), static_cast<const double *>(x),
                  static_cast<double *>(y));
    return go(static_cast<const float *>(vals), static_cast<const float *>(x),
              static_cast<float *>(y));
}

hipError_t launch_spmv_tiles(int dtype, int items, int64_t n, const int32_t *pos,
                             const int32_t *crd, const void *vals, const void *x, void *y,
                             const Tiles &t, int64_t stride, bool exact_chunks, int variant,
                             double *carry, hipStream_t s) {
    if (dtype == SPL_F64)
        return spmv_tiles_dispatch<double>(items, n, pos, crd, static_cast<const double *>(vals),
                                           static_cast<const double *>(x),
                                           static_cast<double *>(y), t, stride, exact_chunks,
                                           variant, carry, s);
    return spmv_tiles_dispatch<float>(items, n, pos, crd, static_cast<const float *>(vals),
                                      static_cast<const float *>(x), static_cast<float *>(y), t,
                                      stride, exact_chunks, variant, carry, s);
}

}  // namespace spl
