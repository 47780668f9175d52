// Transposition of a (Dense, Compressed) matrix: the CSR arrays of B^T from
// those of B.  The format language stores CSC as (Dense, Compressed) over
// the reversed dimension order (Sec. II-B), so a CSC matrix A is the CSR of
// A^T and this call turns it into A's CSR, on which every CSR leaf runs.
//
// Entries are read in B's order, sorted by (row, column), and stably sorted
// by column with an LSD radix sort of 8-bit digits: a stable sort by column
// of a row-major sequence is the column-major sequence, i.e. B^T's CSR with
// rows sorted.  Each pass cuts the sequence into tiles of 4,096 entries;
// k_radix_counts counts the tile's digits (LDS integer counters), one scan
// over the digit-major count matrix gives every (digit, tile) its output
// offset, and k_radix_scatter ranks every entry among the tile's entries of
// its digit in sequence order -- in rounds of 256 consecutive entries,
// wave-level digit matching by ballots, the four waves' counts through LDS
// -- and writes it at offset + rank.  Integer only, no order-dependent
// atomics: the result is deterministic and bit-exact.  k_transpose_emit then
// writes B^T's pos (from the sorted columns), crd (the source rows, by a
// binary search of each source position in B's pos) and vals.
#include "device.hpp"
#include "internal.hpp"

namespace spl {
namespace {

constexpr int kRadixBits = 8;
constexpr int kDigits = 1 << kRadixBits;
constexpr int kRounds = 16;
constexpr int kRadixTile = kBlock * kRounds;  // 4,096 entries per tile

__device__ __forceinline__ int digit_of(int32_t key, int shift) {
    return (static_cast<uint32_t>(key) >> shift) & (kDigits - 1);
}

// counts[1 + d * ntiles + t] = number of entries of tile t with digit d
// (the leading slot is the scan's), keys from `keys` or, on the first pass,
// from crd directly.
__global__ __launch_bounds__(kBlock) void k_radix_counts(int64_t n, const int32_t *__restrict__ keys,
                                                         int shift, int64_t ntiles,
                                                         int32_t *__restrict__ counts) {
    __shared__ int32_t s_cnt[kDigits];
    s_cnt[threadIdx.x] = 0;  // kBlock == kDigits
    __syncthreads();
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kRadixTile;
#pragma unroll 4
    for (int r = 0; r < kRounds; ++r) {
        const int64_t e = base + r * kBlock + threadIdx.x;
        if (e < n) atomicAdd(&s_cnt[digit_of(keys[e], shift)], 1);
    }
    __syncthreads();
    counts[1 + static_cast<int64_t>(threadIdx.x) * ntiles + blockIdx.x] = s_cnt[threadIdx.x];
}

// Stable scatter of one pass: entry e of the tile goes to
// offsets[d * ntiles + t] + (entries of digit d before e in the tile).
// vals_in == nullptr on the first pass: the payload is the entry's index.
__global__ __launch_bounds__(kBlock) void k_radix_scatter(
    int64_t n, const int32_t *__restrict__ keys_in, const int32_t *__restrict__ vals_in,
    int shift, int64_t ntiles, const int32_t *__restrict__ offsets,
    int32_t *__restrict__ keys_out, int32_t *__restrict__ vals_out) {
    __shared__ int32_t s_base[kDigits];        // tile offset + entries placed so far
    __shared__ int32_t s_wcnt[kBlock / kWave][kDigits];
    const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    s_base[tid] = offsets[static_cast<int64_t>(tid) * ntiles + blockIdx.x];
    const uint64_t lt = lane ? (~0ull >> (kWave - lane)) : 0ull;  // lanes below this one
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kRadixTile;
    for (int r = 0; r < kRounds; ++r) {
#pragma unroll
        for (int w = 0; w < kBlock / kWave; ++w) s_wcnt[w][tid] = 0;
        __syncthreads();  // also orders s_base's updates of the previous round
        const int64_t e = base + r * kBlock + tid;
        const bool valid = e < n;
        const int32_t key = valid ? keys_in[e] : 0;
        const int32_t val = valid ? (vals_in ? vals_in[e] : static_cast<int32_t>(e)) : 0;
        const int d = digit_of(key, shift);
        // lanes of this wave holding the same digit
        uint64_t same = __ballot(valid);
#pragma unroll
        for (int b = 0; b < kRadixBits; ++b) {
            const uint64_t ones = __ballot(valid && ((d >> b) & 1));
            same &= ((d >> b) & 1) ? ones : ~ones;
        }
        const int before = __popcll(same & lt);
        if (valid && before == 0) s_wcnt[wave][d] = __popcll(same);
        __syncthreads();
        if (valid) {
            int rank = s_base[d] + before;
            for (int w = 0; w < wave; ++w) rank += s_wcnt[w][d];
            keys_out[rank] = key;
            vals_out[rank] = val;
        }
        __syncthreads();
        int add = 0;
#pragma unroll
        for (int w = 0; w < kBlock / kWave; ++w) add += s_wcnt[w][tid];
        s_base[tid] += add;
    }
}

// B^T's arrays from the sorted (column, source position) pairs: pos[c] is
// the first output position of column c (columns without entries repeat
// the next one's), crd the source row, vals the source value.
template <typename V>
__global__ __launch_bounds__(kBlock) void k_transpose_emit(
    int64_t n, int64_t m, int64_t nnz, const int32_t *__restrict__ pos,
    const int32_t *__restrict__ keys, const int32_t *__restrict__ src, const V *__restrict__ vals,
    int32_t *__restrict__ tpos, int32_t *__restrict__ tcrd, V *__restrict__ tvals) {
    const int64_t q = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (q >= nnz) return;
    const int32_t c = keys[q];
    const int32_t prev = q ? keys[q - 1] : -1;
    for (int64_t k = prev + 1; k <= c; ++k) tpos[k] = static_cast<int32_t>(q);
    if (q == nnz - 1)
        for (int64_t k = c + 1; k <= m; ++k) tpos[k] = static_cast<int32_t>(nnz);
    const int32_t p = src[q];
    // the row holding position p: the last i with pos[i] <= p
    int64_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (pos[mid] <= p)
            lo = mid;
        else
            hi = mid;
    }
    tcrd[q] = static_cast<int32_t>(lo);
    tvals[q] = vals[p];
}

__global__ __launch_bounds__(kBlock) void k_fill_zero(int64_t count, int32_t *__restrict__ out) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i < count) out[i] = 0;
}

}  // namespace

int transpose_passes(int64_t m) {
    int bits = 0;
    while (bits < 31 && (static_cast<int64_t>(1) << bits) < m) ++bits;
    return bits ? (bits + kRadixBits - 1) / kRadixBits : 1;
}

size_t transpose_ws_bytes(int64_t nnz, int64_t m) {
    auto up = [](size_t v) { return (v + 255) & ~static_cast<size_t>(255); };
    const int64_t tiles = ceil_div(nnz > 0 ? nnz : 1, kRadixTile);
    const int64_t cells = tiles * kDigits;
    (void)m;
    return 4 * up(static_cast<size_t>(nnz > 0 ? nnz : 1) * 4) +
           up(static_cast<size_t>(cells + 1) * 4) +
           up(static_cast<size_t>(spadd3_scan_tiles(cells)) * 8) + up(8);
}

hipError_t launch_transpose(int vtype, int64_t n, int64_t m, int64_t nnz, const int32_t *pos,
                            const int32_t *crd, const void *vals, int32_t *tpos, int32_t *tcrd,
                            void *tvals, void *ws, hipStream_t s) {
    hipError_t e;
    if (nnz == 0) {
        k_fill_zero<<<dim3(static_cast<unsigned>(ceil_div(m + 1, kBlock))), kBlock, 0, s>>>(m + 1,
                                                                                          tpos);
        return hipGetLastError();
    }
    auto up = [](size_t v) { return (v + 255) & ~static_cast<size_t>(255); };
    char *w = static_cast<char *>(ws);
    int32_t *k0 = reinterpret_cast<int32_t *>(w);
    w += up(static_cast<size_t>(nnz) * 4);
    int32_t *v0 = reinterpret_cast<int32_t *>(w);
    w += up(static_cast<size_t>(nnz) * 4);
    int32_t *k1 = reinterpret_cast<int32_t *>(w);
    w += up(static_cast<size_t>(nnz) * 4);
    int32_t *v1 = reinterpret_cast<int32_t *>(w);
    w += up(static_cast<size_t>(nnz) * 4);
    const int64_t tiles = ceil_div(nnz, kRadixTile);
    const int64_t cells = tiles * kDigits;
    int32_t *counts = reinterpret_cast<int32_t *>(w);
    w += up(static_cast<size_t>(cells + 1) * 4);
    int64_t *tile_sum = reinterpret_cast<int64_t *>(w);
    w += up(static_cast<size_t>(spadd3_scan_tiles(cells)) * 8);
    int64_t *total = reinterpret_cast<int64_t *>(w);

    const int passes = transpose_passes(m);
    const int32_t *kin = crd;
    const int32_t *vin = nullptr;
    int32_t *kout = k0, *vout = v0;
    const dim3 grid(static_cast<unsigned>(tiles));
    for (int pass = 0; pass < passes; ++pass) {
        const int shift = pass * kRadixBits;
        k_radix_counts<<<grid, kBlock, 0, s>>>(nnz, kin, shift, tiles, counts);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = launch_pos_scan(cells, counts, tile_sum, total, s)) != hipSuccess) return e;
        k_radix_scatter<<<grid, kBlock, 0, s>>>(nnz, kin, vin, shift, tiles, counts, kout, vout);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        kin = kout;
        vin = vout;
        kout = kout == k0 ? k1 : k0;
        vout = vout == v0 ? v1 : v0;
    }
    const dim3 eg(static_cast<unsigned>(ceil_div(nnz, kBlock)));
    if (vtype == SPL_F64)
        k_transpose_emit<double><<<eg, kBlock, 0, s>>>(n, m, nnz, pos, kin, vin,
                                                        static_cast<const double *>(vals), tpos,
                                                        tcrd, static_cast<double *>(tvals));
    else if (vtype == SPL_F32)
        k_transpose_emit<float><<<eg, kBlock, 0, s>>>(n, m, nnz, pos, kin, vin,
                                                       static_cast<const float *>(vals), tpos, tcrd,
                                                       static_cast<float *>(tvals));
    else
        k_transpose_emit<bf16><<<eg, kBlock, 0, s>>>(n, m, nnz, pos, kin, vin,
                                                      static_cast<const bf16 *>(vals), tpos, tcrd,
                                                      static_cast<bf16 *>(tvals));
    return hipGetLastError();
}

}  // namespace spl
