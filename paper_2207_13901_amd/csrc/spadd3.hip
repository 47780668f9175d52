// SpAdd3 leaf  A(i,j) = B(i,j) + C(i,j) + D(i,j)  for CSR operands (paper
// Sec. VI-A), fused so no pairwise intermediate is built, with the output
// assembled in two phases (Sec. V-B): a symbolic phase counts the union of
// the three coordinate lists of every row and an exclusive scan turns the
// counts into A.pos; the numeric phase writes A.crd and A.vals at those
// positions with no synchronization between rows.  Row split only: the
// non-zero split does not apply to a sum of CSR operands (Sec. VI-A, CPU
// results).
//
// One lane per row merges the three sorted coordinate lists; values are
// summed in operand order B, C, D over the operands present (a cancellation
// to zero keeps its coordinate).  The scan is three passes: per-workgroup
// totals, one workgroup scanning the totals, per-workgroup rescan.  The
// symbolic phase copies the workgroup's input coordinates to LDS with
// coalesced loads first, and the numeric phase stages the output in LDS so
// that its stores are coalesced: one lane per row reading or storing
// straight to HBM keeps far more partly used lines open than the caches
// hold.
#include "device.hpp"
#include "internal.hpp"

namespace spl {
namespace {

constexpr int kScanItems = 16;
constexpr int kScanTile = kBlock * kScanItems;

struct Csr3 {
    const int32_t *bp, *bc, *cp, *cc, *dp, *dc;
};

// Where a workgroup reads the three operands' coordinates from: the
// operands themselves, or an LDS copy of the workgroup's ranges (element q
// of operand X at x[q - ox]).
struct Crd3 {
    const int32_t *b, *c, *d;
    int32_t ob, oc, od;
};

// Where a workgroup reads the three operands' values from (as Crd3).
template <typename V>
struct Vals3 {
    const V *b, *c, *d;
    int32_t ob, oc, od;
};

// Three-way merge of one row's sorted coordinate lists, resumable: next()
// yields the union's coordinates in increasing order; with values, the sum
// over the operands present in operand order B, C, D.
struct Merge3 {
    static constexpr int32_t kInf = 0x7fffffff;
    int32_t a, ae, b, be, d, de, xa, xb, xd;

    __device__ __forceinline__ Merge3(const Csr3 &m, const Crd3 &x, int64_t i) {
        a = m.bp[i];
        ae = m.bp[i + 1];
        b = m.cp[i];
        be = m.cp[i + 1];
        d = m.dp[i];
        de = m.dp[i + 1];
        xa = a < ae ? x.b[a - x.ob] : kInf;
        xb = b < be ? x.c[b - x.oc] : kInf;
        xd = d < de ? x.d[d - x.od] : kInf;
    }

    __device__ __forceinline__ bool done() const { return min(xa, min(xb, xd)) == kInf; }

    // Advance past the smallest remaining coordinate c; returns c.  Values
    // of operand X at position q are read at vals.X[q - vals.oX].
    template <bool kValues, typename V>
    __device__ __forceinline__ int32_t next(const Crd3 &x, const Vals3<V> &v, V &sum) {
        const int32_t c = min(xa, min(xb, xd));
        V s = 0;
        if (xa == c) {
            if (kValues) s = v.b[a - v.ob];
            ++a;
            xa = a < ae ? x.b[a - x.ob] : kInf;
        }
        if (xb == c) {
            if (kValues) s = s + v.c[b - v.oc];
            ++b;
            xb = b < be ? x.c[b - x.oc] : kInf;
        }
        if (xd == c) {
            if (kValues) s = s + v.d[d - v.od];
            ++d;
            xd = d < de ? x.d[d - x.od] : kInf;
        }
        sum = s;
        return c;
    }
};

// Coordinates of the workgroup's rows [r0, r1) per operand staged in LDS.
// One lane per row reading its row straight from HBM keeps a few lines per
// lane open at once, more than the L1 and L2 hold, so lines are fetched
// several times; the coalesced copy reads each once.  When an operand's run
// exceeds kStageCap the workgroup reads the operands directly.
constexpr int kStageCap = 2560;

__device__ __forceinline__ Crd3 stage_crd(const Csr3 &m, int64_t r0, int64_t r1,
                                          int32_t (*s_x)[kStageCap]) {
    const int32_t b0 = m.bp[r0], c0 = m.cp[r0], d0 = m.dp[r0];
    const int32_t nb = m.bp[r1] - b0, nc = m.cp[r1] - c0, nd = m.dp[r1] - d0;
    if (nb > kStageCap || nc > kStageCap || nd > kStageCap) return Crd3{m.bc, m.cc, m.dc, 0, 0, 0};
    for (int k = threadIdx.x; k < nb; k += kBlock) s_x[0][k] = m.bc[b0 + k];
    for (int k = threadIdx.x; k < nc; k += kBlock) s_x[1][k] = m.cc[c0 + k];
    for (int k = threadIdx.x; k < nd; k += kBlock) s_x[2][k] = m.dc[d0 + k];
    __syncthreads();
    return Crd3{s_x[0], s_x[1], s_x[2], b0, c0, d0};
}

__global__ __launch_bounds__(kBlock) void k_spadd3_count(int64_t n, Csr3 m, int32_t *apos) {
    __shared__ int32_t s_x[3][kStageCap];
    const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kBlock;
    const int64_t r1 = r0 + kBlock < n ? r0 + kBlock : n;
    const int64_t i = r0 + threadIdx.x;
    const Crd3 x = stage_crd(m, r0, r1, s_x);
    if (i == 0) apos[0] = 0;
    if (i >= n) return;
    Merge3 mg(m, x, i);
    int32_t k = 0;
    float unused;
    const Vals3<float> none{nullptr, nullptr, nullptr, 0, 0, 0};
    while (!mg.done()) {
        mg.next<false, float>(x, none, unused);
        ++k;
    }
    apos[i + 1] = k;
}

// Numeric phase.  The 256 rows of a workgroup own one contiguous run of the
// output, [apos[r0], apos[r0 + 256]), written in windows of kFillCap
// entries: in each window every lane continues its row's merge from where
// it stopped, emitting into LDS the entries whose output index falls in the
// window, and the workgroup then writes the window with coalesced stores.
// Each row is merged once whatever its length; only one row's lane works
// in the windows a long row fills alone.  The inputs are read directly:
// staging them as well would halve the workgroups per CU, which costs more
// than the repeated line fetches it saves.
constexpr int kFillCap = 2048;

// STAGE 0: inputs read directly; 1: the workgroup's coordinate runs staged
// in LDS (as the count phase does); 2: coordinates and values staged, with a
// smaller output window.  Runs longer than kStageCap fall back to direct
// reads for the whole workgroup.
template <typename V, int STAGE>
__global__ __launch_bounds__(kBlock) void k_spadd3_fill(int64_t n, Csr3 m, const V *bv,
                                                        const V *cv, const V *dv,
                                                        const int32_t *apos, int32_t *acrd,
                                                        V *aval) {
    constexpr int kWin = STAGE == 2 ? 1024 : kFillCap;
    __shared__ int32_t s_crd[kWin];
    __shared__ V s_val[kWin];
    __shared__ int32_t s_x[STAGE ? 3 : 1][STAGE ? kStageCap : 1];
    __shared__ V s_v[STAGE == 2 ? 3 : 1][STAGE == 2 ? kStageCap : 1];
    const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kBlock;
    const int64_t r1 = r0 + kBlock < n ? r0 + kBlock : n;
    const int64_t i = r0 + threadIdx.x;
    Crd3 x{m.bc, m.cc, m.dc, 0, 0, 0};
    Vals3<V> vv{bv, cv, dv, 0, 0, 0};
    if constexpr (STAGE > 0) {
        const int32_t b0 = m.bp[r0], c0 = m.cp[r0], d0 = m.dp[r0];
        const int32_t nb = m.bp[r1] - b0, nc = m.cp[r1] - c0, nd = m.dp[r1] - d0;
        if (nb <= kStageCap && nc <= kStageCap && nd <= kStageCap) {
            for (int k = threadIdx.x; k < nb; k += kBlock) s_x[0][k] = m.bc[b0 + k];
            for (int k = threadIdx.x; k < nc; k += kBlock) s_x[1][k] = m.cc[c0 + k];
            for (int k = threadIdx.x; k < nd; k += kBlock) s_x[2][k] = m.dc[d0 + k];
            x = Crd3{s_x[0], s_x[1], s_x[2], b0, c0, d0};
            if constexpr (STAGE == 2) {
                for (int k = threadIdx.x; k < nb; k += kBlock) s_v[0][k] = bv[b0 + k];
                for (int k = threadIdx.x; k < nc; k += kBlock) s_v[1][k] = cv[c0 + k];
                for (int k = threadIdx.x; k < nd; k += kBlock) s_v[2][k] = dv[d0 + k];
                vv = Vals3<V>{s_v[0], s_v[1], s_v[2], b0, c0, d0};
            }
            __syncthreads();
        }
    }
    const int64_t base = apos[r0];
    const int64_t total = apos[r1] - base;
    const bool mine = i < n;
    int64_t k = mine ? apos[i] - base : 0;
    const int64_t hi = mine ? apos[i + 1] - base : 0;
    Merge3 mg(m, x, mine ? i : r0);
    for (int64_t w = 0; w < total; w += kWin) {
        const int64_t we = w + kWin < total ? w + kWin : total;
        for (; k < hi && k < we; ++k) {
            V sum;
            const int32_t c = mg.next<true, V>(x, vv, sum);
            s_crd[k - w] = c;
            s_val[k - w] = sum;
        }
        __syncthreads();
        for (int64_t q = threadIdx.x; q < we - w; q += kBlock) {
            store_stream(acrd + base + w + q, s_crd[q]);
            store_stream(aval + base + w + q, s_val[q]);
        }
        __syncthreads();
    }
}

// Element i of the scanned sequence: x[i], or with window bounds the window
// length max(end[i] - begin[i], 0).
__device__ __forceinline__ int32_t scan_value(const int32_t *x, const int32_t *begin,
                                              const int32_t *end, int64_t i) {
    if (!begin) return x[i];
    const int32_t len = end[i] - begin[i];
    return len > 0 ? len : 0;
}

// Block sums of the sequence's elements [0, n) in tiles of kScanTile.
__global__ __launch_bounds__(kBlock) void k_scan_tile_sums(int64_t n, const int32_t *x,
                                                           const int32_t *begin,
                                                           const int32_t *end,
                                                           int64_t *tile_sum) {
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile;
    int64_t acc = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const int64_t i = base + j * kBlock + threadIdx.x;
        if (i < n) acc += scan_value(x, begin, end, i);
    }
    __shared__ int64_t s[kBlock];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = s[0];
}

// Exclusive scan of the tile sums by one workgroup; total to *total.
__global__ __launch_bounds__(kBlock) void k_scan_tile_prefix(int64_t ntiles, int64_t *tile_sum,
                                                             int64_t *total) {
    __shared__ int64_t s[kBlock];
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < ntiles; b0 += kBlock) {
        const int64_t i = b0 + threadIdx.x;
        const int64_t v = i < ntiles ? tile_sum[i] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < kBlock; off <<= 1) {
            const int64_t add = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
            __syncthreads();
            s[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < ntiles) tile_sum[i] = carry + s[threadIdx.x] - v;
        carry += s[kBlock - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

// x[i] <- tile prefix + inclusive scan within the tile, i.e. with x =
// counts at apos + 1 this leaves apos[i+1] = sum of counts[0..i] (in place;
// with window bounds the values are the window lengths instead of x).  The
// tile goes through LDS so that the loads and stores are coalesced; each
// thread scans 16 consecutive elements there (padded: element e at
// e + e / 16, so the threads' runs fall in different banks).
__global__ __launch_bounds__(kBlock) void k_scan_tile_apply(int64_t n, int32_t *x,
                                                            const int32_t *begin,
                                                            const int32_t *end,
                                                            const int64_t *tile_sum,
                                                            int32_t *head) {
    if (head && blockIdx.x == 0 && threadIdx.x == 0) *head = 0;  // the leading 0 of a pos array
    constexpr int kPad = kScanTile + kScanTile / kScanItems;
    __shared__ int64_t s_v[kPad];
    __shared__ int64_t s[kBlock];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const int e = j * kBlock + threadIdx.x;
        const int64_t i = base + e;
        s_v[e + e / kScanItems] = i < n ? scan_value(x, begin, end, i) : 0;
    }
    __syncthreads();
    const int e0 = threadIdx.x * kScanItems;
    const int p0 = e0 + e0 / kScanItems;  // this thread's run, unpadded inside
    int64_t run = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        run += s_v[p0 + j];
        s_v[p0 + j] = run;
    }
    s[threadIdx.x] = run;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        const int64_t add = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += add;
        __syncthreads();
    }
    const int64_t before = tile_sum[blockIdx.x] + s[threadIdx.x] - run;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) s_v[p0 + j] += before;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const int e = j * kBlock + threadIdx.x;
        const int64_t i = base + e;
        if (i < n) x[i] = static_cast<int32_t>(s_v[e + e / kScanItems]);
    }
}

}  // namespace

int64_t spadd3_scan_tiles(int64_t n) { return ceil_div(n > 0 ? n : 1, kScanTile); }

hipError_t launch_window_offsets(int64_t n, const int32_t *begin, const int32_t *end,
                                 int32_t *vpos, int64_t *tile_sum, int64_t *total, hipStream_t s) {
    // vpos[0] = 0 and vpos[1..n] the inclusive scan of the window lengths
    const int64_t nt = spadd3_scan_tiles(n);
    k_scan_tile_sums<<<dim3(static_cast<unsigned>(nt)), kBlock, 0, s>>>(n, nullptr, begin, end,
                                                                        tile_sum);
    hipError_t e;
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_scan_tile_prefix<<<1, kBlock, 0, s>>>(nt, tile_sum, total);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_scan_tile_apply<<<dim3(static_cast<unsigned>(nt)), kBlock, 0, s>>>(n, vpos + 1, begin, end,
                                                                         tile_sum, vpos);
    return hipGetLastError();
}

hipError_t launch_pos_scan(int64_t n, int32_t *apos, int64_t *tile_sum, int64_t *total,
                           hipStream_t s) {
    // apos[1..n] hold counts: scanned in place, apos[0] = 0
    const int64_t nt = spadd3_scan_tiles(n);
    k_scan_tile_sums<<<dim3(static_cast<unsigned>(nt)), kBlock, 0, s>>>(n, apos + 1, nullptr,
                                                                        nullptr, tile_sum);
    hipError_t e;
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_scan_tile_prefix<<<1, kBlock, 0, s>>>(nt, tile_sum, total);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_scan_tile_apply<<<dim3(static_cast<unsigned>(nt)), kBlock, 0, s>>>(n, apos + 1, nullptr,
                                                                         nullptr, tile_sum, apos);
    return hipGetLastError();
}

hipError_t launch_spadd3_symbolic(int64_t n, const int32_t *bp, const int32_t *bc,
                                  const int32_t *cp, const int32_t *cc, const int32_t *dp,
                                  const int32_t *dc, int32_t *apos, int64_t *tile_sum,
                                  int64_t *total, hipStream_t s) {
    Csr3 m{bp, bc, cp, cc, dp, dc};
    const int64_t rows_grid = ceil_div(n > 0 ? n : 1, kBlock);
    k_spadd3_count<<<dim3(static_cast<unsigned>(rows_grid)), kBlock, 0, s>>>(n, m, apos);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nt = spadd3_scan_tiles(n);
    k_scan_tile_sums<<<dim3(static_cast<unsigned>(nt)), kBlock, 0, s>>>(n, apos + 1, nullptr,
                                                                        nullptr, tile_sum);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_scan_tile_prefix<<<1, kBlock, 0, s>>>(nt, tile_sum, total);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_scan_tile_apply<<<dim3(static_cast<unsigned>(nt)), kBlock, 0, s>>>(n, apos + 1, nullptr,
                                                                         nullptr, tile_sum, nullptr);
    return hipGetLastError();
}

template <typename V>
hipError_t spadd3_fill(int stage, int64_t n, const Csr3 &m, const void *bv, const void *cv,
                       const void *dv, const int32_t *apos, int32_t *acrd, void *aval,
                       hipStream_t s) {
    dim3 grid(static_cast<unsigned>(ceil_div(n, kBlock)));
    auto go = [&](auto kern) {
        kern<<<grid, kBlock, 0, s>>>(n, m, static_cast<const V *>(bv), static_cast<const V *>(cv),
                                     static_cast<const V *>(dv), apos, acrd, static_cast<V *>(aval));
        return hipGetLastError();
    };
    if (stage == 1) return go(k_spadd3_fill<V, 1>);
    if (stage == 2) return go(k_spadd3_fill<V, 2>);
    return go(k_spadd3_fill<V, 0>);
}

hipError_t launch_spadd3_numeric(int vtype, int64_t n, const int32_t *bp, const int32_t *bc,
                                 const void *bv, const int32_t *cp, const int32_t *cc,
                                 const void *cv, const int32_t *dp, const int32_t *dc,
                                 const void *dv, const int32_t *apos, int32_t *acrd, void *aval,
                                 int stage, hipStream_t s) {
    Csr3 m{bp, bc, cp, cc, dp, dc};
    if (n == 0) return hipSuccess;
    if (vtype == SPL_F64) return spadd3_fill<double>(stage, n, m, bv, cv, dv, apos, acrd, aval, s);
    return spadd3_fill<float>(stage, n, m, bv, cv, dv, apos, acrd, aval, s);
}

}  // namespace spl
