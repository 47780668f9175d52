// SpAdd3 leaf  A(i,j) = B(i,j) + C(i,j) + D(i,j)  for CSR operands (paper
// Sec. VI-A), fused so no pairwise intermediate is built, with the output
// assembled in two phases (Sec. V-B): a symbolic phase counts the union of
// the three coordinate lists of every row and an exclusive scan turns the
// counts into A.pos; the numeric phase writes A.crd and A.vals at those
// positions with no synchronization between rows.  Row split only: the
// non-zero split does not apply to a sum of CSR operands (Sec. VI-A, CPU
// results).
//
// Values are summed in operand order B, C, D over the operands present (a
// cancellation to zero keeps its coordinate).  The symbolic phase copies
// the workgroup's input coordinates to LDS with coalesced loads, and one
// lane per row merges the three sorted coordinate lists there to count the
// union.  The scan is three passes: per-workgroup totals, one workgroup
// scanning the totals, per-workgroup rescan.  The numeric phase's default
// form works by ranks: with the coordinates staged, every input entry finds
// its own output slot by binary search in the other operands' rows, so the
// work is spread over all lanes and every input line is read with coalesced
// loads.  The merge forms (one lane per row, output staged in LDS windows
// so that its stores are coalesced) remain as schedule variants: one lane
// per row reading or storing straight to HBM keeps far more partly used
// lines open than the caches hold, and a window is filled only by the lanes
// whose rows reach into it.
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

// Copies three runs of n3[X] <= PER * kBlock consecutive coordinates from
// src[X] to dst[X] in LDS.  Every lane issues all its loads before any store
// (past a run: 0, with no access), so the copy costs one memory round trip,
// not one per loop iteration.
template <int PER>
__device__ __forceinline__ void stage3(const int32_t *const *src, const int32_t *n3,
                                       int32_t *const *dst) {
    const int t = threadIdx.x;
    uint32_t v[3][PER];
#pragma unroll
    for (int X = 0; X < 3; ++X) {
        const __amdgpu_buffer_rsrc_t rc = span_rsrc(src[X], 4u * n3[X]);
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int k = j * kBlock + t;
            v[X][j] = buf_u32(rc, k < n3[X] ? 4u * k : kBufOut);
        }
    }
#pragma unroll
    for (int X = 0; X < 3; ++X)
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int k = j * kBlock + t;
            if (k < n3[X]) dst[X][k] = static_cast<int32_t>(v[X][j]);
        }
}

// Coordinates of the workgroup's rows [r0, r1) per operand staged in LDS.
// One lane per row reading its row straight from HBM keeps a few lines per
// lane open at once, more than the L1 and L2 hold, so lines are fetched
// several times; the coalesced copy reads each once.  When an operand's run
// exceeds kStageCap the workgroup reads the operands directly.
constexpr int kStageCap = 2560;

// Stages the coordinate runs of rows [r0, r1) when each fits kStageCap and
// returns whether it did (then with the workgroup synchronized); first3
// gets the runs' first positions.
__device__ __forceinline__ bool stage_crd(const Csr3 &m, int64_t r0, int64_t r1,
                                          int32_t (*s_x)[kStageCap], int32_t *first3) {
    first3[0] = m.bp[r0];
    first3[1] = m.cp[r0];
    first3[2] = m.dp[r0];
    const int32_t n3[3] = {m.bp[r1] - first3[0], m.cp[r1] - first3[1], m.dp[r1] - first3[2]};
    if (n3[0] > kStageCap || n3[1] > kStageCap || n3[2] > kStageCap) return false;
    const int32_t *src[3] = {m.bc + first3[0], m.cc + first3[1], m.dc + first3[2]};
    int32_t *dst[3] = {s_x[0], s_x[1], s_x[2]};
    stage3<kStageCap / kBlock>(src, n3, dst);
    __syncthreads();
    return true;
}

// Union size of row i's coordinate lists read through x (HBM).
__device__ __forceinline__ int32_t union_count(const Csr3 &m, const Crd3 &x, int64_t i) {
    Merge3 mg(m, x, i);
    int32_t k = 0;
    float unused;
    const Vals3<float> none{nullptr, nullptr, nullptr, 0, 0, 0};
    while (!mg.done()) {
        mg.next<false, float>(x, none, unused);
        ++k;
    }
    return k;
}

// The same from the staged runs s_x (first positions f), without branches:
// each step takes the smallest head, advances every list holding it and
// reads all three heads again at indices clamped into the stage, so a step
// is one round of LDS reads instead of up to three behind lane-masked
// branches.
__device__ __forceinline__ int32_t union_count_staged(const Csr3 &m, int32_t (*s_x)[kStageCap],
                                                      const int32_t *f, int64_t i) {
    constexpr int32_t kInf = Merge3::kInf;
    int32_t p[3] = {m.bp[i] - f[0], m.cp[i] - f[1], m.dp[i] - f[2]};
    const int32_t e[3] = {m.bp[i + 1] - f[0], m.cp[i + 1] - f[1], m.dp[i + 1] - f[2]};
    auto head = [&](int X) {
        const int32_t q = p[X] < kStageCap ? p[X] : kStageCap - 1;
        const int32_t v = s_x[X][q];
        return p[X] < e[X] ? v : kInf;
    };
    int32_t h[3] = {head(0), head(1), head(2)};
    int32_t k = 0;
    while (min(h[0], min(h[1], h[2])) != kInf) {
        const int32_t c = min(h[0], min(h[1], h[2]));
#pragma unroll
        for (int X = 0; X < 3; ++X) p[X] += h[X] == c ? 1 : 0;
#pragma unroll
        for (int X = 0; X < 3; ++X) h[X] = head(X);
        ++k;
    }
    return k;
}

__global__ __launch_bounds__(kBlock) void k_spadd3_count(int64_t n, Csr3 m, int32_t *apos) {
    __shared__ int32_t s_x[3][kStageCap];
    const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kBlock;
    const int64_t r1 = r0 + kBlock < n ? r0 + kBlock : n;
    const int64_t i = r0 + threadIdx.x;
    int32_t f[3];
    const bool staged = stage_crd(m, r0, r1, s_x, f);
    if (i == 0) apos[0] = 0;
    if (i >= n) return;
    // the staged path is code of its own, so that it reads LDS directly
    // rather than through generic (flat) loads
    if (staged)
        apos[i + 1] = union_count_staged(m, s_x, f, i);
    else
        apos[i + 1] = union_count(m, Crd3{m.bc, m.cc, m.dc, 0, 0, 0}, i);
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

// The workgroup's rows [r0, r1) merged a lane per row into output windows
// of kWin entries in LDS (w_crd, w_val), each window written with coalesced
// stores.
template <typename V, int kWin>
__device__ __forceinline__ void fill_windows(int64_t n, const Csr3 &m, const Crd3 &x,
                                             const Vals3<V> &vv, const int32_t *apos,
                                             int32_t *acrd, V *aval, int64_t r0, int64_t r1,
                                             int32_t *w_crd, V *w_val) {
    const int64_t i = r0 + threadIdx.x;
    const int64_t base = apos[r0];
    const int64_t total = apos[r1] - base;
    const bool mine = i < r1;
    int64_t k = mine ? apos[i] - base : 0;
    const int64_t hi = mine ? apos[i + 1] - base : 0;
    Merge3 mg(m, x, mine ? i : r0);
    for (int64_t w = 0; w < total; w += kWin) {
        const int64_t we = w + kWin < total ? w + kWin : total;
        for (; k < hi && k < we; ++k) {
            V sum;
            const int32_t c = mg.next<true, V>(x, vv, sum);
            w_crd[k - w] = c;
            w_val[k - w] = sum;
        }
        __syncthreads();
        for (int64_t q = threadIdx.x; q < we - w; q += kBlock) {
            store_stream(acrd + base + w + q, w_crd[q]);
            store_stream(aval + base + w + q, w_val[q]);
        }
        __syncthreads();
    }
}

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
    if constexpr (STAGE > 0) {
        // the staged path is a copy of its own, so that it reads LDS directly
        int32_t f[3];
        if (stage_crd(m, r0, r1, s_x, f)) {
            const Crd3 x{s_x[0], s_x[1], s_x[2], f[0], f[1], f[2]};
            if constexpr (STAGE == 2) {
                const int32_t nv[3] = {m.bp[r1] - f[0], m.cp[r1] - f[1], m.dp[r1] - f[2]};
                const V *src[3] = {bv + f[0], cv + f[1], dv + f[2]};
#pragma unroll
                for (int X = 0; X < 3; ++X)
                    for (int k = threadIdx.x; k < nv[X]; k += kBlock) s_v[X][k] = src[X][k];
                __syncthreads();
                fill_windows<V, kWin>(n, m, x, Vals3<V>{s_v[0], s_v[1], s_v[2], f[0], f[1], f[2]},
                                      apos, acrd, aval, r0, r1, s_crd, s_val);
            } else {
                fill_windows<V, kWin>(n, m, x, Vals3<V>{bv, cv, dv, 0, 0, 0}, apos, acrd, aval,
                                      r0, r1, s_crd, s_val);
            }
            return;
        }
    }
    fill_windows<V, kWin>(n, m, Crd3{m.bc, m.cc, m.dc, 0, 0, 0}, Vals3<V>{bv, cv, dv, 0, 0, 0},
                          apos, acrd, aval, r0, r1, s_crd, s_val);
}

// Numeric phase by ranks.  The workgroup's coordinate runs of the three
// operands are staged in LDS, and every input entry then finds its output
// slot by itself, a lane per entry: an entry of C duplicates one of B when
// B's row holds its coordinate, an entry of D when B's or C's row does; the
// first operand holding a coordinate owns it and writes it at
//   A.pos[i] + #(B_i < x) + #(owned C_i < x) + #(owned D_i < x),
// the counts from lower bounds by binary search in the staged rows less the
// duplicates below them, which come from one ballot of the duplicate flags
// per 64 entries and a prefix over those words.  The owner adds the values
// of the duplicates in the order B, C, D as the merge does.  Every input
// line is read with coalesced loads (values by their owner lanes, the
// duplicates' values gathered from lines their neighbours read), and no lane
// walks a whole row.  Runs longer than kRankCap fall back to the windowed
// merge for that workgroup.  A workgroup takes 128 rows with its 256 lanes
// (5 entries a lane and operand, 22 KB of LDS): 0.142 ms on three 1e6-row
// operands of 8 entries a row, against 0.153 with 192 rows (7 a lane,
// 31 KB), 0.166 with 256 (9 a lane, 40 KB, 4 workgroups a CU) and 0.149
// with 64 (3 a lane): more workgroups per CU until a lane has too little
// to overlap.
constexpr int kRankRows = 128;                 // rows per workgroup
constexpr int kRankCap = 1280;                 // entries per operand and workgroup
constexpr int kRankPer = kRankCap / kBlock;     // entries per lane and operand
constexpr int kRankChunks = kRankCap / 64 + 1;  // ballot words, one spare for a full run
static_assert(kRankCap % kBlock == 0, "whole entries per lane");
static_assert(kRankRows <= 256 && kRankRows <= kBlock, "a row index fits a byte, a lane per row");
static_assert(kRankChunks <= 64, "one wave scans the ballot words");

// Value at byte offset `off` of a buffer (0 past its range, with no access).
__device__ __forceinline__ float buf_load(const float *, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ double buf_load(const double *, __amdgpu_buffer_rsrc_t r,
                                           uint32_t off) {
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
    const u32x2 w = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
    return __hiloint2double(static_cast<int>(w[1]), static_cast<int>(w[0]));
}

__device__ __forceinline__ int lower_bound_lds(const int32_t *a, int lo, int hi, int32_t x) {
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// Flagged entries among the first k of a run: the prefix of k's 64-entry
// word plus the flags below k inside it.
__device__ __forceinline__ int flags_below(const uint64_t *mask, const int32_t *pre, int k) {
    const int c = k >> 6;
    return pre[c] + __popcll(mask[c] & ((1ull << (k & 63)) - 1));
}

// LDS of the rank forms: the coordinate runs, the row of each staged entry
// (relative to the workgroup's first row), the rows' starts in the runs,
// the duplicate flags of C and D with their per-word prefixes, and a
// per-row constant of the output slots.
struct RankLds {
    int32_t x[3][kRankCap];
    uint8_t row[3][kRankCap];
    int32_t start[3][kRankRows + 1];
    uint64_t mask[2][kRankChunks];
    int32_t pre[2][kRankChunks];
    int32_t base[kRankRows];

    __device__ __forceinline__ int lb(int X, int r, int32_t v) const {
        return lower_bound_lds(x[X], start[X][r], start[X][r + 1], v);
    }
    __device__ __forceinline__ bool holds(int X, int r, int p, int32_t v) const {
        return p < start[X][r + 1] && x[X][p] == v;
    }
    // owned entries of C (X = 1) or D (X = 2) before staged index k of the run
    __device__ __forceinline__ int owned(int X, int k) const {
        return k - flags_below(mask[X - 1], pre[X - 1], k);
    }
    __device__ __forceinline__ bool dup(int X, int e) const {
        return (mask[X - 1][e >> 6] >> (e & 63)) & 1;
    }
};

// What the flag pass found for a lane's entries of C and D, kept for the
// output pass: the row (8 bits) and the lower bounds in B's row and, for D,
// in C's row (12 bits each, kRankCap <= 4096).
struct RankSeen {
    uint32_t c[kRankPer], d[kRankPer];
};
static_assert(kRankCap <= 4096, "staged indices fit 12 bits");

// Stages rows [r0, r0 + nr) whose runs (n3 entries from first3) fit, flags
// the duplicates and sets the per-row constants
//   base[r] = apos[r] - apos[r0] - start_B[r] - owned_C(start_C[r]) - owned_D(start_D[r]),
// so that an entry's output slot, relative to the workgroup's first output,
// is base[r] plus its counts before it.
// Ends with the workgroup synchronized.
__device__ void rank_prepare(const Csr3 &m, int64_t r0, int nr, const int32_t *first3,
                             const int32_t *n3, const int32_t *apos, RankLds &L,
                             RankSeen &S) {
    const int t = threadIdx.x;
    const int32_t *pos[3] = {m.bp, m.cp, m.dp};
    const int32_t *crd[3] = {m.bc, m.cc, m.dc};
    const int32_t *src[3] = {crd[0] + first3[0], crd[1] + first3[1], crd[2] + first3[2]};
    int32_t *dst[3] = {L.x[0], L.x[1], L.x[2]};
    stage3<kRankPer>(src, n3, dst);
#pragma unroll
    for (int X = 0; X < 3; ++X)
        for (int r = t; r <= nr; r += kBlock) L.start[X][r] = pos[X][r0 + r] - first3[X];
    __syncthreads();
    if (t < nr) {
#pragma unroll
        for (int X = 0; X < 3; ++X)
            for (int k = L.start[X][t]; k < L.start[X][t + 1]; ++k) L.row[X][k] = t;
    }
    __syncthreads();
    const int lane = t & 63, wave = t >> 6;
#pragma unroll
    for (int j = 0; j < kRankPer; ++j) {  // C entries that B's row holds
        const int e = j * kBlock + t;
        bool d = false;
        S.c[j] = 0;
        if (e < n3[1]) {
            const int r = L.row[1][e];
            const int32_t v = L.x[1][e];
            const int p = L.lb(0, r, v);
            d = L.holds(0, r, p, v);
            S.c[j] = r | (p << 8);
        }
        const uint64_t word = __ballot(d);
        if (lane == 0) L.mask[0][4 * j + wave] = word;
    }
#pragma unroll
    for (int j = 0; j < kRankPer; ++j) {  // D entries that B's or C's row holds
        const int e = j * kBlock + t;
        bool d = false;
        S.d[j] = 0;
        if (e < n3[2]) {
            const int r = L.row[2][e];
            const int32_t v = L.x[2][e];
            const int p = L.lb(0, r, v), q = L.lb(1, r, v);
            d = L.holds(0, r, p, v) || L.holds(1, r, q, v);
            S.d[j] = r | (p << 8) | (q << 20);
        }
        const uint64_t word = __ballot(d);
        if (lane == 0) L.mask[1][4 * j + wave] = word;
    }
    static_assert(kBlock == 256, "four waves: word 4j + wave holds entries j*256 + 64*wave ..");
    __syncthreads();
    if (wave < 2) {  // exclusive prefix of the flag counts per word: wave 0 for C, 1 for D
        const int words = (n3[1 + wave] + 63) >> 6;
        int cnt = 0;
        if (lane < kRankChunks) {
            if (lane < words)
                cnt = __popcll(L.mask[wave][lane]);
            else
                L.mask[wave][lane] = 0;
        }
        int incl = cnt;
        for (int d = 1; d < 64; d <<= 1) {
            const int v = __shfl_up(incl, d);
            if (lane >= d) incl += v;
        }
        if (lane < kRankChunks) L.pre[wave][lane] = incl - cnt;
    }
    __syncthreads();
    if (t < nr)
        L.base[t] = apos[r0 + t] - apos[r0] - L.start[0][t] - L.owned(1, L.start[1][t]) -
                    L.owned(2, L.start[2][t]);
    __syncthreads();
}

// Output slot and value loads of entry j of operand X, when it owns its
// coordinate (o = -1 otherwise): s1 / s2 are the byte offsets of the values
// of C / D at that coordinate when they hold it (kBufOut when not).
template <int X, typename V>
__device__ __forceinline__ void rank_slot(const RankLds &L, const RankSeen &S, int j, int n,
                                          int32_t &o, int32_t &x, uint32_t &s1, uint32_t &s2) {
    const int e = j * kBlock + threadIdx.x;
    s1 = kBufOut;
    s2 = kBufOut;
    o = -1;
    x = 0;
    if (e < n && (X == 0 || !L.dup(X, e))) {
        int r, slot;
        if constexpr (X == 0) {  // B owns all its entries
            r = L.row[0][e];
            x = L.x[0][e];
            const int p = L.lb(1, r, x), q = L.lb(2, r, x);
            if (L.holds(1, r, p, x)) s1 = static_cast<uint32_t>(sizeof(V) * p);
            if (L.holds(2, r, q, x)) s2 = static_cast<uint32_t>(sizeof(V) * q);
            slot = e + L.owned(1, p) + L.owned(2, q);
        } else if constexpr (X == 1) {  // B does not hold it
            r = S.c[j] & 255;
            x = L.x[1][e];
            const int p = S.c[j] >> 8, q = L.lb(2, r, x);
            if (L.holds(2, r, q, x)) s2 = static_cast<uint32_t>(sizeof(V) * q);
            slot = p + L.owned(1, e) + L.owned(2, q);
        } else {  // neither B nor C holds it
            r = S.d[j] & 255;
            x = L.x[2][e];
            const int p = (S.d[j] >> 8) & 4095, q = S.d[j] >> 20;
            slot = p + L.owned(1, q) + L.owned(2, e);
        }
        o = L.base[r] + slot;
    }
}

// Entries J0 .. J0 + kRankGroup - 1 of each operand that own their
// coordinate, written at their output slots (relative to the workgroup's
// first output at acrd, aval).  First the searches in LDS, then the loads
// of the values of the later operands holding the coordinates, all at
// once, then the sums (own: the entries' own values, loaded with the
// staging) and stores.  The three operands' entries of a group fall in
// about the same rows, so the group fills its output lines while the L2
// still holds them (one operand after another left them partly written
// and evicted: 2.3 times the output's bytes written).  Groups of three
// entries per operand (at 256 rows a workgroup: 0.167 ms on three 1e6-row
// operands, against 0.175 for groups of one, fewer loads in flight, and
// 0.189 for one operand after another).
constexpr int kRankGroup = 3;

template <int J0, typename V>
__device__ __forceinline__ void rank_emit(const RankLds &L, const RankSeen &S,
                                          const V *const *vals, const __amdgpu_buffer_rsrc_t *rv,
                                          const V (*own)[kRankPer], const int32_t *n3,
                                          int32_t *acrd, V *aval) {
    // the last group may be short
    constexpr int NJ = J0 + kRankGroup <= kRankPer ? kRankGroup : kRankPer - J0;
    int32_t o[3][kRankGroup], xs[3][kRankGroup];
    V g1[kRankGroup], g2[2][kRankGroup];
    uint32_t has1 = 0, has2 = 0;  // bit 3X + jj: entry adds C's value (X = 0) / D's (X < 2)
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
        uint32_t s1, s2;
        rank_slot<0, V>(L, S, J0 + jj, n3[0], o[0][jj], xs[0][jj], s1, s2);
        g1[jj] = buf_load(vals[1], rv[1], s1);
        g2[0][jj] = buf_load(vals[2], rv[2], s2);
        has1 |= static_cast<uint32_t>(s1 != kBufOut) << jj;
        has2 |= static_cast<uint32_t>(s2 != kBufOut) << jj;
        rank_slot<1, V>(L, S, J0 + jj, n3[1], o[1][jj], xs[1][jj], s1, s2);
        g2[1][jj] = buf_load(vals[2], rv[2], s2);
        has2 |= static_cast<uint32_t>(s2 != kBufOut) << (kRankGroup + jj);
        rank_slot<2, V>(L, S, J0 + jj, n3[2], o[2][jj], xs[2][jj], s1, s2);
    }
#pragma unroll
    for (int X = 0; X < 3; ++X)
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj) {
            if (o[X][jj] < 0) continue;
            // the merge's order: B's value, else 0, then + C's, then + D's
            V v = X == 0 ? own[0][J0 + jj] : V(0) + own[X][J0 + jj];
            if (X == 0 && ((has1 >> jj) & 1)) v = v + g1[jj];
            if (X < 2 && ((has2 >> (kRankGroup * X + jj)) & 1)) v = v + g2[X < 2 ? X : 0][jj];
            acrd[o[X][jj]] = xs[X][jj];
            aval[o[X][jj]] = v;
        }
}

template <typename V>
__global__ __launch_bounds__(kBlock) void k_spadd3_rank(int64_t n, Csr3 m, const V *bv,
                                                        const V *cv, const V *dv,
                                                        const int32_t *apos, int32_t *acrd,
                                                        V *aval) {
    __shared__ __align__(16) RankLds L;
    constexpr int kRankWin = 1024;  // output window of the fallback merge
    static_assert(kRankWin * (4 + sizeof(V)) <= sizeof(L.x), "fallback windows fit the stage");
    const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kRankRows;
    const int64_t r1 = r0 + kRankRows < n ? r0 + kRankRows : n;
    const int nr = static_cast<int>(r1 - r0);
    const int32_t first3[3] = {m.bp[r0], m.cp[r0], m.dp[r0]};
    const int32_t n3[3] = {m.bp[r1] - first3[0], m.cp[r1] - first3[1], m.dp[r1] - first3[2]};
    if (n3[0] > kRankCap || n3[1] > kRankCap || n3[2] > kRankCap) {
        fill_windows<V, kRankWin>(n, m, Crd3{m.bc, m.cc, m.dc, 0, 0, 0},
                                  Vals3<V>{bv, cv, dv, 0, 0, 0}, apos, acrd, aval, r0, r1,
                                  &L.x[0][0], reinterpret_cast<V *>(&L.x[0][0] + kRankWin));
        return;
    }
    const V *vals[3] = {bv, cv, dv};
    __amdgpu_buffer_rsrc_t rv[3];
    V own[3][kRankPer];  // the lane's entries' values, in flight with the staging
#pragma unroll
    for (int X = 0; X < 3; ++X) {
        rv[X] = span_rsrc(vals[X] + first3[X], sizeof(V) * n3[X]);
#pragma unroll
        for (int j = 0; j < kRankPer; ++j) {
            const int e = j * kBlock + threadIdx.x;
            own[X][j] = buf_load(vals[X], rv[X],
                                 e < n3[X] ? static_cast<uint32_t>(sizeof(V) * e) : kBufOut);
        }
    }
    RankSeen S;
    rank_prepare(m, r0, nr, first3, n3, apos, L, S);
    const int32_t out0 = apos[r0];
    rank_emit<0>(L, S, vals, rv, own, n3, acrd + out0, aval + out0);
    rank_emit<3>(L, S, vals, rv, own, n3, acrd + out0, aval + out0);
    static_assert(kRankPer == 5 && kRankGroup == 3, "groups of 3 and 2");
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
    const dim3 rows_grid(static_cast<unsigned>(ceil_div(n > 0 ? n : 1, kBlock)));
    k_spadd3_count<<<rows_grid, kBlock, 0, s>>>(n, m, apos);
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
    if (stage == 3) {
        k_spadd3_rank<V><<<dim3(static_cast<unsigned>(ceil_div(n, kRankRows))), kBlock, 0, s>>>(
            n, m, static_cast<const V *>(bv), static_cast<const V *>(cv),
            static_cast<const V *>(dv), apos, acrd, static_cast<V *>(aval));
        return hipGetLastError();
    }
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
