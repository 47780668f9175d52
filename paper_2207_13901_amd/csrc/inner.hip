// Inner product of two sparse tensors with different patterns (the TIN
// statement with no free index, Sec. II-A): a = sum over the coordinates
// both store of B * C.  The co-iteration intersects the operands level by
// level (the paper's coordinate-tree iteration, Sec. IV-C): a unit of work
// is one stored coordinate of B's last-but-one level — a position of a CSR
// matrix, a fiber of a CSF tensor — whose coordinate is looked up in C's
// segment of the same parent by binary search; for a fiber the two sorted
// last-level coordinate lists are then merged.
//
// A workgroup takes kUnitIters * 256 consecutive units, a lane every 256th.
// The parent of each unit comes from the parent pos entries of the
// workgroup's unit range, staged in LDS, and so do C's parent pos entries
// and the C coordinates that can match: units are sorted by (parent,
// coordinate), so the matches of the range lie between the first position
// of C's first parent holding a coordinate at or past the range's first,
// and the last position of C's last parent holding one at or below the
// range's last.  The searches then run in LDS.  Those range bounds come from
// a pre-pass (k_inner_bounds, a lane per workgroup boundary, all searching
// at once) rather than from a serial search at the start of each workgroup.  When more than kParents
// parents or kCStage C coordinates fall in the range, each lane searches
// pos and crd in HBM instead.  Products are summed in double: each lane,
// then a fixed tree over the workgroup into one partial per workgroup,
// then a fixed-order final pass (k_inner_final), so the result does not
// depend on timing.
#include "device.hpp"
#include "internal.hpp"

namespace spl {
namespace {

constexpr int kParents = 1024;   // parents staged per workgroup
constexpr int kCStage = 2560;    // C coordinates staged per workgroup
constexpr int kUnitIters = 8;    // units per lane

// Largest r in [lo, hi) with pos[r] <= u (the parent holding unit u); I is
// the index type (32-bit where the indices are LDS offsets, fewer VALU
// instructions a step).
template <typename I, typename P>
__device__ __forceinline__ I parent_of(const P &pos, I lo, I hi, I u) {
    while (hi - lo > 1) {
        const I mid = (lo + hi) >> 1;
        if (static_cast<I>(pos(mid)) <= u)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// First position in the sorted crd[lo, hi) whose coordinate is at least j
// (UPPER false) or above j (UPPER true).
template <bool UPPER>
__device__ __forceinline__ int64_t bound_sorted(const int32_t *__restrict__ crd, int64_t lo,
                                                int64_t hi, int32_t j) {
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (UPPER ? crd[mid] <= j : crd[mid] < j)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// Position of coordinate j in the sorted crd[lo, hi), or -1.
template <typename I, typename C>
__device__ __forceinline__ I find_sorted(const C &crd, I lo, I hi, int32_t j) {
    while (lo < hi) {
        const I mid = (lo + hi) >> 1;
        const int32_t v = crd(mid);
        if (v == j) return mid;
        if (v < j)
            lo = mid + 1;
        else
            hi = mid;
    }
    return -1;
}

// Range bounds of every workgroup: for boundary b (unit u_b = b * span,
// capped at units), the parent of u_b and the first C position of that
// parent whose coordinate is at least u_b's (the start of workgroup b), and
// the parent of u_b - 1 and the first C position of that parent whose
// coordinate is above u_b - 1's (the end of workgroup b - 1).
__global__ __launch_bounds__(kBlock) void k_inner_bounds(int64_t n, int64_t units, int64_t span,
                                                         int64_t parts,
                                                         const int32_t *__restrict__ bpos,
                                                         const int32_t *__restrict__ bcrd,
                                                         const int32_t *__restrict__ cpos,
                                                         const int32_t *__restrict__ ccrd,
                                                         int64_t *__restrict__ bnd) {
    const int64_t b = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (b > parts) return;
    const int64_t ub = b * span < units ? b * span : units;
    auto gpos = [&](int64_t r) { return bpos[r]; };
    int64_t ra = 0, ca = 0, rb = 0, cb = 0;
    if (ub < units) {
        ra = parent_of<int64_t>(gpos, 0, n, ub);
        ca = bound_sorted<false>(ccrd, cpos[ra], cpos[ra + 1], bcrd[ub]);
    }
    if (ub > 0) {
        rb = parent_of<int64_t>(gpos, 0, n, ub - 1);
        cb = bound_sorted<true>(ccrd, cpos[rb], cpos[rb + 1], bcrd[ub - 1]);
    }
    bnd[4 * b] = ra;
    bnd[4 * b + 1] = ca;
    bnd[4 * b + 2] = rb;
    bnd[4 * b + 3] = cb;
}

template <typename V, int ORDER>
__global__ __launch_bounds__(kBlock) void k_inner_general(
    int64_t n, int64_t units, const int32_t *__restrict__ bpos, const int32_t *__restrict__ bcrd,
    const int32_t *__restrict__ bpos2, const int32_t *__restrict__ bcrd2,
    const V *__restrict__ bv, const int32_t *__restrict__ cpos, const int32_t *__restrict__ ccrd,
    const int32_t *__restrict__ cpos2, const int32_t *__restrict__ ccrd2,
    const V *__restrict__ cv, const int64_t *__restrict__ bnd, double *__restrict__ part) {
    __shared__ int32_t s_pos[kParents + 1];   // B's parent pos entries of the range
    __shared__ int32_t s_cpos[kParents + 1];  // C's
    __shared__ int32_t s_ccrd[kCStage];       // C's coordinates that can match
    __shared__ double s_sum[kBlock / kWave];
    static_assert(kBlock / kWave == 4, "four waves per workgroup");
    const int64_t u0 = static_cast<int64_t>(blockIdx.x) * (kBlock * kUnitIters);
    const int64_t u1 = u0 + kBlock * kUnitIters < units ? u0 + kBlock * kUnitIters : units;
    auto gpos = [&](int64_t r) { return bpos[r]; };
    const int64_t w = blockIdx.x;
    const int64_t r0 = bnd[4 * w], c0 = bnd[4 * w + 1];
    const int64_t cnt = bnd[4 * w + 6] - r0 + 1, c1 = bnd[4 * w + 7];
    const bool staged = cnt <= kParents && c1 - c0 <= kCStage;
    if (staged) {
        for (int64_t k = threadIdx.x; k <= cnt; k += kBlock) {
            s_pos[k] = bpos[r0 + k];
            s_cpos[k] = cpos[r0 + k];
        }
        for (int64_t k = threadIdx.x; k < c1 - c0; k += kBlock) s_ccrd[k] = ccrd[c0 + k];
    }
    __syncthreads();

    // Unit and position indices fit in 32 bits (they index arrays whose
    // sizes are int32 pos entries), and so do the staged LDS offsets.
    double acc = 0.0;
    int32_t jv[kUnitIters];  // the lane's coordinates, loaded together
    // (bounds compared in 64 bits: the last range may end past 2^31 - 1)
#pragma unroll
    for (int it = 0; it < kUnitIters; ++it) {
        const int64_t u = u0 + it * kBlock + threadIdx.x;
        jv[it] = u < u1 ? bcrd[u] : 0;
    }
    const int32_t cnt32 = static_cast<int32_t>(cnt);
    const int32_t c0s = static_cast<int32_t>(c0), c1s = static_cast<int32_t>(c1);
    int32_t rk = 0;  // staged parent index of the lane's previous unit (units ascend)
#pragma unroll
    for (int it = 0; it < kUnitIters; ++it) {
        const int64_t u64 = u0 + it * kBlock + threadIdx.x;
        if (u64 >= u1) break;
        const int32_t u = static_cast<int32_t>(u64);
        const int32_t j = jv[it];
        int32_t g;
        if (staged) {
            rk = parent_of<int32_t>([&](int32_t k) { return s_pos[k]; }, rk, cnt32, u);
            // C's positions of this parent, clipped to the staged range
            const int32_t lo = s_cpos[rk] > c0s ? s_cpos[rk] : c0s;
            const int32_t hi = s_cpos[rk + 1] < c1s ? s_cpos[rk + 1] : c1s;
            g = find_sorted<int32_t>([&](int32_t k) { return s_ccrd[k]; }, lo - c0s, hi - c0s, j);
            if (g >= 0) g += c0s;
        } else {
            const int64_t r = parent_of<int64_t>(gpos, r0, r0 + cnt, u);
            g = static_cast<int32_t>(
                find_sorted<int64_t>([&](int64_t k) { return ccrd[k]; }, cpos[r], cpos[r + 1], j));
        }
        if (g < 0) continue;
        if (ORDER == 2) {
            acc += to_f64(bv[u]) * to_f64(cv[g]);
        } else {
            int32_t p = bpos2[u], q = cpos2[g];
            const int32_t pe = bpos2[u + 1], qe = cpos2[g + 1];
            while (p < pe && q < qe) {
                // values loaded with the coordinates (one round of loads a step)
                const int32_t kb = bcrd2[p], kc = ccrd2[q];
                const V vb = bv[p], vc = cv[q];
                if (kb == kc) acc += to_f64(vb) * to_f64(vc);
                p += kb <= kc ? 1 : 0;
                q += kc <= kb ? 1 : 0;
            }
        }
    }
    // fixed order: a butterfly in each wave, then the four wave sums in order
    acc = group_sum<kWave>(acc);
    if ((threadIdx.x & (kWave - 1)) == 0) s_sum[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = ((s_sum[0] + s_sum[1]) + s_sum[2]) + s_sum[3];
}

}  // namespace

int64_t inner_general_parts(int64_t units) {
    return ceil_div(units > 0 ? units : 1, kBlock * kUnitIters);
}

namespace {
size_t part_bytes(int64_t parts) { return (static_cast<size_t>(parts) * 8 + 255) / 256 * 256; }
}  // namespace

size_t inner_general_ws(int64_t units) {
    const int64_t parts = inner_general_parts(units);
    return part_bytes(parts) + static_cast<size_t>(parts + 1) * 4 * sizeof(int64_t);
}

hipError_t launch_inner_general(int vtype, int order, int64_t n, int64_t units,
                                const int32_t *bpos, const int32_t *bcrd, const int32_t *bpos2,
                                const int32_t *bcrd2, const void *bv, const int32_t *cpos,
                                const int32_t *ccrd, const int32_t *cpos2, const int32_t *ccrd2,
                                const void *cv, void *ws, double *out, hipStream_t s) {
    const int64_t parts = inner_general_parts(units);
    double *part = static_cast<double *>(ws);
    int64_t *bnd = reinterpret_cast<int64_t *>(static_cast<char *>(ws) + part_bytes(parts));
    if (units > 0) {
        k_inner_bounds<<<dim3(static_cast<unsigned>(ceil_div(parts + 1, kBlock))), kBlock, 0, s>>>(
            n, units, kBlock * kUnitIters, parts, bpos, bcrd, cpos, ccrd, bnd);
        dim3 grid(static_cast<unsigned>(parts));
        auto go = [&](auto kern, auto *b, auto *c) {
            kern<<<grid, kBlock, 0, s>>>(n, units, bpos, bcrd, bpos2, bcrd2, b, cpos, ccrd, cpos2,
                                         ccrd2, c, bnd, part);
        };
        if (vtype == SPL_F64) {
            const double *b = static_cast<const double *>(bv), *c = static_cast<const double *>(cv);
            if (order == 2) go(k_inner_general<double, 2>, b, c);
            else go(k_inner_general<double, 3>, b, c);
        } else {
            const float *b = static_cast<const float *>(bv), *c = static_cast<const float *>(cv);
            if (order == 2) go(k_inner_general<float, 2>, b, c);
            else go(k_inner_general<float, 3>, b, c);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return launch_inner_final(units > 0 ? parts : 0, part, out, s);
}

}  // namespace spl
