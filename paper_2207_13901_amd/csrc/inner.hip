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
constexpr int kLockstep = 2;     // fibers a lane merges in lockstep

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

// 4-byte integer at byte offset `off` of a buffer (0 past its range); the
// default cache policy, since neighbouring lanes' fibers share lines.
__device__ __forceinline__ int32_t load_i32(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return static_cast<int32_t>(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
// 4- or 8-byte value at byte offset `off` of a buffer (0 past its range).
__device__ __forceinline__ float load_val(const float *, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ double load_val(const double *, __amdgpu_buffer_rsrc_t r,
                                           uint32_t off) {
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
    const u32x2 w = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
    return __hiloint2double(static_cast<int>(w[1]), static_cast<int>(w[0]));
}

// BUF (CSF operands whose last-level arrays each fit a buffer descriptor's
// range; nnzb, nnzc, cunits size them): the lane's fibers are merged
// kLockstep at a time in lockstep, every step loading the next coordinates
// and values of both at once (a lane with nothing to load reads 0 past the
// descriptor's range, without a branch), so the lane's chain of dependent
// loads is about half as long (0.956 -> 0.891 ms on the 1e8-nonzero tensor;
// 4 at a time: 0.930, 8: slower still, as lanes load for fibers that have
// ended; these loads keep the default cache policy, since neighbouring
// lanes' fibers share lines: with the non-temporal hint, 1.08).  Without
// BUF the fibers are merged one after another.
template <typename V, int ORDER, bool BUF = false>
__global__ __launch_bounds__(kBlock) void k_inner_general(
    int64_t n, int64_t units, const int32_t *__restrict__ bpos, const int32_t *__restrict__ bcrd,
    const int32_t *__restrict__ bpos2, const int32_t *__restrict__ bcrd2,
    const V *__restrict__ bv, const int32_t *__restrict__ cpos, const int32_t *__restrict__ ccrd,
    const int32_t *__restrict__ cpos2, const int32_t *__restrict__ ccrd2,
    const V *__restrict__ cv, const int64_t *__restrict__ bnd, double *__restrict__ part,
    int64_t nnzb, int64_t nnzc, int64_t cunits) {
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
        // every lane issues all its loads before any store (past a run: 0,
        // with no access), so the copy costs one round of loads, not one
        // per loop iteration
        constexpr int kPosPer = (kParents + 1 + kBlock - 1) / kBlock;
        constexpr int kCPer = (kCStage + kBlock - 1) / kBlock;
        const int np = static_cast<int>(cnt) + 1;
        const int nc = c1 > c0 ? static_cast<int>(c1 - c0) : 0;
        const __amdgpu_buffer_rsrc_t rp = span_rsrc(bpos + r0, 4u * np);
        const __amdgpu_buffer_rsrc_t rq = span_rsrc(cpos + r0, 4u * np);
        const __amdgpu_buffer_rsrc_t rc = span_rsrc(ccrd + c0, 4u * nc);
        uint32_t a[kPosPer], b[kPosPer], c[kCPer];
#pragma unroll
        for (int i = 0; i < kPosPer; ++i) {
            const int k = i * kBlock + threadIdx.x;
            a[i] = buf_u32(rp, k < np ? 4u * k : kBufOut);
            b[i] = buf_u32(rq, k < np ? 4u * k : kBufOut);
        }
#pragma unroll
        for (int i = 0; i < kCPer; ++i) {
            const int k = i * kBlock + threadIdx.x;
            c[i] = buf_u32(rc, k < nc ? 4u * k : kBufOut);
        }
#pragma unroll
        for (int i = 0; i < kPosPer; ++i) {
            const int k = i * kBlock + threadIdx.x;
            if (k < np) {
                s_pos[k] = static_cast<int32_t>(a[i]);
                s_cpos[k] = static_cast<int32_t>(b[i]);
            }
        }
#pragma unroll
        for (int i = 0; i < kCPer; ++i) {
            const int k = i * kBlock + threadIdx.x;
            if (k < nc) s_ccrd[k] = static_cast<int32_t>(c[i]);
        }
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
    if constexpr (BUF && ORDER == 3) {
        // the C fiber matching each of the lane's fibers (-1: none)
        int32_t gq[kUnitIters];
#pragma unroll
        for (int it = 0; it < kUnitIters; ++it) {
            const int64_t u64 = u0 + it * kBlock + threadIdx.x;
            gq[it] = -1;
            if (u64 >= u1) continue;
            const int32_t u = static_cast<int32_t>(u64);
            const int32_t j = jv[it];
            if (staged) {
                rk = parent_of<int32_t>([&](int32_t k) { return s_pos[k]; }, rk, cnt32, u);
                const int32_t lo = s_cpos[rk] > c0s ? s_cpos[rk] : c0s;
                const int32_t hi = s_cpos[rk + 1] < c1s ? s_cpos[rk + 1] : c1s;
                const int32_t g =
                    find_sorted<int32_t>([&](int32_t k) { return s_ccrd[k]; }, lo - c0s, hi - c0s, j);
                gq[it] = g >= 0 ? g + c0s : -1;
            } else {
                const int64_t r = parent_of<int64_t>(gpos, r0, r0 + cnt, u);
                gq[it] = static_cast<int32_t>(find_sorted<int64_t>(
                    [&](int64_t k) { return ccrd[k]; }, cpos[r], cpos[r + 1], j));
            }
        }
        const __amdgpu_buffer_rsrc_t rbp = span_rsrc(bpos2, 4u * static_cast<uint32_t>(units + 1));
        const __amdgpu_buffer_rsrc_t rcp = span_rsrc(cpos2, 4u * static_cast<uint32_t>(cunits + 1));
        const __amdgpu_buffer_rsrc_t rbc = span_rsrc(bcrd2, 4u * static_cast<uint32_t>(nnzb));
        const __amdgpu_buffer_rsrc_t rcc = span_rsrc(ccrd2, 4u * static_cast<uint32_t>(nnzc));
        const __amdgpu_buffer_rsrc_t rbv =
            span_rsrc(bv, static_cast<uint32_t>(sizeof(V)) * static_cast<uint32_t>(nnzb));
        const __amdgpu_buffer_rsrc_t rcv =
            span_rsrc(cv, static_cast<uint32_t>(sizeof(V)) * static_cast<uint32_t>(nnzc));
#pragma unroll
        for (int g0 = 0; g0 < kUnitIters; g0 += kLockstep) {
            // both fibers' position ranges of the group, all at once
            int32_t p[kLockstep], pe[kLockstep], q[kLockstep], qe[kLockstep];
#pragma unroll
            for (int i = 0; i < kLockstep; ++i) {
                const int it = g0 + i;
                const int64_t u = u0 + it * kBlock + threadIdx.x;
                const bool hit = gq[it] >= 0;
                const uint32_t ob = hit ? 4u * static_cast<uint32_t>(u) : kBufOut;
                const uint32_t oc = hit ? 4u * static_cast<uint32_t>(gq[it]) : kBufOut;
                p[i] = load_i32(rbp, ob);
                pe[i] = load_i32(rbp, ob + 4);
                q[i] = load_i32(rcp, oc);
                qe[i] = load_i32(rcp, oc + 4);
            }
            for (;;) {  // one merge step of every fiber of the group
                int32_t kb[kLockstep], kc[kLockstep];
                V vb[kLockstep], vc[kLockstep];
                bool any = false;
#pragma unroll
                for (int i = 0; i < kLockstep; ++i) {
                    const bool act = p[i] < pe[i] && q[i] < qe[i];
                    any = any || act;
                    const uint32_t ob = act ? 4u * static_cast<uint32_t>(p[i]) : kBufOut;
                    const uint32_t oc = act ? 4u * static_cast<uint32_t>(q[i]) : kBufOut;
                    kb[i] = load_i32(rbc, ob);
                    kc[i] = load_i32(rcc, oc);
                    vb[i] = load_val(bv, rbv, act ? static_cast<uint32_t>(sizeof(V)) * p[i] : kBufOut);
                    vc[i] = load_val(cv, rcv, act ? static_cast<uint32_t>(sizeof(V)) * q[i] : kBufOut);
                }
                if (!any) break;
#pragma unroll
                for (int i = 0; i < kLockstep; ++i) {
                    if (!(p[i] < pe[i] && q[i] < qe[i])) continue;
                    if (kb[i] == kc[i]) acc += to_f64(vb[i]) * to_f64(vc[i]);
                    p[i] += kb[i] <= kc[i] ? 1 : 0;
                    q[i] += kc[i] <= kb[i] ? 1 : 0;
                }
            }
        }
    } else
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
                                const void *cv, int64_t nnzb, int64_t nnzc, int64_t cunits,
                                void *ws, double *out, hipStream_t s) {
    const int64_t parts = inner_general_parts(units);
    double *part = static_cast<double *>(ws);
    int64_t *bnd = reinterpret_cast<int64_t *>(static_cast<char *>(ws) + part_bytes(parts));
    if (units > 0) {
        k_inner_bounds<<<dim3(static_cast<unsigned>(ceil_div(parts + 1, kBlock))), kBlock, 0, s>>>(
            n, units, kBlock * kUnitIters, parts, bpos, bcrd, cpos, ccrd, bnd);
        dim3 grid(static_cast<unsigned>(parts));
        auto go = [&](auto kern, auto *b, auto *c) {
            kern<<<grid, kBlock, 0, s>>>(n, units, bpos, bcrd, bpos2, bcrd2, b, cpos, ccrd, cpos2,
                                         ccrd2, c, bnd, part, nnzb, nnzc, cunits);
        };
        // the lockstep merge when every last-level array fits a descriptor
        const size_t vb = vtype == SPL_F64 ? 8 : 4;
        auto fits = [](int64_t count, size_t bytes) {
            return count >= 0 && static_cast<uint64_t>(count) * bytes <= kBufRange;
        };
        const bool buf = order == 3 && fits(nnzb, vb) && fits(nnzc, vb) && fits(units + 1, 4) &&
                         fits(cunits + 1, 4);
        if (vtype == SPL_F64) {
            const double *b = static_cast<const double *>(bv), *c = static_cast<const double *>(cv);
            if (order == 2) go(k_inner_general<double, 2>, b, c);
            else if (buf) go(k_inner_general<double, 3, true>, b, c);
            else go(k_inner_general<double, 3>, b, c);
        } else {
            const float *b = static_cast<const float *>(bv), *c = static_cast<const float *>(cv);
            if (order == 2) go(k_inner_general<float, 2>, b, c);
            else if (buf) go(k_inner_general<float, 3, true>, b, c);
            else go(k_inner_general<float, 3>, b, c);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return launch_inner_final(units > 0 ? parts : 0, part, out, s);
}

}  // namespace spl
