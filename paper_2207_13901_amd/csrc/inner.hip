// Inner product of two sparse tensors with different patterns (the TIN
// statement with no free index, Sec. II-A): a = sum over the coordinates
// both store of B * C.  The co-iteration intersects the operands level by
// level (the paper's coordinate-tree iteration, Sec. IV-C): a unit of work
// is one stored coordinate of B's last-but-one level — a position of a CSR
// matrix, a fiber of a CSF tensor — whose coordinate is looked up in C's
// segment of the same parent by binary search; for a fiber the two sorted
// last-level coordinate lists are then merged.
//
// One lane per unit, 256 units per workgroup.  The parent of each unit comes
// from the parent pos entries of the workgroup's unit range, staged in LDS
// (a binary search there; a per-lane search of pos in HBM when more than
// kParents parents overlap the range).  Products are summed in double: each
// lane, then a fixed tree over the workgroup into one partial per
// workgroup, then a fixed-order final pass (k_inner_final), so the result
// does not depend on timing.
#include "device.hpp"
#include "internal.hpp"

namespace spl {
namespace {

constexpr int kParents = 1024;

// Largest r in [lo, hi) with pos[r] <= u (the parent holding unit u).
template <typename P>
__device__ __forceinline__ int64_t parent_of(const P &pos, int64_t lo, int64_t hi, int64_t u) {
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (static_cast<int64_t>(pos(mid)) <= u)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Position of coordinate j in the sorted crd[lo, hi), or -1.
__device__ __forceinline__ int64_t find_sorted(const int32_t *__restrict__ crd, int64_t lo,
                                               int64_t hi, int32_t j) {
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        const int32_t v = crd[mid];
        if (v == j) return mid;
        if (v < j)
            lo = mid + 1;
        else
            hi = mid;
    }
    return -1;
}

template <typename V, int ORDER>
__global__ __launch_bounds__(kBlock) void k_inner_general(
    int64_t n, int64_t units, const int32_t *__restrict__ bpos, const int32_t *__restrict__ bcrd,
    const int32_t *__restrict__ bpos2, const int32_t *__restrict__ bcrd2,
    const V *__restrict__ bv, const int32_t *__restrict__ cpos, const int32_t *__restrict__ ccrd,
    const int32_t *__restrict__ cpos2, const int32_t *__restrict__ ccrd2,
    const V *__restrict__ cv, double *__restrict__ part) {
    __shared__ int32_t s_pos[kParents + 1];
    __shared__ int64_t s_r0, s_cnt;
    __shared__ double s_sum[kBlock];
    const int64_t u0 = static_cast<int64_t>(blockIdx.x) * kBlock;
    const int64_t u1 = u0 + kBlock < units ? u0 + kBlock : units;
    auto gpos = [&](int64_t r) { return bpos[r]; };
    if (threadIdx.x == 0) {
        const int64_t r0 = parent_of(gpos, 0, n, u0);
        const int64_t r1 = parent_of(gpos, r0, n, u1 - 1);
        s_r0 = r0;
        s_cnt = r1 - r0 + 1;
    }
    __syncthreads();
    const int64_t r0 = s_r0, cnt = s_cnt;
    const bool staged = cnt <= kParents;
    if (staged)
        for (int64_t k = threadIdx.x; k <= cnt; k += kBlock) s_pos[k] = bpos[r0 + k];
    __syncthreads();

    double acc = 0.0;
    const int64_t u = u0 + threadIdx.x;
    if (u < u1) {
        const int64_t r = staged ? r0 + parent_of([&](int64_t k) { return s_pos[k]; }, 0, cnt, u)
                                 : parent_of(gpos, r0, n, u);
        const int64_t g = find_sorted(ccrd, cpos[r], cpos[r + 1], bcrd[u]);
        if (g >= 0) {
            if (ORDER == 2) {
                acc = to_f64(bv[u]) * to_f64(cv[g]);
            } else {
                int64_t p = bpos2[u], pe = bpos2[u + 1];
                int64_t q = cpos2[g], qe = cpos2[g + 1];
                while (p < pe && q < qe) {
                    const int32_t kb = bcrd2[p], kc = ccrd2[q];
                    if (kb == kc) acc += to_f64(bv[p++]) * to_f64(cv[q++]);
                    else if (kb < kc) ++p;
                    else ++q;
                }
            }
        }
    }
    s_sum[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) s_sum[threadIdx.x] += s_sum[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s_sum[0];
}

}  // namespace

int64_t inner_general_parts(int64_t units) { return ceil_div(units > 0 ? units : 1, kBlock); }

hipError_t launch_inner_general(int vtype, int order, int64_t n, int64_t units,
                                const int32_t *bpos, const int32_t *bcrd, const int32_t *bpos2,
                                const int32_t *bcrd2, const void *bv, const int32_t *cpos,
                                const int32_t *ccrd, const int32_t *cpos2, const int32_t *ccrd2,
                                const void *cv, double *part, double *out, hipStream_t s) {
    const int64_t parts = inner_general_parts(units);
    if (units > 0) {
        dim3 grid(static_cast<unsigned>(parts));
        auto go = [&](auto kern, auto *b, auto *c) {
            kern<<<grid, kBlock, 0, s>>>(n, units, bpos, bcrd, bpos2, bcrd2, b, cpos, ccrd, cpos2,
                                         ccrd2, c, part);
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
