// Device-side helpers shared by the spleaf kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spl {

constexpr int kWave = 64;
constexpr int kBlock = 256;  // 4 waves per workgroup everywhere

// BF16 storage type: the upper 16 bits of an IEEE binary32.
struct bf16 {
    uint16_t bits;
};

__device__ __forceinline__ float to_f32(bf16 v) {
    return __uint_as_float(static_cast<uint32_t>(v.bits) << 16);
}
__device__ __forceinline__ float to_f32(float v) { return v; }
__device__ __forceinline__ double to_f64(double v) { return v; }
__device__ __forceinline__ double to_f64(float v) { return static_cast<double>(v); }
__device__ __forceinline__ double to_f64(bf16 v) { return static_cast<double>(to_f32(v)); }

// Widen a stored value to the accumulation type Acc.
template <typename Acc, typename V>
__device__ __forceinline__ Acc widen(V v);
template <> __device__ __forceinline__ double widen<double, double>(double v) { return v; }
template <> __device__ __forceinline__ double widen<double, float>(float v) { return v; }
template <> __device__ __forceinline__ float widen<float, float>(float v) { return v; }
template <> __device__ __forceinline__ float widen<float, bf16>(bf16 v) { return to_f32(v); }

// Narrow an accumulator to the stored output type (round to nearest even).
template <typename O, typename Acc>
__device__ __forceinline__ O narrow(Acc v) { return static_cast<O>(v); }

// Non-temporal streaming loads for arrays read exactly once (crd, vals):
// keeps them from evicting the gathered dense operand from the caches.
template <typename T>
__device__ __forceinline__ T load_stream(const T *p) {
    return __builtin_nontemporal_load(p);
}
__device__ __forceinline__ bf16 load_stream(const bf16 *p) {
    bf16 r;
    r.bits = __builtin_nontemporal_load(&p->bits);
    return r;
}

// Non-temporal stores for outputs written exactly once, so that the
// streamed results do not evict the gathered dense operand from L2/MALL.
template <typename T>
__device__ __forceinline__ void store_stream(T *p, T v) {
    __builtin_nontemporal_store(v, p);
}

// Sum over aligned groups of L lanes (L a power of two <= 64) with xor
// butterflies; every lane of the group ends with the group total.
template <int L, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, L);
    return v;
}

// Merge-path search (Merrill and Garland, SC'16) over the sequence of row
// ends `ends[0..nr)` and the positions base, base+1, ..., base+np-1.  A row
// end e precedes position q when e <= q.  Returns the number of row ends
// among the first d merged items.
template <typename EndFn>
__device__ __forceinline__ int64_t merge_search(int64_t d, int64_t nr, int64_t np,
                                                int64_t base, EndFn end_at) {
    int64_t lo = d > np ? d - np : 0;
    int64_t hi = d < nr ? d : nr;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (static_cast<int64_t>(end_at(mid)) <= base + d - mid - 1)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

__host__ __device__ __forceinline__ int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// End of the next chunk of a leaf workgroup walking the merged sequence of
// row ends and positions from (ci, cp), inside partition piece `piece`
// (bounds trow/tpos[piece+1]): the piece's end if it lies within `chunk`
// items, else the merge-path point `chunk` items ahead, found by thread 0
// with a binary search over pos.  Writes (ei, ep) to s_next and returns the
// piece the walk is in afterwards.  Contains a workgroup barrier; every
// thread must call it.
__device__ __forceinline__ int64_t chunk_end(const int32_t *__restrict__ pos,
                                             const int32_t *__restrict__ trow,
                                             const int32_t *__restrict__ tpos, int64_t piece,
                                             int64_t ci, int64_t cp, int chunk,
                                             int64_t *s_next) {
    const int64_t bi = trow[piece + 1], bp = tpos[piece + 1];
    const bool whole = bi + bp - ci - cp <= chunk;
    if (threadIdx.x == 0) {
        if (whole) {
            s_next[0] = bi;
            s_next[1] = bp;
        } else {
            const int64_t k = merge_search(chunk, bi - ci, bp - cp, cp,
                                           [&](int64_t m) { return pos[ci + m + 1]; });
            s_next[0] = ci + k;
            s_next[1] = cp + chunk - k;
        }
    }
    __syncthreads();
    return whole ? piece + 1 : piece;
}

}  // namespace spl
