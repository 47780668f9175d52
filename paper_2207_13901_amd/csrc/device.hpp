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

// Rows of a dense operand read and written VEC consecutive elements per lane
// (VEC > 1: one vector access of VEC elements, 16 bytes except for 4 BF16;
// the address must be aligned to the access size).
typedef float vf32x4 __attribute__((ext_vector_type(4)));
typedef double vf64x2 __attribute__((ext_vector_type(2)));
typedef uint32_t vu32x4 __attribute__((ext_vector_type(4)));

template <int VEC, typename Acc>
__device__ __forceinline__ void load_row(const float *p, Acc (&o)[VEC]) {
    if constexpr (VEC == 1) {
        o[0] = *p;
    } else {
        static_assert(VEC == 4, "FP32 rows: 1 or 4 per lane");
        const vf32x4 v = *reinterpret_cast<const vf32x4 *>(p);
        o[0] = v.x;
        o[1] = v.y;
        o[2] = v.z;
        o[3] = v.w;
    }
}
template <int VEC, typename Acc>
__device__ __forceinline__ void load_row(const double *p, Acc (&o)[VEC]) {
    if constexpr (VEC == 1) {
        o[0] = *p;
    } else {
        static_assert(VEC == 2, "FP64 rows: 1 or 2 per lane");
        const vf64x2 v = *reinterpret_cast<const vf64x2 *>(p);
        o[0] = v.x;
        o[1] = v.y;
    }
}
template <int VEC, typename Acc>
__device__ __forceinline__ void load_row(const bf16 *p, Acc (&o)[VEC]) {
    if constexpr (VEC == 1) {
        o[0] = to_f32(*p);
    } else if constexpr (VEC == 4) {
        typedef uint32_t vu32x2 __attribute__((ext_vector_type(2)));
        const vu32x2 v = *reinterpret_cast<const vu32x2 *>(p);  // 8-byte access
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            o[2 * k] = __uint_as_float(v[k] << 16);
            o[2 * k + 1] = __uint_as_float(v[k] & 0xffff0000u);
        }
    } else {
        static_assert(VEC == 8, "BF16 rows: 1, 4 or 8 per lane");
        // element 2k in the low half of word k (little-endian)
        const vu32x4 v = *reinterpret_cast<const vu32x4 *>(p);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            o[2 * k] = __uint_as_float(v[k] << 16);
            o[2 * k + 1] = __uint_as_float(v[k] & 0xffff0000u);
        }
    }
}

template <int VEC, typename Acc>
__device__ __forceinline__ void store_row(float *p, const Acc (&a)[VEC]) {
    if constexpr (VEC == 1) {
        __builtin_nontemporal_store(static_cast<float>(a[0]), p);
    } else {
#pragma unroll
        for (int q = 0; q < VEC; q += 4) {
            vf32x4 v = {static_cast<float>(a[q]), static_cast<float>(a[q + 1]),
                        static_cast<float>(a[q + 2]), static_cast<float>(a[q + 3])};
            __builtin_nontemporal_store(v, reinterpret_cast<vf32x4 *>(p + q));
        }
    }
}
template <int VEC, typename Acc>
__device__ __forceinline__ void store_row(double *p, const Acc (&a)[VEC]) {
    if constexpr (VEC == 1) {
        __builtin_nontemporal_store(static_cast<double>(a[0]), p);
    } else {
        static_assert(VEC == 2, "FP64 rows: 1 or 2 per lane");
        vf64x2 v = {static_cast<double>(a[0]), static_cast<double>(a[1])};
        __builtin_nontemporal_store(v, reinterpret_cast<vf64x2 *>(p));
    }
}

// VEC consecutive elements of a gathered dense row, held as loaded: FP32
// and FP64 as values, BF16 packed two per 32-bit register and widened only
// when read (at), so a row segment in flight takes half the registers.
template <int VEC, typename BT>
struct RowVec {
    BT v[VEC];
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int k = 0; k < VEC; ++k) v[k] = 0;
    }
    __device__ __forceinline__ void load(const BT *p) { load_row<VEC>(p, v); }
    // 16 bytes at byte offset `off` of buffer `r` (4 FP32 or 2 FP64)
    __device__ __forceinline__ void load_buf(__amdgpu_buffer_rsrc_t r, uint32_t off) {
        static_assert(VEC * sizeof(BT) == 16, "16-byte lanes");
        typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
        const u32x4 x = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
        // (__builtin_bit_cast of a vector element here compiled to a
        // one-dword load: the integer-to-float intrinsics instead)
        if constexpr (sizeof(BT) == 4) {
#pragma unroll
            for (int k = 0; k < VEC; ++k) v[k] = __uint_as_float(x[k]);
        } else {
#pragma unroll
            for (int k = 0; k < VEC; ++k) v[k] = __hiloint2double(x[2 * k + 1], x[2 * k]);
        }
    }
    __device__ __forceinline__ BT at(int k) const { return v[k]; }
};
template <int VEC>
struct RowVec<VEC, bf16> {
    static constexpr int kWords = VEC == 1 ? 1 : VEC / 2;
    uint32_t w[kWords];
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int k = 0; k < kWords; ++k) w[k] = 0;
    }
    __device__ __forceinline__ void load(const bf16 *p) {
        if constexpr (VEC == 1) {
            w[0] = static_cast<uint32_t>(p->bits) << 16;
        } else if constexpr (VEC == 4) {
            typedef uint32_t vu32x2 __attribute__((ext_vector_type(2)));
            const vu32x2 x = *reinterpret_cast<const vu32x2 *>(p);  // 8-byte access
            w[0] = x[0];
            w[1] = x[1];
        } else {
            static_assert(VEC == 8, "BF16 rows: 1, 4 or 8 per lane");
            const vu32x4 x = *reinterpret_cast<const vu32x4 *>(p);  // 16-byte access
#pragma unroll
            for (int k = 0; k < 4; ++k) w[k] = x[k];
        }
    }
    // 8 (VEC 4) or 16 (VEC 8) bytes at byte offset `off` of buffer `r`
    __device__ __forceinline__ void load_buf(__amdgpu_buffer_rsrc_t r, uint32_t off) {
        if constexpr (VEC == 4) {
            typedef uint32_t vu32x2 __attribute__((ext_vector_type(2)));
            const vu32x2 x = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
            w[0] = x[0];
            w[1] = x[1];
        } else {
            static_assert(VEC == 8, "BF16 buffer rows: 4 or 8 per lane");
            const vu32x4 x = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
#pragma unroll
            for (int k = 0; k < 4; ++k) w[k] = x[k];
        }
    }
    // element 2k sits in the low half of word k (little-endian)
    __device__ __forceinline__ float at(int k) const {
        if constexpr (VEC == 1) return __uint_as_float(w[0]);
        return __uint_as_float((k & 1) ? (w[k >> 1] & 0xffff0000u) : (w[k >> 1] << 16));
    }
};

// Buffer loads for gathers that must not branch.  A lane's load is issued
// whether or not the lane needs it: a lane that does not passes kBufOut as
// its offset, which lies past every descriptor range used here, so the
// hardware's range check returns 0 without touching memory.  With no
// per-lane branch around them, the compiler counts the loads exactly and
// waits for each result only when it is used; a load inside a lane-masked
// branch makes it assume the worst and wait for nearly everything before
// the next dependent load (for a batch of gathers: one or two in flight).
// Ranges are at most kBufRange bytes (internal.hpp), so the offsets of
// every in-bounds access fit 32 bits; callers keep to spans of that size.
constexpr uint32_t kBufOut = 0xFFFFFFF0u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t span_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, bytes, 0x00020000);
}
// 4-byte element at byte offset `off`.  AUX is the cache policy: 2 (the
// default) non-temporal, for arrays streamed once; 0 where later loads of
// the same lines follow (neighbouring lanes or the next instructions).
template <int AUX = 2>
__device__ __forceinline__ uint32_t buf_u32(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, AUX);
}
template <int AUX = 2>
__device__ __forceinline__ float buf_val(const float *, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, AUX));
}
template <int AUX = 2>
__device__ __forceinline__ float buf_val(const bf16 *, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __uint_as_float(static_cast<uint32_t>(__builtin_amdgcn_raw_buffer_load_b16(r, off, 0, AUX))
                           << 16);
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
template <typename P>
__device__ __forceinline__ int64_t chunk_end(const P *__restrict__ pos,
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
                                           [&](int64_t m) { return static_cast<int64_t>(pos[ci + m + 1]); });
            s_next[0] = ci + k;
            s_next[1] = cp + chunk - k;
        }
    }
    __syncthreads();
    return whole ? piece + 1 : piece;
}

}  // namespace spl
