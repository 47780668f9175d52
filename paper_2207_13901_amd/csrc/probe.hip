// Memory-system probes used to put the leaf kernels' numbers in context:
//  - k_probe_stream: streams a buffer once (16-byte vector loads), the HBM
//    read ceiling for the streamed arrays (crd, vals, pos);
//  - k_probe_gather: reads `count` rows of `row_bytes` bytes at pseudo-random
//    row indices of a table (a SplitMix64 hash of the request number), the
//    ceiling for the random dense-operand gathers of SpMV/SpMM/MTTKRP/SDDMM
//    when the table does not fit in the caches;
//  - k_probe_gather_vec: the same gathers with 16-byte lanes.
// Both reduce what they read into one double per workgroup so nothing is
// optimized away.
#include "device.hpp"
#include "internal.hpp"

namespace spl {
namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ void block_store_sum(float v, double *out) {
    __shared__ float s[kBlock];
    s[threadIdx.x] = v;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = s[0];
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kBlock) void k_probe_stream(const f32x4 *__restrict__ buf,
                                                         int64_t n4, double *__restrict__ out) {
    float acc = 0.f;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n4; i += stride) {
        const f32x4 v = __builtin_nontemporal_load(buf + i);
        acc += v.x + v.y + v.z + v.w;
    }
    block_store_sum(acc, out);
}

// W lanes read one row of W * 4 bytes; each wave reads 64 / W rows per step.
template <int W>
__global__ __launch_bounds__(kBlock) void k_probe_gather(const float *__restrict__ table,
                                                         int64_t rows, int64_t count,
                                                         double *__restrict__ out) {
    // each lane group keeps kInFlight independent row reads outstanding
    constexpr int kInFlight = 8;
    float acc = 0.f;
    const int lane = threadIdx.x % W;
    const int64_t groups = static_cast<int64_t>(gridDim.x) * (kBlock / W);
    const int64_t g0 = static_cast<int64_t>(blockIdx.x) * (kBlock / W) + threadIdx.x / W;
    // rows used: the largest power of two <= rows, so the index is a mask
    // (a 64-bit modulo would make the probe compute-bound)
    uint64_t mask = 1;
    while (mask * 2 <= static_cast<uint64_t>(rows)) mask *= 2;
    mask -= 1;
    for (int64_t q0 = g0 * kInFlight; q0 < count; q0 += groups * kInFlight) {
        float v[kInFlight];
#pragma unroll
        for (int u = 0; u < kInFlight; ++u) {
            const int64_t q = q0 + u;
            const int64_t r = static_cast<int64_t>(mix64(static_cast<uint64_t>(q)) & mask);
            v[u] = q < count ? table[r * W + lane] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < kInFlight; ++u) acc += v[u];
    }
    block_store_sum(acc, out);
}

// As k_probe_gather with 16-byte lanes: W lanes read one row of W * 16
// bytes (the same rows per step as W * 4 four-byte lanes, in a quarter of
// the load instructions).
template <int W>
__global__ __launch_bounds__(kBlock) void k_probe_gather_vec(const f32x4 *__restrict__ table,
                                                             int64_t rows, int64_t count,
                                                             double *__restrict__ out) {
    constexpr int kInFlight = 8;
    float acc = 0.f;
    const int lane = threadIdx.x % W;
    const int64_t groups = static_cast<int64_t>(gridDim.x) * (kBlock / W);
    const int64_t g0 = static_cast<int64_t>(blockIdx.x) * (kBlock / W) + threadIdx.x / W;
    uint64_t mask = 1;
    while (mask * 2 <= static_cast<uint64_t>(rows)) mask *= 2;
    mask -= 1;
    for (int64_t q0 = g0 * kInFlight; q0 < count; q0 += groups * kInFlight) {
        f32x4 v[kInFlight];
#pragma unroll
        for (int u = 0; u < kInFlight; ++u) {
            const int64_t q = q0 + u;
            const int64_t r = static_cast<int64_t>(mix64(static_cast<uint64_t>(q)) & mask);
            v[u] = q < count ? table[r * W + lane] : f32x4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int u = 0; u < kInFlight; ++u) acc += v[u].x + v[u].y + v[u].z + v[u].w;
    }
    block_store_sum(acc, out);
}

}  // namespace

hipError_t launch_probe(int kind, const void *buf, int64_t bytes, int64_t row_bytes,
                        int64_t count, double *out, int64_t blocks, hipStream_t s) {
    dim3 grid(static_cast<unsigned>(blocks));
    if (kind == 0) {
        k_probe_stream<<<grid, kBlock, 0, s>>>(static_cast<const f32x4 *>(buf), bytes / 16, out);
        return hipGetLastError();
    }
    if (kind == 2) {
        const f32x4 *t4 = static_cast<const f32x4 *>(buf);
        switch (row_bytes) {
        case 16: k_probe_gather_vec<1><<<grid, kBlock, 0, s>>>(t4, bytes / 16, count, out); break;
        case 64: k_probe_gather_vec<4><<<grid, kBlock, 0, s>>>(t4, bytes / 64, count, out); break;
        case 256: k_probe_gather_vec<16><<<grid, kBlock, 0, s>>>(t4, bytes / 256, count, out); break;
        default: k_probe_gather_vec<8><<<grid, kBlock, 0, s>>>(t4, bytes / 128, count, out); break;
        }
        return hipGetLastError();
    }
    const float *t = static_cast<const float *>(buf);
    switch (row_bytes) {
    case 4: k_probe_gather<1><<<grid, kBlock, 0, s>>>(t, bytes / 4, count, out); break;
    case 8: k_probe_gather<2><<<grid, kBlock, 0, s>>>(t, bytes / 8, count, out); break;
    case 32: k_probe_gather<8><<<grid, kBlock, 0, s>>>(t, bytes / 32, count, out); break;
    case 64: k_probe_gather<16><<<grid, kBlock, 0, s>>>(t, bytes / 64, count, out); break;
    case 256: k_probe_gather<64><<<grid, kBlock, 0, s>>>(t, bytes / 256, count, out); break;
    default: k_probe_gather<32><<<grid, kBlock, 0, s>>>(t, bytes / 128, count, out); break;
    }
    return hipGetLastError();
}

}  // namespace spl
