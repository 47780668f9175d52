// Content check of one Compressed level (paper Sec. III-B): pos starts at 0,
// never decreases and ends at the child count; every crd lies in
// [0, extent) and increases strictly within its segment.  Integer atomics
// record the failure kinds (bit mask) and the smallest failing parent.
#include "device.hpp"
#include "internal.hpp"

namespace spl {
namespace {

__global__ __launch_bounds__(kBlock) void k_validate(int64_t parents, const int32_t *__restrict__ pos,
                                                     const int32_t *__restrict__ crd,
                                                     int64_t children, int64_t extent,
                                                     unsigned long long *flags) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i > parents) return;
    unsigned code = 0;
    if (i == 0 && pos[0] != 0) code |= 1u;
    if (i == parents) {
        if (static_cast<int64_t>(pos[parents]) != children) code |= 4u;
    } else {
        const int64_t p0 = pos[i], p1 = pos[i + 1];
        if (p1 < p0) {
            code |= 2u;
        } else if (p0 >= 0 && p1 <= children) {
            int64_t prev = -1;
            for (int64_t p = p0; p < p1; ++p) {
                const int64_t c = crd[p];
                if (c < 0 || c >= extent) code |= 8u;
                if (c <= prev) code |= 16u;
                prev = c;
            }
        } else {
            code |= 4u;
        }
    }
    if (code) {
        atomicOr(reinterpret_cast<unsigned *>(flags), code);
        atomicMin(flags + 1, static_cast<unsigned long long>(i));
    }
}

}  // namespace

hipError_t launch_validate_level(int64_t parents, const int32_t *pos, const int32_t *crd,
                                 int64_t children, int64_t extent, int64_t *flags,
                                 hipStream_t s) {
    const int64_t work = parents + 1;
    k_validate<<<dim3(static_cast<unsigned>((work + kBlock - 1) / kBlock)), kBlock, 0, s>>>(
        parents, pos, crd, children, extent, reinterpret_cast<unsigned long long *>(flags));
    return hipGetLastError();
}

}  // namespace spl
