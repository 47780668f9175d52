// Learned schedule selection: cheap sparsity features of a CSR matrix and a
// small fully connected network (7 -> 64 -> 64 -> K, ReLU) that predicts,
// for each of K candidate schedules, its time relative to the best one.
// Training and inference run in these kernels; every reduction over the
// batch or the matrix has a fixed order, so results are reproducible.
//
// Parameter layout (FP32, one flat array):
//   W1[64][7], b1[64], W2[64][64], b2[64], W3[K][64], b3[K]  (K <= 256).
#include "device.hpp"
#include "internal.hpp"

namespace spl {
namespace {

constexpr int kIn = 7;
constexpr int kHid = 64;
constexpr int kFeatBlocks = 1024;

struct Layout {
    int64_t w1, b1, w2, b2, w3, b3, total;
};

__host__ __device__ inline Layout layout(int K) {
    Layout L;
    L.w1 = 0;
    L.b1 = L.w1 + kHid * kIn;
    L.w2 = L.b1 + kHid;
    L.b2 = L.w2 + kHid * kHid;
    L.w3 = L.b2 + kHid;
    L.b3 = L.w3 + static_cast<int64_t>(K) * kHid;
    L.total = L.b3 + K;
    return L;
}

// Per-workgroup partial sums of the feature statistics over rows:
// [sum deg, sum deg^2, max deg, max |col - row|, sum row span, empty rows].
__global__ __launch_bounds__(kBlock) void k_feature_partials(int64_t n, const int32_t *__restrict__ pos,
                                                             const int32_t *__restrict__ crd,
                                                             double *__restrict__ part) {
    double s1 = 0, s2 = 0, mx = 0, bw = 0, span = 0, empty = 0;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n; i += stride) {
        const int32_t p0 = pos[i], p1 = pos[i + 1];
        const double d = static_cast<double>(p1 - p0);
        s1 += d;
        s2 += d * d;
        mx = fmax(mx, d);
        if (p1 > p0) {
            const double first = crd[p0], last = crd[p1 - 1];
            const double row = static_cast<double>(i);
            bw = fmax(bw, fmax(fabs(first - row), fabs(last - row)));
            span += last - first + 1.0;
        } else {
            empty += 1.0;
        }
    }
    __shared__ double s[6][kBlock];
    s[0][threadIdx.x] = s1;
    s[1][threadIdx.x] = s2;
    s[2][threadIdx.x] = mx;
    s[3][threadIdx.x] = bw;
    s[4][threadIdx.x] = span;
    s[5][threadIdx.x] = empty;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            s[0][threadIdx.x] += s[0][threadIdx.x + w];
            s[1][threadIdx.x] += s[1][threadIdx.x + w];
            s[2][threadIdx.x] = fmax(s[2][threadIdx.x], s[2][threadIdx.x + w]);
            s[3][threadIdx.x] = fmax(s[3][threadIdx.x], s[3][threadIdx.x + w]);
            s[4][threadIdx.x] += s[4][threadIdx.x + w];
            s[5][threadIdx.x] += s[5][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = s[threadIdx.x][0];
}

// Combine the partials (fixed order) and write the 7 features:
//  log2(rows), log2(nnz+1), mean degree, log2(1 + degree variance),
//  log2(1 + max degree), log2(1 + bandwidth), mean row span / columns.
__global__ __launch_bounds__(kBlock) void k_feature_final(int64_t n, int64_t m, int64_t nblocks,
                                                          const double *__restrict__ part,
                                                          float *__restrict__ feat) {
    __shared__ double s[6][kBlock];
    double a[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t b = threadIdx.x; b < nblocks; b += kBlock) {
        a[0] += part[b * 6 + 0];
        a[1] += part[b * 6 + 1];
        a[2] = fmax(a[2], part[b * 6 + 2]);
        a[3] = fmax(a[3], part[b * 6 + 3]);
        a[4] += part[b * 6 + 4];
        a[5] += part[b * 6 + 5];
    }
    for (int k = 0; k < 6; ++k) s[k][threadIdx.x] = a[k];
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            s[0][threadIdx.x] += s[0][threadIdx.x + w];
            s[1][threadIdx.x] += s[1][threadIdx.x + w];
            s[2][threadIdx.x] = fmax(s[2][threadIdx.x], s[2][threadIdx.x + w]);
            s[3][threadIdx.x] = fmax(s[3][threadIdx.x], s[3][threadIdx.x + w]);
            s[4][threadIdx.x] += s[4][threadIdx.x + w];
            s[5][threadIdx.x] += s[5][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double rows = static_cast<double>(n > 0 ? n : 1);
        const double nnz = s[0][0];
        const double mean = nnz / rows;
        const double var = fmax(0.0, s[1][0] / rows - mean * mean);
        const double nonempty = fmax(1.0, rows - s[5][0]);
        feat[0] = static_cast<float>(log2(rows));
        feat[1] = static_cast<float>(log2(nnz + 1.0));
        feat[2] = static_cast<float>(mean);
        feat[3] = static_cast<float>(log2(1.0 + var));
        feat[4] = static_cast<float>(log2(1.0 + s[2][0]));
        feat[5] = static_cast<float>(log2(1.0 + s[3][0]));
        feat[6] = static_cast<float>(s[4][0] / nonempty / static_cast<double>(m > 0 ? m : 1));
    }
}

// Forward pass, one workgroup of 64 lanes per sample: lane j computes hidden
// unit j of each layer.  Inputs are standardized with (mu, istd) when given:
// x = (X - mu) * istd.  Activations go to
// act = [H1 (B x 64), H2 (B x 64), x (B x 7)] for the backward pass.
__global__ __launch_bounds__(kHid) void k_mlp_forward(int K, const float *__restrict__ P,
                                                      const float *__restrict__ X,
                                                      const float *__restrict__ norm, int64_t B,
                                                      float *__restrict__ Y, float *__restrict__ act) {
    const Layout L = layout(K);
    const int64_t b = blockIdx.x;
    const int j = threadIdx.x;
    __shared__ float s_x[kIn];
    __shared__ float s_h1[kHid];
    __shared__ float s_h2[kHid];
    if (j < kIn) {
        float x = X[b * kIn + j];
        if (norm) x = (x - norm[j]) * norm[kIn + j];
        s_x[j] = x;
        if (act) act[2 * B * kHid + b * kIn + j] = x;
    }
    __syncthreads();
    float z = P[L.b1 + j];
    for (int i = 0; i < kIn; ++i) z += P[L.w1 + j * kIn + i] * s_x[i];
    const float h1 = z > 0.f ? z : 0.f;
    s_h1[j] = h1;
    __syncthreads();
    z = P[L.b2 + j];
    for (int i = 0; i < kHid; ++i) z += P[L.w2 + j * kHid + i] * s_h1[i];
    const float h2 = z > 0.f ? z : 0.f;
    s_h2[j] = h2;
    if (act) {
        act[b * kHid + j] = h1;
        act[B * kHid + b * kHid + j] = h2;
    }
    __syncthreads();
    for (int k = j; k < K; k += kHid) {
        float y = P[L.b3 + k];
        for (int i = 0; i < kHid; ++i) y += P[L.w3 + static_cast<int64_t>(k) * kHid + i] * s_h2[i];
        Y[b * K + k] = y;
    }
}

// Backward pass for the mean squared error L = mean_{b,k} (Y - T)^2, one
// workgroup per sample: per-sample gradients of the pre-activations
// dZ = [dZ1 (B x 64), dZ2 (B x 64), dZ3 (B x K)] and the per-sample loss.
__global__ __launch_bounds__(kHid) void k_mlp_backward_sample(int K, const float *__restrict__ P,
                                                              int64_t B, const float *__restrict__ Y,
                                                              const float *__restrict__ T,
                                                              const float *__restrict__ act,
                                                              float *__restrict__ dZ,
                                                              float *__restrict__ loss_b) {
    const Layout L = layout(K);
    const int64_t b = blockIdx.x;
    const int j = threadIdx.x;
    const float scale = 2.0f / static_cast<float>(B * K);
    __shared__ float s_d3[256];
    __shared__ float s_d2[kHid];
    __shared__ float s_l[kHid];
    float l = 0.f;
    for (int k = j; k < K; k += kHid) {
        const float e = Y[b * K + k] - T[b * K + k];
        l += e * e;
        const float d = scale * e;
        s_d3[k] = d;
        dZ[2 * B * kHid + b * K + k] = d;
    }
    s_l[j] = l;
    __syncthreads();
    const float h2 = act[B * kHid + b * kHid + j];
    float g = 0.f;
    for (int k = 0; k < K; ++k) g += P[L.w3 + static_cast<int64_t>(k) * kHid + j] * s_d3[k];
    const float d2 = h2 > 0.f ? g : 0.f;
    s_d2[j] = d2;
    dZ[B * kHid + b * kHid + j] = d2;
    __syncthreads();
    const float h1 = act[b * kHid + j];
    g = 0.f;
    for (int i = 0; i < kHid; ++i) g += P[L.w2 + i * kHid + j] * s_d2[i];
    dZ[b * kHid + j] = h1 > 0.f ? g : 0.f;
    if (j == 0) {
        float t = 0.f;
        for (int i = 0; i < kHid; ++i) t += s_l[i];
        loss_b[b] = t;
    }
}

// Parameter gradients: one lane per parameter, summing over the batch in
// sample order.  grad has the parameter layout; loss = mean squared error.
__global__ __launch_bounds__(kBlock) void k_mlp_grad(int K, int64_t B,
                                                     const float *__restrict__ act,
                                                     const float *__restrict__ dZ,
                                                     const float *__restrict__ loss_b,
                                                     float *__restrict__ grad,
                                                     float *__restrict__ loss) {
    const Layout L = layout(K);
    const int64_t q = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (q == 0 && loss) {
        float t = 0.f;
        for (int64_t b = 0; b < B; ++b) t += loss_b[b];
        *loss = t / static_cast<float>(B * K);
    }
    if (q >= L.total) return;
    const float *H1 = act, *H2 = act + B * kHid, *X = act + 2 * B * kHid;
    const float *D1 = dZ, *D2 = dZ + B * kHid, *D3 = dZ + 2 * B * kHid;
    float g = 0.f;
    if (q < L.b1) {  // W1[j][i]
        const int j = static_cast<int>(q / kIn), i = static_cast<int>(q % kIn);
        for (int64_t b = 0; b < B; ++b) g += D1[b * kHid + j] * X[b * kIn + i];
    } else if (q < L.w2) {  // b1[j]
        const int j = static_cast<int>(q - L.b1);
        for (int64_t b = 0; b < B; ++b) g += D1[b * kHid + j];
    } else if (q < L.b2) {  // W2[j][i]
        const int64_t r = q - L.w2;
        const int j = static_cast<int>(r / kHid), i = static_cast<int>(r % kHid);
        for (int64_t b = 0; b < B; ++b) g += D2[b * kHid + j] * H1[b * kHid + i];
    } else if (q < L.w3) {  // b2[j]
        const int j = static_cast<int>(q - L.b2);
        for (int64_t b = 0; b < B; ++b) g += D2[b * kHid + j];
    } else if (q < L.b3) {  // W3[k][i]
        const int64_t r = q - L.w3;
        const int k = static_cast<int>(r / kHid), i = static_cast<int>(r % kHid);
        for (int64_t b = 0; b < B; ++b) g += D3[b * K + k] * H2[b * kHid + i];
    } else {  // b3[k]
        const int k = static_cast<int>(q - L.b3);
        for (int64_t b = 0; b < B; ++b) g += D3[b * K + k];
    }
    grad[q] = g;
}

// Adam (Kingma and Ba, ICLR 2015) with bias correction at step t >= 1.
__global__ __launch_bounds__(kBlock) void k_adam(int64_t n, float *__restrict__ P,
                                                 float *__restrict__ m, float *__restrict__ v,
                                                 const float *__restrict__ g, float lr, float b1,
                                                 float b2, float eps, float c1, float c2) {
    const int64_t q = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (q >= n) return;
    const float gq = g[q];
    const float mq = b1 * m[q] + (1.f - b1) * gq;
    const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
    m[q] = mq;
    v[q] = vq;
    const float mh = mq / c1, vh = vq / c2;
    P[q] -= lr * mh / (sqrtf(vh) + eps);
}

}  // namespace

int64_t mlp_param_count(int K) { return layout(K).total; }
int64_t feature_ws_bytes() { return kFeatBlocks * 6 * sizeof(double); }

hipError_t launch_features(int64_t n, int64_t m, const int32_t *pos, const int32_t *crd,
                           double *part, float *feat, hipStream_t s) {
    k_feature_partials<<<kFeatBlocks, kBlock, 0, s>>>(n, pos, crd, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_feature_final<<<1, kBlock, 0, s>>>(n, m, kFeatBlocks, part, feat);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(int K, const float *P, const float *X, const float *norm,
                              int64_t B, float *Y, float *act, hipStream_t s) {
    if (B == 0) return hipSuccess;
    k_mlp_forward<<<dim3(static_cast<unsigned>(B)), kHid, 0, s>>>(K, P, X, norm, B, Y, act);
    return hipGetLastError();
}

hipError_t launch_mlp_backward(int K, const float *P, int64_t B, const float *Y, const float *T,
                               const float *act, float *dZ, float *loss_b, float *grad,
                               float *loss, hipStream_t s) {
    if (B == 0) return hipSuccess;
    k_mlp_backward_sample<<<dim3(static_cast<unsigned>(B)), kHid, 0, s>>>(K, P, B, Y, T, act, dZ,
                                                                           loss_b);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t n = layout(K).total;
    k_mlp_grad<<<dim3(static_cast<unsigned>(ceil_div(n, kBlock))), kBlock, 0, s>>>(
        K, B, act, dZ, loss_b, grad, loss);
    return hipGetLastError();
}

hipError_t launch_adam(int64_t n, float *P, float *m, float *v, const float *g, float lr, float b1,
                       float b2, float eps, int step, hipStream_t s) {
    const float c1 = 1.f - powf(b1, static_cast<float>(step));
    const float c2 = 1.f - powf(b2, static_cast<float>(step));
    k_adam<<<dim3(static_cast<unsigned>(ceil_div(n, kBlock))), kBlock, 0, s>>>(n, P, m, v, g, lr,
                                                                               b1, b2, eps, c1, c2);
    return hipGetLastError();
}

}  // namespace spl
