// Kernels of the cost-model MLP (16 -> 64 -> 64 -> 2, ReLU), the learned
// replacement of the paper's shallow cost network (Section 4.2, "Shallow
// NNs"): a matrix-core GEMM with bf16 operands and fp32 accumulation, fused
// bias / ReLU / ReLU-mask epilogues, column sums for bias gradients, the
// mean-squared-error gradient and Adam.
#include "hb_internal.h"

namespace hb {

namespace {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// float32 -> bf16 bits, round to nearest, ties to even (finite inputs)
__device__ inline short to_bf16(float x) {
    uint32_t b = __float_as_uint(x);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return (short)(b >> 16);
}

// One wave computes a 16 x 16 tile of C = op(A) op(B) with the 16x16x16
// bf16 matrix instruction.  Operand layout of that instruction: lane l holds
// A[l % 16][4 (l / 16) + e] and B[4 (l / 16) + e][l % 16], e = 0..3, and
// receives D[4 (l / 16) + e][l % 16].
__global__ __launch_bounds__(64) void k_gemm(const GemmArgs g) {
    const int l = threadIdx.x;
    const int tm = blockIdx.x * 16, tn = blockIdx.y * 16;
    const int r16 = l & 15, kq = (l >> 4) * 4;
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < g.K; k0 += 16) {
        v4s a, b;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int k = k0 + kq + e;
            const int i = tm + r16, j = tn + r16;
            float av = 0.f, bv = 0.f;
            if (i < g.M && k < g.K) av = g.transA ? g.A[(size_t)k * g.lda + i] : g.A[(size_t)i * g.lda + k];
            if (j < g.N && k < g.K) bv = g.transB ? g.B[(size_t)j * g.ldb + k] : g.B[(size_t)k * g.ldb + j];
            a[e] = to_bf16(av);
            b[e] = to_bf16(bv);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int i = tm + (l >> 4) * 4 + e, j = tn + r16;
        if (i >= g.M || j >= g.N) continue;
        float v = acc[e];
        if (g.bias) v += g.bias[j];
        if (g.mask && !(g.mask[(size_t)i * g.ldc + j] > 0.f)) v = 0.f;
        g.C[(size_t)i * g.ldc + j] = v;
        if (g.relu) g.relu[(size_t)i * g.ldc + j] = v > 0.f ? v : 0.f;
    }
}

// out[j] = sum_i A[i][j], one thread per column
__global__ void k_colsum(const float* __restrict__ A, int rows, int cols, float* __restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= cols) return;
    float s = 0.f;
    for (int i = 0; i < rows; ++i) s += A[(size_t)i * cols + j];
    out[j] = s;
}

// dY = 2 (Y - T) / (rows * cols); sum of squared errors into *sse
__global__ void k_mse_grad(const float* __restrict__ Y, const float* __restrict__ T, int n, float scale,
                           float* __restrict__ dY, float* __restrict__ sse) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    float e2 = 0.f;
    if (x < n) {
        const float d = Y[x] - T[x];
        dY[x] = 2.f * d * scale;
        e2 = d * d;
    }
    for (int o = 32; o > 0; o >>= 1) e2 += __shfl_xor(e2, o);
    if ((threadIdx.x & 63) == 0 && sse) atomicAdd(sse, e2);
}

__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int n, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const float gx = g[x];
    const float mx = b1 * m[x] + (1.f - b1) * gx;
    const float vx = b2 * v[x] + (1.f - b2) * gx * gx;
    m[x] = mx;
    v[x] = vx;
    w[x] -= lr * (mx * c1) / (sqrtf(vx * c2) + eps);
}

// Inference of the whole network, 16 rows per wave step, with the
// activations never leaving registers.  Each layer computes the transposed
// product Y^T = W^T X^T: with the matrix instruction's layouts its result
// D[o][row] sits exactly where the next layer's B operand X^T[k][row] is
// expected, so no transpose is needed.  W^T tiles are the A operands, kept
// in registers across the wave's row tiles.  Operands are rounded to bf16
// as in k_gemm; bias, ReLU and accumulation stay fp32.
constexpr int kIn = 16, kHid = 64;
constexpr int kW1 = 0, kB1 = kW1 + kIn * kHid, kW2 = kB1 + kHid, kB2 = kW2 + kHid * kHid;
constexpr int kW3 = kB2 + kHid, kB3 = kW3 + kHid * 2;

__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ W, const float* __restrict__ x,
                                                     uint64_t n, float* __restrict__ y) {
    const int l = threadIdx.x & 63;
    const int r16 = l & 15, kq = (l >> 4) * 4;
    // A operands: W^T[o][k] = W[k][o]; lane holds A[r16][kq + e]
    v4s a1[4], a2[4][4], a3[4];
#pragma unroll
    for (int ot = 0; ot < 4; ++ot)
#pragma unroll
        for (int e = 0; e < 4; ++e) a1[ot][e] = to_bf16(W[kW1 + (kq + e) * kHid + ot * 16 + r16]);
#pragma unroll
    for (int ot = 0; ot < 4; ++ot)
#pragma unroll
        for (int kt = 0; kt < 4; ++kt)
#pragma unroll
            for (int e = 0; e < 4; ++e) a2[ot][kt][e] = to_bf16(W[kW2 + (kt * 16 + kq + e) * kHid + ot * 16 + r16]);
#pragma unroll
    for (int kt = 0; kt < 4; ++kt)
#pragma unroll
        for (int e = 0; e < 4; ++e) a3[kt][e] = r16 < 2 ? to_bf16(W[kW3 + (kt * 16 + kq + e) * 2 + r16]) : (short)0;
    // biases at the D positions o = ot * 16 + kq + e
    float b1[4][4], b2[4][4], b3[4];
#pragma unroll
    for (int ot = 0; ot < 4; ++ot)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            b1[ot][e] = W[kB1 + ot * 16 + kq + e];
            b2[ot][e] = W[kB2 + ot * 16 + kq + e];
        }
#pragma unroll
    for (int e = 0; e < 4; ++e) b3[e] = kq + e < 2 ? W[kB3 + kq + e] : 0.f;

    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    for (uint64_t t = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); t * 16 < n; t += waves) {
        const uint64_t row = t * 16 + r16;
        // B operand of layer 1: X^T[k][row], lane holds k = kq + e
        v4s xb;
#pragma unroll
        for (int e = 0; e < 4; ++e) xb[e] = to_bf16(row < n ? x[row * kIn + kq + e] : 0.f);
        v4s h1[4];
#pragma unroll
        for (int ot = 0; ot < 4; ++ot) {
            v4f acc = {0.f, 0.f, 0.f, 0.f};
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1[ot], xb, acc, 0, 0, 0);
#pragma unroll
            for (int e = 0; e < 4; ++e) h1[ot][e] = to_bf16(fmaxf(acc[e] + b1[ot][e], 0.f));
        }
        v4s h2[4];
#pragma unroll
        for (int ot = 0; ot < 4; ++ot) {
            v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kt = 0; kt < 4; ++kt) acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a2[ot][kt], h1[kt], acc, 0, 0, 0);
#pragma unroll
            for (int e = 0; e < 4; ++e) h2[ot][e] = to_bf16(fmaxf(acc[e] + b2[ot][e], 0.f));
        }
        v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kt = 0; kt < 4; ++kt) acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a3[kt], h2[kt], acc, 0, 0, 0);
        // D[o][row]: o = kq + e, outputs 0 and 1 on lanes 0..15
        if (kq == 0 && row < n) {
            y[row * 2 + 0] = acc[0] + b3[0];
            y[row * 2 + 1] = acc[1] + b3[1];
        }
    }
}

}  // namespace

hipError_t launch_mlp_forward(const float* W, const float* x, uint64_t n, float* y, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const uint64_t tiles = (n + 15) / 16;
    const unsigned blocks = (unsigned)std::min<uint64_t>((tiles + 3) / 4, 4096);
    k_mlp_forward<<<blocks, 256, 0, s>>>(W, x, n, y);
    return hipGetLastError();
}

hipError_t launch_gemm(const GemmArgs& g, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    dim3 grid((g.M + 15) / 16, (g.N + 15) / 16);
    k_gemm<<<grid, 64, 0, s>>>(g);
    return hipGetLastError();
}

hipError_t launch_colsum(const float* A, int rows, int cols, float* out, hipStream_t s) {
    k_colsum<<<(cols + 63) / 64, 64, 0, s>>>(A, rows, cols, out);
    return hipGetLastError();
}

hipError_t launch_mse_grad(const float* Y, const float* T, int n, float scale, float* dY, float* sse,
                           hipStream_t s) {
    k_mse_grad<<<(n + 255) / 256, 256, 0, s>>>(Y, T, n, scale, dY, sse);
    return hipGetLastError();
}

hipError_t launch_adam(float* w, const float* g, float* m, float* v, int n, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t s) {
    k_adam<<<(n + 255) / 256, 256, 0, s>>>(w, g, m, v, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

}  // namespace hb
