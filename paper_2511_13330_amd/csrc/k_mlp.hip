// Kernels of the learned pulse proposal: a small multilayer perceptron with
// bfloat16 operands and FP32 accumulation on gfx950 MFMA
// (v_mfma_f32_16x16x16bf16_1k), GELU hidden layers and an amax*sigmoid head.
//
// One generic product C[i][j] = sum_k A(i,k) B(k,j) with arbitrary operand
// strides covers the forward (X W^T), the input gradient (G W) and the weight
// gradient (G^T X). A workgroup of four waves computes a 64 x 64 output tile;
// operand tiles of 64 x 32 are staged through LDS with the k index contiguous,
// so every lane reads its four consecutive k values of A and B in one 8-byte
// load. Epilogues are fused: bias + GELU (bf16 activations for the next
// product), bias + scaled sigmoid (head), and the GELU derivative of the
// backward pass.
#include "tile.hpp"
#include "internal.hpp"

namespace lmag {

typedef short s4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

constexpr int MT = 64, KT = 32, KP = KT + 8;   // tile edge, k step, padded LDS row

__global__ void __launch_bounds__(256) k_mlp_gemm(MlpGemmArgs a) {
  __shared__ uint16_t As[MT][KP];
  __shared__ uint16_t Bs[MT][KP];   // B tile stored transposed: Bs[j][k]
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, g = l >> 4, c = l & 15;
  const int wr = w >> 1, wc = w & 1;
  const int m0 = blockIdx.y * MT, n0 = blockIdx.x * MT;
  const uint16_t* A = a.A;
  const uint16_t* B = a.B;
  f4v acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4v{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < a.K; k0 += KT) {
    // stage: 64 x 32 elements of each operand, 8 per thread
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int idx = e * 256 + tid;
      const int r = idx / KT, kk = idx % KT;
      const int gi = m0 + r, gk = k0 + kk, gj = n0 + r;
      As[r][kk] = (gi < a.M && gk < a.K) ? A[(int64_t)gi * a.lda_r + (int64_t)gk * a.lda_c] : (uint16_t)0;
      Bs[r][kk] = (gj < a.N && gk < a.K) ? B[(int64_t)gk * a.ldb_r + (int64_t)gj * a.ldb_c] : (uint16_t)0;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < KT; ks += 16) {
      s4v av[2], bv[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const uint16_t* pa = &As[wr * 32 + i * 16 + c][ks + 4 * g];
        const uint16_t* pb = &Bs[wc * 32 + i * 16 + c][ks + 4 * g];
#pragma unroll
        for (int v = 0; v < 4; ++v) { av[i][v] = (short)pa[v]; bv[i][v] = (short)pb[v]; }
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // epilogue: element (row, col) of block (i, j) register r
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wr * 32 + i * 16 + 4 * g + r;
        const int col = n0 + wc * 32 + j * 16 + c;
        if (row >= a.M || col >= a.N) continue;
        const int64_t o = (int64_t)row * a.N + col;
        float v = acc[i][j][r];
        switch (a.mode) {
          case MLP_STORE:          // C (fp32)
            a.C32[o] = v;
            break;
          case MLP_BIAS_GELU:      // pre = v + b ; Y = bf16(gelu(pre))
            v += a.bias[col];
            if (a.C32) a.C32[o] = v;
            a.C16[o] = f2bf(gelu_f(v));
            break;
          case MLP_BIAS_SIGMOID:   // z = v + b ; Y = scale * sigmoid(z)
            v += a.bias[col];
            if (a.C32) a.C32[o] = v;
            a.Y32[o] = a.scale / (1.0f + expf(-v));
            break;
          case MLP_GELU_GRAD: {    // G_prev = v * gelu'(pre_prev): fp32 and bf16
            const float gp = v * gelu_grad_f(a.aux[o]);
            if (a.C32) a.C32[o] = gp;
            a.C16[o] = f2bf(gp);
            break;
          }
        }
      }
}

hipError_t launch_mlp_gemm(const MlpGemmArgs& a, hipStream_t s) {
  if (a.M <= 0 || a.N <= 0) return hipSuccess;
  const dim3 g((a.N + MT - 1) / MT, (a.M + MT - 1) / MT);
  hipLaunchKernelGGL(k_mlp_gemm, g, dim3(256), 0, s, a);
  return hipGetLastError();
}

// db[j] = sum_i G[i][j] in a fixed order (one thread per column).
__global__ void k_colsum(const float* G, int rows, int cols, float* out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cols) return;
  double s = 0.0;
  for (int i = 0; i < rows; ++i) s += (double)G[(int64_t)i * cols + j];
  out[j] = (float)s;
}

hipError_t launch_colsum(const float* G, int rows, int cols, float* out, hipStream_t s) {
  if (cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_colsum, dim3((cols + 255) / 256), dim3(256), 0, s, G, rows, cols, out);
  return hipGetLastError();
}

// MSE of sigmoid(z) against y: per-block partial sums in a fixed order, then a
// single-block final sum; dz = 2 (p - y) p (1 - p) / count.
constexpr int MSE_BLOCKS = 256;

__global__ void k_mse_partial(const float* z, const float* y, int64_t n, float* dz32, uint16_t* dz16,
                              double* part) {
  __shared__ double red[256];
  double s = 0.0;
  const double inv = 1.0 / (double)n;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float p = 1.0f / (1.0f + expf(-z[i]));
    const float d = p - y[i];
    s += (double)d * (double)d;
    const float g = (float)(2.0 * inv) * d * p * (1.0f - p);
    if (dz32) dz32[i] = g;
    if (dz16) dz16[i] = f2bf(g);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_mse_final(const double* part, int nb, int64_t n, double* loss) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < nb; ++i) s += part[i];
  *loss = s / (double)n;
}

hipError_t launch_mse(const float* z, const float* y, int64_t n, float* dz32, uint16_t* dz16,
                      double* part, double* loss, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mse_partial, dim3(MSE_BLOCKS), dim3(256), 0, s, z, y, n, dz32, dz16, part);
  hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(64), 0, s, (const double*)part, MSE_BLOCKS, n, loss);
  return hipGetLastError();
}

__global__ void k_cast_bf16(const float* in, uint16_t* out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = f2bf(in[i]);
}

hipError_t launch_cast_bf16(const float* in, uint16_t* out, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cast_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

}  // namespace lmag
