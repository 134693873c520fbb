// Block-tiled path in a real representation. Every matrix of the path (the
// Liouvillian basis, the Magnus exponents and their commutators, the slice
// exponentials, the chain and scan products, the target channel) maps
// Hermitian matrices to Hermitian matrices, so in the orthonormal basis of
// Hermitian operators
//   |k><k|,  (|k><l| + |l><k|) / sqrt 2,  i (|k><l| - |l><k|) / sqrt 2  (k < l)
// it is a real n x n matrix (n = d^2). The change of basis T is unitary (2 x 2
// blocks on the index pairs p = k + l d, q = l + k d), so products, traces and
// the process fidelity are those of the column-stacking form up to rounding,
// and the propagator goes back to column stacking as T^dag (I + R) T. A real
// product is one MFMA product where the complex one takes three (3M), on tiles
// of half the bytes.
#include <hip/hip_runtime.h>
#include <algorithm>
#include <cmath>

#include "tile.hpp"
#include "internal.hpp"
#include "big.hpp"
#include "pade.hpp"

namespace lmag {

namespace {

typedef float f4v __attribute__((ext_vector_type(4)));

// Real 64 x 64 register tile in the 16x16x4 MFMA output layout: lane (w, g, c)
// holds column 16 w + c and rows 16 q + 4 g + r in v[q][r].
struct RTR {
  f4v v[4];
};

__device__ __forceinline__ void rr_zero(RTR& X) {
#pragma unroll
  for (int q = 0; q < 4; ++q) X.v[q] = f4v{0.f, 0.f, 0.f, 0.f};
}
__device__ __forceinline__ void rr_load(RTR& X, const float* __restrict__ M, int ld) {
  const Lane L;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) X.v[q][r] = M[(size_t)(16 * q + 4 * L.g + r) * ld + L.col];
}
__device__ __forceinline__ void rr_store(const RTR& X, float* __restrict__ M, int ld) {
  const Lane L;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) M[(size_t)(16 * q + 4 * L.g + r) * ld + L.col] = X.v[q][r];
}
__device__ __forceinline__ void rr_scale(RTR& X, float a) {
#pragma unroll
  for (int q = 0; q < 4; ++q) X.v[q] *= a;
}
__device__ __forceinline__ void rr_axpy(RTR& Y, float a, const RTR& X) {
#pragma unroll
  for (int q = 0; q < 4; ++q) Y.v[q] += a * X.v[q];
}
__device__ __forceinline__ void rr_add_diag(RTR& X, float a) {
  const Lane L;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (16 * q + 4 * L.g + r == L.col) X.v[q][r] += a;
}

__device__ __forceinline__ const float* rmat(const void* base, const int32_t* idx, int b, size_t nn) {
  return reinterpret_cast<const float*>(base) + (size_t)(idx ? idx[b] : b) * nn;
}

// LDS pitch of a staged A tile in floats: 68 = 64 + 4 puts the 16-byte reads of
// one column position by 16 consecutive rows on 16 different bank groups.
constexpr int RPITCH = 68;

// acc += A B, A staged in LDS (pitch RPITCH), B in registers; k = 16 kb + 4 g + t
// as in the register layout, so each lane reads its four A values of a k-block
// with one 16-byte load.
__device__ __forceinline__ void rr_gemm(RTR& acc, const float* __restrict__ A, const RTR& B) {
  const Lane L;
  const int g = L.g, c = L.c;
  f4v cur[4], nxt[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) cur[q] = *reinterpret_cast<const f4v*>(A + (16 * q + c) * RPITCH + 4 * g);
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) {
    if (kb + 1 < 4) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        nxt[q] = *reinterpret_cast<const f4v*>(A + (16 * q + c) * RPITCH + 16 * (kb + 1) + 4 * g);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const float b = B.v[kb][t];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc.v[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(cur[q][t], b, acc.v[q], 0, 0, 0);
    }
    __builtin_amdgcn_sched_barrier(0);
    if (kb + 1 < 4) {
#pragma unroll
      for (int q = 0; q < 4; ++q) cur[q] = nxt[q];
    }
  }
}

__device__ __forceinline__ void rr_stage(const RTR& X, float* S) {
  const Lane L;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) S[(16 * q + 4 * L.g + r) * RPITCH + L.col] = X.v[q][r];
}

}  // namespace

// C_b = alpha A_b B_b + beta D_b + beta2 D2_b + gamma I (and the optional second
// output C2 = c2_c C + c2_e E2 + c2_gamma I), real FP32, one 64 x 64 output tile
// per workgroup: the A tile staged in LDS, the B tile in registers. Entries
// with pred <= thresh copy D_b (A_b when D is null) into C_b. XCD as the
// complex kernels: a one-dimensional grid with every product on one XCD.
template <bool XCD, bool PIPE>
__global__ void __launch_bounds__(WG) k_rgemm(BigGemmArgs g) {
  __shared__ __attribute__((aligned(16))) float sa[64 * RPITCH];
  const int Tn = g.n / 64;
  const size_t nn = (size_t)g.n * g.n;
  int b, ti, tj;
  if constexpr (XCD) {
    const int Lb = blockIdx.x, per = gridDim.x / 8;
    const int logical = (Lb % 8) * per + Lb / 8;
    b = logical / (Tn * Tn);
    ti = (logical % (Tn * Tn)) / Tn;
    tj = logical % Tn;
  } else {
    b = blockIdx.y;
    ti = blockIdx.x / Tn;
    tj = blockIdx.x % Tn;
  }
  const size_t off = (size_t)ti * 64 * g.n + tj * 64;
  float* C = const_cast<float*>(rmat(g.C, g.Ci, b, nn));
  const float* D = g.D ? rmat(g.D, g.Di, b, nn) : nullptr;
  const bool active = !g.pred || g.pred[(size_t)(g.Ci ? g.Ci[b] : b) * g.pred_stride] > g.pred_thresh;
  if (!active) {
    RTR X;
    rr_load(X, (D ? D : rmat(g.A, g.Ai, b, nn)) + off, g.n);
    rr_store(X, C + off, g.n);
    return;
  }
  const float* A = rmat(g.A, g.Ai, b, nn) + (size_t)ti * 64 * g.n;
  const float* B = rmat(g.B, g.Bi, b, nn) + tj * 64;
  RTR acc, At, Bt;
  rr_zero(acc);
  if constexpr (PIPE) {
    // the next k-step's tiles are requested before this step's products
    rr_load(At, A, g.n);
    rr_load(Bt, B, g.n);
    for (int tk = 0; tk < Tn; ++tk) {
      __syncthreads();
      rr_stage(At, sa);
      __syncthreads();
      const RTR Bc = Bt;
      if (tk + 1 < Tn) {
        rr_load(At, A + (tk + 1) * 64, g.n);
        rr_load(Bt, B + (size_t)(tk + 1) * 64 * g.n, g.n);
      }
      rr_gemm(acc, sa, Bc);
    }
  } else {
    for (int tk = 0; tk < Tn; ++tk) {
      rr_load(At, A + tk * 64, g.n);
      rr_load(Bt, B + (size_t)tk * 64 * g.n, g.n);
      __syncthreads();
      rr_stage(At, sa);
      __syncthreads();
      rr_gemm(acc, sa, Bt);
    }
  }
  rr_scale(acc, (float)g.alpha);
  if (D && g.beta != 0.0) {
    RTR Dt;
    rr_load(Dt, D + off, g.n);
    rr_axpy(acc, (float)g.beta, Dt);
  }
  if (g.D2 && g.beta2 != 0.0) {
    RTR Dt;
    rr_load(Dt, rmat(g.D2, g.D2i, b, nn) + off, g.n);
    rr_axpy(acc, (float)g.beta2, Dt);
  }
  if (g.gamma != 0.0 && ti == tj) rr_add_diag(acc, (float)g.gamma);
  rr_store(acc, C + off, g.n);
  if (g.C2) {
    rr_scale(acc, (float)g.c2_c);
    if (g.E2) {
      RTR Et;
      rr_load(Et, rmat(g.E2, g.E2i, b, nn) + off, g.n);
      rr_axpy(acc, (float)g.c2_e, Et);
    }
    if (g.c2_gamma != 0.0 && ti == tj) rr_add_diag(acc, (float)g.c2_gamma);
    rr_store(acc, const_cast<float*>(rmat(g.C2, g.C2i, b, nn)) + off, g.n);
  }
}

// Real product kernel 1: a 128 x 128 output tile per workgroup, four waves in
// a 2 x 2 arrangement each owning 64 x 64 (16 accumulator blocks), k-steps of
// 32 with the A tile (128 x 32) and the transposed B tile (128 x 32) staged in
// LDS, so that every lane reads its four consecutive k values of an operand with
// one 16-byte load (pitch 36 floats: 16 rows at one k offset hit 16 different
// bank groups). Twice the products per staged byte of the 64 x 64 kernel.
// n must be a multiple of 128.
constexpr int R2P = 36;   // LDS pitch (floats) of the 32-wide staged tiles

__global__ void __launch_bounds__(WG) k_rgemm128(BigGemmArgs g) {
  __shared__ __attribute__((aligned(16))) float sa[128 * R2P];
  __shared__ __attribute__((aligned(16))) float sb[128 * R2P];   // B^T: [column][k]
  const int T2 = g.n / 128;
  const size_t nn = (size_t)g.n * g.n;
  const int b = blockIdx.y, ti = blockIdx.x / T2, tj = blockIdx.x % T2;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, gq = l >> 4, c = l & 15;
  const int wr = w >> 1, wc = w & 1;   // this wave's 64 x 64 quadrant
  const size_t off = (size_t)ti * 128 * g.n + tj * 128;
  float* C = const_cast<float*>(rmat(g.C, g.Ci, b, nn));
  const float* D = g.D ? rmat(g.D, g.Di, b, nn) : nullptr;
  const bool active = !g.pred || g.pred[(size_t)(g.Ci ? g.Ci[b] : b) * g.pred_stride] > g.pred_thresh;
  // element (rb, cb, r) of this lane: row 64 wr + 16 rb + 4 gq + r, column 64 wc + 16 cb + c
  auto at = [&](int rb, int cb, int r) {
    return (size_t)(64 * wr + 16 * rb + 4 * gq + r) * g.n + 64 * wc + 16 * cb + c;
  };
  if (!active) {
    const float* src = (D ? D : rmat(g.A, g.Ai, b, nn)) + off;
    for (int rb = 0; rb < 4; ++rb)
      for (int cb = 0; cb < 4; ++cb)
        for (int r = 0; r < 4; ++r) C[off + at(rb, cb, r)] = src[at(rb, cb, r)];
    return;
  }
  const float* A = rmat(g.A, g.Ai, b, nn) + (size_t)ti * 128 * g.n;
  const float* B = rmat(g.B, g.Bi, b, nn) + tj * 128;
  f4v acc[4][4];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) acc[rb][cb] = f4v{0.f, 0.f, 0.f, 0.f};
  // staging: A rows (128 x 32): thread -> row tid / 2, k 16 (tid & 1) .. +15 (four f4v);
  // B rows k (32 x 128): thread -> k tid / 8, columns 16 (tid & 7) .. +15
  const int ar = tid >> 1, ak = 16 * (tid & 1);
  const int bk = tid >> 3, bc = 16 * (tid & 7);
  for (int k0 = 0; k0 < g.n; k0 += 32) {
    f4v va[4], vb[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      va[i] = *reinterpret_cast<const f4v*>(A + (size_t)ar * g.n + k0 + ak + 4 * i);
      vb[i] = *reinterpret_cast<const f4v*>(B + (size_t)(k0 + bk) * g.n + bc + 4 * i);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      *reinterpret_cast<f4v*>(sa + ar * R2P + ak + 4 * i) = va[i];
      // B^T row (column of B) bc + 4 i + j, k-granule (bk / 4) permuted by the
      // column's 16-block index, so that the eight threads of one k row, whose
      // columns are 16 apart, write eight different banks
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int col = bc + 4 * i + j;
        sb[col * R2P + 4 * ((bk >> 2) ^ ((col >> 4) & 7)) + (bk & 3)] = vb[i][j];
      }
    }
    __syncthreads();
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
      f4v av[4], bv[4];
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
        av[rb] = *reinterpret_cast<const f4v*>(sa + (64 * wr + 16 * rb + c) * R2P + 16 * kb + 4 * gq);
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
        bv[cb] = *reinterpret_cast<const f4v*>(sb + (64 * wc + 16 * cb + c) * R2P +
                                               4 * ((4 * kb + gq) ^ ((4 * wc + cb) & 7)));
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
          for (int cb = 0; cb < 4; ++cb)
            acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[rb][t], bv[cb][t], acc[rb][cb], 0, 0, 0);
    }
  }
  const float al = (float)g.alpha, be = (float)g.beta, be2 = (float)g.beta2;
  const float* D2 = g.D2 ? rmat(g.D2, g.D2i, b, nn) + off : nullptr;
  const float* E2 = g.E2 ? rmat(g.E2, g.E2i, b, nn) + off : nullptr;
  float* C2 = g.C2 ? const_cast<float*>(rmat(g.C2, g.C2i, b, nn)) + off : nullptr;
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const size_t e = at(rb, cb, r);
        float v = al * acc[rb][cb][r];
        if (D && g.beta != 0.0) v += be * D[off + e];
        if (D2 && g.beta2 != 0.0) v += be2 * D2[e];
        const bool diag = ti == tj && wr == wc && rb == cb && 4 * gq + r == c;
        if (diag && g.gamma != 0.0) v += (float)g.gamma;
        C[off + e] = v;
        if (C2) {
          float v2 = (float)g.c2_c * v;
          if (E2) v2 += (float)g.c2_e * E2[e];
          if (diag && g.c2_gamma != 0.0) v2 += (float)g.c2_gamma;
          C2[e] = v2;
        }
      }
}

hipError_t launch_rgemm(const BigGemmArgs& g, hipStream_t s) {
  if (g.batch <= 0) return hipSuccess;
  if (g.C2 && g.pred) return hipErrorInvalidValue;
  if (g.transA || g.transB) return hipErrorInvalidValue;
  const int Tn = g.n / 64;
  const size_t total = (size_t)Tn * Tn * g.batch;
  const bool xcd = Tn <= 16 && total % 8 == 0 && total <= 0x7fffffff;
  if (g.variant == 1 && Tn % 2 == 0)
    hipLaunchKernelGGL(k_rgemm128, dim3((Tn / 2) * (Tn / 2), g.batch), dim3(WG), 0, s, g);
  else if (g.variant == 5 && xcd)
    hipLaunchKernelGGL((k_rgemm<true, false>), dim3((unsigned)total), dim3(WG), 0, s, g);
  else if (g.variant == 7 && xcd)
    hipLaunchKernelGGL((k_rgemm<true, true>), dim3((unsigned)total), dim3(WG), 0, s, g);
  else if (g.variant == 2 || g.variant == 7)
    hipLaunchKernelGGL((k_rgemm<false, true>), dim3(Tn * Tn, g.batch), dim3(WG), 0, s, g);
  else
    hipLaunchKernelGGL((k_rgemm<false, false>), dim3(Tn * Tn, g.batch), dim3(WG), 0, s, g);
  return hipGetLastError();
}

// Y_b = a X_b + c Z_b + d I, real FP32, four elements per 16-byte vector, four
// vectors per thread and pass; a = 0 reads no X; a *= 2^-s of entry Yi[b] when
// ms is set.
__global__ void __launch_bounds__(256) k_raxpby(BigAxpbyArgs g) {
  constexpr int U = 4;
  const int nv = g.n * g.n / 4;
  const size_t nn = (size_t)g.n * g.n;
  const int b = blockIdx.y;
  const f4v* X = reinterpret_cast<const f4v*>(rmat(g.X, g.Xi, b, nn));
  const f4v* Z = g.Z ? reinterpret_cast<const f4v*>(rmat(g.Z, g.Zi, b, nn)) : nullptr;
  f4v* Y = reinterpret_cast<f4v*>(const_cast<float*>(rmat(g.Y, g.Yi, b, nn)));
  double ad = g.a;
  if (g.ms) ad = ldexp(ad, -(int)g.ms[2 * (size_t)(g.Yi ? g.Yi[b] : b) + 1]);
  const float a = (float)ad, c = (float)g.c;
  const bool rx = ad != 0.0;
  const int stride = gridDim.x * 256;
  for (int v0 = blockIdx.x * 256 + threadIdx.x; v0 < nv; v0 += U * stride) {
    f4v xv[U], zv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int v = v0 + u * stride;
      if (v < nv) {
        if (rx) xv[u] = X[v];
        if (Z) zv[u] = Z[v];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int v = v0 + u * stride;
      if (v < nv) {
        f4v y = f4v{0.f, 0.f, 0.f, 0.f};
        if (rx) y = a * xv[u];
        if (Z) y += c * zv[u];
        if (g.d != 0.0) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int e = 4 * v + j;
            if (e / g.n == e % g.n) y[j] += (float)g.d;
          }
        }
        Y[v] = y;
      }
    }
  }
}

hipError_t launch_raxpby(const BigAxpbyArgs& g, hipStream_t s) {
  if (g.batch <= 0) return hipSuccess;
  auto misaligned = [](const void* p) { return ((uintptr_t)p & 15) != 0; };
  if (misaligned(g.X) || misaligned(g.Y) || misaligned(g.Z)) return hipErrorInvalidValue;
  const size_t nv = (size_t)g.n * g.n / 4;
  const dim3 grid((unsigned)std::min<size_t>(std::max<size_t>((nv + 1023) / 1024, 1), 1024), g.batch);
  hipLaunchKernelGGL(k_raxpby, grid, dim3(256), 0, s, g);
  return hipGetLastError();
}

// Omega_n = sum_j alpha_{n,j} B_j tile by tile for S consecutive slices per
// workgroup (each basis tile fetched once for the S), with the FP64 column sums
// of |Omega| over the tile's rows: part[slice][tile row][col].
template <int S>
__global__ void __launch_bounds__(WG) k_romega(BigOmegaArgs g) {
  const int Tn = g.n / 64;
  const size_t nn = (size_t)g.n * g.n;
  const int s0 = blockIdx.y * S;
  const int t = blockIdx.x, ti = t / Tn, tj = t % Tn;
  const float* basis = (const float*)g.basis;
  RTR X[S];
#pragma unroll
  for (int q = 0; q < S; ++q) rr_zero(X[q]);
  const int j0 = g.tile_ptr ? g.tile_ptr[t] : 0, j1 = g.tile_ptr ? g.tile_ptr[t + 1] : g.nb;
  for (int e = j0; e < j1; ++e) {
    const int j = g.tile_ptr ? g.tile_j[e] : e;
    double aj[S];
    bool any = false;
#pragma unroll
    for (int q = 0; q < S; ++q) {
      aj[q] = s0 + q < g.n_slices ? g.alpha[(size_t)(s0 + q) * g.nb + j] : 0.0;
      any |= aj[q] != 0.0;
    }
    if (!any) continue;
    RTR Bt;
    rr_load(Bt, basis + (size_t)j * nn + (size_t)ti * 64 * g.n + tj * 64, g.n);
#pragma unroll
    for (int q = 0; q < S; ++q)
      if (aj[q] != 0.0) rr_axpy(X[q], (float)aj[q], Bt);
  }
  const Lane L;
#pragma unroll
  for (int q = 0; q < S; ++q) {
    const int slice = s0 + q;
    if (slice >= g.n_slices) break;
    rr_store(X[q], (float*)g.omega + (size_t)slice * nn + (size_t)ti * 64 * g.n + tj * 64, g.n);
    double sum = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int r = 0; r < 4; ++r) sum += fabs((double)X[q].v[a][r]);
    sum += __shfl_xor(sum, 16);
    sum += __shfl_xor(sum, 32);
    if (L.g == 0) g.part[((size_t)slice * Tn + ti) * g.n + tj * 64 + L.col] = sum;
  }
}

// Column sums of |Omega| of dense exponents (sixth order, assembled by products).
__global__ void __launch_bounds__(WG) k_rcolsum(BigOmegaArgs g) {
  const int Tn = g.n / 64;
  const size_t nn = (size_t)g.n * g.n;
  const int slice = blockIdx.y, ti = blockIdx.x / Tn, tj = blockIdx.x % Tn;
  RTR X;
  rr_load(X, (const float*)g.omega + (size_t)slice * nn + (size_t)ti * 64 * g.n + tj * 64, g.n);
  const Lane L;
  double sum = 0.0;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int r = 0; r < 4; ++r) sum += fabs((double)X.v[a][r]);
  sum += __shfl_xor(sum, 16);
  sum += __shfl_xor(sum, 32);
  if (L.g == 0) g.part[((size_t)slice * Tn + ti) * g.n + tj * 64 + L.col] = sum;
}

// (m, s) and the Neumann level count of every slice from its FP64 column sums,
// then Omega / 2^s in place.
__global__ void __launch_bounds__(256) k_rnorm(BigOmegaArgs g) {
  __shared__ double red[256];
  __shared__ int sc_sh;
  const int Tn = g.n / 64;
  const int slice = blockIdx.x;
  double mx = 0.0;
  for (int col = threadIdx.x; col < g.n; col += 256) {
    double cs = 0.0;
    for (int ti = 0; ti < Tn; ++ti) cs += g.part[((size_t)slice * Tn + ti) * g.n + col];
    mx = fmax(mx, cs);
    if (!(cs == cs)) mx = cs;   // NaN propagates
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      const double o = red[threadIdx.x + off];
      red[threadIdx.x] = (o == o) ? fmax(red[threadIdx.x], o) : o;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double v = red[0];
    int m, s;
    big_choose_ms<float>(v, m, s);
    g.ms[2 * (size_t)slice] = (int8_t)m;
    g.ms[2 * (size_t)slice + 1] = (int8_t)s;
    if (g.nlev) {
      const int lv = big_neumann_levels<float>(ldexp(v, -s), g.b3);
      g.nlev[slice] = (int8_t)(lv > 0 ? lv : kBigNeumannLevels);
    }
    sc_sh = s;
  }
  __syncthreads();
  const int s = sc_sh;
  if (s == 0) return;
  const float f = (float)ldexp(1.0, -s);
  const size_t nn = (size_t)g.n * g.n;
  float* X = (float*)g.omega + (size_t)slice * nn;
  for (size_t e = threadIdx.x; e < nn; e += 256) X[e] *= f;
}

hipError_t launch_romega(const BigOmegaArgs& g, hipStream_t s) {
  if (g.n_slices <= 0) return hipSuccess;
  const int Tn = g.n / 64;
  constexpr int S = kBigSlicesPerGroup;
  hipLaunchKernelGGL((k_romega<S>), dim3(Tn * Tn, (g.n_slices + S - 1) / S), dim3(WG), 0, s, g);
  if (g.ms) hipLaunchKernelGGL(k_rnorm, dim3(g.n_slices), dim3(256), 0, s, g);
  return hipGetLastError();
}

hipError_t launch_rnorm_dense(const BigOmegaArgs& g, hipStream_t s) {
  if (g.n_slices <= 0) return hipSuccess;
  const int Tn = g.n / 64;
  hipLaunchKernelGGL(k_rcolsum, dim3(Tn * Tn, g.n_slices), dim3(WG), 0, s, g);
  hipLaunchKernelGGL(k_rnorm, dim3(g.n_slices), dim3(256), 0, s, g);
  return hipGetLastError();
}

// Per-tile partial traces Re Tr(K_n B_j) = sum_{a,b} K[a][b] B_j[b][a] for S
// consecutive slices per workgroup: the K tile transposed once through LDS, the
// basis tile (tj, ti) read untransposed; lane partials in FP32, the sums over
// lanes and tiles in FP64.
template <int S>
__global__ void __launch_bounds__(WG) k_rtraces_part(BigTraceArgs g) {
  __shared__ float sk[64 * 65];
  __shared__ double red[4][S][MAX_BIG_NB];
  const int Tn = g.n / 64;
  const size_t nn = (size_t)g.n * g.n;
  const int s0 = blockIdx.y * S, tile = blockIdx.x;
  const int ti = tile / Tn, tj = tile % Tn;
  const float* basis = (const float*)g.basis;
  const Lane L;
  const int bt = tj * Tn + ti;
  for (int e = threadIdx.x; e < 4 * S * g.nb; e += WG) (&red[0][0][0])[(e / g.nb) * MAX_BIG_NB + e % g.nb] = 0.0;
  const int j0 = g.tile_ptr ? g.tile_ptr[bt] : 0, j1 = g.tile_ptr ? g.tile_ptr[bt + 1] : g.nb;
  RTR Kt[S];
#pragma unroll
  for (int q = 0; q < S; ++q) {
    if (j1 > j0 && s0 + q < g.n_slices) {
      RTR X;
      rr_load(X, (const float*)g.K + (size_t)(s0 + q) * nn + (size_t)ti * 64 * g.n + tj * 64, g.n);
      __syncthreads();
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) sk[(16 * a + 4 * L.g + r) * 65 + L.col] = X.v[a][r];
      __syncthreads();
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) Kt[q].v[a][r] = sk[L.col * 65 + 16 * a + 4 * L.g + r];
    } else {
      rr_zero(Kt[q]);
    }
  }
  __syncthreads();
  for (int e = j0; e < j1; ++e) {
    const int j = g.tile_ptr ? g.tile_j[e] : e;
    RTR Bt;
    rr_load(Bt, basis + (size_t)j * nn + (size_t)tj * 64 * g.n + ti * 64, g.n);
#pragma unroll
    for (int q = 0; q < S; ++q) {
      float part = 0.f;
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) part = fmaf(Kt[q].v[a][r], Bt.v[a][r], part);
      double acc = (double)part;
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o);
      if (L.l == 0) red[L.w][q][j] = acc;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < S * g.nb; e += WG) {
    const int q = e / g.nb, j = e % g.nb;
    if (s0 + q < g.n_slices)
      g.part[((size_t)(s0 + q) * Tn * Tn + tile) * g.nb + j] = (red[0][q][j] + red[1][q][j]) + (red[2][q][j] + red[3][q][j]);
  }
}

hipError_t launch_rtraces(const BigTraceArgs& g, hipStream_t s) {
  if (g.n_slices <= 0) return hipSuccess;
  const int Tn = g.n / 64;
  constexpr int S = kBigSlicesPerGroup;
  hipLaunchKernelGGL((k_rtraces_part<S>), dim3(Tn * Tn, (g.n_slices + S - 1) / S), dim3(WG), 0, s, g);
  return launch_btraces_sum(g, s);
}

// F_item = Tr(R_T^T R_U) / d^2 = sum_{a,b} st[a][b] R_U[b][a] / d^2 (st = R_T^T,
// FP64), R_U = I + the item's inclusive prefix (stored as R - I).
__global__ void k_rfidelity(BigFidArgs g) {
  __shared__ double red[256];
  const int item = blockIdx.x;
  const size_t nn = (size_t)g.n * g.n;
  const float* U = (const float*)g.U + (size_t)g.U_index[item] * nn;
  const double* S = g.st64 + (size_t)g.target[item] * nn;
  double acc = 0.0;
  for (size_t e = threadIdx.x; e < nn; e += 256) {
    const size_t a = e / g.n, c = e % g.n;
    acc += S[e] * ((double)U[c * g.n + a] + (a == c ? 1.0 : 0.0));
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) g.F[g.F_index ? g.F_index[item] : item] = red[0] / ((double)g.d * g.d);
}

hipError_t launch_rfidelity(const BigFidArgs& g, hipStream_t s) {
  if (g.n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rfidelity, dim3(g.n_items), dim3(256), 0, s, g);
  return hipGetLastError();
}

namespace {
// Entries of T (rows a, columns i) for a = k + l d: T[a][a] and T[a][partner].
struct TPair {
  int partner;      // l + k d (a itself on the diagonal k == l)
  double sr, si;    // T[a][a]
  double pr, pi;    // T[a][partner]
};
__device__ __forceinline__ TPair t_row(int a, int d) {
  const int k = a % d, l = a / d;
  const double h = 0.70710678118654752440;
  if (k == l) return {a, 1.0, 0.0, 0.0, 0.0};
  if (k < l) return {l + k * d, h, 0.0, h, 0.0};   // (v_kl + v_lk) / sqrt 2
  return {l + k * d, 0.0, h, 0.0, -h};             // i (v_kl - v_lk) / sqrt 2 of the pair (l, k)
}
}  // namespace

// R = T S T^dag for nmat complex FP64 superoperators S (row-major n x n) into
// real FP64 R; the imaginary part, zero for a Hermiticity-preserving S, is
// dropped.
__global__ void k_to_real(const cpx<double>* S, int d, int nmat, double* R) {
  const int n = d * d;
  const size_t nn = (size_t)n * n;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < nn * nmat; e += (size_t)gridDim.x * blockDim.x) {
    const size_t m = e / nn, idx = e % nn;
    const int a = (int)(idx / n), b = (int)(idx % n);
    const cpx<double>* Sm = S + m * nn;
    const TPair ta = t_row(a, d), tb = t_row(b, d);
    const int ia[2] = {a, ta.partner}, jb[2] = {b, tb.partner};
    const double ar[2] = {ta.sr, ta.pr}, ai[2] = {ta.si, ta.pi};
    const double br[2] = {tb.sr, tb.pr}, bi[2] = {tb.si, tb.pi};
    double re = 0.0;
    for (int x = 0; x < (a == ta.partner ? 1 : 2); ++x)
      for (int y = 0; y < (b == tb.partner ? 1 : 2); ++y) {
        const cpx<double> s = Sm[(size_t)ia[x] * n + jb[y]];
        // Re(T[a][i] S[i][j] conj(T[b][j]))
        const double ur = ar[x] * s.re - ai[x] * s.im, ui = ar[x] * s.im + ai[x] * s.re;
        re += ur * br[y] + ui * bi[y];
      }
    R[e] = re;
  }
}

hipError_t launch_to_real(const double* S, int d, int nmat, double* R, hipStream_t s) {
  if (nmat <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_to_real, dim3(1024), dim3(256), 0, s, (const cpx<double>*)S, d, nmat, R);
  return hipGetLastError();
}

// U_item = T^dag (I + R) T in column stacking, complex FP32 (R from the item's
// inclusive prefix, stored as R - I): S_out[Yi[b]] from R[Xi[b]].
__global__ void k_from_real(const float* R, const int32_t* Xi, int d, cpx<float>* out, const int32_t* Yi) {
  const int n = d * d;
  const size_t nn = (size_t)n * n;
  const int b = blockIdx.y;
  const float* Rm = R + (size_t)Xi[b] * nn;
  cpx<float>* O = out + (size_t)Yi[b] * nn;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < nn; idx += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx / n), j = (int)(idx % n);
    // S[i][j] = sum_{a in {i, pi}, c in {j, pj}} conj(T[a][i]) R[a][c] T[c][j]
    const TPair ti = t_row(i, d), tj = t_row(j, d);
    const int as[2] = {i, ti.partner}, cs[2] = {j, tj.partner};
    double re = 0.0, im = 0.0;
    for (int x = 0; x < (i == ti.partner ? 1 : 2); ++x) {
      const int a = as[x];
      const TPair ta = t_row(a, d);
      const double tr = (a == i) ? ta.sr : ta.pr, tim = (a == i) ? ta.si : ta.pi;   // T[a][i]
      for (int y = 0; y < (j == tj.partner ? 1 : 2); ++y) {
        const int c = cs[y];
        const TPair tc = t_row(c, d);
        const double ur = (c == j) ? tc.sr : tc.pr, ui = (c == j) ? tc.si : tc.pi;   // T[c][j]
        const double r = (double)Rm[(size_t)a * n + c] + (a == c ? 1.0 : 0.0);
        // conj(T[a][i]) r T[c][j]
        const double pr = tr * ur + tim * ui, pim = tr * ui - tim * ur;
        re += r * pr;
        im += r * pim;
      }
    }
    O[idx] = cpx<float>{(float)re, (float)im};
  }
}

hipError_t launch_from_real(const float* R, const int32_t* Xi, int d, int batch, void* out, const int32_t* Yi,
                            hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_from_real, dim3(256, batch), dim3(256), 0, s, R, Xi, d, (cpx<float>*)out, Yi);
  return hipGetLastError();
}

// flags[j][t] = 1 if tile t of real FP64 basis element j has a nonzero entry.
__global__ void k_rtile_flags(const double* basis, int nb, int n, uint8_t* flags) {
  __shared__ int any;
  const int Tn = n / 64;
  const int t = blockIdx.x, j = blockIdx.y;
  const int ti = t / Tn, tj = t % Tn;
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  const double* B = basis + (size_t)j * n * n + (size_t)ti * 64 * n + tj * 64;
  int nz = 0;
  for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) nz |= B[(size_t)(e / 64) * n + e % 64] != 0.0;
  if (nz) any = 1;   // benign race: every writer stores 1
  __syncthreads();
  if (threadIdx.x == 0) flags[(size_t)j * Tn * Tn + t] = (uint8_t)any;
}

hipError_t launch_rtile_flags(const double* basis, int nb, int n, uint8_t* flags, hipStream_t s) {
  const int Tn = n / 64;
  hipLaunchKernelGGL(k_rtile_flags, dim3(Tn * Tn, nb), dim3(256), 0, s, basis, nb, n, flags);
  return hipGetLastError();
}

// FP64 -> FP32 copy of a real array.
__global__ void k_rcast(const double* in, float* out, size_t count) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (size_t)gridDim.x * blockDim.x)
    out[e] = (float)in[e];
}

hipError_t launch_rcast(const double* in, float* out, size_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_rcast, dim3(1024), dim3(256), 0, s, in, out, count);
  return hipGetLastError();
}

}  // namespace lmag

namespace lmag {

// The 64 x 64 slice kernels in the same basis (d <= 8): tiles stay complex in
// memory, with zero imaginary parts, and each product takes one real MFMA.
// Indices at or beyond d^2 (the zero padding of a tile) map to themselves.
namespace {
__device__ __forceinline__ TPair t_row_pad(int a, int d) {
  return a < d * d ? t_row(a, d) : TPair{a, 1.0, 0.0, 0.0, 0.0};
}
}  // namespace

// In place, one workgroup per 64 x 64 tile: R = Re(T S T^dag) of a complex
// FP64 tile S, written back as (R, 0), and as complex FP32 into out32 when
// given. The real part is the whole of T S T^dag for a Hermiticity-preserving
// S; for any other S it is the projection that a real first-order change of R
// sees (Re Tr(G^dag dS) = Tr(Re(T G T^dag)^T dR) for real dR), which is what a
// gradient seed needs.
__global__ void __launch_bounds__(256) k_tile_to_real(cpx<double>* tiles, int d, cpx<float>* out32) {
  __shared__ cpx<double> S[64 * 64];
  cpx<double>* X = tiles + (size_t)blockIdx.x * 4096;
  for (int e = threadIdx.x; e < 4096; e += 256) S[e] = X[e];
  __syncthreads();
  for (int e = threadIdx.x; e < 4096; e += 256) {
    const int a = e / 64, b = e % 64;
    const TPair ta = t_row_pad(a, d), tb = t_row_pad(b, d);
    const int ia[2] = {a, ta.partner}, jb[2] = {b, tb.partner};
    const double ar[2] = {ta.sr, ta.pr}, ai[2] = {ta.si, ta.pi};
    const double br[2] = {tb.sr, tb.pr}, bi[2] = {tb.si, tb.pi};
    double re = 0.0;
    for (int x = 0; x < (a == ta.partner ? 1 : 2); ++x)
      for (int y = 0; y < (b == tb.partner ? 1 : 2); ++y) {
        const cpx<double> s = S[ia[x] * 64 + jb[y]];
        const double ur = ar[x] * s.re - ai[x] * s.im, ui = ar[x] * s.im + ai[x] * s.re;
        re += ur * br[y] + ui * bi[y];   // Re(T[a][i] S[i][j] conj(T[b][j]))
      }
    X[e] = cpx<double>{re, 0.0};
    if (out32) out32[(size_t)blockIdx.x * 4096 + e] = cpx<float>{(float)re, 0.f};
  }
}

hipError_t launch_tile_to_real(double* tiles, int count, int d, float* out32, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (d < 1 || d > 8) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_tile_to_real, dim3(count), dim3(256), 0, s, (cpx<double>*)tiles, d, (cpx<float>*)out32);
  return hipGetLastError();
}

// In place, one workgroup per item: the n x n complex FP32 matrix (n = d^2)
// at out + items[b].src n^2 holds a real matrix R in its real parts and
// becomes T^dag R T, column stacking.
__global__ void __launch_bounds__(256) k_out_from_real(cpx<float>* out, const Item* items, int d) {
  __shared__ float R[64 * 64];
  const int n = d * d;
  cpx<float>* X = out + (size_t)items[blockIdx.x].src * n * n;
  for (int e = threadIdx.x; e < n * n; e += 256) R[e] = X[e].re;
  __syncthreads();
  for (int e = threadIdx.x; e < n * n; e += 256) {
    const int i = e / n, j = e % n;
    // X[i][j] = sum over a in {i, p(i)}, c in {j, p(j)} of conj(T[a][i]) R[a][c] T[c][j]
    const TPair ti = t_row(i, d), tj = t_row(j, d);
    const int as[2] = {i, ti.partner}, cs[2] = {j, tj.partner};
    double re = 0.0, im = 0.0;
    for (int x = 0; x < (i == ti.partner ? 1 : 2); ++x) {
      const int a = as[x];
      const TPair ta = t_row(a, d);
      const double tr = (a == i) ? ta.sr : ta.pr, tim = (a == i) ? ta.si : ta.pi;   // T[a][i]
      for (int y = 0; y < (j == tj.partner ? 1 : 2); ++y) {
        const int c = cs[y];
        const TPair tc = t_row(c, d);
        const double ur = (c == j) ? tc.sr : tc.pr, ui = (c == j) ? tc.si : tc.pi;   // T[c][j]
        const double r = (double)R[a * n + c];
        re += r * (tr * ur + tim * ui);
        im += r * (tr * ui - tim * ur);
      }
    }
    X[e] = cpx<float>{(float)re, (float)im};
  }
}

hipError_t launch_out_from_real(void* out, const Item* items, int n_items, int d, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  if (d < 1 || d > 8) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_out_from_real, dim3(n_items), dim3(256), 0, s, (cpx<float>*)out, items, d);
  return hipGetLastError();
}

}  // namespace lmag
