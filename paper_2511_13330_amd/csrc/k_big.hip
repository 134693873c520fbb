// Block-tiled kernels for superoperators larger than one 64x64 tile
// (n = 64 T, T = n / 64 tiles per side; 4 spins: n = 256, 6 spins: n = 4096).
//
// Every per-slice step of the Pade / Frechet pipeline is a batched operation
// over many n x n matrices (all slices, or all chunks for the ordered
// products). The product kernel assigns one 64 x 64 output tile of one matrix
// to a workgroup, which accumulates over the T tiles of the contraction with
// the register-tile MFMA product of tile.hpp (A tile staged through LDS, B tile
// in registers). Matrices are row-major n x n, interleaved complex.
#include "tile.hpp"
#include "internal.hpp"
#include "big.hpp"
#include "pade.hpp"

#include <algorithm>
#include <type_traits>

namespace lmag {

template <typename T> struct BigShared {
  cpx<T> slot[64 * PITCH];
  double red[8];
};

template <typename T>
__device__ __forceinline__ const cpx<T>* mat(const void* base, const int32_t* idx, int b, size_t nn) {
  return reinterpret_cast<const cpx<T>*>(base) + (size_t)(idx ? idx[b] : b) * nn;
}

// C_b = alpha * op(A_b) op(B_b) + beta * D_b + beta2 * D2_b + gamma * I, for every batch entry
// b with (pred == null or pred[b] != 0); other entries copy D_b (or A_b when
// D is null) into C_b. op = transpose when the flag is set.
// XCD = true takes a one-dimensional grid of Tn^2 * batch workgroups (a
// multiple of 8) and gives every product whole to one XCD: workgroups are
// dispatched round-robin over the eight XCDs, so hardware slot L runs on XCD
// L mod 8 and is given product tile (L mod 8) * (grid / 8) + L / 8. An XCD then
// works through consecutive products, each one's operand tiles fetched into its
// own L2 once and re-read there by the product's other output tiles.
// (batch entry, tile row, tile column) of this workgroup.
template <bool XCD>
__device__ __forceinline__ void tile_of_block(int Tn, int& b, int& ti, int& tj) {
  if constexpr (XCD) {
    const int L = blockIdx.x, per = gridDim.x / 8;
    const int logical = (L % 8) * per + L / 8;
    b = logical / (Tn * Tn);
    ti = (logical % (Tn * Tn)) / Tn;
    tj = logical % Tn;
  } else {
    b = blockIdx.y;
    ti = blockIdx.x / Tn;
    tj = blockIdx.x % Tn;
  }
}

// Epilogue of the register-B kernels: C = alpha acc + beta D + beta2 D2 +
// gamma I, then the optional second output C2 = c2_c C + c2_e E2 + c2_gamma I.
template <typename T>
__device__ __forceinline__ void bgemm_epilogue(const BigGemmArgs& g, RT<T>& acc, int b, int ti, int tj,
                                               cpx<T>* C, const cpx<T>* D) {
  const size_t nn = (size_t)g.n * g.n;
  const size_t off = (size_t)ti * 64 * g.n + tj * 64;
  rt_scale(acc, (T)g.alpha);
  if (D && g.beta != 0.0) {
    RT<T> Dt;
    rt_load<T, false>(Dt, D + off, g.n);
    rt_axpy(acc, (T)g.beta, Dt);
  }
  if (g.D2 && g.beta2 != 0.0) {
    RT<T> Dt;
    rt_load<T, false>(Dt, mat<T>(g.D2, g.D2i, b, nn) + off, g.n);
    rt_axpy(acc, (T)g.beta2, Dt);
  }
  if (g.gamma != 0.0 && ti == tj) rt_add_diag(acc, (T)g.gamma);
  rt_store<T, false>(acc, C + off, g.n);
  if (g.C2) {
    // second output from the same tile: C2 = c2_c C + c2_e E2 + c2_gamma I
    rt_scale(acc, (T)g.c2_c);
    if (g.E2) {
      RT<T> Et;
      rt_load<T, false>(Et, mat<T>(g.E2, g.E2i, b, nn) + off, g.n);
      rt_axpy(acc, (T)g.c2_e, Et);
    }
    if (g.c2_gamma != 0.0 && ti == tj) rt_add_diag(acc, (T)g.c2_gamma);
    cpx<T>* C2 = const_cast<cpx<T>*>(mat<T>(g.C2, g.C2i, b, nn));
    rt_store<T, false>(acc, C2 + off, g.n);
  }
}

template <typename T, bool TA, bool TB, bool XCD, bool PIPE>
__device__ __forceinline__ void bgemm_body(const BigGemmArgs& g, BigShared<T>& sh) {
  const int Tn = g.n / 64;
  const size_t nn = (size_t)g.n * g.n;
  int b, ti, tj;
  tile_of_block<XCD>(Tn, b, ti, tj);
  cpx<T>* C = const_cast<cpx<T>*>(mat<T>(g.C, g.Ci, b, nn));
  const cpx<T>* D = g.D ? mat<T>(g.D, g.Di, b, nn) : nullptr;
  const bool active = !g.pred || g.pred[(size_t)(g.Ci ? g.Ci[b] : b) * g.pred_stride] > g.pred_thresh;
  if (!active) {
    const cpx<T>* src = D ? D : mat<T>(g.A, g.Ai, b, nn);
    RT<T> X;
    rt_load<T, false>(X, src + (size_t)ti * 64 * g.n + tj * 64, g.n);
    rt_store<T, false>(X, C + (size_t)ti * 64 * g.n + tj * 64, g.n);
    return;
  }
  const cpx<T>* A = mat<T>(g.A, g.Ai, b, nn);
  const cpx<T>* B = mat<T>(g.B, g.Bi, b, nn);
  RT<T> acc;
  rt_zero(acc);
  for (int tk = 0; tk < Tn; ++tk) {
    // A tile (ti, tk) of op(A): op(A)[ti][tk] = TA ? A[tk][ti]^T : A[ti][tk]
    RT<T> At, Bt;
    if (TA) rt_load<T, true>(At, A + (size_t)tk * 64 * g.n + ti * 64, g.n);
    else rt_load<T, false>(At, A + (size_t)ti * 64 * g.n + tk * 64, g.n);
    // without the pipeline (fewer registers) the B tile is fetched after the
    // A tile has gone to LDS, so that the two are never live together
    if (PIPE) {
      if (TB) rt_load<T, true>(Bt, B + (size_t)tj * 64 * g.n + tk * 64, g.n);
      else rt_load<T, false>(Bt, B + (size_t)tk * 64 * g.n + tj * 64, g.n);
    }
    __syncthreads();
    rt_store<T, false>(At, sh.slot, PITCH);
    if (!PIPE) {
      if (TB) rt_load<T, true>(Bt, B + (size_t)tj * 64 * g.n + tk * 64, g.n);
      else rt_load<T, false>(Bt, B + (size_t)tk * 64 * g.n + tj * 64, g.n);
    }
    __syncthreads();
    gemm_acc<T, false, PITCH, PIPE>(acc, sh.slot, Bt);
  }
  bgemm_epilogue<T>(g, acc, b, ti, tj, C, D);
}

template <typename T, bool TA, bool TB, bool XCD = false>
__global__ void __launch_bounds__(WG) k_bgemm(BigGemmArgs g) {
  __shared__ BigShared<T> sh;
  bgemm_body<T, TA, TB, XCD, true>(g, sh);
}

// Three resident workgroups per CU (three waves per SIMD, at most 168
// registers): the k-step loads of one workgroup hide behind the products of
// two others; the A operands are read from LDS without the software pipeline
// of the two-workgroup kernel, which needs more registers.
template <bool XCD>
__global__ void __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(3, 3)))
k_bgemm_occ3(BigGemmArgs g) {
  __shared__ BigShared<float> sh;
  bgemm_body<float, false, false, XCD, false>(g, sh);
}

// Kernel 8 (single precision, no transposes): one 64 x 64 output tile per
// workgroup like kernel 0, with each A tile brought into LDS by the direct
// global-to-LDS loads (no registers, no LDS stores by the waves) into one of
// two buffers, so that the next k-step's A tile and B tile are in flight while
// the current step's products run; one barrier per k-step. The A tile is kept
// unpadded and row-major with the 16-byte granules of each row permuted
// (granule G of row R at position G ^ (R & 15)): a 16-byte read of one granule
// position by the 16 lanes that hold rows 16 q .. 16 q + 15 then touches 16
// different bank groups, and a load instruction, whose 64 lanes fill 1 KB of
// LDS in lane order, reads a permutation of two contiguous 512-byte rows.
constexpr int DMA_TILE = 64 * 64;   // complex elements of one LDS A buffer

__device__ __forceinline__ void dma_a_tile(const cpx<float>* At, int ld, cpx<float>* buf) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int chunk = 8 * w + i;                 // 1 KB of LDS: rows 2 chunk, 2 chunk + 1
    const int r = 2 * chunk + (l >> 5);
    const int G = (l & 31) ^ (r & 15);           // the granule that lands at position l & 31
    __builtin_amdgcn_global_load_lds((const void*)(At + (size_t)r * ld + 2 * G),
                                     (__attribute__((address_space(3))) void*)(buf + chunk * 128), 16, 0, 0);
  }
}

// acc += A B for the A tile in LDS (layout above) and B in registers (RT), in
// the 3M form, k = 16 kb + 4 g + t as in the RT layout. mid() runs after the
// first half of the k-steps, whose B registers are dead by then: the next
// step's B tile is requested there, so that it never doubles the B registers.
template <typename F>
__device__ __forceinline__ void mma_dma(RT<float>& acc, const cpx<float>* buf, const RT<float>& B,
                                        const F& mid) {
  const Lane L;
  const int g = L.g, c = L.c;
  const char* base = reinterpret_cast<const char*>(buf) + c * 512;   // row 16 q + c, q = 0 below
  vec4<float>::type k1[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) k1[q] = vec4<float>::type{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) {
    if (kb == 2) {
      __builtin_amdgcn_sched_barrier(0);
      mid();
      __builtin_amdgcn_sched_barrier(0);
    }
    const int G0 = 8 * kb + 2 * g;
    float4 a[4][2];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const char* row = base + q * 16 * 512;
      a[q][0] = *reinterpret_cast<const float4*>(row + ((G0 ^ c) << 4));
      a[q][1] = *reinterpret_cast<const float4*>(row + (((G0 + 1) ^ c) << 4));
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const float br = B.re[kb][t], bi = B.im[kb][t];
      const float nsum = -(br + bi), diff = bi - br;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float4& v = a[q][t >> 1];
        const float are = (t & 1) ? v.z : v.x, aim = (t & 1) ? v.w : v.y;
        k1[q] = mfma4<float>(are + aim, br, k1[q]);
        acc.re[q] = mfma4<float>(aim, nsum, acc.re[q]);
        acc.im[q] = mfma4<float>(are, diff, acc.im[q]);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) { acc.re[q] += k1[q]; acc.im[q] += k1[q]; }
}

template <bool XCD>
__global__ void __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(2, 2))) k_bgemm_dma(BigGemmArgs g) {
  __shared__ __attribute__((aligned(16))) cpx<float> abuf[2 * DMA_TILE];
  const int Tn = g.n / 64;
  const size_t nn = (size_t)g.n * g.n;
  int b, ti, tj;
  tile_of_block<XCD>(Tn, b, ti, tj);
  cpx<float>* C = const_cast<cpx<float>*>(mat<float>(g.C, g.Ci, b, nn));
  const cpx<float>* D = g.D ? mat<float>(g.D, g.Di, b, nn) : nullptr;
  const bool active = !g.pred || g.pred[(size_t)(g.Ci ? g.Ci[b] : b) * g.pred_stride] > g.pred_thresh;
  if (!active) {
    const cpx<float>* src = D ? D : mat<float>(g.A, g.Ai, b, nn);
    RT<float> X;
    rt_load<float, false>(X, src + (size_t)ti * 64 * g.n + tj * 64, g.n);
    rt_store<float, false>(X, C + (size_t)ti * 64 * g.n + tj * 64, g.n);
    return;
  }
  const cpx<float>* Arow = mat<float>(g.A, g.Ai, b, nn) + (size_t)ti * 64 * g.n;
  const cpx<float>* Bcol = mat<float>(g.B, g.Bi, b, nn) + tj * 64;
  RT<float> acc, Bt, Bn;
  rt_zero(acc);
  dma_a_tile(Arow, g.n, abuf);
  rt_load<float, false>(Bt, Bcol, g.n);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  for (int tk = 0; tk < Tn; ++tk) {
    const bool more = tk + 1 < Tn;
    // buffer (tk + 1) & 1 was last read by step tk - 1, which every wave has
    // left at the barrier that ended it
    if (more) dma_a_tile(Arow + (tk + 1) * 64, g.n, abuf + ((tk + 1) & 1) * DMA_TILE);
    mma_dma(acc, abuf + (tk & 1) * DMA_TILE, Bt, [&] {
      if (more) rt_load<float, false>(Bn, Bcol + (size_t)(tk + 1) * 64 * g.n, g.n);
    });
    if (more) {
      __builtin_amdgcn_s_waitcnt(0);   // this wave's loads into LDS and registers
      __syncthreads();                 // every wave's
      rt_copy(Bt, Bn);
    }
  }
  bgemm_epilogue<float>(g, acc, b, ti, tj, C, D);
}

// Two output tiles per workgroup (variant 4; single precision, no transposes):
// 512 threads, waves 0-3 compute tile (ti, 2p) and waves 4-7 tile (ti, 2p + 1).
// The register-tile column of a lane is 16 w + c, so the second half's lanes
// address columns 64..127 of the pair from the same base pointer. Each k-step's
// A tile is loaded and staged in LDS once (by the first half) for both tiles.
__global__ void __launch_bounds__(2 * WG) k_bgemm_pair(BigGemmArgs g) {
  __shared__ BigShared<float> sh;
  const int Tn = g.n / 64;
  const size_t nn = (size_t)g.n * g.n;
  const int b = blockIdx.y, half = threadIdx.x >> 8;
  const int ti = blockIdx.x / (Tn / 2), tj0 = 2 * (blockIdx.x % (Tn / 2));
  const size_t base = (size_t)ti * 64 * g.n + tj0 * 64;
  cpx<float>* C = const_cast<cpx<float>*>(mat<float>(g.C, g.Ci, b, nn));
  const cpx<float>* D = g.D ? mat<float>(g.D, g.Di, b, nn) : nullptr;
  const bool active = !g.pred || g.pred[(size_t)(g.Ci ? g.Ci[b] : b) * g.pred_stride] > g.pred_thresh;
  if (!active) {
    const cpx<float>* src = D ? D : mat<float>(g.A, g.Ai, b, nn);
    RT<float> X;
    rt_load<float, false>(X, src + base, g.n);
    rt_store<float, false>(X, C + base, g.n);
    return;
  }
  const cpx<float>* A = mat<float>(g.A, g.Ai, b, nn);
  const cpx<float>* B = mat<float>(g.B, g.Bi, b, nn);
  RT<float> acc;
  rt_zero(acc);
  for (int tk = 0; tk < Tn; ++tk) {
    RT<float> At, Bt;
    if (half == 0) rt_load<float, false>(At, A + (size_t)ti * 64 * g.n + tk * 64, g.n);
    rt_load<float, false>(Bt, B + (size_t)tk * 64 * g.n + tj0 * 64, g.n);
    __syncthreads();
    if (half == 0) rt_store<float, false>(At, sh.slot, PITCH);
    __syncthreads();
    gemm_acc<float, false, PITCH>(acc, sh.slot, Bt);
  }
  rt_scale(acc, (float)g.alpha);
  if (D && g.beta != 0.0) {
    RT<float> Dt;
    rt_load<float, false>(Dt, D + base, g.n);
    rt_axpy(acc, (float)g.beta, Dt);
  }
  if (g.D2 && g.beta2 != 0.0) {
    RT<float> Dt;
    rt_load<float, false>(Dt, mat<float>(g.D2, g.D2i, b, nn) + base, g.n);
    rt_axpy(acc, (float)g.beta2, Dt);
  }
  if (g.gamma != 0.0 && ti == tj0 + half) {
    // the diagonal of this half's own tile: row == column - 64 half
    const Lane L;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (L.row<float>(q, r) == L.col - 64 * half) acc.re[q][r] += (float)g.gamma;
  }
  rt_store<float, false>(acc, C + base, g.n);
}

// Quadrant variants (single precision, no transposes): wave w of the
// workgroup owns the 32 x 32 quadrant (w >> 1, w & 1) of the 64 x 64 output
// tile. Both operand tiles of a k-step sit in LDS; every thread loads its share
// of the next k-step's tiles into registers (coalesced 16-byte loads) before
// the current products run, so the global loads drain under the MFMAs.
// SHAPE 16: v_mfma_f32_16x16x4f32 on 2 x 2 blocks of 16 x 16 per quadrant,
//   A operand lane (g, c) = (l / 16, l % 16) holds A[c][k = g], output row of
//   register r is 4 g + r, column c.
// SHAPE 32: v_mfma_f32_32x32x2f32 on the whole quadrant, A operand lane l
//   holds A[l % 32][k = l / 32], B operand B[k = l / 32][l % 32], output row of
//   register r is 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32.
// Complex products use the 3M form of tile.hpp.
struct QuadShared {
  cpx<float> a[64 * PITCH];
  cpx<float> b[64 * PITCH];
};

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));

__device__ __forceinline__ void quad_fetch(f4 (&r)[8], const cpx<float>* M, size_t ld, int tid) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int idx = tid + 256 * i, row = idx >> 5, c2 = idx & 31;
    r[i] = *reinterpret_cast<const f4*>(M + (size_t)row * ld + 2 * c2);
  }
}

__device__ __forceinline__ void quad_stage(const f4 (&r)[8], cpx<float>* S, int tid) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int idx = tid + 256 * i, row = idx >> 5, c2 = idx & 31;
    S[row * PITCH + 2 * c2] = cpx<float>{r[i].x, r[i].y};
    S[row * PITCH + 2 * c2 + 1] = cpx<float>{r[i].z, r[i].w};
  }
}

// Split-bf16 products (variant 3): every FP32 operand value v is written as
// three bfloat16 pieces v = v1 + v2 + v3 (v1 = bf16(v), v2 = bf16(v - v1),
// v3 = bf16(v - v1 - v2); each difference is exact in FP32, so the pieces hold
// all 24 significand bits), and a real product sum_k a_k b_k is formed from the
// six cross terms a_i b_j with i + j <= 4 on v_mfma_f32_16x16x32_bf16
// (products of bf16 pieces are exact, accumulation is FP32). The dropped terms
// a_2 b_3, a_3 b_2, a_3 b_3 are below 2^-24 |a||b| relative: FP32-level error.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ void split3(float v, bf16x8 (&p)[3], int i) {
  const __bf16 h = (__bf16)v;
  const float r1 = v - (float)h;
  const __bf16 m = (__bf16)r1;
  p[0][i] = h;
  p[1][i] = m;
  p[2][i] = (__bf16)(r1 - (float)m);
}

template <int SHAPE, bool SPLIT = false>
__global__ void __launch_bounds__(WG) k_bgemm_q(BigGemmArgs g) {
  __shared__ QuadShared sh;
  const int Tn = g.n / 64;
  const size_t nn = (size_t)g.n * g.n;
  const int b = blockIdx.y;
  const int ti = blockIdx.x / Tn, tj = blockIdx.x % Tn;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int qi = w >> 1, qj = w & 1;
  cpx<float>* C = const_cast<cpx<float>*>(mat<float>(g.C, g.Ci, b, nn));
  const cpx<float>* D = g.D ? mat<float>(g.D, g.Di, b, nn) : nullptr;
  const bool active = !g.pred || g.pred[(size_t)(g.Ci ? g.Ci[b] : b) * g.pred_stride] > g.pred_thresh;
  if (!active) {
    const cpx<float>* src = D ? D : mat<float>(g.A, g.Ai, b, nn);
    RT<float> X;
    rt_load<float, false>(X, src + (size_t)ti * 64 * g.n + tj * 64, g.n);
    rt_store<float, false>(X, C + (size_t)ti * 64 * g.n + tj * 64, g.n);
    return;
  }
  const cpx<float>* A = mat<float>(g.A, g.Ai, b, nn) + (size_t)ti * 64 * g.n;   // row block ti
  const cpx<float>* B = mat<float>(g.B, g.Bi, b, nn) + tj * 64;                 // column block tj
  constexpr int NB = SHAPE == 16 ? 2 : 1;      // MFMA blocks per quadrant side
  constexpr int NACC = SHAPE == 16 ? 4 : 16;   // accumulator registers per block
  typedef typename std::conditional<SHAPE == 16, f4, f16v>::type acc_t;
  acc_t k1[NB][NB], cr[NB][NB], ci[NB][NB];
#pragma unroll
  for (int x = 0; x < NB; ++x)
#pragma unroll
    for (int y = 0; y < NB; ++y)
#pragma unroll
      for (int r = 0; r < NACC; ++r) { k1[x][y][r] = 0.f; cr[x][y][r] = 0.f; ci[x][y][r] = 0.f; }
  f4 ra[8], rb[8];
  quad_fetch(ra, A, g.n, tid);
  quad_fetch(rb, B, g.n, tid);
  for (int tk = 0; tk < Tn; ++tk) {
    __syncthreads();
    quad_stage(ra, sh.a, tid);
    quad_stage(rb, sh.b, tid);
    __syncthreads();
    if (tk + 1 < Tn) {
      quad_fetch(ra, A + (tk + 1) * 64, g.n, tid);
      quad_fetch(rb, B + (size_t)(tk + 1) * 64 * g.n, g.n, tid);
    }
    if constexpr (SPLIT) {
      // 16x16x32 bf16 MFMA: lane (gg, c) holds k = 32 kk + 8 gg + i, i = 0..7,
      // of row c (A) and of column c (B); A and B agree on the k of each slot
      const int gg = l >> 4, c = l & 15;
      for (int kk = 0; kk < 2; ++kk) {
        bf16x8 ap[NB][3][3], bp[NB][3][3];   // [block][operand][piece]
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int k = 32 * kk + 8 * gg + i;
#pragma unroll
          for (int x = 0; x < NB; ++x) {
            const cpx<float> av = sh.a[(qi * 32 + x * 16 + c) * PITCH + k];
            split3(av.re + av.im, ap[x][0], i);
            split3(av.im, ap[x][1], i);
            split3(av.re, ap[x][2], i);
          }
#pragma unroll
          for (int y = 0; y < NB; ++y) {
            const cpx<float> bv = sh.b[k * PITCH + qj * 32 + y * 16 + c];
            split3(bv.re, bp[y][0], i);
            split3(-(bv.re + bv.im), bp[y][1], i);
            split3(bv.im - bv.re, bp[y][2], i);
          }
        }
#pragma unroll
        for (int x = 0; x < NB; ++x)
#pragma unroll
          for (int y = 0; y < NB; ++y) {
            // pieces (i, j) with i + j <= 4 (1-based): (1,1) (1,2) (2,1) (1,3) (3,1) (2,2)
            constexpr int PI[6] = {0, 0, 1, 0, 2, 1}, PJ[6] = {0, 1, 0, 2, 0, 1};
#pragma unroll
            for (int t = 0; t < 6; ++t) {
              k1[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[x][0][PI[t]], bp[y][0][PJ[t]], k1[x][y], 0, 0, 0);
              cr[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[x][1][PI[t]], bp[y][1][PJ[t]], cr[x][y], 0, 0, 0);
              ci[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[x][2][PI[t]], bp[y][2][PJ[t]], ci[x][y], 0, 0, 0);
            }
          }
      }
    } else if constexpr (SHAPE == 16) {
      const int gg = l >> 4, c = l & 15;
#pragma unroll 4
      for (int kk = 0; kk < 16; ++kk) {
        const int k = 4 * kk + gg;
        cpx<float> av[NB], bv[NB];
#pragma unroll
        for (int x = 0; x < NB; ++x) av[x] = sh.a[(qi * 32 + x * 16 + c) * PITCH + k];
#pragma unroll
        for (int y = 0; y < NB; ++y) bv[y] = sh.b[k * PITCH + qj * 32 + y * 16 + c];
#pragma unroll
        for (int x = 0; x < NB; ++x) {
          const float asum = av[x].re + av[x].im;
#pragma unroll
          for (int y = 0; y < NB; ++y) {
            const float nsum = -(bv[y].re + bv[y].im), diff = bv[y].im - bv[y].re;
            k1[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(asum, bv[y].re, k1[x][y], 0, 0, 0);
            cr[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[x].im, nsum, cr[x][y], 0, 0, 0);
            ci[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[x].re, diff, ci[x][y], 0, 0, 0);
          }
        }
      }
    } else {
      const int h = l >> 5, c = l & 31;
#pragma unroll 4
      for (int kk = 0; kk < 32; ++kk) {
        const int k = 2 * kk + h;
        const cpx<float> av = sh.a[(qi * 32 + c) * PITCH + k];
        const cpx<float> bv = sh.b[k * PITCH + qj * 32 + c];
        const float nsum = -(bv.re + bv.im), diff = bv.im - bv.re;
        k1[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(av.re + av.im, bv.re, k1[0][0], 0, 0, 0);
        cr[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(av.im, nsum, cr[0][0], 0, 0, 0);
        ci[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(av.re, diff, ci[0][0], 0, 0, 0);
      }
    }
  }
  // epilogue: C = alpha (K1 + Cr, K1 + Ci) + beta D + beta2 D2 + gamma I
  const cpx<float>* D2 = g.D2 ? mat<float>(g.D2, g.D2i, b, nn) : nullptr;
  const float al = (float)g.alpha, be = (float)g.beta, be2 = (float)g.beta2, ga = (float)g.gamma;
#pragma unroll
  for (int x = 0; x < NB; ++x)
#pragma unroll
    for (int y = 0; y < NB; ++y)
#pragma unroll
      for (int r = 0; r < NACC; ++r) {
        int row, col;
        if constexpr (SHAPE == 16) {
          row = qi * 32 + x * 16 + 4 * (l >> 4) + r;
          col = qj * 32 + y * 16 + (l & 15);
        } else {
          row = qi * 32 + 8 * (r >> 2) + 4 * (l >> 5) + (r & 3);
          col = qj * 32 + (l & 31);
        }
        const size_t e = (size_t)(ti * 64 + row) * g.n + tj * 64 + col;
        cpx<float> v{al * (k1[x][y][r] + cr[x][y][r]), al * (k1[x][y][r] + ci[x][y][r])};
        if (D && g.beta != 0.0) { const cpx<float> d = D[e]; v.re += be * d.re; v.im += be * d.im; }
        if (D2 && g.beta2 != 0.0) { const cpx<float> d = D2[e]; v.re += be2 * d.re; v.im += be2 * d.im; }
        if (g.gamma != 0.0 && ti == tj && row == col) v.re += ga;
        C[e] = v;
      }
}

hipError_t launch_bgemm(int prec, const BigGemmArgs& g_in, hipStream_t s) {
  if (g_in.batch <= 0) return hipSuccess;
  if (g_in.C2 && g_in.pred) return hipErrorInvalidValue;   // the copy path writes no C2
  BigGemmArgs g = g_in;
  // a second output is written by the register-B kernels (0, 5, 6, 7, 8) only
  if (g.C2 && g.variant >= 1 && g.variant <= 4) g.variant = 0;
  const int Tn = g.n / 64;
  const dim3 grid(Tn * Tn, g.batch);
  if (prec == 32 && !g.transA && !g.transB && g.variant == 4 && Tn % 2 == 0) {
    hipLaunchKernelGGL(k_bgemm_pair, dim3(Tn * Tn / 2, g.batch), dim3(2 * WG), 0, s, g);
    return hipGetLastError();
  }
  const bool xcd_ok = Tn <= 16 && ((size_t)Tn * Tn * g.batch) % 8 == 0 &&
                      (size_t)Tn * Tn * g.batch <= 0x7fffffff;
  if (prec == 32 && !g.transA && !g.transB && g.variant == 8) {
    if (xcd_ok) hipLaunchKernelGGL(k_bgemm_dma<true>, dim3(Tn * Tn * g.batch), dim3(WG), 0, s, g);
    else hipLaunchKernelGGL(k_bgemm_dma<false>, grid, dim3(WG), 0, s, g);
    return hipGetLastError();
  }
  if (prec == 32 && !g.transA && !g.transB && g.variant == 7 && xcd_ok) {
    hipLaunchKernelGGL(k_bgemm_occ3<true>, dim3(Tn * Tn * g.batch), dim3(WG), 0, s, g);
    return hipGetLastError();
  }
  if (prec == 32 && !g.transA && !g.transB && (g.variant == 6 || g.variant == 7)) {
    hipLaunchKernelGGL(k_bgemm_occ3<false>, grid, dim3(WG), 0, s, g);
    return hipGetLastError();
  }
  if (prec == 32 && !g.transA && !g.transB && g.variant == 5 && xcd_ok) {
    hipLaunchKernelGGL((k_bgemm<float, false, false, true>), dim3(Tn * Tn * g.batch), dim3(WG), 0, s, g);
    return hipGetLastError();
  }
  if (prec == 32 && !g.transA && !g.transB && g.variant == 1) {
    hipLaunchKernelGGL(k_bgemm_q<16>, grid, dim3(WG), 0, s, g);
    return hipGetLastError();
  }
  if (prec == 32 && !g.transA && !g.transB && g.variant == 2) {
    hipLaunchKernelGGL(k_bgemm_q<32>, grid, dim3(WG), 0, s, g);
    return hipGetLastError();
  }
  if (prec == 32 && !g.transA && !g.transB && g.variant == 3) {
    hipLaunchKernelGGL((k_bgemm_q<16, true>), grid, dim3(WG), 0, s, g);
    return hipGetLastError();
  }
#define LMAG_BG(T, a, b) hipLaunchKernelGGL((k_bgemm<T, a, b>), grid, dim3(WG), 0, s, g)
  if (prec == 32) {
    if (g.transA && g.transB) LMAG_BG(float, true, true);
    else if (g.transA) LMAG_BG(float, true, false);
    else if (g.transB) LMAG_BG(float, false, true);
    else LMAG_BG(float, false, false);
  } else {
    if (g.transA && g.transB) LMAG_BG(double, true, true);
    else if (g.transA) LMAG_BG(double, true, false);
    else if (g.transB) LMAG_BG(double, false, true);
    else LMAG_BG(double, false, false);
  }
#undef LMAG_BG
  return hipGetLastError();
}

// Y_b = a X_b + c Z_b + d I (elementwise, batched; Z may be null). Each
// thread moves 16-byte vectors (two FP32 or one FP64 complex element), four
// per pass with the loads issued ahead of the stores; a = 0 reads no X.
template <typename T> struct Vec16;
template <> struct Vec16<float> { using type = float4; };
template <> struct Vec16<double> { using type = double2; };

template <typename T>
__device__ __forceinline__ void axpby_vec(typename Vec16<T>::type& y, T a, const typename Vec16<T>::type* x,
                                          T c, const typename Vec16<T>::type* z) {
  if constexpr (sizeof(T) == 4) {
    y = make_float4(0.f, 0.f, 0.f, 0.f);
    if (x) { y.x = a * x->x; y.y = a * x->y; y.z = a * x->z; y.w = a * x->w; }
    if (z) { y.x += c * z->x; y.y += c * z->y; y.z += c * z->z; y.w += c * z->w; }
  } else {
    y = make_double2(0.0, 0.0);
    if (x) { y.x = a * x->x; y.y = a * x->y; }
    if (z) { y.x += c * z->x; y.y += c * z->y; }
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_baxpby(BigAxpbyArgs g) {
  using V = typename Vec16<T>::type;
  constexpr int per = 16 / (2 * sizeof(T));   // complex elements per vector
  constexpr int U = 4;
  const int nv = g.n * g.n / per;             // n <= 4096: fits in int
  const size_t nn = (size_t)g.n * g.n;
  const int b = blockIdx.y;
  const V* X = reinterpret_cast<const V*>(mat<T>(g.X, g.Xi, b, nn));
  const V* Z = g.Z ? reinterpret_cast<const V*>(mat<T>(g.Z, g.Zi, b, nn)) : nullptr;
  V* Y = reinterpret_cast<V*>(const_cast<cpx<T>*>(mat<T>(g.Y, g.Yi, b, nn)));
  double ad = g.a;
  if (g.ms) ad = ldexp(ad, -(int)g.ms[2 * (size_t)(g.Yi ? g.Yi[b] : b) + 1]);
  const T a = (T)ad, c = (T)g.c;
  const bool rx = ad != 0.0;
  const int stride = gridDim.x * 256;
  for (int v0 = blockIdx.x * 256 + threadIdx.x; v0 < nv; v0 += U * stride) {
    V xv[U], zv[U];
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
        V y;
        axpby_vec<T>(y, a, rx ? &xv[u] : nullptr, c, Z ? &zv[u] : nullptr);
        if (g.d != 0.0) {
#pragma unroll
          for (int j = 0; j < per; ++j) {
            const int e = v * per + j;
            if (e / g.n == e % g.n) {
              if constexpr (sizeof(T) == 4) { if (j == 0) y.x += (T)g.d; else y.z += (T)g.d; }
              else y.x += (T)g.d;
            }
          }
        }
        Y[v] = y;
      }
    }
  }
}

// The same one complex element at a time, for base pointers that are not
// 16-byte aligned (a caller's output buffer may start anywhere on 8 bytes).
template <typename T>
__global__ void __launch_bounds__(256) k_baxpby_scalar(BigAxpbyArgs g) {
  const size_t nn = (size_t)g.n * g.n;
  const int b = blockIdx.y;
  const cpx<T>* X = mat<T>(g.X, g.Xi, b, nn);
  const cpx<T>* Z = g.Z ? mat<T>(g.Z, g.Zi, b, nn) : nullptr;
  cpx<T>* Y = const_cast<cpx<T>*>(mat<T>(g.Y, g.Yi, b, nn));
  double a = g.a;
  if (g.ms) a = ldexp(a, -(int)g.ms[2 * (size_t)(g.Yi ? g.Yi[b] : b) + 1]);
  for (int e = blockIdx.x * 256 + threadIdx.x; e < (int)nn; e += gridDim.x * 256) {
    cpx<T> y;
    y.re = T(0);
    y.im = T(0);
    if (a != 0.0) { const cpx<T> x = X[e]; y.re = (T)a * x.re; y.im = (T)a * x.im; }
    if (Z) { const cpx<T> z = Z[e]; y.re += (T)g.c * z.re; y.im += (T)g.c * z.im; }
    if (g.d != 0.0 && e / g.n == e % g.n) y.re += (T)g.d;
    Y[e] = y;
  }
}

hipError_t launch_baxpby(int prec, const BigAxpbyArgs& g, hipStream_t s) {
  if (g.batch <= 0) return hipSuccess;
  auto misaligned = [](const void* p) { return ((uintptr_t)p & 15) != 0; };
  if (misaligned(g.X) || misaligned(g.Y) || misaligned(g.Z)) {
    const size_t nn = (size_t)g.n * g.n;
    const dim3 grid((unsigned)std::min<size_t>((nn + 255) / 256, 1024), g.batch);
    if (prec == 32) hipLaunchKernelGGL(k_baxpby_scalar<float>, grid, dim3(256), 0, s, g);
    else hipLaunchKernelGGL(k_baxpby_scalar<double>, grid, dim3(256), 0, s, g);
    return hipGetLastError();
  }
  const size_t nv = (size_t)g.n * g.n / (prec == 32 ? 2 : 1);
  // about four vectors per thread per matrix (1024 per workgroup), at most 1024 workgroups
  const dim3 grid((unsigned)std::min<size_t>(std::max<size_t>((nv + 1023) / 1024, 1), 1024), g.batch);
  if (prec == 32) hipLaunchKernelGGL(k_baxpby<float>, grid, dim3(256), 0, s, g);
  else hipLaunchKernelGGL(k_baxpby<double>, grid, dim3(256), 0, s, g);
  return hipGetLastError();
}

// Omega_n = sum_j alpha_{n,j} B_j tile by tile; partial FP64 column 1-norms of
// every 64-row block: part[slice][tile_row][col].
template <typename T, int S>
__global__ void __launch_bounds__(WG) k_bomega(BigOmegaArgs g) {
  const int Tn = g.n / 64;
  const size_t nn = (size_t)g.n * g.n;
  const int s0 = blockIdx.y * S;
  const int ti = blockIdx.x / Tn, tj = blockIdx.x % Tn;
  const cpx<T>* basis = (const cpx<T>*)g.basis;
  // S consecutive slices per workgroup: each basis tile is fetched once for all S
  RT<T> X[S];
#pragma unroll
  for (int q = 0; q < S; ++q) rt_zero(X[q]);
  const int t = blockIdx.x;
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
    RT<T> Bt;
    rt_load<T, false>(Bt, basis + (size_t)j * nn + (size_t)ti * 64 * g.n + tj * 64, g.n);
#pragma unroll
    for (int q = 0; q < S; ++q)
      if (aj[q] != 0.0) rt_axpy(X[q], (T)aj[q], Bt);
  }
  const Lane L;
#pragma unroll
  for (int q = 0; q < S; ++q) {
    const int slice = s0 + q;
    if (slice >= g.n_slices) break;
    cpx<T>* out = (cpx<T>*)g.omega + (size_t)slice * nn;
    rt_store<T, false>(X[q], out + (size_t)ti * 64 * g.n + tj * 64, g.n);
    // column sums of |X| over this tile's 64 rows
    double sum = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double u = (double)X[q].re[a][r], v = (double)X[q].im[a][r];
        sum += sqrt(u * u + v * v);
      }
    sum += __shfl_xor(sum, 16);
    sum += __shfl_xor(sum, 32);
    if (L.g == 0) g.part[((size_t)slice * Tn + ti) * g.n + tj * 64 + L.col] = sum;
  }
}

// Per slice: ||Omega||_1 from the partial column sums, (m, s) and Neumann
// levels; then Omega <- Omega / 2^s.
template <typename T>
__global__ void __launch_bounds__(256) k_bnorm(BigOmegaArgs g) {
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
    big_choose_ms<T>(v, m, s);
    g.ms[2 * (size_t)slice] = (int8_t)m;
    g.ms[2 * (size_t)slice + 1] = (int8_t)s;
    if (g.nlev) {
      const int lv = big_neumann_levels<T>(ldexp(v, -s), g.b3);
      g.nlev[slice] = (int8_t)(lv > 0 ? lv : kBigNeumannLevels);
    }
    sc_sh = s;
  }
  __syncthreads();
  const int s = sc_sh;
  if (s == 0) return;
  const T f = (T)ldexp(1.0, -s);
  const size_t nn = (size_t)g.n * g.n;
  cpx<T>* X = (cpx<T>*)g.omega + (size_t)slice * nn;
  for (size_t e = threadIdx.x; e < nn; e += 256) { X[e].re *= f; X[e].im *= f; }
}

// Partial FP64 column 1-norms of dense matrices (as k_bomega's second half):
// part[slice][tile_row][col].
template <typename T>
__global__ void __launch_bounds__(WG) k_bcolsum(BigOmegaArgs g) {
  const int Tn = g.n / 64;
  const size_t nn = (size_t)g.n * g.n;
  const int slice = blockIdx.y;
  const int ti = blockIdx.x / Tn, tj = blockIdx.x % Tn;
  RT<T> X;
  rt_load<T, false>(X, (const cpx<T>*)g.omega + (size_t)slice * nn + (size_t)ti * 64 * g.n + tj * 64, g.n);
  const Lane L;
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double a = (double)X.re[q][r], b = (double)X.im[q][r];
      s += sqrt(a * a + b * b);
    }
  s += __shfl_xor(s, 16);
  s += __shfl_xor(s, 32);
  if (L.g == 0) g.part[((size_t)slice * Tn + ti) * g.n + tj * 64 + L.col] = s;
}

// Omega = sum_j alpha_j B_j with its partial column norms; with ms set, also
// the per-slice (m, s), Neumann levels and the scaling Omega / 2^s.
hipError_t launch_bomega(int prec, const BigOmegaArgs& g, hipStream_t s) {
  if (g.n_slices <= 0) return hipSuccess;
  const int Tn = g.n / 64;
  constexpr int S = kBigSlicesPerGroup;
  const dim3 grid(Tn * Tn, (g.n_slices + S - 1) / S);
  if (prec == 32) {
    hipLaunchKernelGGL((k_bomega<float, S>), grid, dim3(WG), 0, s, g);
    if (g.ms) hipLaunchKernelGGL(k_bnorm<float>, dim3(g.n_slices), dim3(256), 0, s, g);
  } else {
    hipLaunchKernelGGL((k_bomega<double, S>), grid, dim3(WG), 0, s, g);
    if (g.ms) hipLaunchKernelGGL(k_bnorm<double>, dim3(g.n_slices), dim3(256), 0, s, g);
  }
  return hipGetLastError();
}

// (m, s), Neumann levels and the scaling Omega / 2^s of dense exponents held
// in g.omega (the sixth-order slices, assembled by products).
hipError_t launch_bnorm_dense(int prec, const BigOmegaArgs& g, hipStream_t s) {
  if (g.n_slices <= 0) return hipSuccess;
  const int Tn = g.n / 64;
  if (prec == 32) {
    hipLaunchKernelGGL(k_bcolsum<float>, dim3(Tn * Tn, g.n_slices), dim3(WG), 0, s, g);
    hipLaunchKernelGGL(k_bnorm<float>, dim3(g.n_slices), dim3(256), 0, s, g);
  } else {
    hipLaunchKernelGGL(k_bcolsum<double>, dim3(Tn * Tn, g.n_slices), dim3(WG), 0, s, g);
    hipLaunchKernelGGL(k_bnorm<double>, dim3(g.n_slices), dim3(256), 0, s, g);
  }
  return hipGetLastError();
}

// g[slice][j] = Re sum_x K^T[x] B_j[x]: partial sums per (slice, tile) in
// part[slice][tile][j], then a fixed-order reduction over tiles.
template <typename T, int S>
__global__ void __launch_bounds__(WG) k_btraces_part(BigTraceArgs g) {
  __shared__ BigShared<T> sh;
  __shared__ double red[4][S][MAX_BIG_NB];
  const int Tn = g.n / 64;
  const size_t nn = (size_t)g.n * g.n;
  const int s0 = blockIdx.y * S, tile = blockIdx.x;
  const int ti = tile / Tn, tj = tile % Tn;
  const cpx<T>* basis = (const cpx<T>*)g.basis;
  const Lane L;
  // Re Tr(K B_j) over this tile = Re sum_{a,b} K[a][b] B_j[b][a] (a in row block
  // ti, b in column block tj): with trans_basis the K tile is transposed once
  // through LDS and paired with the untransposed basis tile (tj, ti), whose
  // rows the lanes then read contiguously; otherwise K and B_j pair as stored
  const int bt = g.trans_basis ? tj * Tn + ti : tile;
  for (int e = threadIdx.x; e < 4 * S * g.nb; e += WG) (&red[0][0][0])[(e / g.nb) * MAX_BIG_NB + e % g.nb] = 0.0;
  const int j0 = g.tile_ptr ? g.tile_ptr[bt] : 0, j1 = g.tile_ptr ? g.tile_ptr[bt + 1] : g.nb;
  RT<T> Kt[S];
#pragma unroll
  for (int q = 0; q < S; ++q) {
    if (j1 > j0 && s0 + q < g.n_slices) {
      const cpx<T>* K = (const cpx<T>*)g.K + (size_t)(s0 + q) * nn + (size_t)ti * 64 * g.n + tj * 64;
      if (g.trans_basis) {
        RT<T> X;
        rt_load<T, false>(X, K, g.n);
        __syncthreads();
        rt_store<T, false>(X, sh.slot, PITCH);
        __syncthreads();
        rt_load<T, true>(Kt[q], sh.slot, PITCH);
      } else {
        rt_load<T, false>(Kt[q], K, g.n);
      }
    } else {
      rt_zero(Kt[q]);
    }
  }
  __syncthreads();
  for (int e = j0; e < j1; ++e) {
    const int j = g.tile_ptr ? g.tile_j[e] : e;
    RT<T> Bt;
    rt_load<T, false>(Bt, basis + (size_t)j * nn + (size_t)(bt / Tn) * 64 * g.n + (bt % Tn) * 64, g.n);
#pragma unroll
    for (int q = 0; q < S; ++q) {
      // a lane's 16 terms in the compute precision, the sums over lanes and
      // tiles in FP64
      T part = T(0);
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          part = fma(Kt[q].re[a][r], Bt.re[a][r], part);
          part = fma(-Kt[q].im[a][r], Bt.im[a][r], part);
        }
      double acc = (double)part;
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
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

__global__ void k_btraces_sum(BigTraceArgs g) {
  const int slice = blockIdx.x;
  const int Tn = g.n / 64;
  for (int j = threadIdx.x; j < g.nb; j += blockDim.x) {
    double s = 0.0;
    for (int t = 0; t < Tn * Tn; ++t) s += g.part[((size_t)slice * Tn * Tn + t) * g.nb + j];
    g.gtrace[(size_t)(g.first_slice + slice) * g.nb + j] = s;
  }
}

__global__ void k_tile_flags(const cpx<double>* basis, int nb, int n, uint8_t* flags) {
  __shared__ int any;
  const int Tn = n / 64;
  const int t = blockIdx.x, j = blockIdx.y;
  const int ti = t / Tn, tj = t % Tn;
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  const cpx<double>* B = basis + (size_t)j * n * n + (size_t)ti * 64 * n + tj * 64;
  int nz = 0;
  for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) {
    const cpx<double> v = B[(size_t)(e / 64) * n + e % 64];
    nz |= (v.re != 0.0 || v.im != 0.0);
  }
  if (nz) any = 1;   // benign race: every writer stores 1
  __syncthreads();
  if (threadIdx.x == 0) flags[(size_t)j * Tn * Tn + t] = (uint8_t)any;
}

hipError_t launch_tile_flags(const double* basis, int nb, int n, uint8_t* flags, hipStream_t s) {
  const int Tn = n / 64;
  hipLaunchKernelGGL(k_tile_flags, dim3(Tn * Tn, nb), dim3(256), 0, s, (const cpx<double>*)basis, nb, n,
                     flags);
  return hipGetLastError();
}

hipError_t launch_btraces(int prec, const BigTraceArgs& g, hipStream_t s) {
  if (g.n_slices <= 0) return hipSuccess;
  const int Tn = g.n / 64;
  constexpr int S = kBigSlicesPerGroup;
  const dim3 grid(Tn * Tn, (g.n_slices + S - 1) / S);
  if (prec == 32) hipLaunchKernelGGL((k_btraces_part<float, S>), grid, dim3(WG), 0, s, g);
  else hipLaunchKernelGGL((k_btraces_part<double, S>), grid, dim3(WG), 0, s, g);
  return launch_btraces_sum(g, s);
}

hipError_t launch_btraces_sum(const BigTraceArgs& g, hipStream_t s) {
  hipLaunchKernelGGL(k_btraces_sum, dim3(g.n_slices), dim3(64), 0, s, g);
  return hipGetLastError();
}

// F_item = Re Tr(S_T^dag U) / d^2 = Re sum_{a,b} S_T^dag[a][b] U[b][a] / d^2 in FP64.
template <typename T>
__global__ void k_bfidelity(BigFidArgs g) {
  __shared__ double red[2][256];
  const int item = blockIdx.x;
  const size_t nn = (size_t)g.n * g.n;
  const cpx<T>* U = (const cpx<T>*)g.U + (size_t)g.U_index[item] * nn;
  const cpx<double>* S = (const cpx<double>*)g.st64 + (size_t)g.target[item] * nn;
  double re = 0.0, im = 0.0;
  for (size_t e = threadIdx.x; e < nn; e += 256) {
    const size_t a = e / g.n, c = e % g.n;
    const cpx<double> x = S[e];
    const cpx<T> y = U[c * g.n + a];
    re += x.re * (double)y.re - x.im * (double)y.im;
    im += x.re * (double)y.im + x.im * (double)y.re;
    if (a == c) { re += x.re; im += x.im; }   // U is stored as U - I
  }
  red[0][threadIdx.x] = re;
  red[1][threadIdx.x] = im;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      red[0][threadIdx.x] += red[0][threadIdx.x + off];
      red[1][threadIdx.x] += red[1][threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double inv = 1.0 / ((double)g.d * g.d);
    g.F[g.F_index ? g.F_index[item] : item] = red[0][0] * inv;
  }
}

hipError_t launch_bfidelity(int prec, const BigFidArgs& g, hipStream_t s) {
  if (g.n_items <= 0) return hipSuccess;
  if (prec == 32) hipLaunchKernelGGL(k_bfidelity<float>, dim3(g.n_items), dim3(256), 0, s, g);
  else hipLaunchKernelGGL(k_bfidelity<double>, dim3(g.n_items), dim3(256), 0, s, g);
  return hipGetLastError();
}

// Superoperator lift, dissipator and target for general n = d^2 (double).
__global__ void k_blift(const cpx<double>* H, int d, cpx<double>* out) {
  const int n = d * d;
  const size_t nn = (size_t)n * n;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < nn; idx += (size_t)gridDim.x * blockDim.x) {
    const int a = (int)(idx / n), b = (int)(idx % n);
    const int i = a % d, j = a / d, k = b % d, l = b / d;
    double zr = 0.0, zi = 0.0;
    if (j == l) { zr += H[i * d + k].re; zi += H[i * d + k].im; }
    if (i == k) { zr -= H[l * d + j].re; zi -= H[l * d + j].im; }
    out[idx] = cpx<double>{zi, -zr};
  }
}

__global__ void k_bdissipator(const cpx<double>* Ls, int n_jump, int d, const cpx<double>* LdL,
                              cpx<double>* out) {
  const int n = d * d;
  const size_t nn = (size_t)n * n;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < nn; idx += (size_t)gridDim.x * blockDim.x) {
    const int a = (int)(idx / n), b = (int)(idx % n);
    const int i = a % d, j = a / d, k = b % d, l = b / d;
    double re = 0.0, im = 0.0;
    for (int q = 0; q < n_jump; ++q) {
      const cpx<double>* L = Ls + (size_t)q * d * d;
      const cpx<double>* M = LdL + (size_t)q * d * d;
      const cpx<double> x = L[j * d + l], y = L[i * d + k];
      re += x.re * y.re + x.im * y.im;
      im += x.re * y.im - x.im * y.re;
      if (j == l) { re -= 0.5 * M[i * d + k].re; im -= 0.5 * M[i * d + k].im; }
      if (i == k) { re -= 0.5 * M[l * d + j].re; im -= 0.5 * M[l * d + j].im; }
    }
    out[idx] = cpx<double>{re, im};
  }
}

// M_q = L_q^dag L_q (d x d, one thread per entry)
__global__ void k_ldl(const cpx<double>* Ls, int n_jump, int d, cpx<double>* out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n_jump * d * d) return;
  const int q = idx / (d * d), x = (idx / d) % d, y = idx % d;
  const cpx<double>* L = Ls + (size_t)q * d * d;
  double re = 0.0, im = 0.0;
  for (int z = 0; z < d; ++z) {
    const cpx<double> p = L[z * d + x], r = L[z * d + y];
    re += p.re * r.re + p.im * r.im;
    im += p.re * r.im - p.im * r.re;
  }
  out[idx] = cpx<double>{re, im};
}

__global__ void k_btargets(const cpx<double>* U, int n_targets, int d, cpx<double>* st64, cpx<float>* st32) {
  const int n = d * d;
  const size_t nn = (size_t)n * n;
  const int t = blockIdx.y;
  const cpx<double>* Ut = U + (size_t)t * d * d;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < nn; idx += (size_t)gridDim.x * blockDim.x) {
    const int r = (int)(idx / n), c = (int)(idx % n);
    const int k = r % d, l = r / d, i = c % d, j = c / d;
    const cpx<double> x = Ut[j * d + l], y = Ut[i * d + k];
    const cpx<double> o{x.re * y.re + x.im * y.im, x.im * y.re - x.re * y.im};
    st64[(size_t)t * nn + idx] = o;
    if (st32) st32[(size_t)t * nn + idx] = cpx<float>{(float)o.re, (float)o.im};
  }
}

hipError_t launch_blift(const double* H, int d, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_blift, dim3(1024), dim3(256), 0, s, (const cpx<double>*)H, d, (cpx<double>*)out);
  return hipGetLastError();
}
hipError_t launch_bdissipator(const double* Ls, int n_jump, int d, double* ldl, double* out, hipStream_t s) {
  if (n_jump > 0)
    hipLaunchKernelGGL(k_ldl, dim3((n_jump * d * d + 255) / 256), dim3(256), 0, s, (const cpx<double>*)Ls,
                       n_jump, d, (cpx<double>*)ldl);
  hipLaunchKernelGGL(k_bdissipator, dim3(1024), dim3(256), 0, s, (const cpx<double>*)Ls, n_jump, d,
                     (const cpx<double>*)ldl, (cpx<double>*)out);
  return hipGetLastError();
}
hipError_t launch_btargets(const double* U, int n_targets, int d, double* st64, float* st32, hipStream_t s) {
  hipLaunchKernelGGL(k_btargets, dim3(256, n_targets), dim3(256), 0, s, (const cpx<double>*)U, n_targets, d,
                     (cpx<double>*)st64, (cpx<float>*)st32);
  return hipGetLastError();
}

}  // namespace lmag
