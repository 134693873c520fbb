// Register-tile primitives for 64 x 64 complex superoperator tiles on gfx950.
//
// A workgroup of 256 threads (four wave64s, one per SIMD) owns one tile. The
// register tile ("RT") layout follows the output layout of the 16x16x4 MFMA:
// thread (wave w, lane l), g = l / 16, c = l % 16, holds column j = 16 w + c and
// the sixteen rows i = 16 q + sub(g, r) (q, r in 0..3) in re[q][r], im[q][r],
// where sub(g, r) is the MFMA output row of register r in lane group g.
// Because MFMA contractions may use any permutation of the summation index as
// long as both operands use the same one, a tile in this layout is directly the
// B operand of the next product (k = 16 kb + sub(g, t) sits in register (kb, t)):
// chains of products never leave registers. The A operand is read from LDS (or
// from global memory), row-major with a padded pitch, in either orientation.
//
// Complex products in FP64 use four real MFMAs (4M method): Cr += Ar Br - Ai Bi,
// Ci += Ar Bi + Ai Br. In FP32 they use three (3M, Gauss's trick):
// K1 = (Ar + Ai) Br, Cr += K1 - Ai (Br + Bi), Ci += K1 + Ar (Bi - Br); its
// normwise error bound is a small constant times that of the 4M method.
#pragma once
#include <type_traits>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lmag {

constexpr int TN = 64;        // tile edge (superoperator dimension of the fast path)
constexpr int PITCH = 65;     // LDS row pitch in complex elements (one 8-byte bank pair of skew)
constexpr int WG = 256;       // threads per workgroup

template <typename T> struct cpx { T re, im; };

template <typename T> struct vec4;
template <> struct vec4<float> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct vec4<double> { typedef double type __attribute__((ext_vector_type(4))); };

template <typename T>
__device__ __forceinline__ typename vec4<T>::type mfma4(T a, T b, typename vec4<T>::type c);
template <>
__device__ __forceinline__ vec4<float>::type mfma4<float>(float a, float b, vec4<float>::type c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <>
__device__ __forceinline__ vec4<double>::type mfma4<double>(double a, double b, vec4<double>::type c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <typename T> struct RT {
  typename vec4<T>::type re[4], im[4];
};

// Row, inside a 16-row block, of accumulator register r of lane group g in the
// 16x16x4 MFMA output. Single precision: 4 g + r. Double precision interleaves
// the lane groups: g + 4 r (measured on gfx950).
template <typename T> struct Sub;
template <> struct Sub<float> {
  static __device__ __forceinline__ constexpr int row(int g, int r) { return 4 * g + r; }
  static __device__ __forceinline__ constexpr int grp(int s) { return s >> 2; }   // s = row & 15
  static __device__ __forceinline__ constexpr int reg(int s) { return s & 3; }
};
template <> struct Sub<double> {
  static __device__ __forceinline__ constexpr int row(int g, int r) { return g + 4 * r; }
  static __device__ __forceinline__ constexpr int grp(int s) { return s & 3; }
  static __device__ __forceinline__ constexpr int reg(int s) { return s >> 2; }
};

struct Lane {
  int w, l, g, c, col;
  __device__ __forceinline__ Lane() {
    const int tid = threadIdx.x;
    w = tid >> 6; l = tid & 63; g = l >> 4; c = l & 15; col = 16 * w + c;
  }
  template <typename T>
  __device__ __forceinline__ int row(int q, int r) const { return 16 * q + Sub<T>::row(g, r); }
};

template <typename T> __device__ __forceinline__ void rt_zero(RT<T>& X) {
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) { X.re[q][r] = T(0); X.im[q][r] = T(0); }
}

// X += v I
template <typename T> __device__ __forceinline__ void rt_add_diag(RT<T>& X, T v) {
  const Lane L;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (L.template row<T>(q, r) == L.col) X.re[q][r] += v;
}

template <typename T> __device__ __forceinline__ void rt_identity(RT<T>& X) {
  rt_zero(X);
  rt_add_diag(X, T(1));
}

// Y = a X + b I (real a, b)
template <typename T> __device__ __forceinline__ void rt_poly1(RT<T>& Y, const RT<T>& X, T a, T b) {
#pragma unroll
  for (int q = 0; q < 4; ++q) { Y.re[q] = a * X.re[q]; Y.im[q] = a * X.im[q]; }
  rt_add_diag(Y, b);
}

// Y += a X
template <typename T> __device__ __forceinline__ void rt_axpy(RT<T>& Y, T a, const RT<T>& X) {
#pragma unroll
  for (int q = 0; q < 4; ++q) { Y.re[q] += a * X.re[q]; Y.im[q] += a * X.im[q]; }
}

template <typename T> __device__ __forceinline__ void rt_scale(RT<T>& Y, T a) {
#pragma unroll
  for (int q = 0; q < 4; ++q) { Y.re[q] *= a; Y.im[q] *= a; }
}

template <typename T> __device__ __forceinline__ void rt_copy(RT<T>& Y, const RT<T>& X) {
#pragma unroll
  for (int q = 0; q < 4; ++q) { Y.re[q] = X.re[q]; Y.im[q] = X.im[q]; }
}

// Load a row-major 64x64 complex matrix (row stride ld elements) into RT.
// TRANS = true loads the plain transpose.
template <typename T, bool TRANS>
__device__ __forceinline__ void rt_load(RT<T>& X, const cpx<T>* __restrict__ M, int ld) {
  const Lane L;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = L.template row<T>(q, r), j = L.col;
      const cpx<T> v = TRANS ? M[(size_t)j * ld + i] : M[(size_t)i * ld + j];
      X.re[q][r] = v.re; X.im[q][r] = v.im;
    }
}

template <typename T, bool TRANS>
__device__ __forceinline__ void rt_store(const RT<T>& X, cpx<T>* __restrict__ M, int ld) {
  const Lane L;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = L.template row<T>(q, r), j = L.col;
      cpx<T> v; v.re = X.re[q][r]; v.im = X.im[q][r];
      if (TRANS) M[(size_t)j * ld + i] = v; else M[(size_t)i * ld + j] = v;
    }
}

// No extra work inside a product (see gemm_acc's hook).
struct NoHook {
  __device__ __forceinline__ void operator()(int) const {}
};

// acc += alpha-free X * Y where X is read from memory (LDS or global) row-major
// with pitch PA, in orientation TA (false: X = A, true: X = A^T), and Y is an RT.
// acc and B must be different register tiles.
// PIPE (single precision): issue the next k-step's A loads ahead of this
// step's MFMAs and pin that order; off where registers are too tight for it.
// hook(st) runs at each of the 16 k-steps st, ahead of that step's MFMAs: a
// share of a global tile load or store placed there drains while the matrix
// cores work, where the whole transfer issued at once would stall the wave.
template <typename T, bool TA, int PA, bool PIPE = true, typename H = NoHook>
__device__ __forceinline__ void gemm_acc(RT<T>& acc, const cpx<T>* __restrict__ A, const RT<T>& B,
                                         const H& hook = H{}) {
  constexpr bool hooked = !std::is_same<H, NoHook>::value;
  const Lane L;
  const int g = L.g, c = L.c;
  if constexpr (sizeof(T) == 4) {
    // 3M: K1 = (Ar + Ai) Br, Cr += K1 - Ai (Br + Bi), Ci += K1 + Ar (Bi - Br).
    // Software-pipelined over the 16 k-steps (kb, t): the next step's four A
    // values are requested before this step's 12 MFMAs, which cover the LDS
    // latency.
    typename vec4<T>::type k1[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) k1[q] = typename vec4<T>::type{0.f, 0.f, 0.f, 0.f};
    auto ld = [&](int st, int q) {
      const int kb = st >> 2, t = st & 3;
      return TA ? A[(16 * kb + Sub<T>::row(g, t)) * PA + 16 * q + c]
                : A[(16 * q + c) * PA + 16 * kb + Sub<T>::row(g, t)];
    };
    if constexpr (!PIPE) {
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) {
        cpx<T> a[4][4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int t = 0; t < 4; ++t) a[q][t] = ld(4 * kb + t, q);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          if constexpr (hooked) {
            __builtin_amdgcn_sched_barrier(0);
            hook(4 * kb + t);
            __builtin_amdgcn_sched_barrier(0);
          }
          const T br = B.re[kb][t], bi = B.im[kb][t];
          const T nsum = -(br + bi), diff = bi - br;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            k1[q] = mfma4<T>(a[q][t].re + a[q][t].im, br, k1[q]);
            acc.re[q] = mfma4<T>(a[q][t].im, nsum, acc.re[q]);
            acc.im[q] = mfma4<T>(a[q][t].re, diff, acc.im[q]);
          }
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) { acc.re[q] += k1[q]; acc.im[q] += k1[q]; }
      return;
    }
    cpx<T> cur[4], nxt[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) cur[q] = ld(0, q);
#pragma unroll
    for (int st = 0; st < 16; ++st) {
      if (st + 1 < 16) {
#pragma unroll
        for (int q = 0; q < 4; ++q) nxt[q] = ld(st + 1, q);
      }
      hook(st);
      // keep the scheduler from sinking these loads next to their use
      __builtin_amdgcn_sched_barrier(0);
      const T br = B.re[st >> 2][st & 3], bi = B.im[st >> 2][st & 3];
      const T nsum = -(br + bi), diff = bi - br;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        k1[q] = mfma4<T>(cur[q].re + cur[q].im, br, k1[q]);
        acc.re[q] = mfma4<T>(cur[q].im, nsum, acc.re[q]);
        acc.im[q] = mfma4<T>(cur[q].re, diff, acc.im[q]);
      }
      __builtin_amdgcn_sched_barrier(0);
      if (st + 1 < 16) {
#pragma unroll
        for (int q = 0; q < 4; ++q) cur[q] = nxt[q];
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) { acc.re[q] += k1[q]; acc.im[q] += k1[q]; }
  } else {
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
      cpx<T> a[4][4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int t = 0; t < 4; ++t)
          a[q][t] = TA ? A[(16 * kb + Sub<T>::row(g, t)) * PA + 16 * q + c]
                       : A[(16 * q + c) * PA + 16 * kb + Sub<T>::row(g, t)];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        hook(4 * kb + t);
        const T br = B.re[kb][t], bi = B.im[kb][t], nbi = -bi;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          acc.re[q] = mfma4<T>(a[q][t].re, br, acc.re[q]);
          acc.im[q] = mfma4<T>(a[q][t].re, bi, acc.im[q]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          acc.re[q] = mfma4<T>(a[q][t].im, nbi, acc.re[q]);
          acc.im[q] = mfma4<T>(a[q][t].im, br, acc.im[q]);
        }
      }
    }
  }
}

// Real tiles in LDS (single precision; the real mode of the slice kernels): a
// row-major 64 x 64 float array with a row pitch of RPITCH_LDS floats, in the
// memory of a complex slot. Rows are 16-byte aligned, and a lane's four k
// values of one 16-wide k block are adjacent: one 16-byte read per (q, kb).
constexpr int RPITCH_LDS = 68;

// S[row][col] = X.re (the imaginary parts are not stored)
template <typename T>
__device__ __forceinline__ void rl_store(const RT<T>& X, T* __restrict__ S) {
  const Lane L;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) S[L.template row<T>(q, r) * RPITCH_LDS + L.col] = X.re[q][r];
}

// X.re = S, X.im = 0
template <typename T>
__device__ __forceinline__ void rl_load(RT<T>& X, const T* __restrict__ S) {
  const Lane L;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      X.re[q][r] = S[L.template row<T>(q, r) * RPITCH_LDS + L.col];
      X.im[q][r] = T(0);
    }
}

// acc.re += A B.re for a real A in LDS (rl_store layout) and a real register
// tile B; acc.im is left as it is. Lane (w, g, c) reads A[16 q + c][16 kb +
// 4 g .. 4 g + 3]: the k values of the kb block's four MFMA steps t (k = 16 kb
// + 4 g + t, the order in which B holds them). hook(st), st = 4 kb + t, runs
// ahead of step st's MFMAs as in gemm_acc. PIPE: the next block's reads are
// issued before the current block's MFMAs.
template <typename T, bool PIPE = true, typename H = NoHook>
__device__ __forceinline__ void gemm_rl(RT<T>& acc, const T* __restrict__ A, const RT<T>& B,
                                        const H& hook = H{}) {
  static_assert(sizeof(T) == 4, "real LDS tiles are single precision");
  typedef float f4rl __attribute__((ext_vector_type(4)));
  constexpr bool hooked = !std::is_same<H, NoHook>::value;
  const Lane L;
  const T* base = A + L.c * RPITCH_LDS + 4 * L.g;
  auto ld = [&](int kb, int q) -> f4rl {
    return *reinterpret_cast<const f4rl*>(base + 16 * q * RPITCH_LDS + 16 * kb);
  };
  f4rl cur[4], nxt[4];
  if constexpr (PIPE) {
#pragma unroll
    for (int q = 0; q < 4; ++q) cur[q] = ld(0, q);
  }
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) {
    if constexpr (PIPE) {
      if (kb + 1 < 4) {
#pragma unroll
        for (int q = 0; q < 4; ++q) nxt[q] = ld(kb + 1, q);
      }
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) cur[q] = ld(kb, q);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if constexpr (hooked) {
        __builtin_amdgcn_sched_barrier(0);
        hook(4 * kb + t);
        __builtin_amdgcn_sched_barrier(0);
      }
      const T br = B.re[kb][t];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc.re[q] = mfma4<T>(cur[q][t], br, acc.re[q]);
    }
    if constexpr (PIPE) {
      if (kb + 1 < 4) {
#pragma unroll
        for (int q = 0; q < 4; ++q) cur[q] = nxt[q];
      }
    }
  }
}

// Column 1-norm max_j sum_i |X_ij| accumulated in FP64. red: 4 doubles of LDS.
template <typename T>
__device__ __forceinline__ double rt_norm1(const RT<T>& X, double* red) {
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
#pragma unroll
  for (int off = 8; off >= 1; off >>= 1) s = fmax(s, __shfl_xor(s, off));
  __syncthreads();
  if (L.l == 0) red[L.w] = s;
  __syncthreads();
  const double m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  return m;
}

// Wave + workgroup sum of one double per thread. red: 4 doubles of LDS.
__device__ __forceinline__ double wg_sum(double s, double* red) {
  const Lane L;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
  __syncthreads();
  if (L.l == 0) red[L.w] = s;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

template <typename T> __device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  cpx<T> o; o.re = a.re * b.re - a.im * b.im; o.im = a.re * b.im + a.im * b.re; return o;
}
template <typename T> __device__ __forceinline__ cpx<T> cinv(cpx<T> a) {
  const T den = a.re * a.re + a.im * a.im;
  cpx<T> o; o.re = a.re / den; o.im = -a.im / den; return o;
}

// In-place Gauss-Jordan inverse without pivoting. Valid for column diagonally
// dominant X (the Pade denominators used here are, by the choice of degree and
// scaling). Step k is the rank-1 update X <- X - u v^T with
//   u_i = X[i][k] (i != k), u_k = X[k][k] - 1,
//   v_j = X[k][j] / X[k][k] (j != k), v_k = 1 + 1 / X[k][k],
// which performs the elimination and stores the inverse's column k in place.
// colbuf: 2 x 64 complex of LDS (double-buffered broadcast of column k).
template <typename T>
__device__ __forceinline__ void rt_gj_inverse(RT<T>& X, cpx<T>* colbuf) {
  const Lane L;
#pragma unroll
  for (int k = 0; k < 64; ++k) {
    cpx<T>* cb = colbuf + (k & 1) * 64;
    const int kq = k >> 4, kg = Sub<T>::grp(k & 15), kr = Sub<T>::reg(k & 15), kc = k & 15;
    if (L.w == kq && L.c == kc) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          cpx<T> v; v.re = X.re[q][r]; v.im = X.im[q][r];
          cb[L.template row<T>(q, r)] = v;
        }
    }
        T xk_r = T(0), xk_i = T(0);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (q == kq && r == kr) { xk_r = X.re[q][r]; xk_i = X.im[q][r]; }
    const T xr = __shfl(xk_r, 16 * kg + L.c);
    const T xi = __shfl(xk_i, 16 * kg + L.c);
    __syncthreads();
    const cpx<T> piv = cb[k];
    const cpx<T> pinv = cinv(piv);
    cpx<T> xk; xk.re = xr; xk.im = xi;
    cpx<T> v = cmul(xk, pinv);
    if (L.col == k) { v.re = T(1) + pinv.re; v.im = pinv.im; }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = L.template row<T>(q, r);
        cpx<T> u = cb[i];
        if (i == k) { u.re = piv.re - T(1); u.im = piv.im; }
        X.re[q][r] -= u.re * v.re - u.im * v.im;
        X.im[q][r] -= u.re * v.im + u.im * v.re;
      }
  }
  __syncthreads();
}

}  // namespace lmag
