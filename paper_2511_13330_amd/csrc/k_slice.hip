// Per-slice kernels of the Lindblad-Magnus path on 64x64 superoperator tiles.
//
// Forward (one workgroup per chunk of consecutive slices, persistent grid):
//   Omega_n = sum_j alpha_{n,j} B_j                (Eq. 8 lift, Eq. 13 + GL2 term)
//   ||Omega_n||_1 in FP64 -> Pade degree m, scaling exponent s
//   S_n = r_m(Omega_n / 2^s)^(2^s), r_m = q_m^{-1} p_m   (Eq. 14)
//   P <- S_n P  (chunk-local ordered product, later slices on the left, Eq. 15)
// Backward (same chunks, slices in reverse order), per slice n:
//   M_n^T = Z_n^T P_loc,n^T,  K_n^T = L(Omega_n^T, M_n^T) (Pade Frechet derivative),
//   g_{n,j} = Re Tr(K_n B_j),  Z_{n-1}^T = S_n^T Z_n^T.
// The backward works with transposed tiles so that every product keeps its
// running factor in registers as the B operand (see tile.hpp).
#include "tile.hpp"
#include "internal.hpp"

namespace lmag {

template <typename T> struct Cfg;
template <> struct Cfg<float> { static constexpr int NLDS = 4; };
template <> struct Cfg<double> { static constexpr int NLDS = 2; };

constexpr int SLOT = 64 * PITCH;
constexpr int TILE = 64 * 64;
constexpr int MAXNB = 32;

// theta_m (Higham 2005): largest ||A||_1 with backward error of r_m below the
// unit roundoff. Single precision uses m = 3 only; double uses m in {3, 5, 7}.
// For these (m, theta) the denominator q_m(A) is column diagonally dominant
// (sum_j>=1 b_j theta^j < 1), so Gauss-Jordan needs no pivoting.
__constant__ double c_theta32_3 = 4.258730016922831e-1;
__constant__ double c_theta64[3] = {1.495585217958292e-2, 2.539398330063230e-1,
                                     9.504178996162932e-1};

template <typename T> struct Shared {
  cpx<T> slots[Cfg<T>::NLDS * SLOT];
  cpx<T> colbuf[128];
  double red[4 * MAXNB];
  int sidx;
};

template <typename T, int K>
__device__ __forceinline__ cpx<T>* slot(Shared<T>& sh, cpx<T>* gs) {
  if constexpr (K < Cfg<T>::NLDS) return sh.slots + K * SLOT;
  else return gs + (K - Cfg<T>::NLDS) * SLOT;
}

template <typename T, bool TRANS>
__device__ __forceinline__ void put(const RT<T>& X, cpx<T>* S) { rt_store<T, TRANS>(X, S, PITCH); }

template <typename T>
__device__ __forceinline__ void mm(RT<T>& acc, const cpx<T>* A, const RT<T>& B) {
  gemm_acc<T, false, PITCH>(acc, A, B);
}

template <typename T>
__device__ __forceinline__ void choose_ms(double nrm, int& m, int& s) {
  s = 0;
  if constexpr (sizeof(T) == 4) {
    m = 3;
    const double th = c_theta32_3;
    if (nrm > th) {
      s = (int)ceil(log2(nrm / th));
      while (s < 62 && ldexp(nrm, -s) > th) ++s;
    }
  } else {
    if (nrm <= c_theta64[0]) m = 3;
    else if (nrm <= c_theta64[1]) m = 5;
    else {
      m = 7;
      const double th = c_theta64[2];
      if (nrm > th) {
        s = (int)ceil(log2(nrm / th));
        while (s < 62 && ldexp(nrm, -s) > th) ++s;
      }
    }
  }
  if (!(nrm == nrm)) { m = 3; s = 0; }  // NaN input: propagate NaN, no scaling loop
  if (s < 0) s = 0;
  if (s > 62) s = 62;
}

template <typename T, bool TRANS>
__device__ __forceinline__ void build_omega(RT<T>& X, const cpx<T>* __restrict__ basis, int nb,
                                            const double* __restrict__ alpha) {
  rt_zero(X);
  for (int j = 0; j < nb; ++j) {
    const double aj = alpha[j];
    if (aj == 0.0) continue;
    RT<T> B;
    rt_load<T, TRANS>(B, basis + (size_t)j * TILE, 64);
    rt_axpy(X, (T)aj, B);
  }
}

template <typename T>
__device__ __forceinline__ const double* pade_b(const PadeTable& pt, int m) {
  return m == 3 ? pt.b3 : (m == 5 ? pt.b5 : pt.b7);
}

template <typename T> __device__ __forceinline__ cpx<T>* tile_at(void* base, size_t idx) {
  return reinterpret_cast<cpx<T>*>(base) + idx * TILE;
}

// One slice forward; returns S_n in R. A_out-side stores go to the workspace
// when ws != null.
template <typename T>
__device__ void fwd_slice(RT<T>& R, Shared<T>& sh, cpx<T>* gs, const SliceArgs& a, int n) {
  const Lane L;
  RT<T> A;
  build_omega<T, false>(A, (const cpx<T>*)a.basis, a.nb, a.alpha + (size_t)n * a.nb);
  const double nrm = rt_norm1(A, sh.red);
  int m, s;
  choose_ms<T>(nrm, m, s);
  if (s) rt_scale(A, (T)ldexp(1.0, -s));
  const double* b = pade_b<T>(a.pade, m);
  const bool st = a.store && a.ws_tiles;
  cpx<T>* ws = st ? tile_at<T>(a.ws_tiles, (size_t)n * WS_TILES) : nullptr;

  __syncthreads();
  put<T, false>(A, slot<T, 0>(sh, gs));
  __syncthreads();
  RT<T> A2;
  rt_zero(A2);
  mm(A2, slot<T, 0>(sh, gs), A);
  if (st) rt_store<T, false>(A2, ws + WS_A2 * TILE, 64);
  RT<T> W, V;
  rt_poly1(W, A2, (T)b[3], (T)b[1]);
  rt_poly1(V, A2, (T)b[2], (T)b[0]);
  if (m >= 5) {
    put<T, false>(A2, slot<T, 1>(sh, gs));
    __syncthreads();
    RT<T> A4;
    rt_zero(A4);
    mm(A4, slot<T, 1>(sh, gs), A2);
    rt_axpy(W, (T)b[5], A4);
    rt_axpy(V, (T)b[4], A4);
    if (m == 7) {
      RT<T> A6;
      rt_zero(A6);
      mm(A6, slot<T, 1>(sh, gs), A4);
      rt_axpy(W, (T)b[7], A6);
      rt_axpy(V, (T)b[6], A6);
    }
  }
  RT<T> U;
  rt_zero(U);
  mm(U, slot<T, 0>(sh, gs), W);
  // P = V + U (in U), Q = V - U (in V)
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const auto vr = V.re[q], vi = V.im[q];
    V.re[q] = vr - U.re[q]; V.im[q] = vi - U.im[q];
    U.re[q] = vr + U.re[q]; U.im[q] = vi + U.im[q];
  }
  rt_gj_inverse(V, sh.colbuf);
  if (st) rt_store<T, false>(V, ws + WS_QINV * TILE, 64);
  put<T, false>(V, slot<T, 1>(sh, gs));
  __syncthreads();
  rt_zero(R);
  mm(R, slot<T, 1>(sh, gs), U);
  if (st) rt_store<T, false>(R, ws + WS_S * TILE, 64);
  for (int k = 0; k < s; ++k) {
    __syncthreads();
    put<T, false>(R, slot<T, 2>(sh, gs));
    __syncthreads();
    RT<T> R2;
    rt_zero(R2);
    mm(R2, slot<T, 2>(sh, gs), R);
    rt_copy(R, R2);
  }
  if (a.ms && L.w == 0 && L.l == 0) {
    a.ms[2 * (size_t)n] = (int8_t)m;
    a.ms[2 * (size_t)n + 1] = (int8_t)s;
  }
}

template <typename T>
__device__ __forceinline__ int grab(Shared<T>& sh, int* counter) {
  __syncthreads();
  if (threadIdx.x == 0) sh.sidx = atomicAdd(counter, 1);
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(sh.sidx);
}

template <typename T>
__global__ void __launch_bounds__(WG, 1) k_forward(SliceArgs a) {
  __shared__ Shared<T> sh;
  cpx<T>* gs = a.gscratch ? reinterpret_cast<cpx<T>*>(a.gscratch) + (size_t)blockIdx.x * 2 * SLOT
                          : nullptr;
  for (;;) {
    const int idx = grab(sh, a.counter);
    if (idx >= a.n_chunks) break;
    const Chunk ch = a.chunks[idx];
    RT<T> P;
    rt_identity(P);
    for (int k = 0; k < ch.count; ++k) {
      const int n = ch.first + k;
      if (a.store && a.ws_tiles)
        rt_store<T, false>(P, tile_at<T>(a.ws_tiles, (size_t)n * WS_TILES + WS_PLOC), 64);
      RT<T> S;
      fwd_slice<T>(S, sh, gs, a, n);
      __syncthreads();
      put<T, false>(S, slot<T, 3>(sh, gs));
      __syncthreads();
      RT<T> Pn;
      rt_zero(Pn);
      mm(Pn, slot<T, 3>(sh, gs), P);
      rt_copy(P, Pn);
    }
    rt_store<T, false>(P, tile_at<T>(a.totals, (size_t)ch.chunk), 64);
  }
}

// One slice backward in the transposed frame. Z holds Z_n^T on entry and
// Z_{n-1}^T on exit.
template <typename T>
__device__ void bwd_slice(RT<T>& Z, Shared<T>& sh, cpx<T>* gs, const SliceArgs& a, int n) {
  const Lane L;
  const cpx<T>* ws = tile_at<T>(a.ws_tiles, (size_t)n * WS_TILES);
  const int m = a.ms[2 * (size_t)n], s = a.ms[2 * (size_t)n + 1];
  const double* b = pade_b<T>(a.pade, m);
  const T sc = (T)ldexp(1.0, -s);

  // E = M_n^T / 2^s,  M_n^T = Z_n^T P_loc,n^T
  __syncthreads();
  put<T, false>(Z, slot<T, 0>(sh, gs));
  __syncthreads();
  RT<T> E;
  {
    RT<T> Pl;
    rt_load<T, true>(Pl, ws + WS_PLOC * TILE, 64);
    rt_zero(E);
    mm(E, slot<T, 0>(sh, gs), Pl);
  }
  if (s) rt_scale(E, sc);
  RT<T> A;
  build_omega<T, true>(A, (const cpx<T>*)a.basis, a.nb, a.alpha + (size_t)n * a.nb);
  if (s) rt_scale(A, sc);
  __syncthreads();
  put<T, false>(A, slot<T, 0>(sh, gs));
  put<T, false>(E, slot<T, 1>(sh, gs));
  __syncthreads();
  RT<T> L2;
  rt_zero(L2);
  mm(L2, slot<T, 0>(sh, gs), E);
  mm(L2, slot<T, 1>(sh, gs), A);
  RT<T> W, LW, LV;
  {
    RT<T> A2;
    rt_load<T, true>(A2, ws + WS_A2 * TILE, 64);
    rt_poly1(W, A2, (T)b[3], (T)b[1]);
    rt_poly1(LW, L2, (T)b[3], T(0));
    rt_poly1(LV, L2, (T)b[2], T(0));
    if (m >= 5) {
      put<T, false>(A2, slot<T, 2>(sh, gs));
      put<T, false>(L2, slot<T, 3>(sh, gs));
      __syncthreads();
      RT<T> A4, L4;
      rt_zero(A4);
      mm(A4, slot<T, 2>(sh, gs), A2);
      rt_zero(L4);
      mm(L4, slot<T, 2>(sh, gs), L2);
      mm(L4, slot<T, 3>(sh, gs), A2);
      rt_axpy(W, (T)b[5], A4);
      rt_axpy(LW, (T)b[5], L4);
      rt_axpy(LV, (T)b[4], L4);
      if (m == 7) {
        RT<T> T6;
        rt_zero(T6);
        mm(T6, slot<T, 3>(sh, gs), A4);   // L2 A4
        mm(T6, slot<T, 2>(sh, gs), L4);   // A2 L4
        rt_axpy(LW, (T)b[7], T6);
        rt_axpy(LV, (T)b[6], T6);
        rt_zero(T6);
        mm(T6, slot<T, 2>(sh, gs), A4);   // A6
        rt_axpy(W, (T)b[7], T6);
      }
    }
  }
  // L_U = A L_W + E W
  RT<T> LU;
  rt_zero(LU);
  mm(LU, slot<T, 0>(sh, gs), LW);
  mm(LU, slot<T, 1>(sh, gs), W);
  // L_Q = L_V - L_U (into LW), L_P = L_V + L_U (into LU)
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const auto vr = LV.re[q], vi = LV.im[q];
    LW.re[q] = vr - LU.re[q]; LW.im[q] = vi - LU.im[q];
    LU.re[q] = vr + LU.re[q]; LU.im[q] = vi + LU.im[q];
  }
  RT<T> R;
  rt_load<T, true>(R, ws + WS_S * TILE, 64);   // r_m(A)^T
  __syncthreads();
  put<T, false>(LW, slot<T, 1>(sh, gs));
  {
    RT<T> Qi;
    rt_load<T, true>(Qi, ws + WS_QINV * TILE, 64);
    put<T, false>(Qi, slot<T, 2>(sh, gs));
  }
  __syncthreads();
  // X = L_P - L_Q R ; L = Q^{-1} X
  {
    RT<T> Tm;
    rt_zero(Tm);
    mm(Tm, slot<T, 1>(sh, gs), R);
#pragma unroll
    for (int q = 0; q < 4; ++q) { LU.re[q] -= Tm.re[q]; LU.im[q] -= Tm.im[q]; }
  }
  RT<T> K;
  rt_zero(K);
  mm(K, slot<T, 2>(sh, gs), LU);
  for (int k = 0; k < s; ++k) {
    __syncthreads();
    put<T, false>(R, slot<T, 0>(sh, gs));
    put<T, false>(K, slot<T, 1>(sh, gs));
    __syncthreads();
    RT<T> Kn, Rn;
    rt_zero(Kn);
    mm(Kn, slot<T, 0>(sh, gs), K);
    mm(Kn, slot<T, 1>(sh, gs), R);
    rt_zero(Rn);
    mm(Rn, slot<T, 0>(sh, gs), R);
    rt_copy(K, Kn);
    rt_copy(R, Rn);
  }
  // traces Re Tr(K B_j) = Re sum K^T o B_j (elementwise, same positions)
  {
    const cpx<T>* basis = (const cpx<T>*)a.basis;
    for (int j = 0; j < a.nb; ++j) {
      RT<T> B;
      rt_load<T, false>(B, basis + (size_t)j * TILE, 64);
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          acc += (double)K.re[q][r] * (double)B.re[q][r] - (double)K.im[q][r] * (double)B.im[q][r];
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
      if (L.l == 0) sh.red[L.w * MAXNB + j] = acc;
    }
    __syncthreads();
    if (threadIdx.x < (unsigned)a.nb) {
      const int j = threadIdx.x;
      a.gtrace[(size_t)n * a.nb + j] =
          (sh.red[j] + sh.red[MAXNB + j]) + (sh.red[2 * MAXNB + j] + sh.red[3 * MAXNB + j]);
    }
  }
  // Z_{n-1}^T = S_n^T Z_n^T
  __syncthreads();
  put<T, false>(R, slot<T, 0>(sh, gs));
  __syncthreads();
  RT<T> Zn;
  rt_zero(Zn);
  mm(Zn, slot<T, 0>(sh, gs), Z);
  rt_copy(Z, Zn);
}

template <typename T>
__global__ void __launch_bounds__(WG, 1) k_backward(SliceArgs a) {
  __shared__ Shared<T> sh;
  cpx<T>* gs = a.gscratch ? reinterpret_cast<cpx<T>*>(a.gscratch) + (size_t)blockIdx.x * 2 * SLOT
                          : nullptr;
  for (;;) {
    const int idx = grab(sh, a.counter);
    if (idx >= a.n_chunks) break;
    const Chunk ch = a.chunks[idx];
    RT<T> Z;
    rt_load<T, true>(Z, tile_at<T>((void*)a.env, (size_t)ch.chunk), 64);
    for (int k = ch.count - 1; k >= 0; --k) bwd_slice<T>(Z, sh, gs, a, ch.first + k);
  }
}

hipError_t launch_slice_forward(int prec, const SliceArgs& a, int grid, hipStream_t s) {
  if (prec == 32) hipLaunchKernelGGL(k_forward<float>, dim3(grid), dim3(WG), 0, s, a);
  else hipLaunchKernelGGL(k_forward<double>, dim3(grid), dim3(WG), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_slice_backward(int prec, const SliceArgs& a, int grid, hipStream_t s) {
  if (prec == 32) hipLaunchKernelGGL(k_backward<float>, dim3(grid), dim3(WG), 0, s, a);
  else hipLaunchKernelGGL(k_backward<double>, dim3(grid), dim3(WG), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------- unit kernels
template <typename T>
__global__ void __launch_bounds__(WG, 1) k_debug_gemm(const cpx<T>* A, const cpx<T>* B, cpx<T>* C,
                                                      int transA) {
  __shared__ Shared<T> sh;
  RT<T> Bt, acc;
  rt_load<T, false>(Bt, B, 64);
  RT<T> At;
  rt_load<T, false>(At, A, 64);
  if (transA) put<T, true>(At, sh.slots); else put<T, false>(At, sh.slots);
  __syncthreads();
  rt_zero(acc);
  mm(acc, (const cpx<T>*)sh.slots, Bt);
  rt_store<T, false>(acc, C, 64);
}

template <typename T>
__global__ void __launch_bounds__(WG, 1) k_debug_inverse(const cpx<T>* A, cpx<T>* C) {
  __shared__ Shared<T> sh;
  RT<T> X;
  rt_load<T, false>(X, A, 64);
  rt_gj_inverse(X, sh.colbuf);
  rt_store<T, false>(X, C, 64);
}

// exp of one 64x64 tile through the forward slice routine (basis = A, alpha = 1)
template <typename T>
__global__ void __launch_bounds__(WG, 1) k_debug_expm(const cpx<T>* A, cpx<T>* C, int8_t* ms,
                                                      const double* one, cpx<T>* gs, PadeTable pt) {
  __shared__ Shared<T> sh;
  SliceArgs a{};
  a.basis = A; a.nb = 1; a.alpha = one; a.ms = ms; a.pade = pt;
  a.store = 0; a.ws_tiles = nullptr;
  RT<T> R;
  fwd_slice<T>(R, sh, gs, a, 0);
  rt_store<T, false>(R, C, 64);
}

hipError_t launch_debug_gemm(int prec, const void* A, const void* B, void* C, int transA, hipStream_t s) {
  if (prec == 32)
    hipLaunchKernelGGL(k_debug_gemm<float>, dim3(1), dim3(WG), 0, s, (const cpx<float>*)A,
                       (const cpx<float>*)B, (cpx<float>*)C, transA);
  else
    hipLaunchKernelGGL(k_debug_gemm<double>, dim3(1), dim3(WG), 0, s, (const cpx<double>*)A,
                       (const cpx<double>*)B, (cpx<double>*)C, transA);
  return hipGetLastError();
}

hipError_t launch_debug_inverse(int prec, const void* A, void* C, hipStream_t s) {
  if (prec == 32)
    hipLaunchKernelGGL(k_debug_inverse<float>, dim3(1), dim3(WG), 0, s, (const cpx<float>*)A,
                       (cpx<float>*)C);
  else
    hipLaunchKernelGGL(k_debug_inverse<double>, dim3(1), dim3(WG), 0, s, (const cpx<double>*)A,
                       (cpx<double>*)C);
  return hipGetLastError();
}

__device__ double g_one_alpha[1] = {1.0};

hipError_t launch_debug_expm(int prec, const void* A, void* C, int8_t* ms, void* gscratch, PadeTable pt, hipStream_t s) {
  double* one = nullptr;
  hipError_t e = hipGetSymbolAddress((void**)&one, HIP_SYMBOL(g_one_alpha));
  if (e != hipSuccess) return e;
  if (prec == 32)
    hipLaunchKernelGGL(k_debug_expm<float>, dim3(1), dim3(WG), 0, s, (const cpx<float>*)A,
                       (cpx<float>*)C, ms, (const double*)one, (cpx<float>*)gscratch, pt);
  else
    hipLaunchKernelGGL(k_debug_expm<double>, dim3(1), dim3(WG), 0, s, (const cpx<double>*)A,
                       (cpx<double>*)C, ms, (const double*)one, (cpx<double>*)gscratch, pt);
  return hipGetLastError();
}

}  // namespace lmag
