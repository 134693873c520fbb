// Set-up, scan, environment, fidelity and chain-rule kernels.
#include "tile.hpp"
#include "internal.hpp"

namespace lmag {

constexpr int TILE = 64 * 64;

// ------------------------------------------------------------ system set-up
// Eq. 8 with column-stacking vec (vec(rho)[i + d j] = rho[i][j]):
//   (I (x) X)[(i,j),(k,l)] = delta_jl X[i][k]
//   (X^T (x) I)[(i,j),(k,l)] = delta_ik X[l][j]
//   (conj(L) (x) L)[(i,j),(k,l)] = conj(L[j][l]) L[i][k]
// Tiles are 64 x 64, zero outside n = d^2.
__global__ void k_lift(const cpx<double>* H, int d, cpx<double>* out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= TILE) return;
  const int a = idx / 64, b = idx % 64, n = d * d;
  cpx<double> o{0.0, 0.0};
  if (a < n && b < n) {
    const int i = a % d, j = a / d, k = b % d, l = b / d;
    double zr = 0.0, zi = 0.0;
    if (j == l) { zr += H[i * d + k].re; zi += H[i * d + k].im; }
    if (i == k) { zr -= H[l * d + j].re; zi -= H[l * d + j].im; }
    o.re = zi;   // -i z
    o.im = -zr;
  }
  out[idx] = o;
}

__global__ void k_dissipator(const cpx<double>* Ls, int n_jump, int d, cpx<double>* out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= TILE) return;
  const int a = idx / 64, b = idx % 64, n = d * d;
  cpx<double> o{0.0, 0.0};
  if (a < n && b < n) {
    const int i = a % d, j = a / d, k = b % d, l = b / d;
    for (int q = 0; q < n_jump; ++q) {
      const cpx<double>* L = Ls + (size_t)q * d * d;
      // conj(L[j][l]) L[i][k]
      const cpx<double> x = L[j * d + l], y = L[i * d + k];
      o.re += x.re * y.re + x.im * y.im;
      o.im += x.re * y.im - x.im * y.re;
      // - 1/2 delta_jl (L^dag L)[i][k] - 1/2 delta_ik (L^dag L)[l][j]
      if (j == l) {
        for (int z = 0; z < d; ++z) {  // sum_z conj(L[z][i]) L[z][k]
          const cpx<double> p = L[z * d + i], r = L[z * d + k];
          o.re -= 0.5 * (p.re * r.re + p.im * r.im);
          o.im -= 0.5 * (p.re * r.im - p.im * r.re);
        }
      }
      if (i == k) {
        for (int z = 0; z < d; ++z) {  // sum_z conj(L[z][l]) L[z][j]
          const cpx<double> p = L[z * d + l], r = L[z * d + j];
          o.re -= 0.5 * (p.re * r.re + p.im * r.im);
          o.im -= 0.5 * (p.re * r.im - p.im * r.re);
        }
      }
    }
  }
  out[idx] = o;
}

// out = X Y - Y X on 64 x 64 double tiles
__global__ void k_commutator(const cpx<double>* X, const cpx<double>* Y, cpx<double>* out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= TILE) return;
  const int a = idx / 64, b = idx % 64;
  double re = 0.0, im = 0.0;
  for (int k = 0; k < 64; ++k) {
    const cpx<double> x = X[a * 64 + k], y = Y[k * 64 + b];
    const cpx<double> u = Y[a * 64 + k], v = X[k * 64 + b];
    re += (x.re * y.re - x.im * y.im) - (u.re * v.re - u.im * v.im);
    im += (x.re * y.im + x.im * y.re) - (u.re * v.im + u.im * v.re);
  }
  out[idx] = cpx<double>{re, im};
}

__global__ void k_cast(const double* in, float* out, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)in[i];
}

__global__ void k_fill_int(int* p, int v, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_lift(const double* H, int d, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_lift, dim3(TILE / 256), dim3(256), 0, s, (const cpx<double>*)H, d,
                     (cpx<double>*)out);
  return hipGetLastError();
}
hipError_t launch_dissipator(const double* Ls, int n_jump, int d, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_dissipator, dim3(TILE / 256), dim3(256), 0, s, (const cpx<double>*)Ls,
                     n_jump, d, (cpx<double>*)out);
  return hipGetLastError();
}
hipError_t launch_commutator(const double* X, const double* Y, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_commutator, dim3(TILE / 256), dim3(256), 0, s, (const cpx<double>*)X,
                     (const cpx<double>*)Y, (cpx<double>*)out);
  return hipGetLastError();
}
hipError_t launch_cast(const double* in, float* out, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cast, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}
hipError_t launch_fill_int(int* p, int v, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_int, dim3((n + 255) / 256), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

// --------------------------------------------------------- Magnus coefficients
// Basis order: L_c (n_ctrl) | Z_i (n_static) | D | [L_c, D] | [L_c, Z_i] (c-major)
// | [L_p, L_q] (p < q). The last three groups exist for order 2 only.
struct BasisIdx {
  int nc, ns;
  __device__ int L(int c) const { return c; }
  __device__ int Z(int i) const { return nc + i; }
  __device__ int D() const { return nc + ns; }
  __device__ int CD(int c) const { return nc + ns + 1 + c; }
  __device__ int CZ(int c, int i) const { return nc + ns + 1 + nc + c * ns + i; }
  __device__ int CC(int k) const { return nc + ns + 1 + nc + nc * ns + k; }
};

#define LMAG_SQ3 1.7320508075688772

template <typename T>
__device__ void node_values(const AlphaArgs& a, int it, int k, int N, double* a1, double* a2) {
  const T* amps = (const T*)a.amps + (size_t)(a.item_amp_offset[it] + k) * a.n_ctrl;
  const T* nxt = (a.hold_foh && k + 1 < N) ? amps + a.n_ctrl : amps;
  const double l1 = 0.5 - LMAG_SQ3 / 6.0, l2 = 0.5 + LMAG_SQ3 / 6.0;
  for (int c = 0; c < a.n_ctrl; ++c) {
    const double u0 = (double)amps[c], u1 = (double)nxt[c];
    const double eps = a.ctrl_scale ? ((const double*)a.ctrl_scale)[(size_t)a.items[it].src * a.n_ctrl + c] : 1.0;
    a1[c] = eps * (u0 + l1 * (u1 - u0));
    a2[c] = eps * (u0 + l2 * (u1 - u0));
  }
}

template <typename T> __global__ void k_alpha(AlphaArgs a) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= a.n_slices_total) return;
  const int it = a.slice_item[n];
  const Item item = a.items[it];
  const int k = n - item.first_slice;
  double a1[16], a2[16];
  node_values<T>(a, it, k, item.n_slices, a1, a2);
  const BasisIdx B{a.n_ctrl, a.n_static};
  double* al = a.alpha + (size_t)n * a.nb;
  const double h = a.dt, kap = LMAG_SQ3 * h * h / 12.0;
  const double* bc = a.static_coef ? (const double*)a.static_coef + (size_t)item.src * a.n_static : nullptr;
  for (int c = 0; c < a.n_ctrl; ++c) al[B.L(c)] = 0.5 * h * (a1[c] + a2[c]);
  for (int i = 0; i < a.n_static; ++i) al[B.Z(i)] = h * (bc ? bc[i] : 0.0);
  al[B.D()] = h;
  if (a.order == 2) {
    for (int c = 0; c < a.n_ctrl; ++c) {
      const double dc = kap * (a2[c] - a1[c]);
      al[B.CD(c)] = dc;
      for (int i = 0; i < a.n_static; ++i) al[B.CZ(c, i)] = dc * (bc ? bc[i] : 0.0);
    }
    int kk = 0;
    for (int p = 0; p < a.n_ctrl; ++p)
      for (int q = p + 1; q < a.n_ctrl; ++q, ++kk)
        al[B.CC(kk)] = kap * (a2[p] * a1[q] - a2[q] * a1[p]);
  }
}

// Sixth-order slices (three Gauss-Legendre nodes c_k = 1/2 - sqrt(15)/10,
// 1/2, 1/2 + sqrt(15)/10): the coefficients, on the order-1 basis
// {L_c, Z_i, D}, of a1 = h B_2, a2 = (sqrt(15) h / 3)(B_3 - B_1) and
// a3 = (10 h / 3)(B_3 - 2 B_2 + B_1), B_k = L(t_n + c_k h). Output planes
// alpha[p][slice][nb], p = 0, 1, 2 for a1, a2, a3.
#define LMAG_SQ15 3.872983346207417
__device__ __forceinline__ void gl3_fracs(double* lam) {
  lam[0] = 0.5 - LMAG_SQ15 / 10.0; lam[1] = 0.5; lam[2] = 0.5 + LMAG_SQ15 / 10.0;
}

template <typename T>
__device__ void node_values3(const AlphaArgs& a, int it, int k, int N, double (*v)[16]) {
  const T* amps = (const T*)a.amps + (size_t)(a.item_amp_offset[it] + k) * a.n_ctrl;
  const T* nxt = (a.hold_foh && k + 1 < N) ? amps + a.n_ctrl : amps;
  double lam[3];
  gl3_fracs(lam);
  for (int c = 0; c < a.n_ctrl; ++c) {
    const double u0 = (double)amps[c], u1 = (double)nxt[c];
    const double eps = a.ctrl_scale ? ((const double*)a.ctrl_scale)[(size_t)a.items[it].src * a.n_ctrl + c] : 1.0;
    for (int q = 0; q < 3; ++q) v[q][c] = eps * (u0 + lam[q] * (u1 - u0));
  }
}

template <typename T> __global__ void k_alpha6(AlphaArgs a) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= a.n_slices_total) return;
  const int it = a.slice_item[n];
  const Item item = a.items[it];
  const int k = n - item.first_slice;
  double v[3][16];
  node_values3<T>(a, it, k, item.n_slices, v);
  const BasisIdx B{a.n_ctrl, a.n_static};
  const size_t plane = (size_t)a.n_slices_total * a.nb;
  double* p1 = a.alpha + (size_t)n * a.nb;
  double* p2 = p1 + plane;
  double* p3 = p2 + plane;
  const double h = a.dt, w2 = LMAG_SQ15 * h / 3.0, w3 = 10.0 * h / 3.0;
  const double* bc = a.static_coef ? (const double*)a.static_coef + (size_t)item.src * a.n_static : nullptr;
  for (int c = 0; c < a.n_ctrl; ++c) {
    p1[B.L(c)] = h * v[1][c];
    p2[B.L(c)] = w2 * (v[2][c] - v[0][c]);
    p3[B.L(c)] = w3 * (v[2][c] - 2.0 * v[1][c] + v[0][c]);
  }
  for (int i = 0; i < a.n_static; ++i) {
    p1[B.Z(i)] = h * (bc ? bc[i] : 0.0);
    p2[B.Z(i)] = 0.0;
    p3[B.Z(i)] = 0.0;
  }
  p1[B.D()] = h;
  p2[B.D()] = 0.0;
  p3[B.D()] = 0.0;
}

hipError_t launch_alpha6(const AlphaArgs& a, hipStream_t s) {
  if (a.n_slices_total <= 0) return hipSuccess;
  const dim3 g((a.n_slices_total + 127) / 128);
  if (a.prec == 32) hipLaunchKernelGGL(k_alpha6<float>, g, dim3(128), 0, s, a);
  else hipLaunchKernelGGL(k_alpha6<double>, g, dim3(128), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_alpha(const AlphaArgs& a, hipStream_t s) {
  if (a.n_slices_total <= 0) return hipSuccess;
  const dim3 g((a.n_slices_total + 127) / 128);
  if (a.prec == 32) hipLaunchKernelGGL(k_alpha<float>, g, dim3(128), 0, s, a);
  else hipLaunchKernelGGL(k_alpha<double>, g, dim3(128), 0, s, a);
  return hipGetLastError();
}

// --------------------------------------------------------------- targets
// S_T^dag[a][b] = conj(S_T[b][a]); S_T[(i + d j), (k + d l)] = conj(U[j][l]) U[i][k]
// => S_T^dag[k + d l][i + d j] = U[j][l] conj(U[i][k]).
__global__ void k_targets(TargetArgs a) {
  const int t = blockIdx.y;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= TILE) return;
  const int r = idx / 64, cidx = idx % 64, d = a.d, n = d * d;
  cpx<double> o{0.0, 0.0};
  if (r < n && cidx < n) {
    const int k = r % d, l = r / d, i = cidx % d, j = cidx / d;
    const cpx<double>* U = (const cpx<double>*)a.U + (size_t)t * d * d;
    const cpx<double> x = U[j * d + l], y = U[i * d + k];
    o.re = x.re * y.re + x.im * y.im;
    o.im = x.im * y.re - x.re * y.im;
  }
  ((cpx<double>*)a.st64)[(size_t)t * TILE + idx] = o;
  if (a.st32) {
    cpx<float> f{(float)o.re, (float)o.im};
    ((cpx<float>*)a.st32)[(size_t)t * TILE + idx] = f;
  }
}

hipError_t launch_targets(const TargetArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_targets, dim3(TILE / 256, a.n_targets), dim3(256), 0, s, a);
  return hipGetLastError();
}

// -------------------------------------------------------------- scan kernels
template <typename T> struct ScanShared {
  cpx<T> slot[64 * PITCH];
  double red[8];
};

template <typename T>
__device__ __forceinline__ void tile_copy(cpx<T>* dst, const cpx<T>* src) {
  for (int i = threadIdx.x; i < TILE; i += WG) dst[i] = src[i];
}

// Chunk totals, prefixes and suffixes are stored as M - I (with short chunks
// they are near the identity, and an FP32 product of two such matrices would
// accumulate small terms onto O(1) diagonal entries). For global tiles X, Y
// in that form, out = (I + X)(I + Y) - I = X + Y + X Y; X is staged through
// LDS, Y is a register tile.
template <typename T>
__device__ void tile_mul_delta(ScanShared<T>& sh, const cpx<T>* X, const cpx<T>* Y, cpx<T>* out) {
  RT<T> Xr, Yr, acc;
  rt_load<T, false>(Xr, X, 64);
  rt_load<T, false>(Yr, Y, 64);
  __syncthreads();
  rt_store<T, false>(Xr, sh.slot, PITCH);
  __syncthreads();
  rt_copy(acc, Yr);
  rt_axpy(acc, T(1), Xr);
  gemm_acc<T, false, PITCH>(acc, sh.slot, Yr);
  rt_store<T, false>(acc, out, 64);
}

// Hillis-Steele step of the inclusive prefix (later chunks on the left) and of
// the inclusive suffix, over the chunk totals of every item.
template <typename T> __global__ void __launch_bounds__(WG) k_scan_level(ScanArgs a, const int32_t* chunk_item) {
  __shared__ ScanShared<T> sh;
  const int gidx = blockIdx.x;
  const bool suffix = gidx >= a.n_chunks_total;
  const int cidx = suffix ? gidx - a.n_chunks_total : gidx;
  const Item it = a.items[chunk_item[cidx]];
  const int lc = cidx - it.first_chunk, Lc = it.n_chunks, st = a.step;
  const cpx<T>* in = (const cpx<T>*)(suffix ? a.suf_in : a.pre_in);
  cpx<T>* out = (cpx<T>*)(suffix ? a.suf_out : a.pre_out);
  if (!out) return;
  const cpx<T>* self = in + (size_t)cidx * TILE;
  cpx<T>* dst = out + (size_t)cidx * TILE;
  if (!suffix) {
    if (lc >= st) tile_mul_delta<T>(sh, self, in + (size_t)(cidx - st) * TILE, dst);
    else tile_copy<T>(dst, self);
  } else {
    if (lc + st < Lc) tile_mul_delta<T>(sh, in + (size_t)(cidx + st) * TILE, self, dst);
    else tile_copy<T>(dst, self);
  }
}


// W_c = Pre_excl(c) S_T^dag Suf_excl(c); F = Re Tr(S_T^dag U) / d^2 with U the
// item's total, accumulated in FP64 (computed by the item's first chunk).
// Prefixes and suffixes arrive as M - I; the identity is added exactly (in the
// FP64 trace, and as the initial value of the products).
template <typename T> __global__ void __launch_bounds__(WG) k_env(EnvArgs a) {
  __shared__ ScanShared<T> sh;
  const int cidx = blockIdx.x;
  const int itn = a.chunk_item[cidx];
  const Item it = a.items[itn];
  const int lc = cidx - it.first_chunk, Lc = it.n_chunks;
  const cpx<T>* pre = (const cpx<T>*)a.pre;
  const cpx<T>* suf = (const cpx<T>*)a.suf;
  const int tix = a.seed_by_item ? itn : it.target;
  const cpx<T>* st = (const cpx<T>*)a.st + (size_t)tix * TILE;
  if (lc == 0 && (a.F || a.Fim)) {
    const cpx<T>* U = pre + (size_t)(it.first_chunk + Lc - 1) * TILE;
    const cpx<double>* S = (const cpx<double>*)a.st64 + (size_t)tix * TILE;
    double re = 0.0, im = 0.0;
    for (int i = threadIdx.x; i < TILE; i += WG) {
      const int r = i / 64, c = i % 64;
      const cpx<double> x = S[r * 64 + c];
      const cpx<T> y = U[c * 64 + r];
      re += x.re * (double)y.re - x.im * (double)y.im;
      im += x.re * (double)y.im + x.im * (double)y.re;
      if (r == c) { re += x.re; im += x.im; }
    }
    re = wg_sum(re, sh.red);
    im = wg_sum(im, sh.red);
    const double inv = 1.0 / ((double)a.d * (double)a.d);
    if (threadIdx.x == 0) {
      const int fi = a.f_by_src ? it.src : itn;
      if (a.F) a.F[fi] = re * inv;
      if (a.Fim) a.Fim[fi] = im * inv;
    }
  }
  if (!a.env) return;
  cpx<T>* out = (cpx<T>*)a.env + (size_t)cidx * TILE;
  // X = S_T^dag Suf_excl
  RT<T> X;
  if (lc + 1 < Lc) {
    RT<T> Y;
    rt_load<T, false>(Y, suf + (size_t)(cidx + 1) * TILE, 64);
    RT<T> Sr;
    rt_load<T, false>(Sr, st, 64);
    __syncthreads();
    rt_store<T, false>(Sr, sh.slot, PITCH);
    __syncthreads();
    rt_copy(X, Sr);   // S_T^dag (I + Y)
    gemm_acc<T, false, PITCH>(X, sh.slot, Y);
  } else {
    rt_load<T, false>(X, st, 64);
  }
  if (lc > 0) {
    RT<T> Pr;
    rt_load<T, false>(Pr, pre + (size_t)(cidx - 1) * TILE, 64);
    __syncthreads();
    rt_store<T, false>(Pr, sh.slot, PITCH);
    __syncthreads();
    RT<T> W;
    rt_copy(W, X);    // (I + Pr) X
    gemm_acc<T, false, PITCH>(W, sh.slot, X);
    rt_store<T, false>(W, out, 64);
  } else {
    rt_store<T, false>(X, out, 64);
  }
}

hipError_t launch_env(const EnvArgs& a, hipStream_t s) {
  if (a.n_chunks_total <= 0) return hipSuccess;
  if (a.prec == 32) hipLaunchKernelGGL(k_env<float>, dim3(a.n_chunks_total), dim3(WG), 0, s, a);
  else hipLaunchKernelGGL(k_env<double>, dim3(a.n_chunks_total), dim3(WG), 0, s, a);
  return hipGetLastError();
}

// Logical-subspace score of one item per workgroup, in FP64 from the item's
// total U = I + X: Y = U P = P + X P (64 x L), Pi = P^dag Y, then
//   kind 1: D = Pi - T, s = Tr(D^dag D), C = 2 D^dag;
//   kind 2: s = Re Tr(T^dag Pi) / L, C = T^dag / L;
// and the seed M = P C P^dag (ds = Re Tr(M dU)) into the item's tile.
template <typename T>
__global__ void __launch_bounds__(WG) k_logical(LogicalArgs a) {
  __shared__ cpx<double> Y[64][MAX_LOGICAL], Q[64][MAX_LOGICAL], Pi[MAX_LOGICAL][MAX_LOGICAL],
      C[MAX_LOGICAL][MAX_LOGICAL];
  const int itn = blockIdx.x, tid = threadIdx.x, L = a.L;
  const Item it = a.items[itn];
  const cpx<T>* X = (const cpx<T>*)a.pre + (size_t)(it.first_chunk + it.n_chunks - 1) * TILE;
  const cpx<double>* P = (const cpx<double>*)a.P;
  const cpx<double>* Tt = (const cpx<double>*)a.T + (size_t)it.target * L * L;
  {
    const int i = tid & 63, k = tid >> 6;
    if (k < L) {
      cpx<double> y = P[i * L + k];
      for (int j = 0; j < 64; ++j) {
        const cpx<T> x = X[i * 64 + j];
        const cpx<double> p = P[j * L + k];
        y.re += (double)x.re * p.re - (double)x.im * p.im;
        y.im += (double)x.re * p.im + (double)x.im * p.re;
      }
      Y[i][k] = y;
    }
  }
  __syncthreads();
  if (tid < L * L) {
    const int r = tid / L, c = tid % L;
    cpx<double> z{0.0, 0.0};
    for (int i = 0; i < 64; ++i) {
      const cpx<double> p = P[i * L + r], y = Y[i][c];
      z.re += p.re * y.re + p.im * y.im;     // conj(p) y
      z.im += p.re * y.im - p.im * y.re;
    }
    Pi[r][c] = z;
  }
  __syncthreads();
  if (tid == 0) {
    double sc = 0.0;
    for (int r = 0; r < L; ++r)
      for (int c = 0; c < L; ++c) {
        const cpx<double> t = Tt[r * L + c], p = Pi[r][c];
        if (a.kind == 1) {
          const double dr = p.re - t.re, di = p.im - t.im;
          sc += dr * dr + di * di;
          C[c][r] = cpx<double>{2.0 * dr, -2.0 * di};          // 2 D^dag
        } else {
          sc += t.re * p.re + t.im * p.im;                     // Re conj(t) p
          C[c][r] = cpx<double>{t.re / L, -t.im / L};          // T^dag / L
        }
      }
    if (a.kind == 2) sc /= L;
    a.score[a.f_by_src ? it.src : itn] = sc;
  }
  __syncthreads();
  {
    const int i = tid & 63, k = tid >> 6;    // Q = P C
    if (k < L) {
      cpx<double> q{0.0, 0.0};
      for (int b = 0; b < L; ++b) {
        const cpx<double> p = P[i * L + b], c = C[b][k];
        q.re += p.re * c.re - p.im * c.im;
        q.im += p.re * c.im + p.im * c.re;
      }
      Q[i][k] = q;
    }
  }
  __syncthreads();
  cpx<double>* M64 = (cpx<double>*)a.st64 + (size_t)itn * TILE;
  cpx<float>* M32 = a.st32 ? (cpx<float>*)a.st32 + (size_t)itn * TILE : nullptr;
  for (int e = tid; e < TILE; e += WG) {
    const int i = e / 64, j = e % 64;
    cpx<double> m{0.0, 0.0};
    for (int b = 0; b < L; ++b) {            // Q[i][b] conj(P[j][b])
      const cpx<double> q = Q[i][b], p = P[j * L + b];
      m.re += q.re * p.re + q.im * p.im;
      m.im += q.im * p.re - q.re * p.im;
    }
    if (a.real) m.im = 0.0;
    M64[e] = m;
    if (M32) M32[e] = cpx<float>{(float)m.re, (float)m.im};
  }
}

hipError_t launch_logical(const LogicalArgs& a, hipStream_t s) {
  if (a.n_items <= 0) return hipSuccess;
  if (a.prec == 32) hipLaunchKernelGGL(k_logical<float>, dim3(a.n_items), dim3(WG), 0, s, a);
  else hipLaunchKernelGGL(k_logical<double>, dim3(a.n_items), dim3(WG), 0, s, a);
  return hipGetLastError();
}

// S_out[item] = top-left n x n block of the item's total product (stored as U - I)
template <typename T> __global__ void k_extract(ExtractArgs a) {
  const int itn = blockIdx.y;
  const Item it = a.items[itn];
  const cpx<T>* U = (const cpx<T>*)a.pre + (size_t)(it.first_chunk + it.n_chunks - 1) * TILE;
  cpx<T>* out = (cpx<T>*)a.out + (size_t)it.src * a.n * a.n;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < a.n * a.n; i += gridDim.x * blockDim.x) {
    const int r = i / a.n, c = i % a.n;
    cpx<T> v = U[r * 64 + c];
    if (r == c) v.re += T(1);
    out[i] = v;
  }
}

hipError_t launch_extract(const ExtractArgs& a, hipStream_t s) {
  if (a.n_items <= 0) return hipSuccess;
  const dim3 g((a.n * a.n + 255) / 256, a.n_items);
  if (a.prec == 32) hipLaunchKernelGGL(k_extract<float>, g, dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_extract<double>, g, dim3(256), 0, s, a);
  return hipGetLastError();
}

// ------------------------------------------------------------- chain rule
// Per slice: dF/da_{c,1}, dF/da_{c,2} from g_j = Re Tr(K B_j) and the alpha
// formulas; then the node interpolation maps them to u_{n,c} and u_{n+1,c}.
template <typename T>
__device__ void slice_dA(const GradArgs& g, const AlphaArgs& aa, int it, int k, int N, int n,
                         double* dA1, double* dA2) {
  double a1[16], a2[16];
  node_values<T>(aa, it, k, N, a1, a2);
  const BasisIdx B{g.n_ctrl, g.n_static};
  const double* G = g.gtrace + (size_t)n * g.nb;
  const double h = g.dt, kap = LMAG_SQ3 * h * h / 12.0;
  const double* bc = g.static_coef ? (const double*)g.static_coef + (size_t)g.items[it].src * g.n_static : nullptr;
  for (int c = 0; c < g.n_ctrl; ++c) {
    const double base = 0.5 * h * G[B.L(c)];
    double comm = 0.0;
    if (g.order == 2) {
      comm = G[B.CD(c)];
      for (int i = 0; i < g.n_static; ++i) comm += (bc ? bc[i] : 0.0) * G[B.CZ(c, i)];
      comm *= kap;
    }
    dA1[c] = base - comm;
    dA2[c] = base + comm;
  }
  if (g.order == 2) {
    int kk = 0;
    for (int p = 0; p < g.n_ctrl; ++p)
      for (int q = p + 1; q < g.n_ctrl; ++q, ++kk) {
        const double Gp = G[B.CC(kk)];
        dA1[p] += -kap * a2[q] * Gp;
        dA1[q] += kap * a2[p] * Gp;
        dA2[p] += kap * a1[q] * Gp;
        dA2[q] += -kap * a1[p] * Gp;
      }
  }
}

// Sixth order: gtrace holds three planes [p][slice][nb] of Re Tr(G_p B_j) for
// the cotangents G_p of a1, a2, a3; dF/d(node value k of control c) is
// sum_p w_pk Re Tr(G_p L_c) with the weights of a1, a2, a3 in B_1, B_2, B_3.
__device__ void slice_dnodes6(const GradArgs& g, int n, size_t plane, double (*dv)[16]) {
  const BasisIdx B{g.n_ctrl, g.n_static};
  const double h = g.dt, w2 = LMAG_SQ15 * h / 3.0, w3 = 10.0 * h / 3.0;
  const double* G1 = g.gtrace + (size_t)n * g.nb;
  const double* G2 = G1 + plane;
  const double* G3 = G2 + plane;
  for (int c = 0; c < g.n_ctrl; ++c) {
    const double t1 = G1[B.L(c)], t2 = G2[B.L(c)], t3 = G3[B.L(c)];
    dv[0][c] = -w2 * t2 + w3 * t3;
    dv[1][c] = h * t1 - 2.0 * w3 * t3;
    dv[2][c] = w2 * t2 + w3 * t3;
  }
}

template <typename T>
__device__ void item_grad6(const GradArgs& g, int it, int k, double* out) {
  const Item item = g.items[it];
  const int N = item.n_slices;
  const size_t plane = (size_t)g.n_slices_total * g.nb;
  double lam[3], dv[3][16];
  gl3_fracs(lam);
  slice_dnodes6(g, item.first_slice + k, plane, dv);
  for (int c = 0; c < g.n_ctrl; ++c) {
    out[c] = 0.0;
    for (int q = 0; q < 3; ++q)
      out[c] += (!g.hold_foh || k + 1 == N) ? dv[q][c] : (1.0 - lam[q]) * dv[q][c];
  }
  if (g.hold_foh && k > 0) {
    slice_dnodes6(g, item.first_slice + k - 1, plane, dv);
    for (int c = 0; c < g.n_ctrl; ++c)
      for (int q = 0; q < 3; ++q) out[c] += lam[q] * dv[q][c];
  }
  for (int c = 0; c < g.n_ctrl; ++c) {
    const double eps = g.ctrl_scale ? ((const double*)g.ctrl_scale)[(size_t)item.src * g.n_ctrl + c] : 1.0;
    out[c] *= eps * g.inv_d2;
  }
}

template <typename T>
__device__ void item_grad(const GradArgs& g, int it, int k, double* out) {
  if (g.order == 6) {
    item_grad6<T>(g, it, k, out);
    return;
  }
  AlphaArgs aa{};
  aa.amps = g.amps; aa.item_amp_offset = g.item_amp_offset; aa.ctrl_scale = g.ctrl_scale;
  aa.items = g.items;
  aa.n_ctrl = g.n_ctrl; aa.hold_foh = g.hold_foh;
  const Item item = g.items[it];
  const int N = item.n_slices;
  const double l1 = 0.5 - LMAG_SQ3 / 6.0, l2 = 0.5 + LMAG_SQ3 / 6.0;
  double dA1[16], dA2[16];
  slice_dA<T>(g, aa, it, k, N, item.first_slice + k, dA1, dA2);
  for (int c = 0; c < g.n_ctrl; ++c) {
    if (!g.hold_foh || k + 1 == N) out[c] = dA1[c] + dA2[c];
    else out[c] = (1.0 - l1) * dA1[c] + (1.0 - l2) * dA2[c];
  }
  if (g.hold_foh && k > 0) {
    slice_dA<T>(g, aa, it, k - 1, N, item.first_slice + k - 1, dA1, dA2);
    for (int c = 0; c < g.n_ctrl; ++c) out[c] += l1 * dA1[c] + l2 * dA2[c];
  }
  for (int c = 0; c < g.n_ctrl; ++c) {
    const double eps = g.ctrl_scale ? ((const double*)g.ctrl_scale)[(size_t)item.src * g.n_ctrl + c] : 1.0;
    out[c] *= eps * g.inv_d2;
  }
}

// One thread per (group or item, slice).
template <typename T> __global__ void k_grad(GradArgs g, int n_units, int max_slices) {
  const int unit = blockIdx.y;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (unit >= n_units) return;
  double acc[16];
  for (int c = 0; c < g.n_ctrl; ++c) acc[c] = 0.0;
  int it0, cnt;
  if (g.group_first_item) {
    const int b = g.group_first_item[unit], e = g.group_first_item[unit + 1];
    it0 = g.group_items[b];
    cnt = e - b;
    if (k == 0 && threadIdx.x == 0 && g.F_out) {
      double f = 0.0;
      for (int i = b; i < e; ++i) f += g.F_items[g.group_items[i]];
      g.F_out[g.group_global ? g.group_global[unit] : unit] = cnt ? f / cnt : 0.0;
    }
    if (!g.grad || !g.gtrace || k >= g.items[it0].n_slices) return;
    for (int i = b; i < e; ++i) {
      double o[16];
      item_grad<T>(g, g.group_items[i], k, o);
      for (int c = 0; c < g.n_ctrl; ++c) acc[c] += o[c];
    }
    for (int c = 0; c < g.n_ctrl; ++c) acc[c] /= (double)cnt;
  } else {
    it0 = unit;
    if (!g.grad || !g.gtrace || k >= g.items[it0].n_slices) return;
    item_grad<T>(g, it0, k, acc);
  }
  T* gout = (T*)g.grad + (size_t)(g.item_amp_offset[it0] + k) * g.n_ctrl;
  for (int c = 0; c < g.n_ctrl; ++c) gout[c] = (T)acc[c];
}

hipError_t launch_grad(const GradArgs& g, int max_slices, hipStream_t s) {
  const int n_units = g.group_first_item ? g.n_groups : g.n_items;
  if (n_units <= 0 || max_slices <= 0) return hipSuccess;
  const dim3 grid((max_slices + 127) / 128, n_units);
  if (g.prec == 32) hipLaunchKernelGGL(k_grad<float>, grid, dim3(128), 0, s, g, n_units, max_slices);
  else hipLaunchKernelGGL(k_grad<double>, grid, dim3(128), 0, s, g, n_units, max_slices);
  return hipGetLastError();
}

hipError_t launch_scan_level(const ScanArgs& a, const int32_t* chunk_item, hipStream_t s) {
  if (a.n_chunks_total <= 0) return hipSuccess;
  const int nblk = a.suf_out ? 2 * a.n_chunks_total : a.n_chunks_total;
  if (a.prec == 32) hipLaunchKernelGGL(k_scan_level<float>, dim3(nblk), dim3(WG), 0, s, a, chunk_item);
  else hipLaunchKernelGGL(k_scan_level<double>, dim3(nblk), dim3(WG), 0, s, a, chunk_item);
  return hipGetLastError();
}


}  // namespace lmag
