// Per-slice kernels of the Lindblad-Magnus path on 64x64 superoperator tiles.
//
// Exponents (one workgroup per block of slices, bandwidth-parallel):
//   Omega_n = sum_j alpha_{n,j} B_j                (Eq. 8 lift, Eq. 13 + GL2 term)
//   ||Omega_n||_1 in FP64 -> Pade degree m, scaling exponent s; A_n = Omega_n / 2^s
// Forward (one workgroup per chunk of consecutive slices, persistent grid):
//   S_n = r_m(A_n)^(2^s), r_m = q_m^{-1} p_m         (Eq. 14)
//   P <- S_n P  (chunk-local ordered product, later slices on the left, Eq. 15)
// Backward (same chunks, slices in reverse order), per slice n:
//   M_n^T = Z_n^T P_loc,n^T,  K_n^T = L(Omega_n^T, M_n^T) (Pade Frechet derivative),
//   Z_{n-1}^T = S_n^T Z_n^T;  K_n^T replaces A_n in memory.
// Traces (bandwidth-parallel): g_{n,j} = Re Tr(K_n B_j).
// The backward works with transposed tiles so that every product keeps its
// running factor in registers as the B operand (see tile.hpp).
#include "tile.hpp"
#include "internal.hpp"
#include "pade.hpp"

namespace lmag {

template <typename T> struct Cfg;
template <> struct Cfg<float> { static constexpr int NLDS = 4; };
template <> struct Cfg<double> { static constexpr int NLDS = 2; };

constexpr int SLOT = 64 * PITCH;
constexpr int TILE = 64 * 64;
constexpr int MAXNB = 32;
constexpr int NPHASE = 16;

template <typename T> struct Shared {
  alignas(16) cpx<T> slots[Cfg<T>::NLDS * SLOT];   // 16-byte reads of real tiles
  cpx<T> colbuf[128];
  double red[4 * MAXNB];
  long long clk[NPHASE];
  int sidx;
};

template <typename T, int K>
__device__ __forceinline__ cpx<T>* slot(Shared<T>& sh, cpx<T>* gs) {
  if constexpr (K < Cfg<T>::NLDS) return sh.slots + K * SLOT;
  else return gs + (K - Cfg<T>::NLDS) * SLOT;
}

// RE (real mode, single precision): slots hold real tiles in the rl_store
// layout, and the products read them with 16-byte loads along k.
template <typename T, bool TRANS, bool RE = false>
__device__ __forceinline__ void put(const RT<T>& X, cpx<T>* S) {
  if constexpr (RE) rl_store<T>(X, reinterpret_cast<T*>(S));
  else rt_store<T, TRANS>(X, S, PITCH);
}

// a slot back into a register tile
template <typename T, bool RE>
__device__ __forceinline__ void get(RT<T>& X, const cpx<T>* S) {
  if constexpr (RE) rl_load<T>(X, reinterpret_cast<const T*>(S));
  else rt_load<T, false>(X, S, PITCH);
}

template <typename T, bool PIPE = true, bool RE = false>
__device__ __forceinline__ void mm(RT<T>& acc, const cpx<T>* A, const RT<T>& B) {
  if constexpr (RE) gemm_rl<T, PIPE>(acc, reinterpret_cast<const T*>(A), B);
  else gemm_acc<T, false, PITCH, PIPE>(acc, A, B);
}

// mm with a hook that moves a share of a global tile at each k-step
template <typename T, bool PIPE = true, bool RE = false, typename H>
__device__ __forceinline__ void mm(RT<T>& acc, const cpx<T>* A, const RT<T>& B, const H& hook) {
  if constexpr (RE) gemm_rl<T, PIPE, H>(acc, reinterpret_cast<const T*>(A), B, hook);
  else gemm_acc<T, false, PITCH, PIPE, H>(acc, A, B, hook);
}

// Element (row(q, r), col) of this thread in a row-major 64 x 64 tile at M
// (TRANS: in its transpose). Rows split into a uniform part (16 q + the row of
// register r) and a lane part (the row of lane group g); the address is the
// uniform part folded into the base plus one 32-bit lane offset shared by all
// sixteen registers, which keeps the hooks below to a register or two.
template <typename T, bool TRANS, typename E>
__device__ __forceinline__ E* tile_elem(E* M, int q, int r, const Lane& L) {
  const int ru = 16 * q + Sub<T>::row(0, r), rl = Sub<T>::row(L.g, 0);
  E* base = M + (TRANS ? ru : ru * 64);
  return base + (uint32_t)(TRANS ? L.col * 64 + rl : rl * 64 + L.col);
}

// Product hooks: a transfer between a register tile and a row-major 64 x 64
// global tile, spread over k-steps. A load runs at steps S0 .. S0 + 7, two
// registers (q, r), (q, r + 1) per step (for a transposed single-precision
// load these rows are adjacent in memory: one 16-byte access), so that the
// tile has arrived well before the product that follows needs it. A store
// moves register (q, r) = (st / 4, st % 4) at step st.
// RE: the global tile is real, stored as a row-major 64 x 64 array of T in
// the first half of its slot (half the bytes of the complex tile); a load sets
// the imaginary parts to zero.
template <typename T, bool TRANS, int S0 = 0, bool RE = false>
struct TileLoad {
  RT<T>& X;
  const cpx<T>* M;
  __device__ __forceinline__ void operator()(int st) const {
    if (st < S0 || st >= S0 + 8) return;
    const Lane L;
    const int e = 2 * (st - S0), q = e >> 2, r = e & 3;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      if constexpr (RE) {
        X.re[q][r + u] = *tile_elem<T, TRANS>(reinterpret_cast<const T*>(M), q, r + u, L);
        X.im[q][r + u] = T(0);
      } else {
        const cpx<T> v = *tile_elem<T, TRANS>(M, q, r + u, L);
        X.re[q][r + u] = v.re; X.im[q][r + u] = v.im;
      }
    }
  }
};

template <typename T, bool RE = false>
struct TileStore {
  const RT<T>& X;
  cpx<T>* M;
  __device__ __forceinline__ void operator()(int st) const {
    const Lane L;
    const int q = st >> 2, r = st & 3;
    if constexpr (RE) {
      *tile_elem<T, false>(reinterpret_cast<T*>(M), q, r, L) = X.re[q][r];
    } else {
      cpx<T> v; v.re = X.re[q][r]; v.im = X.im[q][r];
      *tile_elem<T, false>(M, q, r, L) = v;
    }
  }
};

// Whole-tile transfers between a register tile and a global tile (pitch 64),
// complex or, with RE, real as in TileLoad.
template <typename T, bool TRANS, bool RE>
__device__ __forceinline__ void gl_load(RT<T>& X, const cpx<T>* M) {
  if constexpr (RE) {
    const T* R = reinterpret_cast<const T*>(M);
    const Lane L;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        X.re[q][r] = *tile_elem<T, TRANS>(R, q, r, L);
        X.im[q][r] = T(0);
      }
  } else {
    rt_load<T, TRANS>(X, M, 64);
  }
}

template <typename T, bool RE>
__device__ __forceinline__ void gl_store(const RT<T>& X, cpx<T>* M) {
  if constexpr (RE) {
    T* R = reinterpret_cast<T*>(M);
    const Lane L;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) *tile_elem<T, false>(R, q, r, L) = X.re[q][r];
  } else {
    rt_store<T, false>(X, M, 64);
  }
}

// Compact store of the support entries of a tile (sparse basis): kpack holds
// this thread's 16-bit mask of support registers and, above it, the slot of its
// first entry; entries go to consecutive slots in register order.
template <typename T>
struct SupportStore {
  const RT<T>& X;
  cpx<T>* M;
  uint32_t kpack;
  __device__ __forceinline__ void operator()(int st) const {
    if ((kpack >> st) & 1u) {
      const int q = st >> 2, r = st & 3;
      cpx<T> v; v.re = X.re[q][r]; v.im = X.im[q][r];
      M[(kpack >> 16) + __builtin_popcount(kpack & ((1u << st) - 1u))] = v;
    }
  }
};

template <typename H1, typename H2, typename H3>
struct Hooks3 {
  H1 h1; H2 h2; H3 h3;
  __device__ __forceinline__ void operator()(int st) const { h1(st); h2(st); h3(st); }
};

template <typename T>
__device__ __forceinline__ const double* pade_b(const PadeTable& pt, int m) {
  return m == 2 ? pt.b2 : (m == 3 ? pt.b3 : (m == 5 ? pt.b5 : pt.b7));
}

template <typename T> __device__ __forceinline__ cpx<T>* tile_at(void* base, size_t idx) {
  return reinterpret_cast<cpx<T>*>(base) + idx * TILE;
}

// Per-phase cycle counters of workgroup 0 (instrumentation; off when clk is null).
// Thread 0 accumulates into LDS so that only the last timestamp lives in registers.
struct Clock {
  long long t = 0;
  long long* acc;
  bool on;
  __device__ __forceinline__ Clock(const long long* clk, long long* lds) : acc(lds),
      on(clk && blockIdx.x == 0 && threadIdx.x == 0) {
    if (on) {
      for (int i = 0; i < NPHASE; ++i) acc[i] = 0;
      t = clock64();
    }
  }
  __device__ __forceinline__ void mark(int p) {
    if (on) { const long long now = clock64(); acc[p] += now - t; t = now; }
  }
  __device__ __forceinline__ void flush(long long* clk) {
    if (on)
      for (int i = 0; i < NPHASE; ++i) clk[i] += acc[i];
  }
};

// Omega_n / 2^s for a block of slices; FP64 column 1-norm selects (m, s).
// Thread t owns column t % 64 and rows 16 (t / 64) .. +15 of every slice.
constexpr int OMEGA_SLICES = 4;

template <typename T>
__global__ void __launch_bounds__(WG) k_omega(SliceArgs a, int n_total) {
  __shared__ double colpart[4][64];
  __shared__ int ms_sh[2];
  const int tid = threadIdx.x, col = tid & 63, rb = (tid >> 6) * 16;
  const int n0 = blockIdx.x * OMEGA_SLICES;
  const cpx<T>* basis = (const cpx<T>*)a.basis;
  cpx<T> acc[OMEGA_SLICES][16];
#pragma unroll
  for (int s = 0; s < OMEGA_SLICES; ++s)
#pragma unroll
    for (int e = 0; e < 16; ++e) { acc[s][e].re = T(0); acc[s][e].im = T(0); }
  for (int j = 0; j < a.nb; ++j) {
    cpx<T> bj[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) bj[e] = basis[(size_t)j * TILE + (rb + e) * 64 + col];
#pragma unroll
    for (int s = 0; s < OMEGA_SLICES; ++s) {
      const int n = n0 + s;
      const T al = n < n_total ? (T)a.alpha[(size_t)n * a.nb + j] : T(0);
#pragma unroll
      for (int e = 0; e < 16; ++e) { acc[s][e].re += al * bj[e].re; acc[s][e].im += al * bj[e].im; }
    }
  }
#pragma unroll
  for (int s = 0; s < OMEGA_SLICES; ++s) {
    const int n = n0 + s;
    if (n >= n_total) break;   // uniform
    double cs = 0.0;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const double x = (double)acc[s][e].re, y = (double)acc[s][e].im;
      cs += sqrt(x * x + y * y);
    }
    __syncthreads();
    colpart[tid >> 6][col] = cs;
    __syncthreads();
    if (tid < 64) {
      double v = (colpart[0][tid] + colpart[1][tid]) + (colpart[2][tid] + colpart[3][tid]);
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off));
      if (tid == 0) {
        int m, sc;
        choose_ms<T>(v, m, sc);
        ms_sh[0] = m; ms_sh[1] = sc;
        a.ms[2 * (size_t)n] = (int8_t)m;
        a.ms[2 * (size_t)n + 1] = (int8_t)sc;
        if (a.nlev)
          a.nlev[n] = (int8_t)inverse_code<T>(ldexp(v, -sc), pade_b<T>(a.pade, m), m, a.inv_mode != 2,
                                              a.pade.ser_max32_2, a.pade.ser_max32_3);
      }
    }
    __syncthreads();
    const T f = (T)ldexp(1.0, -ms_sh[1]);
    cpx<T>* out = tile_at<T>(a.omega, (size_t)n);
    if (a.real) {   // the real tile of the slice kernels' real mode
      T* ro = reinterpret_cast<T*>(out);
#pragma unroll
      for (int e = 0; e < 16; ++e) ro[(rb + e) * 64 + col] = acc[s][e].re * f;
    } else {
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        cpx<T> v; v.re = acc[s][e].re * f; v.im = acc[s][e].im * f;
        out[(rb + e) * 64 + col] = v;
      }
    }
  }
}

// Omega_n / 2^s from the sparse basis: one wave per slice, lane c owns column c.
// Each support entry is summed over its basis terms in ascending j (the order of
// the dense kernel, whose other terms are exact zeros) into registers; the FP64
// column 1-norm selects (m, s). The tile goes out in blocks of OM_RB rows: the
// lane writes its column of the block into LDS (zeros, then its support values
// at their rows: LDS stands in for a register array indexed by row), reads it
// back and stores row-coalesced, so every line of the tile is written once.
template <typename T> struct OmRows { static constexpr int RB = sizeof(T) == 4 ? 8 : 4; };

template <typename T>
__global__ void __launch_bounds__(WG) k_omega_sparse(SliceArgs a, int n_total) {
  constexpr int RB = OmRows<T>::RB;
  __shared__ T al_sh[4][MAXNB];
  __shared__ cpx<T> blk[4][RB][64];   // per wave; each lane uses only its own column
  const int w = threadIdx.x >> 6, c = threadIdx.x & 63;
  const int n = blockIdx.x * 4 + w;
  const bool valid = n < n_total;
  if (valid && c < a.nb) al_sh[w][c] = (T)a.alpha[(size_t)n * a.nb + c];
  __syncthreads();
  if (!valid) return;   // wave-uniform; no barrier follows
  const SparseBasis& sp = a.sp;
  const cpx<T>* val = (const cpx<T>*)sp.pe_val;
  const T* al = al_sh[w];
  const int p0 = sp.col_ptr[c], cnt = sp.col_ptr[c + 1] - p0;
  cpx<T> v[SP_COLCAP];
  int row[SP_COLCAP];
  double cs = 0.0;
#pragma unroll
  for (int q = 0; q < SP_COLCAP; ++q) {
    v[q].re = T(0);
    v[q].im = T(0);
    row[q] = 0;
    if (q < cnt) {
      row[q] = sp.sup_row[p0 + q];
      for (int i = sp.sup_eptr[p0 + q]; i < sp.sup_eptr[p0 + q + 1]; ++i) {
        const T aj = al[sp.pe_j[i]];
        const cpx<T> b = val[i];
        v[q].re += aj * b.re;
        v[q].im += aj * b.im;
      }
      const double x = (double)v[q].re, y = (double)v[q].im;
      cs += sqrt(x * x + y * y);
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) cs = fmax(cs, __shfl_xor(cs, off));
  int m = 3, sc = 0;
  choose_ms<T>(cs, m, sc);
  if (c == 0) {
    a.ms[2 * (size_t)n] = (int8_t)m;
    a.ms[2 * (size_t)n + 1] = (int8_t)sc;
    if (a.nlev)
      a.nlev[n] = (int8_t)inverse_code<T>(ldexp(cs, -sc), pade_b<T>(a.pade, m), m, a.inv_mode != 2,
                                          a.pade.ser_max32_2, a.pade.ser_max32_3);
  }
  const T f = (T)ldexp(1.0, -sc);
  cpx<T>* out = tile_at<T>(a.omega, (size_t)n);
  cpx<T>(*col)[64] = blk[w];
  const cpx<T> zero{T(0), T(0)};
  for (int b = 0; b < 64 / RB; ++b) {
#pragma unroll
    for (int r = 0; r < RB; ++r) col[r][c] = zero;
#pragma unroll
    for (int q = 0; q < SP_COLCAP; ++q)
      if (q < cnt && row[q] / RB == b) {
        cpx<T> x;
        x.re = v[q].re * f;
        x.im = v[q].im * f;
        col[row[q] % RB][c] = x;
      }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      // streaming stores: the tiles (32 KiB per slice) far exceed the caches
      // before the slice kernels read them (measured 1.56 -> 1.46 ms per launch)
      const cpx<T> x = col[r][c];
      if (a.real) {   // the real tile of the slice kernels' real mode
        __builtin_nontemporal_store(x.re, reinterpret_cast<T*>(out) + (b * RB + r) * 64 + c);
      } else {
        cpx<T>* dst = out + (b * RB + r) * 64 + c;
        __builtin_nontemporal_store(x.re, &dst->re);
        __builtin_nontemporal_store(x.im, &dst->im);
      }
    }
  }
}

// Traces from the compact K_n^T (its support positions, stored at the start of
// the slice's exponent tile by the backward): one wave per slice; for each basis
// element the lanes take its entries in a fixed order and the wave sums them
// in FP64.
template <typename T>
__global__ void __launch_bounds__(WG) k_traces_sparse(SliceArgs a, int n_total) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int n = blockIdx.x * 4 + w;
  if (n >= n_total) return;
  const SparseBasis& sp = a.sp;
  const cpx<T>* kc = tile_at<T>(a.omega, (size_t)n);
  const cpx<T>* val = (const cpx<T>*)sp.ent_val;
  for (int j = 0; j < a.nb; ++j) {
    double t = 0.0;
    for (int i = sp.ptr_j[j] + l; i < sp.ptr_j[j + 1]; i += 64) {
      const cpx<T> k = kc[sp.ent_slot[i]];
      const cpx<T> b = val[i];
      t += (double)(k.re * b.re - k.im * b.im);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) t += __shfl_xor(t, off);
    if (l == 0) a.gtrace[(size_t)n * a.nb + j] = t;
  }
}

// The same traces with the slice-invariant entry table and each slice's compact
// K_n^T staged in LDS (dynamic shared memory, laid out by tr_lds_bytes). Lanes
// are grouped by basis element, LPJ lanes each; lane sub of the group of j
// sums the entries ptr_j[j] + sub + LPJ k in ascending k, in FP64, and the
// group is reduced by shuffles in a fixed order, so the result is bitwise
// deterministic. One wave per slice, TR_SPB slices per workgroup.
constexpr int TR_SPB = 32;
constexpr size_t TR_LDS_MAX = 64 * 1024;

template <typename T>
__host__ __device__ inline size_t tr_lds_bytes(int nnz, int n_sup, int nb) {
  return (size_t)nnz * sizeof(cpx<T>) + (size_t)4 * n_sup * sizeof(cpx<T>) +
         (size_t)((nnz + 1) & ~1) * 2 + (size_t)(nb + 1) * 4;
}

template <typename T, int LPJ>
__global__ void __launch_bounds__(WG) k_traces_lds(SliceArgs a, int n_total) {
  extern __shared__ __align__(16) char tr_smem[];
  const SparseBasis& sp = a.sp;
  const int nnz = sp.nnz, nsup = sp.n_sup, nb = a.nb;
  cpx<T>* tval = reinterpret_cast<cpx<T>*>(tr_smem);          // [nnz]
  cpx<T>* kbuf = tval + nnz;                                   // [4][n_sup]
  uint16_t* tslot = reinterpret_cast<uint16_t*>(kbuf + 4 * nsup);   // [nnz]
  int* tptr = reinterpret_cast<int*>(tslot + ((nnz + 1) & ~1));     // [nb + 1]
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const cpx<T>* ev = (const cpx<T>*)sp.ent_val;
  for (int i = tid; i < nnz; i += WG) { tval[i] = ev[i]; tslot[i] = sp.ent_slot[i]; }
  for (int i = tid; i <= nb; i += WG) tptr[i] = sp.ptr_j[i];
  __syncthreads();
  const int j = l / LPJ, sub = l % LPJ;
  cpx<T>* kw = kbuf + w * nsup;
  for (int r = 0; r < TR_SPB / 4; ++r) {
    const int n = blockIdx.x * TR_SPB + 4 * r + w;   // wave-uniform
    const bool valid = n < n_total;
    if (valid) {
      const cpx<T>* kc = tile_at<T>(a.omega, (size_t)n);
      for (int i = l; i < nsup; i += 64) kw[i] = kc[i];
    }
    __syncthreads();   // every wave runs the same rounds
    if (valid && j < nb) {
      double t = 0.0;
      for (int i = tptr[j] + sub; i < tptr[j + 1]; i += LPJ) {
        const cpx<T> k = kw[tslot[i]], b = tval[i];
        t += (double)(k.re * b.re - k.im * b.im);
      }
#pragma unroll
      for (int off = 1; off < LPJ; off <<= 1) t += __shfl_xor(t, off);   // within the group
      if (sub == 0) a.gtrace[(size_t)n * nb + j] = t;
    }
    __syncthreads();   // kw is overwritten next round
  }
}

// g_{n,j} = Re sum_x K^T_n[x] B_j[x] over flat positions x (K^T stored where A_n was).
// Each thread sums its 16 positions in FP32; lanes and waves are combined in FP64.
constexpr int TRACE_SLICES = 4;

template <typename T>
__global__ void __launch_bounds__(WG) k_traces(SliceArgs a, int n_total) {
  __shared__ double red[4][TRACE_SLICES][MAXNB];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int n0 = blockIdx.x * TRACE_SLICES;
  const cpx<T>* basis = (const cpx<T>*)a.basis;
  cpx<T> k[TRACE_SLICES][16];
#pragma unroll
  for (int s = 0; s < TRACE_SLICES; ++s) {
    const int n = n0 + s < n_total ? n0 + s : n_total - 1;
    const cpx<T>* Kt = tile_at<T>(a.omega, (size_t)n);
#pragma unroll
    for (int e = 0; e < 16; ++e) k[s][e] = Kt[tid * 16 + e];
  }
  for (int j = 0; j < a.nb; ++j) {
    cpx<T> bj[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) bj[e] = basis[(size_t)j * TILE + tid * 16 + e];
    double acc[TRACE_SLICES];
#pragma unroll
    for (int s = 0; s < TRACE_SLICES; ++s) {
      T t = T(0);
#pragma unroll
      for (int e = 0; e < 16; ++e) t += k[s][e].re * bj[e].re - k[s][e].im * bj[e].im;
      acc[s] = (double)t;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
      for (int s = 0; s < TRACE_SLICES; ++s) acc[s] += __shfl_xor(acc[s], off);
    if (lane == 0)
#pragma unroll
      for (int s = 0; s < TRACE_SLICES; ++s) red[w][s][j] = acc[s];
  }
  __syncthreads();
  for (int i = tid; i < TRACE_SLICES * a.nb; i += WG) {
    const int s = i / a.nb, j = i % a.nb, n = n0 + s;
    if (n < n_total)
      a.gtrace[(size_t)n * a.nb + j] = (red[0][s][j] + red[1][s][j]) + (red[2][s][j] + red[3][s][j]);
  }
}

// Per-slice codes read inside the slice loops (Pade degree, scaling exponent,
// inverse variant) go through the scalar unit: a load from the constant address
// space. Vector memory operations complete in order, so a vector load here would
// also wait for every tile prefetch and workspace store still in flight. The
// codes are written by an earlier kernel and only read here. The aligned word
// holding the byte never leaves the allocation's page.
__device__ __forceinline__ uint32_t code_word(const int8_t* p) {
  const uintptr_t at = (uintptr_t)p;
  return *(const __attribute__((address_space(4))) uint32_t*)(at & ~(uintptr_t)3) >> ((at & 3) * 8);
}

struct SliceMS { int m, s; };
__device__ __forceinline__ SliceMS slice_ms(const SliceArgs& a, int n) {
  const uint32_t w = code_word(a.ms + 2 * (size_t)n);   // even offset: both bytes in one word
  return {(int)(int8_t)(w & 0xff), (int)(int8_t)((w >> 8) & 0xff)};
}

__device__ __forceinline__ int slice_inverse_code(const SliceArgs& a, int n) {
  return a.nlev ? (int)(int8_t)(code_word(a.nlev + n) & 0xff) : 0;
}

// The codes of one slice, packed in a word: m | s << 8 | inverse code << 16.
struct SliceCode {
  int m, s, K;
};
__device__ __forceinline__ SliceCode unpack_code(uint32_t w) {
  return {(int)(int8_t)(w & 0xff), (int)(int8_t)((w >> 8) & 0xff), (int)(int8_t)((w >> 16) & 0xff)};
}
__device__ __forceinline__ uint32_t slice_code(const SliceArgs& a, int n) {
  const SliceMS ms = slice_ms(a, n);
  return (uint32_t)(ms.m & 0xff) | (uint32_t)(ms.s & 0xff) << 8 |
         (uint32_t)(slice_inverse_code(a, n) & 0xff) << 16;
}

// The codes of up to 64 consecutive slices of a chunk, one slice per lane of
// every wave, fetched by one vector load per 64 slices; a slice takes its code
// with v_readlane (a scalar, for the branches). A scalar load per slice left
// its latency exposed at every slice start, where the code decides the path.
constexpr int CODE_WINDOW = 64;
struct CodeWindow {
  uint32_t v = 0;
  __device__ __forceinline__ void load(const SliceArgs& a, int n0, int cnt) {
    const int l = threadIdx.x & 63;
    v = 0;
    if (l < cnt) {
      const size_t n = (size_t)n0 + l;
      v = (uint32_t)(uint8_t)a.ms[2 * n] | (uint32_t)(uint8_t)a.ms[2 * n + 1] << 8 |
          (a.nlev ? (uint32_t)(uint8_t)a.nlev[n] << 16 : 0u);
    }
  }
  __device__ __forceinline__ uint32_t at(int i) const {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, i);
  }
};

// One slice forward; returns D_n = S_n - I in R. Every matrix near the identity
// is carried as I + X with only X inside the MFMA accumulators: accumulating
// small products onto O(1) diagonal entries in FP32 biases them by a fraction of
// an ulp, and over a chain of thousands of slices that bias adds up linearly.
// With ST, stores go to workspace ws: P_loc (Pl, the chunk product before this
// slice), A^2 (m > 2), Q^{-1} - I and r_m(A) - I (before the squarings). In
// single precision P_loc, A^2 and Q^{-1} - I are stored spread over the k-steps
// of a product that follows the tile's last change (see gemm_acc). r_m(A) - I
// is stored at once: deferring it into the chain product kept it live there and
// made that product spill.
// A holds Omega_n / 2^s (loaded by the caller, which prefetches it during the
// previous slice's chain product).
template <typename T, bool ST, bool RE = false>
__device__ void fwd_slice(RT<T>& R, const RT<T>& A, const RT<T>& Pl, Shared<T>& sh, cpx<T>* gs,
                          const SliceArgs& a, uint32_t code, cpx<T>* ws, Clock& ck) {
  constexpr bool hk = sizeof(T) == 4;   // stores inside products
  const SliceCode sc = unpack_code(code);
  const int m = sc.m, s = sc.s;
  const double* b = pade_b<T>(a.pade, m);   // b[0] = 1
  ck.mark(0);
  constexpr bool st = ST;   // compile-time, so that the stores are straight-line code

  // Slot use: 0 holds A, 1 A^2 then X_Q, 2 Neumann and squaring operands, 3 the
  // chain's D (written by the caller). A write to a slot needs a barrier after
  // its last read only where no barrier has passed since: the previous slice's
  // last reads of slots 0 and 1 (and of 3, by the chain) are all at least one
  // barrier back when this slice first writes them.
  put<T, false, RE>(A, slot<T, 0>(sh, gs));
  __syncthreads();
  RT<T> A2;
  rt_zero(A2);
  // unpipelined: measured faster, and it leaves the kernel without spills
  if constexpr (st && hk) {
    mm<T, false, RE>(A2, slot<T, 0>(sh, gs), A, TileStore<T, RE>{Pl, ws + WS_PLOC * TILE});
  } else {
    if constexpr (st) gl_store<T, RE>(Pl, ws + WS_PLOC * TILE);
    mm<T, false, RE>(A2, slot<T, 0>(sh, gs), A);
  }
  ck.mark(1);
  // single precision stores A^2 during the next product
  if constexpr (st && !hk) gl_store<T, RE>(A2, ws + WS_A2 * TILE);
  const int K = sc.K;
  if (sizeof(T) == 4 && m == 2 && K >= 16) {
    // r_2(A) by its power series, truncated at degree 4 (the selection rule keeps
    // the tail below u/2): D = r_2(A) - I = rho_1 A + A^2 (rho_2 I + rho_3 A + rho_4 A^2),
    // one product, during which A^2 is stored for the adjoint
    const double* r = a.pade.r2;   // computed once on the host
    put<T, false, RE>(A2, slot<T, 1>(sh, gs));
    __syncthreads();
    ck.mark(2);
    RT<T> Bk;   // A again, from LDS: a register copy here makes this branch spill
    get<T, RE>(Bk, slot<T, 0>(sh, gs));
    rt_copy(R, Bk);
    rt_scale(R, (T)r[1]);
    rt_scale(Bk, (T)r[3]);
    rt_axpy(Bk, (T)r[4], A2);
    rt_add_diag(Bk, (T)r[2]);
    ck.mark(3);
    if constexpr (st)
      mm<T, false, RE>(R, slot<T, 1>(sh, gs), Bk, TileStore<T, RE>{A2, ws + WS_A2 * TILE});
    else
      mm<T, false, RE>(R, slot<T, 1>(sh, gs), Bk);
    if constexpr (st) gl_store<T, RE>(R, ws + WS_S * TILE);
  } else {
  RT<T> V;   // the even part minus I
  RT<T> U;   // the odd part
  if (sizeof(T) == 4 && m == 2) {
    // Pade-2: U = b_1 A, V - I = b_2 A^2, no product
    rt_poly1(V, A2, (T)b[2], T(0));
    rt_copy(U, A);
    rt_scale(U, (T)b[1]);
  } else {
  RT<T> W;
  rt_poly1(W, A2, (T)b[3], (T)b[1]);
  rt_poly1(V, A2, (T)b[2], T(0));
  if (sizeof(T) == 8 && m >= 5) {   // single precision uses m in {2, 3} only
    put<T, false, RE>(A2, slot<T, 1>(sh, gs));
    __syncthreads();
    RT<T> A4;
    rt_zero(A4);
    mm<T, true, RE>(A4, slot<T, 1>(sh, gs), A2);
    rt_axpy(W, (T)b[5], A4);
    rt_axpy(V, (T)b[4], A4);
    if (m == 7) {
      RT<T> A6;
      rt_zero(A6);
      mm<T, true, RE>(A6, slot<T, 1>(sh, gs), A4);
      rt_axpy(W, (T)b[7], A6);
      rt_axpy(V, (T)b[6], A6);
    }
  }
  rt_zero(U);
  if constexpr (st && hk)
    mm<T, true, RE>(U, slot<T, 0>(sh, gs), W, TileStore<T, RE>{A2, ws + WS_A2 * TILE});
  else
    mm<T, true, RE>(U, slot<T, 0>(sh, gs), W);
  }
  // P = I + X_P with X_P = (V - I) + U (in U); Q = I + E_Q with E_Q = (V - I) - U (in V)
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const auto vr = V.re[q], vi = V.im[q];
    V.re[q] = vr - U.re[q]; V.im[q] = vi - U.im[q];
    U.re[q] = vr + U.re[q]; U.im[q] = vi + U.im[q];
  }
  ck.mark(2);
  // X_Q = Q^{-1} - I into V
  if (sizeof(T) == 4 && K >= 16) {
    // Pade-3: Q^{-1} = sum_{k<=5} c_k A^k, the power series of 1/q_3 (its tail
    // is below the unit roundoff by the selection rule); c_0 = 1
    const double* c = a.pade.c3;   // computed once on the host
    put<T, false, RE>(A2, slot<T, 1>(sh, gs));
    __syncthreads();
    RT<T> A4;
    rt_zero(A4);
    mm<T, true, RE>(A4, slot<T, 1>(sh, gs), A2);
    RT<T> odd;
    rt_poly1(odd, A2, (T)c[3], (T)c[1]);
    rt_axpy(odd, (T)c[5], A4);
    rt_poly1(V, A2, (T)c[2], T(0));
    rt_axpy(V, (T)c[4], A4);
    mm<T, true, RE>(V, slot<T, 0>(sh, gs), odd);   // X_Q = even - I + A odd
  } else if (K > 0 && K < 16) {
    // binary Neumann product on MFMA: Q^{-1} = (I + F)(I + F^2)(I + F^4)...,
    // F = I - Q = -E_Q; with X = Q^{-1} - I each level is X += F2 + F2 X
    RT<T> F;
#pragma unroll
    for (int q = 0; q < 4; ++q) { F.re[q] = -V.re[q]; F.im[q] = -V.im[q]; }
    rt_copy(V, F);
    for (int k = 1; k < K; ++k) {
      __syncthreads();
      put<T, false, RE>(F, slot<T, 2>(sh, gs));
      __syncthreads();
      RT<T> F2;
      rt_zero(F2);
      mm<T, true, RE>(F2, slot<T, 2>(sh, gs), F);
      __syncthreads();
      put<T, false, RE>(F2, slot<T, 2>(sh, gs));
      __syncthreads();
      RT<T> T1;
      rt_copy(T1, F2);
      mm<T, true, RE>(T1, slot<T, 2>(sh, gs), V);
      rt_axpy(V, T(1), T1);
      rt_copy(F, F2);
    }
  } else {
    rt_add_diag(V, T(1));
    rt_gj_inverse(V, sh.colbuf);
    rt_add_diag(V, T(-1));
  }
  ck.mark(3);
  if constexpr (st && !hk) gl_store<T, RE>(V, ws + WS_QINV * TILE);
  // D = r_m(A) - I = X_Q + X_P + X_Q X_P (slot 1 may still be read by the
  // inverse's last product in other waves)
  __syncthreads();
  put<T, false, RE>(V, slot<T, 1>(sh, gs));
  __syncthreads();
  rt_copy(R, U);
  rt_axpy(R, T(1), V);
  if constexpr (st && hk)
    mm<T, false, RE>(R, slot<T, 1>(sh, gs), U, TileStore<T, RE>{V, ws + WS_QINV * TILE});
  else
    mm<T, true, RE>(R, slot<T, 1>(sh, gs), U);
  if constexpr (st) gl_store<T, RE>(R, ws + WS_S * TILE);
  }
  ck.mark(4);
  // squarings: (I + D)^2 = I + 2 D + D^2
  for (int k = 0; k < s; ++k) {
    __syncthreads();
    put<T, false, RE>(R, slot<T, 2>(sh, gs));
    __syncthreads();
    RT<T> R2;
    rt_copy(R2, R);
    rt_scale(R2, T(2));
    mm<T, true, RE>(R2, slot<T, 2>(sh, gs), R);
    rt_copy(R, R2);
  }
  ck.mark(5);
}

// The chunk's running product P_loc, kept beyond the compute precision: in FP32
// as an FP64 register tile (dre, dim) together with hi, its rounding to FP32,
// which is the operand the MFMA needs; in FP64 as one tile (hi). With the slice
// in the form I + D the step is P <- P + D hi, so the O(1) part of P is never
// rounded to the compute precision along the chain. (A double-float pair of
// FP32 tiles does the same in fewer registers but needs about five times the
// VALU work per step; measured 1.8 % slower on the forward.)
template <typename T> struct RunProd {
  RT<T> hi;
  double dre[4][4], dim[4][4];   // single precision only
};

template <typename T>
__device__ __forceinline__ void rp_identity(RunProd<T>& P) {
  rt_identity(P.hi);
  if constexpr (sizeof(T) == 4) {
    const Lane L;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        P.dre[q][r] = (L.template row<T>(q, r) == L.col) ? 1.0 : 0.0;
        P.dim[q][r] = 0.0;
      }
  }
}

// P += X (float: accumulated in FP64, hi re-rounded; double: hi += X)
template <typename T>
__device__ __forceinline__ void rp_add(RunProd<T>& P, const RT<T>& X) {
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if constexpr (sizeof(T) == 4) {
        P.dre[q][r] += (double)X.re[q][r];
        P.dim[q][r] += (double)X.im[q][r];
        P.hi.re[q][r] = (float)P.dre[q][r];
        P.hi.im[q][r] = (float)P.dim[q][r];
      } else {
        P.hi.re[q][r] += X.re[q][r];
        P.hi.im[q][r] += X.im[q][r];
      }
    }
}

// P <- P + D P (D in LDS or global scratch at Dm; the product uses hi)
template <typename T, bool RE = false>
__device__ __forceinline__ void chain_step(RunProd<T>& P, const cpx<T>* Dm) {
  RT<T> Pn;
  rt_zero(Pn);
  mm<T, false, RE>(Pn, Dm, P.hi);
  rp_add(P, Pn);
}

template <typename T, bool RE = false, typename H>
__device__ __forceinline__ void chain_step(RunProd<T>& P, const cpx<T>* Dm, const H& hook) {
  RT<T> Pn;
  rt_zero(Pn);
  mm<T, false, RE>(Pn, Dm, P.hi, hook);
  rp_add(P, Pn);
}

// stores P - I (the form of chunk totals), rounded once from the FP64 tile in
// single precision
template <typename T>
__device__ __forceinline__ void rp_store_delta(const RunProd<T>& P, cpx<T>* M) {
  const Lane L;
  RT<T> X;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const T d = (L.template row<T>(q, r) == L.col) ? T(1) : T(0);
      if constexpr (sizeof(T) == 4) {
        X.re[q][r] = (T)(P.dre[q][r] - (double)d);
        X.im[q][r] = (T)P.dim[q][r];
      } else {
        X.re[q][r] = P.hi.re[q][r] - d;
        X.im[q][r] = P.hi.im[q][r];
      }
    }
  rt_store<T, false>(X, M, 64);
}

template <typename T>
__device__ __forceinline__ int grab(Shared<T>& sh, int* counter) {
  __syncthreads();
  if (threadIdx.x == 0) sh.sidx = atomicAdd(counter, 1);
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(sh.sidx);
}

// ST: store the per-slice workspace for the adjoint. A separate instantiation:
// with the stores behind a run-time test, the compiler's count of memory
// operations in flight is that of the path without them, and the first use of
// the prefetched Omega tile would also wait for every store.
template <typename T, bool ST, bool RE = false>
__global__ void __launch_bounds__(WG, 1) k_forward(SliceArgs a) {
  __shared__ Shared<T> sh;
  cpx<T>* gs = a.gscratch ? reinterpret_cast<cpx<T>*>(a.gscratch) + (size_t)blockIdx.x * 2 * SLOT
                          : nullptr;
  Clock ck(a.clk, sh.clk);
  for (;;) {
    const int idx = grab(sh, a.counter);
    if (idx >= a.n_chunks) break;
    const Chunk ch = a.chunks[idx];
    RunProd<T> P;
    rp_identity(P);
    RT<T> A;
    gl_load<T, false, RE>(A, tile_at<T>(a.omega, (size_t)ch.first));
    for (int k0 = 0; k0 < ch.count; k0 += CODE_WINDOW) {
      const int k1 = min(ch.count, k0 + CODE_WINDOW);
      CodeWindow cw;
      cw.load(a, ch.first + k0, k1 - k0);
      for (int k = k0; k < k1; ++k) {
        const int n = ch.first + k;
        cpx<T>* ws = ST ? tile_at<T>(a.ws_tiles, (size_t)n * WS_TILES) : nullptr;
        RT<T> D;
        fwd_slice<T, ST, RE>(D, A, P.hi, sh, gs, a, cw.at(k - k0), ws, ck);
        put<T, false, RE>(D, slot<T, 3>(sh, gs));   // slot 3's last reader is the previous chain
        __syncthreads();
        // the next slice's Omega tile, spread over the chain product (the chunk's
        // last slice reloads its own, so that the loads are unconditional)
        chain_step<T, RE>(P, slot<T, 3>(sh, gs),
                          TileLoad<T, false, 0, RE>{A, tile_at<T>(a.omega, (size_t)(k + 1 < ch.count ? n + 1 : n))});
        ck.mark(6);
      }
    }
    rp_store_delta<T>(P, tile_at<T>(a.totals, (size_t)ch.chunk));
  }
  ck.flush(a.clk);
}

// Single precision carries P_loc^T from slice to slice: it is the first tile a
// slice needs, so slice n requests slice n - 1's before its last product.
// Double-precision tiles take twice the registers; there it is loaded in place.
template <typename T> constexpr bool bwd_carry = sizeof(T) == 4;

// One slice backward in the transposed frame. Z holds Z_n^T on entry and
// Z_{n-1}^T on exit. With bwd_carry, Pl and A hold slice n's P_loc^T and
// (Omega_n / 2^s)^T on entry, and on exit those of slice nn (n - 1; at the
// chunk's first slice n itself again: unconditional loads keep the compiler's
// count of operations in flight exact), nx being slice nn's workspace.
// kpack: this thread's compact-K_n^T word (sparse basis), see SparseBasis.
template <typename T, bool RE = false>
__device__ void bwd_slice(RT<T>& Z, RT<T>& Pl, RT<T>& A, Shared<T>& sh, cpx<T>* gs,
                          const SliceArgs& a, int n, uint32_t code, const cpx<T>* ws, int nn,
                          const cpx<T>* nx, Clock& ck, uint32_t kpack) {
  const SliceCode code_n = unpack_code(code);
  const int m = code_n.m, s = code_n.s;
  const double* b = pade_b<T>(a.pade, m);
  const T sc = (T)ldexp(1.0, -s);
  // r_2 by its degree-4 series in the forward: the adjoint differentiates that
  // polynomial and reads A^2 in place of Q^{-1}
  const bool ser2 = sizeof(T) == 4 && m == 2 && code_n.K >= 16;
  // D^T = (r_m(A) - I)^T and (Q^{-1} - I)^T (or A^2). Single precision requests each
  // stored tile one product ahead of its use, spread over that product's
  // k-steps: a wave that requests whole tiles at once stalls on issue (about 4K
  // cycles for three tiles). Double precision loads each where it is needed.
  RT<T> R, Qi;
  ck.mark(10);

  // E = M_n^T / 2^s,  M_n^T = Z_n^T P_loc,n^T
  __syncthreads();
  put<T, false, RE>(Z, slot<T, 0>(sh, gs));
  __syncthreads();
  ck.mark(11);
  RT<T> E;
  rt_zero(E);
  if constexpr (bwd_carry<T>) {
    // (this product and the D product run unpipelined in the complex form,
    // pipelined in the real one: measured faster each)
    if constexpr (RE)   // real mode: Q^{-1} (or A^2) in the second half, three products ahead of its use
      mm<T, true, RE>(E, slot<T, 0>(sh, gs), Pl,
                      Hooks3<TileLoad<T, true, 0, RE>, TileLoad<T, true, 8, RE>, NoHook>{
                          {R, ws + WS_S * TILE}, {Qi, ws + (ser2 ? WS_A2 : WS_QINV) * TILE}, {}});
    else
      mm<T, false, RE>(E, slot<T, 0>(sh, gs), Pl, TileLoad<T, true, 0, RE>{R, ws + WS_S * TILE});
  } else {
    gl_load<T, true, RE>(Pl, ws + WS_PLOC * TILE);
    mm<T, true, RE>(E, slot<T, 0>(sh, gs), Pl);
  }
  if (s) rt_scale(E, sc);
  ck.mark(1);
  if constexpr (!bwd_carry<T>) gl_load<T, true, RE>(A, tile_at<T>(a.omega, (size_t)n));
  __syncthreads();
  put<T, false, RE>(A, slot<T, 0>(sh, gs));
  put<T, false, RE>(E, slot<T, 1>(sh, gs));
  __syncthreads();
  ck.mark(2);
  RT<T> L2;
  rt_zero(L2);
  // real mode: the next slice's P_loc^T arrives during this product (Pl's last
  // use was the E product) and its Omega tile during the next one after A's
  // last use, not in the slice's last product: the loop-carried registers are
  // then complete at the loop's back edge instead of waited for there
  if constexpr (bwd_carry<T> && RE)
    mm<T, true, RE>(L2, slot<T, 0>(sh, gs), E, TileLoad<T, true, 0, RE>{Pl, nx + WS_PLOC * TILE});
  else
    mm<T, true, RE>(L2, slot<T, 0>(sh, gs), E);
  if constexpr (bwd_carry<T> && !RE)
    mm<T, true, RE>(L2, slot<T, 1>(sh, gs), A, TileLoad<T, true, 0, RE>{Qi, ws + (ser2 ? WS_A2 : WS_QINV) * TILE});
  else
    mm<T, true, RE>(L2, slot<T, 1>(sh, gs), A);
  ck.mark(3);
  RT<T> K;
  if (ser2) {
    // the Frechet derivative of the degree-4 polynomial sum_k rho_k A^k:
    // L = rho_1 E + rho_2 L_2 + rho_3 L_3 + rho_4 L_4 with L_3 = L_2 A + A^2 E and
    // L_4 = L_2 A^2 + A^2 L_2, i.e.
    // L = rho_1 E + rho_2 L_2 + L_2 (rho_3 A + rho_4 A^2) + A^2 (rho_3 E + rho_4 L_2).
    // A polynomial's derivative commutes with transposition, so the same formula
    // holds for the transposed operands held here (Qi holds (A^2)^T).
    const double* r = a.pade.r2;
    put<T, false, RE>(L2, slot<T, 2>(sh, gs));
    put<T, false, RE>(Qi, slot<T, 3>(sh, gs));
    __syncthreads();
    ck.mark(4);
    RT<T> Bq, Lq;
    rt_copy(Bq, A);
    rt_scale(Bq, (T)r[3]);
    rt_axpy(Bq, (T)r[4], Qi);
    get<T, RE>(Lq, slot<T, 1>(sh, gs));   // E
    rt_copy(K, Lq);
    rt_scale(K, (T)r[1]);
    rt_axpy(K, (T)r[2], L2);
    rt_scale(Lq, (T)r[3]);
    rt_axpy(Lq, (T)r[4], L2);
    ck.mark(5);
    // both unpipelined in the complex form, pipelined in the real one: measured
    // faster each
    if constexpr (bwd_carry<T> && RE)
      mm<T, true, RE>(K, slot<T, 2>(sh, gs), Bq, TileLoad<T, true, 0, RE>{A, tile_at<T>(a.omega, (size_t)nn)});
    else
      mm<T, false, RE>(K, slot<T, 2>(sh, gs), Bq);
    ck.mark(6);
    mm<T, RE, RE>(K, slot<T, 3>(sh, gs), Lq);
  } else {
  RT<T> W, LW, LV;
  const bool pade2 = sizeof(T) == 4 && m == 2;   // U = b_1 A: L_U = b_1 E, no A^2 needed
  if (pade2) {
    rt_poly1(LV, L2, (T)b[2], T(0));
  } else {
    RT<T> A2;
    gl_load<T, true, RE>(A2, ws + WS_A2 * TILE);
    rt_poly1(W, A2, (T)b[3], (T)b[1]);
    rt_poly1(LW, L2, (T)b[3], T(0));
    rt_poly1(LV, L2, (T)b[2], T(0));
    if (sizeof(T) == 8 && m >= 5) {   // single precision uses m = 3 only
      put<T, false, RE>(A2, slot<T, 2>(sh, gs));
      put<T, false, RE>(L2, slot<T, 3>(sh, gs));
      __syncthreads();
      RT<T> A4, L4;
      rt_zero(A4);
      mm<T, true, RE>(A4, slot<T, 2>(sh, gs), A2);
      rt_zero(L4);
      mm<T, true, RE>(L4, slot<T, 2>(sh, gs), L2);
      mm<T, true, RE>(L4, slot<T, 3>(sh, gs), A2);
      rt_axpy(W, (T)b[5], A4);
      rt_axpy(LW, (T)b[5], L4);
      rt_axpy(LV, (T)b[4], L4);
      if (m == 7) {
        RT<T> T6;
        rt_zero(T6);
        mm<T, true, RE>(T6, slot<T, 3>(sh, gs), A4);   // L2 A4
        mm<T, true, RE>(T6, slot<T, 2>(sh, gs), L4);   // A2 L4
        rt_axpy(LW, (T)b[7], T6);
        rt_axpy(LV, (T)b[6], T6);
        rt_zero(T6);
        mm<T, true, RE>(T6, slot<T, 2>(sh, gs), A4);   // A6
        rt_axpy(W, (T)b[7], T6);
      }
    }
  }
  // L_U = A L_W + E W (Pade-2: b_1 E, E from its copy in LDS)
  ck.mark(4);
  RT<T> LU;
  if (pade2) {
    get<T, RE>(LU, slot<T, 1>(sh, gs));
    rt_scale(LU, (T)b[1]);
  } else {
    rt_zero(LU);
    mm<T, true, RE>(LU, slot<T, 0>(sh, gs), LW);
    mm<T, true, RE>(LU, slot<T, 1>(sh, gs), W);
  }
  ck.mark(5);
  // L_Q = L_V - L_U (into LW), L_P = L_V + L_U (into LU)
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const auto vr = LV.re[q], vi = LV.im[q];
    LW.re[q] = vr - LU.re[q]; LW.im[q] = vi - LU.im[q];
    LU.re[q] = vr + LU.re[q]; LU.im[q] = vi + LU.im[q];
  }
  if constexpr (!bwd_carry<T>) gl_load<T, true, RE>(R, ws + WS_S * TILE);
  // X = L_P - L_Q r_m(A) = (L_P - L_Q) - L_Q D
#pragma unroll
  for (int q = 0; q < 4; ++q) { LU.re[q] -= LW.re[q]; LU.im[q] -= LW.im[q]; }
  __syncthreads();
  put<T, false, RE>(LW, slot<T, 1>(sh, gs));
  if constexpr (!bwd_carry<T>) gl_load<T, true, RE>(Qi, ws + WS_QINV * TILE);
  put<T, false, RE>(Qi, slot<T, 2>(sh, gs));
  __syncthreads();
  ck.mark(6);
  {
    RT<T> Tm;
    rt_zero(Tm);
    if constexpr (bwd_carry<T> && RE)
      mm<T, true, RE>(Tm, slot<T, 1>(sh, gs), R, TileLoad<T, true, 0, RE>{A, tile_at<T>(a.omega, (size_t)nn)});
    else
      mm<T, true, RE>(Tm, slot<T, 1>(sh, gs), R);
#pragma unroll
    for (int q = 0; q < 4; ++q) { LU.re[q] -= Tm.re[q]; LU.im[q] -= Tm.im[q]; }
  }
  // L = Q^{-1} X = X + (Q^{-1} - I) X
  rt_copy(K, LU);
  mm<T, true, RE>(K, slot<T, 2>(sh, gs), LU);
  }
  for (int k = 0; k < s; ++k) {
    __syncthreads();
    put<T, false, RE>(R, slot<T, 0>(sh, gs));
    put<T, false, RE>(K, slot<T, 1>(sh, gs));
    __syncthreads();
    // with R = I + D: K <- R K + K R = 2 K + D K + K D ; D <- 2 D + D D
    RT<T> Kn, Rn;
    rt_copy(Kn, K);
    rt_scale(Kn, T(2));
    mm<T, true, RE>(Kn, slot<T, 0>(sh, gs), K);
    mm<T, true, RE>(Kn, slot<T, 1>(sh, gs), R);
    rt_copy(Rn, R);
    rt_scale(Rn, T(2));
    mm<T, true, RE>(Rn, slot<T, 0>(sh, gs), R);
    rt_copy(K, Kn);
    rt_copy(R, Rn);
  }
  ck.mark(7);
  // K_n^T replaces A_n (whole tile, or only its support positions, compacted,
  // with a sparse basis); the traces Re Tr(K_n B_j) are taken afterwards.
  // Single precision stores it during the last product, together with the
  // next slice's P_loc^T and Omega tile loads.
  cpx<T>* kt = tile_at<T>(a.omega, (size_t)n);
  if constexpr (!bwd_carry<T>) {
    if (a.sp.n_sup > 0) {
#pragma unroll
      for (int st = 0; st < 16; ++st) SupportStore<T>{K, kt, kpack}(st);
    } else {
      rt_store<T, false>(K, kt, 64);
    }
  }
  ck.mark(8);
  // Z_{n-1}^T = S_n^T Z_n^T = Z_n^T + D^T Z_n^T (with s = 0 no wave still reads
  // slot 0 here, but the barrier keeps the waves together: measured faster)
  __syncthreads();
  put<T, false, RE>(R, slot<T, 0>(sh, gs));
  __syncthreads();
  RT<T> Zn;
  rt_copy(Zn, Z);
  if constexpr (bwd_carry<T> && RE) {
    if (a.sp.n_sup > 0)
      mm<T, true, RE>(Zn, slot<T, 0>(sh, gs), Z, SupportStore<T>{K, kt, kpack});
    else
      mm<T, true, RE>(Zn, slot<T, 0>(sh, gs), Z, TileStore<T>{K, kt});
  } else if constexpr (bwd_carry<T>) {
    // P_loc^T (needed first) in the first half of the k-steps, Omega in the second
    const TileLoad<T, true, 0, RE> lp{Pl, nx + WS_PLOC * TILE};
    const TileLoad<T, true, 8, RE> la{A, tile_at<T>(a.omega, (size_t)nn)};
    if (a.sp.n_sup > 0)
      mm<T, true, RE>(Zn, slot<T, 0>(sh, gs), Z,
         Hooks3<SupportStore<T>, TileLoad<T, true, 0, RE>, TileLoad<T, true, 8, RE>>{{K, kt, kpack}, lp, la});
    else
      mm<T, true, RE>(Zn, slot<T, 0>(sh, gs), Z,
         Hooks3<TileStore<T>, TileLoad<T, true, 0, RE>, TileLoad<T, true, 8, RE>>{{K, kt}, lp, la});
  } else {
    mm<T, true, RE>(Zn, slot<T, 0>(sh, gs), Z);
  }
  rt_copy(Z, Zn);
  ck.mark(9);
}

// RC: recompute mode (the chunk's forward is re-run into per-workgroup scratch);
// a separate instantiation so that the stored-workspace kernel carries none of
// its register pressure.
template <typename T, bool RC, bool RE = false>
__global__ void __launch_bounds__(WG, 1) k_backward(SliceArgs a) {
  __shared__ Shared<T> sh;
  cpx<T>* gs = a.gscratch ? reinterpret_cast<cpx<T>*>(a.gscratch) + (size_t)blockIdx.x * 2 * SLOT
                          : nullptr;
  Clock ck(a.clk ? a.clk + 16 : nullptr, sh.clk);
  const uint32_t kpack = a.sp.n_sup > 0 ? a.sp.kpack[threadIdx.x] : 0u;
  for (;;) {
    const int idx = grab(sh, a.counter);
    if (idx >= a.n_chunks) break;
    const Chunk ch = a.chunks[idx];
    cpx<T>* rs = RC ? tile_at<T>(a.rscratch, (size_t)blockIdx.x * a.max_chunk * WS_TILES)
                    : nullptr;
    if (RC) {
      // recompute the chunk's forward into this workgroup's scratch tiles
      RunProd<T> P;
      rp_identity(P);
      RT<T> A;
      gl_load<T, false, RE>(A, tile_at<T>(a.omega, (size_t)ch.first));
      for (int k0 = 0; k0 < ch.count; k0 += CODE_WINDOW) {
        const int k1 = min(ch.count, k0 + CODE_WINDOW);
        CodeWindow cw;
        cw.load(a, ch.first + k0, k1 - k0);
        for (int k = k0; k < k1; ++k) {
          cpx<T>* ws = rs + (size_t)k * WS_TILES * TILE;
          RT<T> D;
          fwd_slice<T, true, RE>(D, A, P.hi, sh, gs, a, cw.at(k - k0), ws, ck);
          if (k + 1 < ch.count) {
            gl_load<T, false, RE>(A, tile_at<T>(a.omega, (size_t)ch.first + k + 1));
            __syncthreads();
            put<T, false, RE>(D, slot<T, 3>(sh, gs));
            __syncthreads();
            chain_step<T, RE>(P, slot<T, 3>(sh, gs));
          }
        }
      }
    }
    auto ws_of = [&](int k) -> const cpx<T>* {
      return rs ? rs + (size_t)k * WS_TILES * TILE
                : tile_at<T>(a.ws_tiles, (size_t)(ch.first + k) * WS_TILES);
    };
    RT<T> Z;
    rt_load<T, true>(Z, tile_at<T>((void*)a.env, (size_t)ch.chunk), 64);
    RT<T> Pl, A;
    if constexpr (bwd_carry<T>) {
      if (RC) __syncthreads();   // the recomputed tiles are read by other threads
      gl_load<T, true, RE>(Pl, ws_of(ch.count - 1) + WS_PLOC * TILE);
      gl_load<T, true, RE>(A, tile_at<T>(a.omega, (size_t)ch.first + ch.count - 1));
      // Wait here, once per chunk, for Z, P_loc and Omega. Otherwise the compiler's
      // count of operations in flight at the loop head is that of this entry
      // path, where nothing follows these loads, and every slice's first wait
      // would also wait for the previous slice's K stores.
      __builtin_amdgcn_s_waitcnt(0);
    }
    ck.mark(0);
    // code windows from the chunk's end: [k0, k1) with k1 - k0 <= 64
    for (int k1 = ch.count; k1 > 0; k1 -= CODE_WINDOW) {
      const int k0 = max(0, k1 - CODE_WINDOW);
      CodeWindow cw;
      cw.load(a, ch.first + k0, k1 - k0);
      for (int k = k1 - 1; k >= k0; --k)
        bwd_slice<T, RE>(Z, Pl, A, sh, gs, a, ch.first + k, cw.at(k - k0), ws_of(k),
                     ch.first + (k > 0 ? k - 1 : 0), ws_of(k > 0 ? k - 1 : 0), ck, kpack);
    }
  }
  ck.flush(a.clk ? a.clk + 16 : nullptr);
}

hipError_t launch_slice_forward(int prec, const SliceArgs& a, int grid, hipStream_t s) {
  const bool st = a.store && a.ws_tiles;
  if (prec == 32 && a.real) {
    if (st) hipLaunchKernelGGL((k_forward<float, true, true>), dim3(grid), dim3(WG), 0, s, a);
    else hipLaunchKernelGGL((k_forward<float, false, true>), dim3(grid), dim3(WG), 0, s, a);
  } else if (prec == 32) {
    if (st) hipLaunchKernelGGL((k_forward<float, true>), dim3(grid), dim3(WG), 0, s, a);
    else hipLaunchKernelGGL((k_forward<float, false>), dim3(grid), dim3(WG), 0, s, a);
  } else {
    if (st) hipLaunchKernelGGL((k_forward<double, true>), dim3(grid), dim3(WG), 0, s, a);
    else hipLaunchKernelGGL((k_forward<double, false>), dim3(grid), dim3(WG), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_omega(int prec, const SliceArgs& a, int n_total, hipStream_t s) {
  if (n_total <= 0) return hipSuccess;
  if (a.sp.n_sup > 0) {
    const dim3 g((n_total + 3) / 4);
    if (prec == 32) hipLaunchKernelGGL(k_omega_sparse<float>, g, dim3(WG), 0, s, a, n_total);
    else hipLaunchKernelGGL(k_omega_sparse<double>, g, dim3(WG), 0, s, a, n_total);
    return hipGetLastError();
  }
  const dim3 g((n_total + OMEGA_SLICES - 1) / OMEGA_SLICES);
  if (prec == 32) hipLaunchKernelGGL(k_omega<float>, g, dim3(WG), 0, s, a, n_total);
  else hipLaunchKernelGGL(k_omega<double>, g, dim3(WG), 0, s, a, n_total);
  return hipGetLastError();
}

hipError_t launch_traces(int prec, const SliceArgs& a, int n_total, hipStream_t s) {
  if (n_total <= 0) return hipSuccess;
  if (a.sp.n_sup > 0) {
    const size_t lds = prec == 32 ? tr_lds_bytes<float>(a.sp.nnz, a.sp.n_sup, a.nb)
                                  : tr_lds_bytes<double>(a.sp.nnz, a.sp.n_sup, a.nb);
    if (lds <= TR_LDS_MAX && a.nb <= 32) {
      const dim3 g((n_total + TR_SPB - 1) / TR_SPB);
      const bool four = a.nb <= 16;   // lanes per basis element: 64 / nb, a power of two
      if (prec == 32) {
        if (four) hipLaunchKernelGGL((k_traces_lds<float, 4>), g, dim3(WG), lds, s, a, n_total);
        else hipLaunchKernelGGL((k_traces_lds<float, 2>), g, dim3(WG), lds, s, a, n_total);
      } else {
        if (four) hipLaunchKernelGGL((k_traces_lds<double, 4>), g, dim3(WG), lds, s, a, n_total);
        else hipLaunchKernelGGL((k_traces_lds<double, 2>), g, dim3(WG), lds, s, a, n_total);
      }
      return hipGetLastError();
    }
    const dim3 g((n_total + 3) / 4);
    if (prec == 32) hipLaunchKernelGGL(k_traces_sparse<float>, g, dim3(WG), 0, s, a, n_total);
    else hipLaunchKernelGGL(k_traces_sparse<double>, g, dim3(WG), 0, s, a, n_total);
    return hipGetLastError();
  }
  const dim3 g((n_total + TRACE_SLICES - 1) / TRACE_SLICES);
  if (prec == 32) hipLaunchKernelGGL(k_traces<float>, g, dim3(WG), 0, s, a, n_total);
  else hipLaunchKernelGGL(k_traces<double>, g, dim3(WG), 0, s, a, n_total);
  return hipGetLastError();
}

hipError_t launch_slice_backward(int prec, const SliceArgs& a, int grid, hipStream_t s) {
  if (prec == 32 && a.real) {
    if (a.recompute) hipLaunchKernelGGL((k_backward<float, true, true>), dim3(grid), dim3(WG), 0, s, a);
    else hipLaunchKernelGGL((k_backward<float, false, true>), dim3(grid), dim3(WG), 0, s, a);
  } else if (prec == 32) {
    if (a.recompute) hipLaunchKernelGGL((k_backward<float, true>), dim3(grid), dim3(WG), 0, s, a);
    else hipLaunchKernelGGL((k_backward<float, false>), dim3(grid), dim3(WG), 0, s, a);
  } else {
    if (a.recompute) hipLaunchKernelGGL((k_backward<double, true>), dim3(grid), dim3(WG), 0, s, a);
    else hipLaunchKernelGGL((k_backward<double, false>), dim3(grid), dim3(WG), 0, s, a);
  }
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
// exp of one tile: k_omega (basis = A, alpha = 1, writes A / 2^s into gs and
// (m, s)) followed by the forward slice routine.
template <typename T>
__global__ void __launch_bounds__(WG, 1) k_debug_expm2(cpx<T>* C, cpx<T>* gs, SliceArgs a) {
  __shared__ Shared<T> sh;
  Clock ck(nullptr, sh.clk);
  RT<T> R, A;
  rt_load<T, false>(A, tile_at<T>(a.omega, 0), 64);
  fwd_slice<T, false>(R, A, A, sh, gs + 2 * SLOT, a, slice_code(a, 0), nullptr, ck);
  rt_add_diag(R, T(1));
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

// gscratch holds 4 slots of 16-byte elements: [0, SLOT) the scaled tile, [2 SLOT, 4 SLOT)
// the double-precision scratch slots.
hipError_t launch_debug_expm(int prec, const void* A, void* C, int8_t* ms, void* gscratch, PadeTable pt, hipStream_t s) {
  double* one = nullptr;
  hipError_t e = hipGetSymbolAddress((void**)&one, HIP_SYMBOL(g_one_alpha));
  if (e != hipSuccess) return e;
  SliceArgs a{};
  a.basis = A; a.nb = 1; a.alpha = one; a.ms = ms; a.pade = pt; a.omega = gscratch;
  a.nlev = (int8_t*)gscratch + 65536;   // past the 64x64 tile, inside slot 0
  a.store = 0; a.ws_tiles = nullptr;
  e = launch_omega(prec, a, 1, s);
  if (e != hipSuccess) return e;
  if (prec == 32)
    hipLaunchKernelGGL(k_debug_expm2<float>, dim3(1), dim3(WG), 0, s, (cpx<float>*)C,
                       (cpx<float>*)gscratch, a);
  else
    hipLaunchKernelGGL(k_debug_expm2<double>, dim3(1), dim3(WG), 0, s, (cpx<double>*)C,
                       (cpx<double>*)gscratch, a);
  return hipGetLastError();
}

}  // namespace lmag
