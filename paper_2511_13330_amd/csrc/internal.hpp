// Internal declarations shared by the host library and the kernel files.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace lmag {

// Pade coefficients b_j = (2m-j)! m! / ((2m)! j! (m-j)!), j = 0..m, and the
// scaling thresholds theta_m, for the degrees this library evaluates.
struct PadeTable {
  double b2[3], b3[4], b5[6], b7[8];
  double ser_max32_2, ser_max32_3;   // largest ||A||_1 for the series of r_2, of 1/q_3 (FP32)
  double r2[8], c3[8];               // power series of r_2, of 1/q_3 (both 1 at degree 0), degrees 0..7
};

// Sparse form of a 64 x 64 basis (built by set_system from its nonzero entries
// B_j[x], x = row * 64 + col). Support positions p (the union of the basis
// supports) are numbered column by column, by ascending row. n_sup = 0 means
// the dense kernels are used (a column with more than SP_COLCAP support rows).
constexpr int SP_COLCAP = 16;
struct SparseBasis {
  int n_sup, nnz;
  const int32_t* col_ptr;   // [65] support positions of column c
  const uint8_t* sup_row;   // [n_sup] row of each support position
  const int32_t* sup_eptr;  // [n_sup + 1] entries of position p: [sup_eptr[p], sup_eptr[p + 1])
  const uint8_t* pe_j;      // [nnz] position-ordered entries (ascending j within a position)
  const void* pe_val;       // [nnz] complex value, compute type
  // Compact K_n^T: the support positions in register-tile order (thread by
  // thread, each thread's registers in order), so a thread's entries are
  // consecutive. kpack[t] = (first slot << 16) | (mask of its 16 registers).
  const uint32_t* kpack;    // [256]
  const int32_t* ptr_j;     // [nb + 1] j-ordered entries of B_j: [ptr_j[j], ptr_j[j + 1])
  const uint16_t* ent_slot; // [nnz] compact slot of each j-ordered entry's position
  const void* ent_val;      // [nnz] complex value, compute type
};

// One chunk of consecutive slices of one item; the unit of work of the slice
// kernels. Slices are numbered globally over the whole call.
struct Chunk {
  int32_t item;        // item index
  int32_t first;       // first global slice index
  int32_t count;       // number of slices
  int32_t chunk;       // global chunk index (into chunk-level arrays)
};

struct Item {
  int32_t first_chunk; // global index of the item's first chunk
  int32_t n_chunks;
  int32_t first_slice; // global index of the item's first slice
  int32_t n_slices;
  int32_t target;      // target index (fidelity calls)
  int32_t group;       // group index or -1
  int32_t src;         // index of the item in the caller's batch
};

// Per-slice workspace tiles (row-major 64x64 complex of the compute type):
// D = r_m(A) - I before the squarings, the chunk's running product before the
// slice, Q^{-1} - I (not written where single precision evaluates r_2 by its
// series), and A^2.
enum { WS_S = 0, WS_PLOC = 1, WS_QINV = 2, WS_A2 = 3, WS_TILES = 4 };

struct SliceArgs {
  const void* basis;        // [nb][64][64] complex, compute type
  int nb;
  const double* alpha;      // [n_slices_total][nb]
  const Chunk* chunks;
  int n_chunks;
  int* counter;             // persistent work counter (zeroed before launch)
  void* ws_tiles;           // [n_slices_total][WS_TILES][64][64] (may be null for propagate)
  int store;                // forward: store per-slice tiles
  void* totals;             // [n_chunks][64][64] chunk products (forward output)
  const void* env;          // [n_chunks][64][64] chunk environments W_c (backward input)
  double* gtrace;           // [n_slices_total][nb] Re Tr(K_n B_j) (backward output)
  int8_t* ms;               // [n_slices_total][2] Pade degree and scaling exponent
  int8_t* nlev;             // [n_slices_total] inverse variant code (see inverse_code)
  int inv_mode;             // 0 automatic; 2 no power series (Neumann or Gauss-Jordan)
  void* gscratch;           // per-workgroup global scratch slots (double precision)
  void* omega;              // [n_slices_total][64][64]: Omega_n / 2^s, then K_n^T (backward;
                            // with a sparse basis only its support positions, compacted)
  long long* clk;           // [32] per-phase cycle counters of workgroup 0, or null
  int recompute;            // backward recomputes each chunk's forward tiles
  int real;                 // FP32 tiles in the basis of Hermitian operators: every tile
                            // is real (zero imaginary parts), one MFMA product each
  void* rscratch;           // [grid][max_chunk][WS_TILES] tiles (recompute mode)
  int max_chunk;            // slices per chunk (scratch stride)
  PadeTable pade;
  SparseBasis sp;           // sparse basis (Omega build, compact K_n^T, traces), or n_sup = 0
};

// launchers (kernel files)
hipError_t launch_slice_forward(int prec, const SliceArgs& a, int grid, hipStream_t s);
hipError_t launch_slice_backward(int prec, const SliceArgs& a, int grid, hipStream_t s);
hipError_t launch_omega(int prec, const SliceArgs& a, int n_total, hipStream_t s);
hipError_t launch_traces(int prec, const SliceArgs& a, int n_total, hipStream_t s);

// system set-up (double precision, padded to 64x64 tiles)
hipError_t launch_lift(const double* H, int d, double* out, hipStream_t s);
hipError_t launch_dissipator(const double* Ls, int n_jump, int d, double* out, hipStream_t s);
hipError_t launch_commutator(const double* X, const double* Y, double* out, hipStream_t s);
hipError_t launch_cast(const double* in, float* out, size_t n, hipStream_t s);
hipError_t launch_fill_int(int* p, int v, int n, hipStream_t s);

struct AlphaArgs {
  int prec;
  const void* amps;          // [total_slices_in_amps][n_ctrl] of the compute type
  const int64_t* item_amp_offset;   // [n_items] slice offset into amps
  const Item* items;
  int n_items;
  const void* static_coef;  // [n_items][n_static] or null (zeros)
  const void* ctrl_scale;   // [n_items][n_ctrl] or null (ones)
  int n_ctrl, n_static, order, hold_foh, nb;
  double dt;
  const int32_t* slice_item;  // [n_slices_total] item of each global slice
  double* alpha;            // out [n_slices_total][nb]
  int n_slices_total;
};
hipError_t launch_alpha(const AlphaArgs& a, hipStream_t s);
// sixth-order slices: coefficient planes [3][n_slices_total][nb] of a1, a2, a3
hipError_t launch_alpha6(const AlphaArgs& a, hipStream_t s);

struct TargetArgs {
  const double* U;          // [n_targets][d][d] complex128
  int n_targets, d;
  double* st64;             // out [n_targets][64][64] complex: S_T^dagger (padded)
  float* st32;              // out, same in float (may be null)
};
hipError_t launch_targets(const TargetArgs& a, hipStream_t s);

// Logical-subspace scores: Pi = P^dag U P (L x L) per item, from the item's
// total U = I + X (stored as X); score s and the seed M (ds = Re Tr(M dU))
// written where the target tiles go, one per item.
constexpr int MAX_LOGICAL = 4;
struct LogicalArgs {
  int prec;
  const Item* items;
  int n_items;
  const void* pre;          // inclusive prefixes (X = U - I at each item's last chunk)
  int kind;                 // 1: ||Pi - T||_F^2, 2: Re Tr(T^dag Pi) / L
  int L;
  const double* P;          // [64][L] complex, row i = superoperator index
  const double* T;          // [n_targets][L][L] complex, row-major
  double* score;            // out, indexed like EnvArgs::F (f_by_src)
  int f_by_src;
  double* st64;             // out [n_items][64][64] complex seed M
  float* st32;              // out, same in float (may be null)
  int real;                 // basis of Hermitian operators: P holds T P, and the seed
                            // keeps its real part (the gradient of a real map)
};
hipError_t launch_logical(const LogicalArgs& a, hipStream_t s);

struct ScanArgs {
  int prec;
  const Item* items;
  int n_items;
  int n_chunks_total;
  int step;                 // 2^k
  const void* pre_in; void* pre_out;   // inclusive prefix arrays [n_chunks][64][64]
  const void* suf_in; void* suf_out;   // inclusive suffix arrays (null = skip)
};
hipError_t launch_scan_level(const ScanArgs& a, const int32_t* chunk_item, hipStream_t s);

struct EnvArgs {
  int prec;
  const Item* items;
  int n_items;
  const int32_t* chunk_item;   // [n_chunks]
  int n_chunks_total;
  const void* pre;          // inclusive prefixes
  const void* suf;          // inclusive suffixes
  const void* st;           // S_T^dagger tiles [n_targets][64][64] compute type
  const double* st64;       // same in double
  void* env;                // out W_c [n_chunks][64][64]
  double* F;                // out (Re), may be null
  double* Fim;              // out (Im), may be null
  int f_by_src;             // index F / Fim by the caller's item index
  int seed_by_item;         // st tiles are per item (logical scores), not per target
  int d;
};
hipError_t launch_env(const EnvArgs& a, hipStream_t s);

struct ExtractArgs {
  int prec;
  const Item* items;
  int n_items;
  const void* pre;          // inclusive prefixes; item total at its last chunk
  void* out;                // [n_items][n][n] complex
  int n;
};
hipError_t launch_extract(const ExtractArgs& a, hipStream_t s);

struct GradArgs {
  int prec;
  const double* gtrace;     // [n_slices_total][nb]
  const void* amps;
  const int64_t* item_amp_offset;
  const Item* items;
  int n_items;
  const void* static_coef;
  const void* ctrl_scale;
  int n_ctrl, n_static, order, hold_foh, nb;
  double dt, inv_d2;
  int n_slices_total;       // sixth order: stride of the three trace planes
  void* grad;               // out, like amps (per item) or per group
  const int32_t* group_first_item;  // [n_groups+1] items sorted by group (null = no groups)
  const int32_t* group_items;       // [n_items]
  int n_groups;
  double* F_items;          // [n_items] per-item fidelity (group mean input)
  double* F_out;            // [n_groups] group means (grouped calls)
  const int32_t* group_global;      // [n_groups] caller's group index of each local group
};
hipError_t launch_grad(const GradArgs& a, int max_slices, hipStream_t s);

struct AdamArgs {
  int64_t n;                // number of parameters
  int64_t row_len;          // parameters per row (row_active granularity)
  void* theta; const void* grad; void* m; void* v;   // compute type
  double lr, beta1, beta2, eps, bc1, bc2, grad_scale, lo, hi;
  const uint8_t* row_active;  // [n / row_len] or null
};
hipError_t launch_adam_project(int prec, const AdamArgs& a, hipStream_t s);

// learned proposal (MLP) kernels
enum { MLP_STORE = 0, MLP_BIAS_GELU = 1, MLP_BIAS_SIGMOID = 2, MLP_GELU_GRAD = 3 };
struct MlpGemmArgs {
  int M, N, K;
  const uint16_t* A; int64_t lda_r, lda_c;   // A(i,k) = A[i*lda_r + k*lda_c] (bf16)
  const uint16_t* B; int64_t ldb_r, ldb_c;   // B(k,j) = B[k*ldb_r + j*ldb_c] (bf16)
  int mode;
  const float* bias;        // [N]
  const float* aux;         // [M][N] pre-activation of the previous layer (GELU_GRAD)
  float scale;              // head scale
  float* C32;               // [M][N] fp32 output (pre-activation / gradient), may be null
  uint16_t* C16;            // [M][N] bf16 output
  float* Y32;               // [M][N] head output
};
hipError_t launch_mlp_gemm(const MlpGemmArgs& a, hipStream_t s);
hipError_t launch_colsum(const float* G, int rows, int cols, float* out, hipStream_t s);
hipError_t launch_mse(const float* z, const float* y, int64_t n, float* dz32, uint16_t* dz16,
                      double* part, double* loss, hipStream_t s);
hipError_t launch_cast_bf16(const float* in, uint16_t* out, int64_t n, hipStream_t s);

// debug / unit-test kernels (single 64x64 tiles)
hipError_t launch_debug_gemm(int prec, const void* A, const void* B, void* C, int transA, hipStream_t s);
hipError_t launch_debug_inverse(int prec, const void* A, void* C, hipStream_t s);
hipError_t launch_debug_expm(int prec, const void* A, void* C, int8_t* ms, void* gscratch, PadeTable pt, hipStream_t s);

}  // namespace lmag
